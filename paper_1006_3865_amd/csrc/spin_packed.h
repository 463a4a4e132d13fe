// spin_packed.h -- the byte-parallel Metropolis update of an aligned 8-site
// group with the four sites of the active colour packed into one dword (the
// row-streaming 2D and plane-streaming 3D kernels).  Same decisions as
// unsat_ising / apply_group in spin_device.h, in fewer operations.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "spin_device.h"

namespace spin {

// Packed form of the update: the four active sites of the group (bytes P,
// P+2, P+4, P+6) gathered into one dword, byte m = site 8g + P + 2m, so that
// each neighbour term is one operation for all four sites.  The other-colour
// bytes of the group I are the neighbours on one side; the other side is I
// moved by one byte with the boundary byte of lw (P = 0: left neighbours
// x-1) or rw (P = 1: right neighbours x+1) shifted in.  Row and plane
// neighbours sit at the active positions of their own dwords.
//   v_perm_b32 selectors (bytes 0-3 of the second operand, 4-7 of the first):
//   even bytes 0x06040200, odd bytes 0x07050301; the shifted dword takes
//   (lw byte 3, I0, I1, I2) = 0x06050403 for P = 0 and (I1, I2, I3, rw byte 0)
//   = 0x00070605 for P = 1 from perm(I, P ? rw : lw).
__device__ __forceinline__ uint32_t gather_bytes(uint32_t lo, uint32_t hi, uint32_t sel) {
  return __builtin_amdgcn_perm(hi, lo, sel);
}

// Selector of the bytes of parity P of an 8-byte group.
__device__ __forceinline__ uint32_t sel_active(uint32_t P) { return P ? 0x07050301u : 0x06040200u; }

// 4u per active site, packed (u = unsatisfied bonds among the 2 + NO neighbours).
template <int NO>
__device__ __forceinline__ uint32_t unsat_packed(uint32_t P, uint32_t c0, uint32_t c1, uint32_t lw, uint32_t rw,
                                                 const uint32_t (&o0)[NO], const uint32_t (&o1)[NO]) {
  const uint32_t sa = sel_active(P), so = sel_active(P ^ 1u);
  const uint32_t A = gather_bytes(c0, c1, sa);
  const uint32_t I = gather_bytes(c0, c1, so);
  const uint32_t N = __builtin_amdgcn_perm(I, P ? rw : lw, P ? 0x00070605u : 0x06050403u);
  uint32_t S = ((A ^ I) & kSignBit) + ((A ^ N) & kSignBit);
#pragma unroll
  for (int i = 0; i < NO; ++i) S += (A ^ gather_bytes(o0[i], o1[i], sa)) & kSignBit;
  return S;
}

// Accept decision for the 4u value i4 and word r: the flip mask m or 0.
template <bool NEVER>
__device__ __forceinline__ uint32_t flip_mask(uint32_t i4, uint32_t r, uint32_t m, const uint32_t* bound_lds,
                                              uint32_t never4) {
  const uint32_t b = *(const uint32_t*)((const char*)bound_lds + i4);
  bool acc = r <= b;
  if (NEVER) acc = acc && (i4 >= never4);
  return acc ? m : 0u;
}

// Apply the four decisions of a packed 4u dword to the group (word r[m] for
// packed byte m, i.e. site 8g + P + 2m).  Byte 1 is extracted by v_perm_b32
// (selector 0x0C gives a zero byte), one operation where a shift and a mask
// would take two.
template <bool NEVER>
__device__ __forceinline__ void apply_packed(uint32_t P, uint32_t& c0, uint32_t& c1, uint32_t S,
                                             const uint32_t r[4], const uint32_t* bound_lds, uint32_t never4) {
  const uint32_t ma = 0xFEu << (8u * P), mb = 0xFEu << (8u * P + 16u);
  const uint32_t f0 = flip_mask<NEVER>(S & 0xFFu, r[0], ma, bound_lds, never4);
  const uint32_t f1 = flip_mask<NEVER>(__builtin_amdgcn_perm(0u, S, 0x0C0C0C01u), r[1], mb, bound_lds, never4);
  const uint32_t f2 = flip_mask<NEVER>(__builtin_amdgcn_ubfe(S, 16u, 8u), r[2], ma, bound_lds, never4);
  const uint32_t f3 = flip_mask<NEVER>(S >> 24, r[3], mb, bound_lds, never4);
  c0 = xor3(c0, f0, f1);
  c1 = xor3(c1, f2, f3);
}

// apply_packed that also adds to acc four times the number of unsatisfied
// bonds of the four active sites after the update (D: lattice dimension).
// S holds 4u per site before it; a flipped site has 2D - u unsatisfied bonds
// afterwards (every one of its bonds changes), so its byte becomes 8D - S_m
// (no byte borrows: S_m <= 8D).  One v_sad_u8 against zero sums the bytes.
template <bool NEVER, int D>
__device__ __forceinline__ void apply_packed_count(uint32_t P, uint32_t& c0, uint32_t& c1, uint32_t S,
                                                   const uint32_t r[4], const uint32_t* bound_lds, uint32_t never4,
                                                   uint32_t& acc) {
  const uint32_t ma = 0xFEu << (8u * P), mb = 0xFEu << (8u * P + 16u);
  const uint32_t f0 = flip_mask<NEVER>(S & 0xFFu, r[0], ma, bound_lds, never4);
  const uint32_t f1 = flip_mask<NEVER>(__builtin_amdgcn_perm(0u, S, 0x0C0C0C01u), r[1], mb, bound_lds, never4);
  const uint32_t f2 = flip_mask<NEVER>(__builtin_amdgcn_ubfe(S, 16u, 8u), r[2], ma, bound_lds, never4);
  const uint32_t f3 = flip_mask<NEVER>(S >> 24, r[3], mb, bound_lds, never4);
  const uint32_t d0 = f0 ^ f1, d1 = f2 ^ f3;
  c0 ^= d0;
  c1 ^= d1;
  const uint32_t F = gather_bytes(d0, d1, sel_active(P));  // 0xFE at the packed sites that flipped
  constexpr uint32_t K = 0x01010101u * (8u * (uint32_t)D);
  const uint32_t Sf = S ^ ((S ^ (K - S)) & F);
  acc = __builtin_amdgcn_sad_u8(Sf, 0u, acc);
}

}  // namespace spin
