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

// 4u per active site, packed (u = unsatisfied bonds among the 2 + NO neighbours);
// 8u with SB = kSignBit8 (bit 3 of each byte carries the sign as well).
constexpr uint32_t kSignBit8 = 0x08080808u;

template <int NO, uint32_t SB = kSignBit>
__device__ __forceinline__ uint32_t unsat_packed(uint32_t P, uint32_t c0, uint32_t c1, uint32_t lw, uint32_t rw,
                                                 const uint32_t (&o0)[NO], const uint32_t (&o1)[NO]) {
  const uint32_t sa = sel_active(P), so = sel_active(P ^ 1u);
  const uint32_t A = gather_bytes(c0, c1, sa);
  const uint32_t I = gather_bytes(c0, c1, so);
  const uint32_t N = __builtin_amdgcn_perm(I, P ? rw : lw, P ? 0x00070605u : 0x06050403u);
  uint32_t S = ((A ^ I) & SB) + ((A ^ N) & SB);
#pragma unroll
  for (int i = 0; i < NO; ++i) S += (A ^ gather_bytes(o0[i], o1[i], sa)) & SB;
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

// Pair table: the bounds of two packed sites in one 8-byte LDS entry.  With
// 8u per byte, the low 16 bits of the packed dword, 8 u0 + 2048 u1, are the
// byte offset of the entry {bound[u0], bound[u1]} of packed sites 0 and 1, the
// high 16 bits that of sites 2 and 3: two shifts or masks and two 8-byte LDS
// reads where the 4u form takes four extractions and four reads.  Z is the
// largest u (the coordination number); the table spans pair_words(Z) dwords.
constexpr uint32_t pair_words(int Z) { return 2u * (uint32_t)Z + 512u * (uint32_t)Z + 2u; }

template <int Z>
__device__ __forceinline__ void fill_pair(uint32_t* pair, const uint32_t* bound, uint32_t t) {
  if (t < (uint32_t)((Z + 1) * (Z + 1))) {
    const uint32_t u0 = t % (uint32_t)(Z + 1), u1 = t / (uint32_t)(Z + 1);
    pair[2u * u0 + 512u * u1] = bound[u0];
    pair[2u * u0 + 512u * u1 + 1u] = bound[u1];
  }
}

// The two pair-table entries of a packed dword S of 8u values: the bounds of
// packed sites 0..3 (byte address pair_lds).
__device__ __forceinline__ uint4 lookup_pair(uint32_t S, const char* pair_lds) {
  const uint2 b01 = *(const uint2*)(pair_lds + (S & 0xFFFFu));
  const uint2 b23 = *(const uint2*)(pair_lds + (S >> 16));
  return make_uint4(b01.x, b01.y, b23.x, b23.y);
}

// Parity-split form of an 8-site group: x = its even bytes (sites 8g, 8g+2,
// 8g+4, 8g+6), y = its odd bytes, so that the active sites of either colour
// are one dword as they stand and a row neighbour's are the same half of its
// group.  Loaded groups are split once, stored groups joined once.
__device__ __forceinline__ uint2 split_group(uint32_t c0, uint32_t c1) {
  return make_uint2(gather_bytes(c0, c1, 0x06040200u), gather_bytes(c0, c1, 0x07050301u));
}
__device__ __forceinline__ uint2 join_group(uint2 s) {
  return make_uint2(gather_bytes(s.x, s.y, 0x05010400u), gather_bytes(s.x, s.y, 0x07030602u));
}

// Decisions of a packed dword of 8u values S (bounds b from lookup_pair) applied to the
// active half A of a parity-split group: byte m of A is packed site m.
template <bool NEVER>
__device__ __forceinline__ uint32_t apply_split(uint32_t A, uint32_t S, uint4 b, const uint32_t r[4],
                                                uint32_t never8) {
  bool a0 = r[0] <= b.x, a1 = r[1] <= b.y, a2 = r[2] <= b.z, a3 = r[3] <= b.w;
  if (NEVER) {
    a0 = a0 && (S & 0xFFu) >= never8;
    a1 = a1 && __builtin_amdgcn_perm(0u, S, 0x0C0C0C01u) >= never8;
    a2 = a2 && __builtin_amdgcn_ubfe(S, 16u, 8u) >= never8;
    a3 = a3 && (S >> 24) >= never8;
  }
  return xor3(xor3(A, a0 ? 0xFEu : 0u, a1 ? 0xFE00u : 0u), a2 ? 0xFE0000u : 0u, a3 ? 0xFE000000u : 0u);
}

// apply_split that also adds to acc four times the number of unsatisfied
// bonds of the four active sites after the update (D: lattice dimension): a
// flipped site has 2D - u unsatisfied bonds afterwards (every one of its bonds
// changes), so its byte becomes 16D - S_m (no byte borrows: S_m <= 16D); the
// bytes are multiples of 8, so halving the dword halves every byte without a
// carry from the byte above, and one v_sad_u8 against zero sums them.  The
// flip mask of the packed sites is the XOR itself.
template <bool NEVER, int D>
__device__ __forceinline__ uint32_t apply_split_count(uint32_t A, uint32_t S, uint4 b, const uint32_t r[4],
                                                      uint32_t never8, uint32_t& acc) {
  bool a0 = r[0] <= b.x, a1 = r[1] <= b.y, a2 = r[2] <= b.z, a3 = r[3] <= b.w;
  if (NEVER) {
    a0 = a0 && (S & 0xFFu) >= never8;
    a1 = a1 && __builtin_amdgcn_perm(0u, S, 0x0C0C0C01u) >= never8;
    a2 = a2 && __builtin_amdgcn_ubfe(S, 16u, 8u) >= never8;
    a3 = a3 && (S >> 24) >= never8;
  }
  const uint32_t F = xor3(a0 ? 0xFEu : 0u, a1 ? 0xFE00u : 0u, a2 ? 0xFE0000u : 0u) ^ (a3 ? 0xFE000000u : 0u);
  constexpr uint32_t K = 0x01010101u * (16u * (uint32_t)D);
  const uint32_t Sf = S ^ ((S ^ (K - S)) & F);
  acc = __builtin_amdgcn_sad_u8(Sf >> 1, 0u, acc);
  return A ^ F;
}

}  // namespace spin
