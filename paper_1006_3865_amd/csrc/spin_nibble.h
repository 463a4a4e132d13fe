// spin_nibble.h -- 8 sites per 32-bit word (4 bits per site) and the
// Metropolis update of such words, shared by the LDS-resident batch kernel
// and the general streaming kernel.
//
// Site 8w+j is nibble j of word w: +1 = 0x1, -1 = 0xF (the low nibble of the
// int8 value), so bits 1..3 of a nibble carry the sign.  (a ^ b) & 0x2 per
// nibble marks an unsatisfied bond (with a coupling nibble, +1 = 0x1 and
// -1 = 0xF, in the XOR for the +-J glass), the sum over the 2d neighbours is
// 2u per nibble (u <= 6), and a flip XORs the nibble with 0xE.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "spin_device.h"

namespace spin {

// int8 spins (0x01 / 0xFF) of 8 consecutive sites <-> one word of nibbles
// (0x1 / 0xF, site j in nibble j).
__device__ __forceinline__ uint32_t pack_nibbles(uint32_t lo, uint32_t hi) {
  uint32_t a = lo & 0x0F0F0F0Fu, b = hi & 0x0F0F0F0Fu;
  a = (a | (a >> 4)) & 0x00FF00FFu;
  b = (b | (b >> 4)) & 0x00FF00FFu;
  a = (a | (a >> 8)) & 0x0000FFFFu;
  b = (b | (b >> 8)) & 0x0000FFFFu;
  return a | (b << 16);
}

__device__ __forceinline__ uint32_t nibbles_to_bytes(uint32_t h) {  // 4 nibbles -> 4 bytes
  uint32_t x = h & 0xFFFFu;
  x = (x | (x << 8)) & 0x00FF00FFu;
  x = (x | (x << 4)) & 0x0F0F0F0Fu;
  const uint32_t neg = (x >> 3) & 0x01010101u;
  return 0x01010101u + (neg << 8) - (neg << 1);  // 0x01 or 0xFF per byte
}

__device__ __forceinline__ void unpack_nibbles(uint32_t w, uint32_t& lo, uint32_t& hi) {
  lo = nibbles_to_bytes(w);
  hi = nibbles_to_bytes(w >> 16);
}

// Unsatisfied-bond count (2u per nibble) of word c with neighbour words.
template <int D, bool EA>
__device__ __forceinline__ uint32_t nib_unsat(uint32_t c, uint32_t lw, uint32_t rw, const uint32_t (&nb)[2 * D - 2],
                                              const uint32_t (&jn)[2 * D]) {
  constexpr uint32_t m = 0x22222222u;
  const uint32_t Lx = __builtin_amdgcn_alignbit(c, lw, 28);  // site x-1 of each nibble
  const uint32_t Rx = __builtin_amdgcn_alignbit(rw, c, 4);   // site x+1
  uint32_t S;
  if (EA) {
    S = (xor3(c, Lx, jn[0]) & m) + (xor3(c, Rx, jn[1]) & m);
#pragma unroll
    for (int k = 0; k < 2 * D - 2; ++k) S += xor3(c, nb[k], jn[2 + k]) & m;
  } else {
    S = ((c ^ Lx) & m) + ((c ^ Rx) & m);
#pragma unroll
    for (int k = 0; k < 2 * D - 2; ++k) S += (c ^ nb[k]) & m;
  }
  return S;
}

// Flip mask (0xE per flipped nibble) for the active nibbles p, p+2, p+4, p+6:
// S is shifted so the active nibbles sit at 0, 2, 4, 6 (constant offsets),
// their 2u values doubled into one byte each (4u: the bound table's byte
// offset, at most 24), the bytes taken out one operation each, and the mask
// shifted back.
template <bool NEVER>
__device__ __forceinline__ uint32_t nib_flips(uint32_t S, uint32_t p, const uint32_t r[4],
                                              const uint32_t* bound, uint32_t never4) {
  const uint32_t T = ((S >> (4u * p)) & 0x0F0F0F0Fu) << 1;  // byte i: 4u of active nibble i
  const uint32_t i4[4] = {T & 0xFFu, __builtin_amdgcn_perm(0u, T, 0x0C0C0C01u), __builtin_amdgcn_ubfe(T, 16u, 8u),
                          T >> 24};
  uint32_t f[4];
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const uint32_t b = *(const uint32_t*)((const char*)bound + i4[i]);
    bool acc = r[i] <= b;
    if (NEVER) acc = acc && (i4[i] >= never4);
    f[i] = acc ? (0xEu << (8 * i)) : 0u;
  }
  return (xor3(f[0], f[1], f[2]) ^ f[3]) << (4u * p);
}

// Global-address-space view of a device pointer (loads with a 32-bit offset
// from a scalar base instead of 64-bit flat addresses).
typedef const __attribute__((address_space(1))) uint32_t gu32;
typedef const __attribute__((address_space(1))) char gc8;
__device__ __forceinline__ gu32* as_global(const uint32_t* p) { return (gu32*)(p); }

// Word i of a global array whose base is the same for the whole wavefront
// and whose byte offsets fit 32 bits: a scalar base plus a 32-bit vector
// offset (no 64-bit address arithmetic per lane).
__device__ __forceinline__ uint32_t ldg_word(gu32* base, uint32_t i) {
  return *reinterpret_cast<gu32*>(reinterpret_cast<gc8*>(base) + (uint64_t)(i << 2));
}

}  // namespace spin
