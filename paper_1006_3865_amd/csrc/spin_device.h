// spin_device.h -- device-side building blocks for gfx950: Philox4x32-10,
// the byte-parallel (four sites per 32-bit register) Metropolis update of an
// aligned 8-site group, and wavefront reductions.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "spin_internal.h"

namespace spin {

// Philox4x32 round multipliers.
constexpr uint32_t kPhiloxM0 = 0xD2511F53u;
constexpr uint32_t kPhiloxM1 = 0xCD9E8D57u;

// Three-input XOR in one VALU op (v_bitop3_b32, truth table 0x96).
__device__ __forceinline__ uint32_t xor3(uint32_t a, uint32_t b, uint32_t c) {
  return __builtin_amdgcn_bitop3_b32(a, b, c, 0x96);
}

// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11): ten rounds of two
// 32x32->64 products (one v_mad_u64_u32 each) and two three-way XORs with
// the precomputed round keys.
__device__ __forceinline__ void philox(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                       const RoundKeys& K, uint32_t r[4]) {
#pragma unroll
  for (int i = 0; i < 10; ++i) {
    const uint64_t p0 = (uint64_t)kPhiloxM0 * c0;
    const uint64_t p1 = (uint64_t)kPhiloxM1 * c2;
    const uint32_t n0 = xor3((uint32_t)(p1 >> 32), c1, K.k0[i]);
    const uint32_t n2 = xor3((uint32_t)(p0 >> 32), c3, K.k1[i]);
    c1 = (uint32_t)p1;
    c3 = (uint32_t)p0;
    c0 = n0;
    c2 = n2;
  }
  r[0] = c0; r[1] = c1; r[2] = c2; r[3] = c3;
}

// Uniform part of a Philox4x32-10 evaluation whose counter words c1, c2, c3
// are the same for the whole wavefront (sweep, replica, colour) and only c0
// varies by lane: the first two rounds are half scalar, so their uniform
// halves are computed once (on the scalar unit) and folded with the round
// keys into single operands.
struct PhiloxUniform {
  uint32_t x1;      // round 1: hi(M0*c0) ^ x1          -> c2 after round 1
  uint32_t x2;      // round 2: hi(M1*c2) ^ x2          -> c0 after round 2
  uint32_t x3;      // round 2: c3_after_round1 ^ x3    -> c2 after round 2 (x3 = hi(M0*u0) ^ k1[1])
  uint32_t x4;      // round 3: hi(M0*c0) ^ x4          -> c2 after round 3 (x4 = lo(M0*u0) ^ k1[2],
                    //          lo(M0*u0) being c3 after round 2)
};

__device__ __forceinline__ PhiloxUniform philox_uniform(uint32_t c1, uint32_t c2, uint32_t c3,
                                                        const RoundKeys& K) {
  PhiloxUniform U;
  const uint64_t p1 = (uint64_t)kPhiloxM1 * c2;
  const uint32_t u0 = (uint32_t)(p1 >> 32) ^ c1 ^ K.k0[0];  // c0 after round 1
  const uint32_t u1 = (uint32_t)p1;                         // c1 after round 1
  U.x1 = c3 ^ K.k1[0];
  U.x2 = u1 ^ K.k0[1];
  const uint64_t q0 = (uint64_t)kPhiloxM0 * u0;
  U.x3 = (uint32_t)(q0 >> 32) ^ K.k1[1];
  U.x4 = (uint32_t)q0 ^ K.k1[2];
  return U;
}

// Waits for the round keys' scalar loads before a loop.  Scalar loads and LDS
// reads share one wait counter: a key first used inside the loop would make
// every iteration wait there for all LDS reads in flight, not only the first.
__device__ __forceinline__ void keys_resident(const RoundKeys& K) {
#pragma unroll
  for (int i = 0; i < 10; ++i) asm volatile("" ::"s"(K.k0[i]), "s"(K.k1[i]));
}

// Philox4x32-10 of counter (c0, c1, c2, c3) given U = philox_uniform(c1, c2, c3)
// and the first product p0 = M0 * c0.
__device__ __forceinline__ void philox_from_p0(uint64_t p0, const PhiloxUniform& U, const RoundKeys& K,
                                               uint32_t r[4]) {
  // round 1
  const uint32_t a2 = (uint32_t)(p0 >> 32) ^ U.x1;
  const uint32_t a3 = (uint32_t)p0;
  // round 2 (c0 after round 1 is uniform: its product is in U)
  const uint64_t p1 = (uint64_t)kPhiloxM1 * a2;
  const uint32_t b0 = (uint32_t)(p1 >> 32) ^ U.x2;
  const uint32_t b1 = (uint32_t)p1;
  const uint32_t b2 = a3 ^ U.x3;
  // round 3 (c3 after round 2 is uniform: folded with its key into x4)
  const uint64_t p2 = (uint64_t)kPhiloxM0 * b0;
  const uint64_t p3 = (uint64_t)kPhiloxM1 * b2;
  uint32_t d0 = xor3((uint32_t)(p3 >> 32), b1, K.k0[2]);
  uint32_t d1 = (uint32_t)p3;
  uint32_t d2 = (uint32_t)(p2 >> 32) ^ U.x4;
  uint32_t d3 = (uint32_t)p2;
  // rounds 4..10
#pragma unroll
  for (int i = 3; i < 10; ++i) {
    const uint64_t q0 = (uint64_t)kPhiloxM0 * d0;
    const uint64_t q1 = (uint64_t)kPhiloxM1 * d2;
    const uint32_t n0 = xor3((uint32_t)(q1 >> 32), d1, K.k0[i]);
    const uint32_t n2 = xor3((uint32_t)(q0 >> 32), d3, K.k1[i]);
    d1 = (uint32_t)q1;
    d3 = (uint32_t)q0;
    d0 = n0;
    d2 = n2;
  }
  r[0] = d0; r[1] = d1; r[2] = d2; r[3] = d3;
}

// Philox4x32-10 of counter (c0, c1, c2, c3) given U = philox_uniform(c1, c2, c3).
__device__ __forceinline__ void philox_lane(uint32_t c0, const PhiloxUniform& U, const RoundKeys& K,
                                            uint32_t r[4]) {
  philox_from_p0((uint64_t)kPhiloxM0 * c0, U, K, r);
}

// philox_lane for the counter c0 = base + v with base uniform, v per lane and
// base + v < 2^32: M0 * c0 = M0 * v + M0 * base, one multiply-add whose 64-bit
// addend mbase = M0 * base (philox_base) is computed on the scalar unit.
// The empty asm keeps the compiler from folding the product back into
// M0 * (base + v), which costs a vector add before the multiply.
__device__ __forceinline__ uint64_t philox_base(uint32_t base) {
  uint64_t m = (uint64_t)kPhiloxM0 * base;
  asm volatile("" : "+s"(m));
  return m;
}

__device__ __forceinline__ void philox_lane_split(uint32_t v, uint64_t mbase, const PhiloxUniform& U,
                                                  const RoundKeys& K, uint32_t r[4]) {
  philox_from_p0((uint64_t)kPhiloxM0 * v + mbase, U, K, r);
}

// ---------------------------------------------------------------------------
// Byte-parallel update of one aligned group of 8 sites along x.
//
// Spin bytes are 0x01 (+1) or 0xFF (-1): every bit from 1 to 7 carries the
// sign, so (a ^ b) & 0x04 per byte is 4 exactly when the two spins differ.
// Summing that over the 2d neighbours gives 4*u per byte, u = number of
// unsatisfied bonds (u <= 6, so no byte overflows).  For a +-J bond the
// coupling byte joins the XOR: the bond is unsatisfied iff s_i J s_j = -1.
// With k = s_i h_i = 2d - 2u the Metropolis rule r < T[k] becomes a lookup
// of a 32-bit bound by the byte value 4u in a small LDS table:
//   bound[u] = T - 1         (accept iff r <= bound; T in [1, 2^32])
//   bound[u] = 0 with u < never_level for T == 0 (rejected separately).
// The flip itself XORs the byte with 0xFE (0x01 <-> 0xFF).
// ---------------------------------------------------------------------------

constexpr uint32_t kSignBit = 0x04040404u;

// 4u per byte for the two centre dwords.  lw / rw: the dword left of c0 and
// right of c1; o0 / o1: the other 2d-2 neighbour dwords (rows / planes).
template <int NO>
__device__ __forceinline__ void unsat_ising(uint32_t c0, uint32_t c1, uint32_t lw, uint32_t rw,
                                            const uint32_t (&o0)[NO], const uint32_t (&o1)[NO],
                                            uint32_t& S0, uint32_t& S1) {
  const uint32_t L0 = __builtin_amdgcn_alignbyte(c0, lw, 3);
  const uint32_t L1 = __builtin_amdgcn_alignbyte(c1, c0, 3);
  const uint32_t R0 = __builtin_amdgcn_alignbyte(c1, c0, 1);
  const uint32_t R1 = __builtin_amdgcn_alignbyte(rw, c1, 1);
  S0 = ((c0 ^ L0) & kSignBit) + ((c0 ^ R0) & kSignBit);
  S1 = ((c1 ^ L1) & kSignBit) + ((c1 ^ R1) & kSignBit);
#pragma unroll
  for (int i = 0; i < NO; ++i) {
    S0 += (c0 ^ o0[i]) & kSignBit;
    S1 += (c1 ^ o1[i]) & kSignBit;
  }
}

// Accept decision for the active byte at bit offset sh of S, word r.
template <bool NEVER>
__device__ __forceinline__ uint32_t flip_bits(uint32_t S, uint32_t sh, uint32_t r,
                                              const uint32_t* bound_lds, uint32_t never4) {
  const uint32_t i4 = __builtin_amdgcn_ubfe(S, sh, 8);  // 4u
  const uint32_t b = *(const uint32_t*)((const char*)bound_lds + i4);
  bool acc = r <= b;
  if (NEVER) acc = acc && (i4 >= never4);
  return acc ? (0xFEu << sh) : 0u;
}

// New value of the 8-site group given 4u per byte, the parity p of the
// active bytes (p, p+2, p+4, p+6) and the four Philox words.
template <bool NEVER>
__device__ __forceinline__ void apply_group(uint32_t& c0, uint32_t& c1, uint32_t S0, uint32_t S1,
                                            uint32_t p, const uint32_t r[4],
                                            const uint32_t* bound_lds, uint32_t never4) {
  const uint32_t sa = 8u * p, sb = 8u * p + 16u;
  const uint32_t f0 = flip_bits<NEVER>(S0, sa, r[0], bound_lds, never4);
  const uint32_t f1 = flip_bits<NEVER>(S0, sb, r[1], bound_lds, never4);
  const uint32_t f2 = flip_bits<NEVER>(S1, sa, r[2], bound_lds, never4);
  const uint32_t f3 = flip_bits<NEVER>(S1, sb, r[3], bound_lds, never4);
  c0 = xor3(c0, f0, f1);
  c1 = xor3(c1, f2, f3);
}

// apply_group with the parity of the active bytes known at compile time.
template <uint32_t P, bool NEVER>
__device__ __forceinline__ void apply_group_p(uint32_t& c0, uint32_t& c1, uint32_t S0, uint32_t S1,
                                              const uint32_t r[4], const uint32_t* bound_lds,
                                              uint32_t never4) {
  constexpr uint32_t sa = 8u * P, sb = 8u * P + 16u;
  const uint32_t f0 = flip_bits<NEVER>(S0, sa, r[0], bound_lds, never4);
  const uint32_t f1 = flip_bits<NEVER>(S0, sb, r[1], bound_lds, never4);
  const uint32_t f2 = flip_bits<NEVER>(S1, sa, r[2], bound_lds, never4);
  const uint32_t f3 = flip_bits<NEVER>(S1, sb, r[3], bound_lds, never4);
  c0 = xor3(c0, f0, f1);
  c1 = xor3(c1, f2, f3);
}

// ---------------------------------------------------------------- reductions

__device__ __forceinline__ int64_t wave_sum(int64_t v) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// Sum over the workgroup; every thread must call it; result valid in thread 0.
template <int NT>
__device__ __forceinline__ int64_t block_sum(int64_t v, int64_t* scratch /* NT/64 */) {
  v = wave_sum(v);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  if (lane == 0) scratch[wid] = v;
  __syncthreads();
  int64_t s = 0;
  if (threadIdx.x == 0) {
#pragma unroll
    for (int i = 0; i < NT / 64; ++i) s += scratch[i];
  }
  __syncthreads();
  return s;
}

// Sum over the 64 lanes of a wavefront (every lane active) of counts below
// 2^26 per lane: an inclusive scan inside each row of 16 lanes by DPP row
// shifts of 1, 2, 4 and 8 lanes (lanes shifted in from outside the row read
// 0), after which lanes 15, 31, 47 and 63 hold the row totals, read with
// readlane.
__device__ __forceinline__ int64_t wave_count_dpp(uint32_t v) {
  int s = (int)v;
  s += __builtin_amdgcn_update_dpp(0, s, 0x111, 0xf, 0xf, true);  // row_shr:1
  s += __builtin_amdgcn_update_dpp(0, s, 0x112, 0xf, 0xf, true);  // row_shr:2
  s += __builtin_amdgcn_update_dpp(0, s, 0x114, 0xf, 0xf, true);  // row_shr:4
  s += __builtin_amdgcn_update_dpp(0, s, 0x118, 0xf, 0xf, true);  // row_shr:8
  return (int64_t)__builtin_amdgcn_readlane(s, 15) + (int64_t)__builtin_amdgcn_readlane(s, 31) +
         (int64_t)__builtin_amdgcn_readlane(s, 47) + (int64_t)__builtin_amdgcn_readlane(s, 63);
}

// Workgroup sum of per-thread counts below 2^26 (DPP within waves, LDS across
// them); every thread must call it; result valid in thread 0.
template <int NT>
__device__ __forceinline__ int64_t block_count_dpp(uint32_t v, int64_t* scratch /* NT/64 */) {
  const int64_t w = wave_count_dpp(v);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  if (lane == 0) scratch[wid] = w;
  __syncthreads();
  int64_t s = 0;
  if (threadIdx.x == 0) {
#pragma unroll
    for (int i = 0; i < NT / 64; ++i) s += scratch[i];
  }
  __syncthreads();
  return s;
}

// Store this workgroup's counts in its record slots.  Every thread calls it
// (it contains barriers); the per-thread counts are below 2^26.  red: >= NT/64
// int64 in LDS.
template <int NT>
__device__ __forceinline__ void record_block(int64_t unsat, int64_t neg, const Record& R,
                                             int64_t* red) {
  const int64_t bu = block_count_dpp<NT>((uint32_t)unsat, red);
  const int64_t bn = block_count_dpp<NT>((uint32_t)neg, red);
  if (threadIdx.x == 0) {
    const unsigned wg = blockIdx.x + gridDim.x * (blockIdx.y + gridDim.y * blockIdx.z);
    R.part[2 * wg] = bu;
    R.part[2 * wg + 1] = bn;
  }
}

}  // namespace spin
