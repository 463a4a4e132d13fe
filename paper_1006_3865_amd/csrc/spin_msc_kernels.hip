// spin_msc_kernels.hip -- multi-spin-coded +-J glass (Sec. 4, last paragraph:
// many disorder realisations at once, combined with multi-spin coding): 32
// systems share the lattice, bit b of every word belongs to system b.
//
// spins: one uint32 per site, bit set = spin -1.  couplings: one uint32 per
// direction and site ([dir][site]), bit set = J -1 for the bond (s, s+e_dir).
// A bond is unsatisfied in system b iff bit b of s_i ^ s_j ^ J is set.  An
// update of site s counts its unsatisfied bonds u (0..2d) in every bit at
// once with a bit-sliced adder (full adders: sum = xor3, carry = majority,
// one v_bitop3 each), then accepts system b iff r < T at k_b = 2d - 2u_b,
// i.e. iff u_b >= u*(r), where u*(r) = #{u < d : r >= T at k = 2d - 2u} is
// one scalar per site (T grows as u grows, and is 2^32 for u >= d).  r is
// the site's shared draw: word
// (s>>1)&3 of Philox counter (s>>3, t, p0, 4 + colour), the chain of the
// oracle's multi-spin-coded mode.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "spin_device.h"
#include "spin_internal.h"
#include "spin_msc.h"

namespace spin {

__device__ __forceinline__ uint32_t maj3(uint32_t a, uint32_t b, uint32_t c) {
  return __builtin_amdgcn_bitop3_b32(a, b, c, 0xE8);
}

// Hot start: bit b of word s is set iff system b's spin is -1, i.e. iff
// bit 31 of word s&3 of Philox(seed, (s>>2, 0, p0 + b, 2)) is clear.
__global__ void k_msc_init(uint32_t* __restrict__ S, uint64_t nquads, RoundKeys K, uint32_t p0) {
  for (uint64_t q = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; q < nquads; q += (uint64_t)gridDim.x * blockDim.x) {
    uint32_t w[4] = {0, 0, 0, 0};
    for (uint32_t b = 0; b < 32; ++b) {
      uint32_t r[4];
      philox((uint32_t)q, 0u, p0 + b, 2u, K, r);
#pragma unroll
      for (int j = 0; j < 4; ++j) w[j] |= ((r[j] >> 31) ^ 1u) << b;
    }
    reinterpret_cast<uint4*>(S)[q] = make_uint4(w[0], w[1], w[2], w[3]);
  }
}

// Couplings: bit b of J[dir][s] is set iff bit 31 of word s&3 of
// Philox(cseed, (s>>2, dir, r0 + b, 3)) is set (J = -1).
__global__ void k_msc_couplings(uint32_t* __restrict__ J, uint64_t nquads, uint32_t d, RoundKeys K, uint32_t r0) {
  for (uint32_t dir = 0; dir < d; ++dir)
    for (uint64_t q = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; q < nquads;
         q += (uint64_t)gridDim.x * blockDim.x) {
      uint32_t w[4] = {0, 0, 0, 0};
      for (uint32_t b = 0; b < 32; ++b) {
        uint32_t r[4];
        philox((uint32_t)q, dir, r0 + b, 3u, K, r);
#pragma unroll
        for (int j = 0; j < 4; ++j) w[j] |= (r[j] >> 31) << b;
      }
      reinterpret_cast<uint4*>(J)[(uint64_t)dir * nquads + q] = make_uint4(w[0], w[1], w[2], w[3]);
    }
}

__device__ __forceinline__ void load8(const uint32_t* p, uint32_t (&v)[8]) {
  const uint4 a = reinterpret_cast<const uint4*>(p)[0];
  const uint4 b = reinterpret_cast<const uint4*>(p)[1];
  v[0] = a.x; v[1] = a.y; v[2] = a.z; v[3] = a.w;
  v[4] = b.x; v[5] = b.y; v[6] = b.z; v[7] = b.w;
}

// Mask of the systems whose unsatisfied count u (bit-sliced u2 u1 u0) is at least us.
__device__ __forceinline__ uint32_t at_least(uint32_t u0, uint32_t u1, uint32_t u2, uint32_t us) {
  uint32_t m = 0xFFFFFFFFu;                         // us == 0
  m = us >= 1 ? (u0 | u1 | u2) : m;
  m = us >= 2 ? (u1 | u2) : m;
  m = us >= 3 ? (u2 | (u1 & u0)) : m;
  return m;
}

// One colour phase: thread = 8-site group g (sites 8g .. 8g+7 of one row);
// its four sites of colour c (offset P = (c + y + z) & 1 inside the group).
template <int D, int P>
__device__ __forceinline__ void msc_group(uint32_t* __restrict__ S, const uint32_t* __restrict__ J,
                                          const MscArgs& a, uint64_t s0, uint32_t x0, uint32_t y, uint32_t z,
                                          const uint32_t (&r)[4]) {
  const uint32_t L = a.L;
  const uint64_t N = a.N, row = (uint64_t)L, plane = (uint64_t)L * L;
  uint32_t c[8], ym[8], yp[8], jx[8], jy[8], jym[8];
  load8(S + s0, c);
  const uint64_t sym = y ? s0 - row : s0 + (L - 1) * row;
  const uint64_t syp = (y + 1 < L) ? s0 + row : s0 - (L - 1) * row;
  load8(S + sym, ym);
  load8(S + syp, yp);
  load8(J + s0, jx);
  load8(J + N + s0, jy);
  load8(J + N + sym, jym);
  uint32_t zm[8], zp[8], jz[8], jzm[8];
  if (D == 3) {
    const uint64_t szm = z ? s0 - plane : s0 + (L - 1) * plane;
    const uint64_t szp = (z + 1 < L) ? s0 + plane : s0 - (L - 1) * plane;
    load8(S + szm, zm);
    load8(S + szp, zp);
    load8(J + 2 * N + s0, jz);
    load8(J + 2 * N + szm, jzm);
  }
  const uint64_t sl = x0 ? s0 - 1 : s0 + L - 1;     // site left of the group
  const uint64_t sr = (x0 + 8 < L) ? s0 + 8 : s0 + 8 - L;
  const uint32_t lw = S[sl], rw = S[sr], jl = J[sl];
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int j = 2 * i + P;
    const uint32_t left = j ? c[j - 1] : lw;
    const uint32_t right = j < 7 ? c[j + 1] : rw;
    const uint32_t jleft = j ? jx[j - 1] : jl;
    const uint32_t s = c[j];
    // unsatisfied bits of the 2d bonds
    const uint32_t b0 = xor3(s, left, jleft), b1 = xor3(s, right, jx[j]);
    const uint32_t b2 = xor3(s, ym[j], jym[j]), b3 = xor3(s, yp[j], jy[j]);
    uint32_t u0, u1, u2;
    if (D == 3) {
      const uint32_t b4 = xor3(s, zm[j], jzm[j]), b5 = xor3(s, zp[j], jz[j]);
      const uint32_t s1 = xor3(b0, b1, b2), c1 = maj3(b0, b1, b2);
      const uint32_t s2 = xor3(b3, b4, b5), c2 = maj3(b3, b4, b5);
      u0 = s1 ^ s2;
      const uint32_t t = s1 & s2;
      u1 = xor3(c1, c2, t);
      u2 = maj3(c1, c2, t);
    } else {
      const uint32_t s1 = xor3(b0, b1, b2), c1 = maj3(b0, b1, b2);
      u0 = s1 ^ b3;
      const uint32_t t = s1 & b3;
      u1 = c1 ^ t;
      u2 = c1 & t;
    }
    // u*(r): thresholds of u = 0 .. d-1 at or below r
    const uint64_t ri = r[i];
    uint32_t us = (ri >= a.thr[0] ? 1u : 0u) + (ri >= a.thr[1] ? 1u : 0u);
    if (D == 3) us += ri >= a.thr[2] ? 1u : 0u;
    c[j] = s ^ at_least(u0, u1, u2, us);
  }
  reinterpret_cast<uint4*>(S + s0)[0] = make_uint4(c[0], c[1], c[2], c[3]);
  reinterpret_cast<uint4*>(S + s0)[1] = make_uint4(c[4], c[5], c[6], c[7]);
}

template <int D>
__global__ __launch_bounds__(256) void k_msc_phase(uint32_t* __restrict__ S, const uint32_t* __restrict__ J,
                                                   MscArgs a) {
  const uint32_t L = a.L, GPR = L / 8;
  const PhiloxUniform U = philox_uniform(a.t, a.p0, 4u + a.colour, a.keys);
  for (uint64_t g = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; g < a.N / 8;
       g += (uint64_t)gridDim.x * blockDim.x) {
    const uint64_t rowi = g / GPR;
    const uint32_t x0 = (uint32_t)(g - rowi * GPR) * 8u;
    const uint32_t y = (uint32_t)(rowi % L), z = (D == 3) ? (uint32_t)(rowi / L) : 0u;
    uint32_t r[4];
    philox_lane((uint32_t)g, U, a.keys, r);
    if (((a.colour + y + z) & 1u) == 0)
      msc_group<D, 0>(S, J, a, g * 8, x0, y, z, r);
    else
      msc_group<D, 1>(S, J, a, g * 8, x0, y, z, r);
  }
}

// E and M of the 32 systems: per workgroup, counts of unsatisfied bonds and
// of negative spins for every bit into part[wg*64 + bit] (unsat) and
// part[wg*64 + 32 + bit] (negative); k_msc_finalize sums the workgroups.
template <int D>
__global__ __launch_bounds__(256) void k_msc_count(const uint32_t* __restrict__ S, const uint32_t* __restrict__ J,
                                                   uint32_t L, uint64_t N, int64_t* __restrict__ part) {
  __shared__ int64_t red[64];
  if (threadIdx.x < 64) red[threadIdx.x] = 0;
  __syncthreads();
  uint32_t cu[32], cn[32];
#pragma unroll
  for (int b = 0; b < 32; ++b) cu[b] = cn[b] = 0;
  const uint64_t row = L, plane = (uint64_t)L * L;
  for (uint64_t s = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; s < N; s += (uint64_t)gridDim.x * blockDim.x) {
    const uint32_t x = (uint32_t)(s % L), y = (uint32_t)((s / L) % L), z = (D == 3) ? (uint32_t)(s / plane) : 0u;
    const uint32_t v = S[s];
    const uint32_t bx = v ^ S[x + 1 < L ? s + 1 : s + 1 - L] ^ J[s];
    const uint32_t by = v ^ S[y + 1 < L ? s + row : s - (L - 1) * row] ^ J[N + s];
    uint32_t bz = 0;
    if (D == 3) bz = v ^ S[z + 1 < L ? s + plane : s - (L - 1) * plane] ^ J[2 * N + s];
#pragma unroll
    for (int b = 0; b < 32; ++b) {
      cu[b] += ((bx >> b) & 1u) + ((by >> b) & 1u) + ((bz >> b) & 1u);
      cn[b] += (v >> b) & 1u;
    }
  }
#pragma unroll
  for (int b = 0; b < 32; ++b) {
    atomicAdd((unsigned long long*)&red[b], (unsigned long long)cu[b]);
    atomicAdd((unsigned long long*)&red[32 + b], (unsigned long long)cn[b]);
  }
  __syncthreads();
  if (threadIdx.x < 64) part[(uint64_t)blockIdx.x * 64 + threadIdx.x] = red[threadIdx.x];
}

__global__ void k_msc_finalize(const int64_t* __restrict__ part, uint32_t nparts, int64_t nb, int64_t N,
                               int64_t* __restrict__ E, int64_t* __restrict__ M) {
  const uint32_t b = threadIdx.x;
  if (b >= 32) return;
  int64_t u = 0, n = 0;
  for (uint32_t w = 0; w < nparts; ++w) {
    u += part[(uint64_t)w * 64 + b];
    n += part[(uint64_t)w * 64 + 32 + b];
  }
  E[b] = -nb + 2 * u;
  M[b] = N - 2 * n;
}

static unsigned blocks_for(uint64_t work, unsigned cap) {
  uint64_t b = (work + 255) / 256;
  return (unsigned)(b < cap ? (b ? b : 1) : cap);
}

hipError_t launch_msc_init(uint32_t* S, uint64_t N, uint64_t seed, uint32_t p0, hipStream_t stream) {
  hipLaunchKernelGGL(k_msc_init, dim3(blocks_for(N / 4, 8192)), dim3(256), 0, stream, S, N / 4, make_round_keys(seed),
                     p0);
  return hipGetLastError();
}

hipError_t launch_msc_couplings(uint32_t* J, uint64_t N, uint32_t d, uint64_t cseed, uint32_t r0, hipStream_t stream) {
  hipLaunchKernelGGL(k_msc_couplings, dim3(blocks_for(N / 4, 8192)), dim3(256), 0, stream, J, N / 4, d,
                     make_round_keys(cseed), r0);
  return hipGetLastError();
}

hipError_t launch_msc_phase(uint32_t* S, const uint32_t* J, const MscArgs& a, uint32_t d, hipStream_t stream) {
  const unsigned blocks = blocks_for(a.N / 8, 1u << 20);
  if (d == 3)
    hipLaunchKernelGGL(k_msc_phase<3>, dim3(blocks), dim3(256), 0, stream, S, J, a);
  else
    hipLaunchKernelGGL(k_msc_phase<2>, dim3(blocks), dim3(256), 0, stream, S, J, a);
  return hipGetLastError();
}

uint32_t msc_count_parts(uint64_t N) { return blocks_for(N, 2048); }

hipError_t launch_msc_measure(const uint32_t* S, const uint32_t* J, uint32_t L, uint32_t d, uint64_t N, int64_t* part,
                              int64_t* E, int64_t* M, hipStream_t stream) {
  const unsigned blocks = msc_count_parts(N);
  if (d == 3)
    hipLaunchKernelGGL(k_msc_count<3>, dim3(blocks), dim3(256), 0, stream, S, J, L, N, part);
  else
    hipLaunchKernelGGL(k_msc_count<2>, dim3(blocks), dim3(256), 0, stream, S, J, L, N, part);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_msc_finalize, dim3(1), dim3(64), 0, stream, part, blocks, (int64_t)d * (int64_t)N, (int64_t)N,
                     E, M);
  return hipGetLastError();
}

}  // namespace spin
