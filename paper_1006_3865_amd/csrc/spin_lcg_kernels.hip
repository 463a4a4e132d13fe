// spin_lcg_kernels.hip -- the canonical chain with linear congruential
// generators in place of Philox, for the RNG-quality experiment (Sec. 4,
// first paragraph).  Every 8-site group g = s>>3 (one "thread" of the
// experiment) owns one generator state; in each colour phase its four sites
// of that colour draw the next four numbers of its stream, in increasing x.
//   32-bit: x -> 1664525 x + 1013904223 (mod 2^32), draw = x;
//   64-bit: x -> 6364136223846793005 x + 1442695040888963407 (mod 2^64),
//           draw = high 32 bits of x.
// Initial states (G = L^d/8 groups):
//   SPIN_RNG_LCG32_ARRAY: state of g = word 0 of Philox (g, 0, replica, 6);
//   SPIN_RNG_LCG32_DISJOINT / SPIN_RNG_LCG64_DISJOINT: one sequence from
//   x0 (words 0 and 1 of Philox (0, 0, replica, 7)), group g starting
//   g * floor(2^P / G) steps after x0.
// The phase kernel reads and writes the int8 spins in global memory: a
// colour-c site reads only colour-(1-c) neighbours, which the phase does not
// write, so the update is race-free in place.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "spin.h"
#include "spin_device.h"
#include "spin_lcg.h"

namespace spin {

constexpr uint64_t kLcg32A = 1664525u, kLcg32C = 1013904223u;
constexpr uint64_t kLcg64A = 6364136223846793005ull, kLcg64C = 1442695040888963407ull;

__device__ __forceinline__ uint64_t lcg_next(uint64_t x, uint32_t mode) {
  if (mode == SPIN_RNG_LCG64_DISJOINT) return x * kLcg64A + kLcg64C;
  return (uint32_t)((uint32_t)x * (uint32_t)kLcg32A + (uint32_t)kLcg32C);
}

__device__ __forceinline__ uint32_t lcg_word(uint64_t x, uint32_t mode) {
  return mode == SPIN_RNG_LCG64_DISJOINT ? (uint32_t)(x >> 32) : (uint32_t)x;
}

// x advanced k steps: the map x -> A x + C applied to itself is x -> A^2 x + (A+1) C; the powers for
// the set bits of k are composed into (ma, mc).
__device__ uint64_t lcg_jump(uint64_t x, uint64_t k, uint32_t mode) {
  const bool wide = mode == SPIN_RNG_LCG64_DISJOINT;
  uint64_t A = wide ? kLcg64A : kLcg32A, C = wide ? kLcg64C : kLcg32C;
  uint64_t ma = 1, mc = 0;
  for (; k; k >>= 1) {
    if (k & 1) {
      mc = A * mc + C;
      ma = A * ma;
    }
    C = (A + 1) * C;
    A = A * A;
  }
  const uint64_t r = ma * x + mc;
  return wide ? r : (uint64_t)(uint32_t)r;
}

__global__ void k_lcg_init(uint64_t* __restrict__ st, uint64_t G, uint32_t mode, RoundKeys K, uint32_t replica) {
  uint32_t w0[4];
  philox(0u, 0u, replica, 7u, K, w0);
  uint64_t x0 = w0[0], len = ((uint64_t)1 << 32) / G;
  if (mode == SPIN_RNG_LCG64_DISJOINT) {
    x0 |= (uint64_t)w0[1] << 32;
    len = UINT64_MAX / G + ((UINT64_MAX % G == G - 1) ? 1u : 0u);  // floor(2^64 / G)
  }
  for (uint64_t g = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; g < G; g += (uint64_t)gridDim.x * blockDim.x) {
    if (mode == SPIN_RNG_LCG32_ARRAY) {
      uint32_t w[4];
      philox((uint32_t)g, 0u, replica, 6u, K, w);
      st[g] = w[0];
    } else {
      st[g] = lcg_jump(x0, g * len, mode);
    }
  }
}

template <int D>
__global__ void k_lcg_phase(int8_t* __restrict__ S, uint64_t* __restrict__ st, LcgArgs a) {
  const uint32_t L = a.L, GPR = L / 8;
  const uint64_t G = a.N / 8, row = L, plane = (uint64_t)L * L;
  for (uint64_t g = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; g < G; g += (uint64_t)gridDim.x * blockDim.x) {
    const uint64_t ri = g / GPR;
    const uint32_t x0 = (uint32_t)(g - ri * GPR) * 8u;
    const uint32_t y = (uint32_t)(ri % L), z = (D == 3) ? (uint32_t)(ri / L) : 0u;
    const uint32_t P = (a.colour + y + z) & 1u;
    uint64_t x = st[g];
#pragma unroll
    for (uint32_t i = 0; i < 4; ++i) {
      const uint32_t xs = x0 + 2 * i + P;
      const uint64_t s = g * 8 + 2 * i + P;
      int h = S[xs ? s - 1 : s + L - 1] + S[xs + 1 < L ? s + 1 : s + 1 - L];
      h += S[y ? s - row : s + (L - 1) * row] + S[y + 1 < L ? s + row : s - (L - 1) * row];
      if (D == 3) h += S[z ? s - plane : s + (L - 1) * plane] + S[z + 1 < L ? s + plane : s - (L - 1) * plane];
      const int sv = S[s];
      x = lcg_next(x, a.mode);
      if ((uint64_t)lcg_word(x, a.mode) < a.T[(sv * h + 2 * D) / 2]) S[s] = (int8_t)(-sv);
    }
    st[g] = x;
  }
}

static unsigned lcg_blocks(uint64_t G) {
  const uint64_t b = (G + 255) / 256;
  return (unsigned)(b < 8192 ? (b ? b : 1) : 8192);
}

hipError_t launch_lcg_init(uint64_t* st, uint64_t G, uint32_t mode, uint64_t seed, uint32_t replica,
                           hipStream_t stream) {
  hipLaunchKernelGGL(k_lcg_init, dim3(lcg_blocks(G)), dim3(256), 0, stream, st, G, mode, make_round_keys(seed),
                     replica);
  return hipGetLastError();
}

hipError_t launch_lcg_phase(int8_t* S, uint64_t* st, uint32_t d, const LcgArgs& a, hipStream_t stream) {
  const uint64_t G = a.N / 8;
  if (d == 3)
    hipLaunchKernelGGL(k_lcg_phase<3>, dim3(lcg_blocks(G)), dim3(256), 0, stream, S, st, a);
  else
    hipLaunchKernelGGL(k_lcg_phase<2>, dim3(lcg_blocks(G)), dim3(256), 0, stream, S, st, a);
  return hipGetLastError();
}

}  // namespace spin
