// spin_heis_kernels.hip -- the classical Heisenberg ferromagnet (continuous
// spins in single precision), the generalisation the paper points to at the
// close of Sec. 4.  Spins are unit vectors stored as float4 (x, y, z, 0) in
// site order.  One launch per colour: a thread updates one site of that
// colour from its 2d neighbours (all of the other colour, untouched by the
// launch), so the update is in place and race-free.
//   draws of site s: hot start Philox (s, 0, replica, 9), update in sweep t,
//   colour c Philox (s, t, replica, 10 + c); u_i = (w_i >> 8) 2^-24;
//   direction (u0, u1): z = 2 u0 - 1, phi = 2 pi u1, rho = sqrt(fma(-z, z, 1)),
//   (rho cos phi, rho sin phi, z);
//   h = neighbour vectors added in the order -x, +x, -y, +y, -z, +z;
//   dE = S.h - S'.h, a.h = fma(a.x, h.x, fma(a.y, h.y, a.z h.z));
//   accept iff dE <= 0 (the Metropolis rule of Sec. 3, Eq. 2, also at beta =
//   inf) or u2 < exp(-(beta dE)).
// cos, sin and exp are evaluated by one stated method (octant reduction of
// u1 and Taylor polynomials; Cody-Waite reduction by ln 2 and a Taylor
// polynomial, scaled by 2^k), every step a single IEEE float operation with
// fused multiply-adds written out and contraction switched off, so each
// result is a definite float.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "spin_device.h"
#include "spin_heis.h"

#pragma clang fp contract(off)

namespace spin {

__device__ __forceinline__ float heis_uniform(uint32_t w) { return (float)(w >> 8) * 0x1p-24f; }

// cos and sin of x in [0, pi/4]: Taylor polynomials to x^10 and x^9, Horner steps in x^2.
__device__ __forceinline__ void heis_cos_sin(float x, float& c, float& sn) {
  const float x2 = x * x;
  float pc = -1.0f / 3628800.0f;
  pc = __builtin_fmaf(pc, x2, 1.0f / 40320.0f);
  pc = __builtin_fmaf(pc, x2, -1.0f / 720.0f);
  pc = __builtin_fmaf(pc, x2, 1.0f / 24.0f);
  pc = __builtin_fmaf(pc, x2, -0.5f);
  c = __builtin_fmaf(pc, x2, 1.0f);
  float ps = 1.0f / 362880.0f;
  ps = __builtin_fmaf(ps, x2, -1.0f / 5040.0f);
  ps = __builtin_fmaf(ps, x2, 1.0f / 120.0f);
  ps = __builtin_fmaf(ps, x2, -1.0f / 6.0f);
  sn = __builtin_fmaf(ps * x2, x, x);
}

// Direction from (u0, u1): z = 2 u0 - 1; the angle 2 pi u1 reduced to its octant o = floor(8 u1) and
// the offset r = 8 u1 - o (exact), the polynomial taken at r pi/4 (even o) or (1 - r) pi/4 (odd o,
// cos and sin swapped), then rotated by the quadrant o >> 1.
__device__ __forceinline__ float4 heis_direction(uint32_t w0, uint32_t w1) {
  const float z = 2.0f * heis_uniform(w0) - 1.0f;
  const float rho = sqrtf(__builtin_fmaf(-z, z, 1.0f));
  const float t = 8.0f * heis_uniform(w1);
  const int o = (int)t;
  const float r = t - (float)o;
  float c, sn;
  heis_cos_sin(((o & 1) ? 1.0f - r : r) * 0.785398163397448309616f, c, sn);
  if (o & 1) {
    const float tmp = c;
    c = sn;
    sn = tmp;
  }
  const int q = o >> 1;
  const float cx = q == 0 ? c : q == 1 ? -sn : q == 2 ? -c : sn;
  const float sy = q == 0 ? sn : q == 1 ? c : q == 2 ? -sn : -c;
  return make_float4(rho * cx, rho * sy, z, 0.0f);
}

// u < exp(y): true for y >= 0, false for y <= -87 (exp(y) < 2^-125), else against 2^k e^r with
// k = floor(y log2(e) + 1/2), r = y - k ln 2 (ln 2 split into a high part exact in float and the
// rest) and e^r by its Taylor polynomial to r^7.
__device__ __forceinline__ bool heis_accept(float u, float y) {
  if (y >= 0.0f) return true;
  if (!(y > -87.0f)) return false;
  const float k = __builtin_floorf(__builtin_fmaf(y, 1.44269504088896340736f, 0.5f));
  float r = __builtin_fmaf(-k, 0.693145751953125f, y);
  r = __builtin_fmaf(-k, 1.428606765330187045e-06f, r);
  float p = 1.0f / 5040.0f;
  p = __builtin_fmaf(p, r, 1.0f / 720.0f);
  p = __builtin_fmaf(p, r, 1.0f / 120.0f);
  p = __builtin_fmaf(p, r, 1.0f / 24.0f);
  p = __builtin_fmaf(p, r, 1.0f / 6.0f);
  p = __builtin_fmaf(p, r, 0.5f);
  p = __builtin_fmaf(p, r, 1.0f);
  p = __builtin_fmaf(p, r, 1.0f);
  return u < __builtin_ldexpf(p, (int)k);
}

__device__ __forceinline__ float heis_dot(const float4& a, const float4& h) {
  return __builtin_fmaf(a.x, h.x, __builtin_fmaf(a.y, h.y, a.z * h.z));
}

__device__ __forceinline__ void heis_add(float4& h, const float4& v) {
  h.x = h.x + v.x;
  h.y = h.y + v.y;
  h.z = h.z + v.z;
}

__global__ void k_heis_init(float4* __restrict__ S, uint64_t N, RoundKeys K, uint32_t replica) {
  for (uint64_t s = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; s < N; s += (uint64_t)gridDim.x * blockDim.x) {
    uint32_t w[4];
    philox((uint32_t)s, 0u, replica, 9u, K, w);
    S[s] = heis_direction(w[0], w[1]);
  }
}

template <int D>
__global__ void k_heis_phase(float4* __restrict__ S, HeisArgs a) {
  const uint32_t L = a.L, half = L / 2;
  const uint64_t row = L, plane = (uint64_t)L * L, n = a.N / 2;
  for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x) {
    const uint64_t ri = i / half;  // row index (y + L z)
    const uint32_t j = (uint32_t)(i - ri * half);
    const uint32_t y = (uint32_t)(ri % L), z = (D == 3) ? (uint32_t)(ri / L) : 0u;
    const uint32_t x = 2 * j + ((a.colour + y + z) & 1u);
    const uint64_t s = ri * L + x;
    float4 h = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
    heis_add(h, S[x ? s - 1 : s + L - 1]);
    heis_add(h, S[x + 1 < L ? s + 1 : s + 1 - L]);
    heis_add(h, S[y ? s - row : s + (L - 1) * row]);
    heis_add(h, S[y + 1 < L ? s + row : s - (L - 1) * row]);
    if (D == 3) {
      heis_add(h, S[z ? s - plane : s + (L - 1) * plane]);
      heis_add(h, S[z + 1 < L ? s + plane : s - (L - 1) * plane]);
    }
    uint32_t w[4];
    philox((uint32_t)s, a.t, a.replica, 10u + a.colour, a.keys, w);
    const float4 cur = S[s];
    const float4 trial = heis_direction(w[0], w[1]);
    const float dE = heis_dot(cur, h) - heis_dot(trial, h);
    if (dE <= 0.0f || heis_accept(heis_uniform(w[2]), -(a.beta * dE))) S[s] = trial;
  }
}

// Per-workgroup sums (E, Mx, My, Mz) in double: E = -sum of the d forward bonds of each site.
template <int D>
__global__ __launch_bounds__(256) void k_heis_measure(const float4* __restrict__ S, uint32_t L, uint64_t N,
                                                      double* __restrict__ part) {
  __shared__ double red[4][256];
  const uint64_t row = L, plane = (uint64_t)L * L;
  double e = 0, mx = 0, my = 0, mz = 0;
  for (uint64_t s = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; s < N; s += (uint64_t)gridDim.x * blockDim.x) {
    const uint32_t x = (uint32_t)(s % L), y = (uint32_t)((s / L) % L), z = (D == 3) ? (uint32_t)(s / plane) : 0u;
    const float4 v = S[s];
    mx += v.x;
    my += v.y;
    mz += v.z;
    const float4 bx = S[x + 1 < L ? s + 1 : s + 1 - L];
    const float4 by = S[y + 1 < L ? s + row : s - (L - 1) * row];
    double b = (double)v.x * bx.x + (double)v.y * bx.y + (double)v.z * bx.z;
    b += (double)v.x * by.x + (double)v.y * by.y + (double)v.z * by.z;
    if (D == 3) {
      const float4 bz = S[z + 1 < L ? s + plane : s - (L - 1) * plane];
      b += (double)v.x * bz.x + (double)v.y * bz.y + (double)v.z * bz.z;
    }
    e -= b;
  }
  red[0][threadIdx.x] = e;
  red[1][threadIdx.x] = mx;
  red[2][threadIdx.x] = my;
  red[3][threadIdx.x] = mz;
  __syncthreads();
  for (uint32_t off = 128; off > 0; off >>= 1) {
    if (threadIdx.x < off)
      for (int k = 0; k < 4; ++k) red[k][threadIdx.x] += red[k][threadIdx.x + off];
    __syncthreads();
  }
  if (threadIdx.x < 4) part[(uint64_t)blockIdx.x * 4 + threadIdx.x] = red[threadIdx.x][0];
}

static unsigned heis_blocks(uint64_t work, unsigned cap) {
  const uint64_t b = (work + 255) / 256;
  return (unsigned)(b < cap ? (b ? b : 1) : cap);
}

uint32_t heis_measure_blocks(uint64_t N) { return heis_blocks(N, 1024); }

hipError_t launch_heis_init(float4* S, uint64_t N, uint64_t seed, uint32_t replica, hipStream_t stream) {
  hipLaunchKernelGGL(k_heis_init, dim3(heis_blocks(N, 8192)), dim3(256), 0, stream, S, N, make_round_keys(seed),
                     replica);
  return hipGetLastError();
}

hipError_t launch_heis_phase(float4* S, uint32_t d, const HeisArgs& a, hipStream_t stream) {
  const unsigned blocks = heis_blocks(a.N / 2, 65535);
  if (d == 3)
    hipLaunchKernelGGL(k_heis_phase<3>, dim3(blocks), dim3(256), 0, stream, S, a);
  else
    hipLaunchKernelGGL(k_heis_phase<2>, dim3(blocks), dim3(256), 0, stream, S, a);
  return hipGetLastError();
}

hipError_t launch_heis_measure(const float4* S, uint32_t L, uint32_t d, uint64_t N, double* part, hipStream_t stream) {
  const unsigned blocks = heis_measure_blocks(N);
  if (d == 3)
    hipLaunchKernelGGL(k_heis_measure<3>, dim3(blocks), dim3(256), 0, stream, S, L, N, part);
  else
    hipLaunchKernelGGL(k_heis_measure<2>, dim3(blocks), dim3(256), 0, stream, S, L, N, part);
  return hipGetLastError();
}

}  // namespace spin
