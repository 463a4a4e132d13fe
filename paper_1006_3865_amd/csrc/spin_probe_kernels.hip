// spin_probe_kernels.hip -- ceiling probes of the hardware the sweep runs on:
// the rate of Philox4x32-10 blocks evaluated exactly as the sweep kernels do
// (philox_uniform + philox_lane), the issue rate of v_mad_u64_u32 and of a
// plain 32-bit VALU operation, and a streaming device copy.  They measure
// what bounds the canonical chain; none is part of it.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "spin.h"
#include "spin_device.h"
#include "spin_internal.h"
#include "spin_phase.h"
#include "spin_probe.h"

namespace spin {

// Each thread evaluates `iters` Philox blocks with counters (i, t, replica,
// colour), i = gid + k * nthreads, and folds the four words of each into one
// value (three XORs per block on top of the generator's own work).
__global__ __launch_bounds__(256) void k_probe_philox(uint32_t* out, uint32_t iters, PhaseArgs a) {
  const uint32_t nthreads = gridDim.x * blockDim.x;
  const uint32_t gid = blockIdx.x * blockDim.x + threadIdx.x;
  const PhiloxUniform U = philox_uniform(a.t, a.replica, a.colour, a.keys);
  uint32_t acc = 0;
  for (uint32_t k = 0; k < iters; ++k) {
    uint32_t r[4];
    philox_lane(gid + k * nthreads, U, a.keys, r);
    acc ^= xor3(r[0], r[1], r[2] ^ r[3]);
  }
  out[gid] = acc;
}

// Eight independent chains of x <- lo(x*K) + hi(x*K): per link one
// v_mad_u64_u32 (the 32x32 -> 64-bit product Philox rounds use) and one
// 32-bit add, i.e. two VALU instructions.
__global__ __launch_bounds__(256) void k_probe_mad64(uint32_t* out, uint32_t iters, uint32_t seed) {
  const uint32_t gid = blockIdx.x * blockDim.x + threadIdx.x;
  uint32_t x[8];
#pragma unroll
  for (int c = 0; c < 8; ++c) x[c] = gid * 2654435761u + (uint32_t)c + seed;
  for (uint32_t k = 0; k < iters; ++k) {
#pragma unroll
    for (int u = 0; u < 4; ++u) {
#pragma unroll
      for (int c = 0; c < 8; ++c) {
        const uint64_t p = (uint64_t)x[c] * 0xD2511F53u;
        x[c] = (uint32_t)p + (uint32_t)(p >> 32);
      }
    }
  }
  uint32_t acc = 0;
#pragma unroll
  for (int c = 0; c < 8; ++c) acc ^= x[c];
  out[gid] = acc;
}

// Eight independent chains of x <- (x ^ K) + y (one v_xad_u32 each): the issue
// rate of a plain full-rate 32-bit VALU operation.
__global__ __launch_bounds__(256) void k_probe_alu32(uint32_t* out, uint32_t iters, uint32_t seed) {
  const uint32_t gid = blockIdx.x * blockDim.x + threadIdx.x;
  uint32_t x[8], y[8];
#pragma unroll
  for (int c = 0; c < 8; ++c) {
    x[c] = gid * 2654435761u + (uint32_t)c + seed;
    y[c] = gid ^ (0x9E3779B9u * (uint32_t)(c + 1));
  }
  for (uint32_t k = 0; k < iters; ++k) {
#pragma unroll
    for (int u = 0; u < 4; ++u) {
#pragma unroll
      for (int c = 0; c < 8; ++c) x[c] = (x[c] ^ 0xCD9E8D57u) + y[c];
    }
  }
  uint32_t acc = 0;
#pragma unroll
  for (int c = 0; c < 8; ++c) acc = xor3(acc, x[c], y[c]);
  out[gid] = acc;
}

// Streaming copy of n 16-byte words, grid-stride.
__global__ __launch_bounds__(256) void k_probe_copy(const uint4* __restrict__ src, uint4* __restrict__ dst,
                                                    uint64_t n) {
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) dst[i] = src[i];
}

}  // namespace spin

using namespace spin;

extern "C" {

int spin_probe_alu(int kind, uint32_t* out, uint32_t blocks, uint32_t iters, uint64_t seed, void* stream) {
  if (!out || blocks == 0 || iters == 0) return set_error(SPIN_EINVAL, "probe: NULL output or zero size");
  hipStream_t s = (hipStream_t)stream;
  if (kind == SPIN_PROBE_PHILOX) {
    PhaseArgs a;
    a.keys = make_round_keys(seed);
    for (int i = 0; i < 8; ++i) a.bound[i] = 0;
    a.never4 = 0;
    a.L = 0;
    a.t = 1;
    a.colour = 0;
    a.replica = 0;
    hipLaunchKernelGGL(k_probe_philox, dim3(blocks), dim3(256), 0, s, out, iters, a);
  } else if (kind == SPIN_PROBE_MAD64) {
    hipLaunchKernelGGL(k_probe_mad64, dim3(blocks), dim3(256), 0, s, out, iters, (uint32_t)seed);
  } else if (kind == SPIN_PROBE_ALU32) {
    hipLaunchKernelGGL(k_probe_alu32, dim3(blocks), dim3(256), 0, s, out, iters, (uint32_t)seed);
  } else {
    return set_error(SPIN_EINVAL, "probe: unknown kind");
  }
  if (hipGetLastError() != hipSuccess) return set_error(SPIN_EDEVICE, "probe launch failed");
  return SPIN_OK;
}

int spin_probe_copy(const void* src, void* dst, uint64_t bytes, uint32_t blocks, void* stream) {
  if (!src || !dst || bytes == 0 || bytes % 16 != 0 || blocks == 0)
    return set_error(SPIN_EINVAL, "probe copy: NULL buffer, zero size or size not a multiple of 16");
  hipLaunchKernelGGL(k_probe_copy, dim3(blocks), dim3(256), 0, (hipStream_t)stream, (const uint4*)src,
                     (uint4*)dst, bytes / 16);
  if (hipGetLastError() != hipSuccess) return set_error(SPIN_EDEVICE, "probe copy launch failed");
  return SPIN_OK;
}

}  // extern "C"
