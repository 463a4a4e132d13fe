// spin_phase.h -- kernel arguments and geometry helpers shared by the
// register-parallel sweep kernels, and the entry points of the streaming
// kernels that live in their own sources (spin_stream2d.hip,
// spin_stream3d.hip).  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "spin_device.h"
#include "spin_internal.h"

namespace spin {

// (v - back) mod L for 0 <= v < L + 2L and back <= L: the coordinate `back`
// sites before v, wrapped periodically.
__device__ __forceinline__ uint32_t wrap_row(uint32_t v, uint32_t back, uint32_t L) {
  uint32_t w = v + L - back;  // in [0, 3L)
  if (w >= L) w -= L;
  if (w >= L) w -= L;
  return w;
}

// Kernel arguments of the register-parallel phase kernels.
struct PhaseArgs {
  RoundKeys keys;
  uint32_t bound[8];
  uint32_t never4;  // 4 * never_level
  uint32_t L;
  uint32_t t;
  uint32_t colour;
  uint32_t replica;
};

inline PhaseArgs phase_args(const Lat& lat, uint32_t t, uint32_t colour, const Accept& acc) {
  PhaseArgs a;
  a.keys = lat.keys;
  for (int i = 0; i < 8; ++i) a.bound[i] = acc.bound[i];
  a.never4 = 4u * acc.never_level;
  a.L = lat.L;
  a.t = t;
  a.colour = colour;
  a.replica = lat.replica;
  return a;
}

// 2D Ising streaming sweep (k_stream2d): L = 8 * threads * G with
// (threads, G) in {(1024, 1), (1024, 2), (512, 1), (512, 2), (256, 2)}.
bool stream2d_shape(uint32_t L, int threads, int* G);
hipError_t launch_stream2d(const Lat& lat, const int8_t* src, int8_t* dst, const PhaseArgs& a, bool never,
                           uint32_t H, const Record* rec, int threads, int G, hipStream_t stream);
// The register-column form of the same sweep (k_stream2c), same shapes; with
// rec it also counts E/M inside the sweep into one partial per workgroup.
hipError_t launch_stream2c(const Lat& lat, const int8_t* src, int8_t* dst, const PhaseArgs& a, bool never,
                           uint32_t H, const Record* rec, int threads, int G, hipStream_t stream);

// 3D Ising streaming sweep: tile.x == L, tile.y = rows per workgroup, tile.z =
// planes per strip, tile.threads = 64 * waves.  L = 512 with (16, 576) or
// (8, 320) runs the register-column kernel (k_stream3r), which can also count
// E/M of its result into rec (*measured = true); the other shapes (L = 512 or
// 1024) run k_stream3d.
bool stream3d_shape(const Lat& lat, const Tile& tile);
uint32_t stream3d_record_parts(const Lat& lat, const Tile& tile);  // 0: the kernel cannot count
hipError_t launch_stream3d(const Lat& lat, const int8_t* src, int8_t* dst, const PhaseArgs& a, bool never,
                           const Tile& tile, const Record* rec, bool* measured, hipStream_t stream);

}  // namespace spin
