// spin_heis.h -- launchers of the classical Heisenberg mode.  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "spin_device.h"

namespace spin {

struct HeisArgs {
  RoundKeys keys;
  uint64_t N;        // sites
  uint32_t L;
  uint32_t t;        // sweep index
  uint32_t replica;
  uint32_t colour;
  float beta;        // beta rounded to float
};

hipError_t launch_heis_init(float4* S, uint64_t N, uint64_t seed, uint32_t replica, hipStream_t stream);
// One colour phase (d = 2 or 3), in place.
hipError_t launch_heis_phase(float4* S, uint32_t d, const HeisArgs& a, hipStream_t stream);
// heis_measure_blocks(N) workgroups each write (E, Mx, My, Mz) as 4 doubles into part.
uint32_t heis_measure_blocks(uint64_t N);
hipError_t launch_heis_measure(const float4* S, uint32_t L, uint32_t d, uint64_t N, double* part, hipStream_t stream);

}  // namespace spin
