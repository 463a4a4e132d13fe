// spin_msc.h -- kernels and launch arguments of the multi-spin-coded +-J
// glass (32 systems per word).  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "spin_internal.h"

namespace spin {

struct MscArgs {
  RoundKeys keys;
  uint64_t thr[3];   // T at k = 2d - 2u for u = 0 .. d-1 (k > 0), as 64-bit values (2^32 never counts)
  uint64_t N;        // sites
  uint32_t L;
  uint32_t t;        // sweep index
  uint32_t p0;       // first replica: third counter word of the shared draws
  uint32_t colour;
};

hipError_t launch_msc_init(uint32_t* S, uint64_t N, uint64_t seed, uint32_t p0, hipStream_t stream);
hipError_t launch_msc_couplings(uint32_t* J, uint64_t N, uint32_t d, uint64_t cseed, uint32_t r0, hipStream_t stream);
hipError_t launch_msc_phase(uint32_t* S, const uint32_t* J, const MscArgs& a, uint32_t d, hipStream_t stream);
// Workgroups of the measurement (each writes 64 int64 partial counts).
uint32_t msc_count_parts(uint64_t N);
// E[b], M[b] (device int64[32] each) of the 32 systems; part: msc_count_parts(N) * 64 int64.
hipError_t launch_msc_measure(const uint32_t* S, const uint32_t* J, uint32_t L, uint32_t d, uint64_t N, int64_t* part,
                              int64_t* E, int64_t* M, hipStream_t stream);

}  // namespace spin
