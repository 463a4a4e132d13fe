// spin_lcg.h -- launchers of the LCG-driven chain (RNG-quality experiment).
// Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace spin {

struct LcgArgs {
  uint64_t T[8];    // acceptance thresholds T[(k+z)/2]
  uint64_t N;       // sites (a multiple of 8)
  uint32_t L;
  uint32_t colour;
  uint32_t mode;    // SPIN_RNG_LCG32_ARRAY, _LCG32_DISJOINT or _LCG64_DISJOINT
};

// Initial states of the G groups' generators (mode as in LcgArgs).
hipError_t launch_lcg_init(uint64_t* st, uint64_t G, uint32_t mode, uint64_t seed, uint32_t replica,
                           hipStream_t stream);
// One colour phase of the Ising lattice S (d = 2 or 3, L % 8 == 0), states st advanced in place.
hipError_t launch_lcg_phase(int8_t* S, uint64_t* st, uint32_t d, const LcgArgs& a, hipStream_t stream);

}  // namespace spin
