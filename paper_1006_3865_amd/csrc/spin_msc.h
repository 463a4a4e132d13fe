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
// J: d*N words; the x bonds in site order, the y and z bonds with each row
// split by x parity (even-x words first).
hipError_t launch_msc_couplings(uint32_t* J, uint64_t N, uint32_t L, uint32_t d, uint64_t cseed, uint32_t r0,
                                hipStream_t stream);
// J6: per 8-site group and colour, the 2d coupling words of each of the 4
// active sites (-x, +x, -y, +y, -z, +z), 2d*N words, built from J.
hipError_t launch_msc_bonds(const uint32_t* J, uint32_t* J6, uint32_t L, uint32_t d, uint64_t N, hipStream_t stream);
hipError_t launch_msc_phase(uint32_t* S, const uint32_t* J6, const MscArgs& a, uint32_t d, hipStream_t stream);
// One sweep per launch, streamed over planes (both colours; ping-pong
// src -> dst): TY rows per workgroup (3D, divides L, <= 32), H planes per
// strip, NT = 256 or 512 threads, XW sites of each row per workgroup (a
// multiple of 8 dividing L); false when the shape does not fit.
bool msc_stream_supported(uint32_t L, uint32_t d, uint32_t TY, uint32_t H, uint32_t NT, uint32_t XW);
hipError_t launch_msc_stream(const uint32_t* src, uint32_t* dst, const uint32_t* J, const MscArgs& a, uint32_t d,
                             uint32_t TY, uint32_t H, uint32_t NT, uint32_t XW, hipStream_t stream);
// 3D L = 128, 256 or 512: one sweep per launch with each row's z column in
// registers and every coupling word read once (ping-pong src -> dst): TY = 4
// or 8 rows per workgroup (TY + 2 wavefronts), H planes per strip (even,
// dividing L).
bool msc_col_supported(uint32_t L, uint32_t d, uint32_t TY, uint32_t H);
hipError_t launch_msc_col(const uint32_t* src, uint32_t* dst, const uint32_t* J, const MscArgs& a, uint32_t d,
                          uint32_t TY, uint32_t H, hipStream_t stream);
// Workgroups of the measurement (each writes 64 int64 partial counts).
uint32_t msc_count_parts(uint64_t N);
// E[b], M[b] (device int64[32] each) of the 32 systems; part: msc_count_parts(N) * 64 int64.
hipError_t launch_msc_measure(const uint32_t* S, const uint32_t* J, uint32_t L, uint32_t d, uint64_t N, int64_t* part,
                              int64_t* E, int64_t* M, hipStream_t stream);

}  // namespace spin
