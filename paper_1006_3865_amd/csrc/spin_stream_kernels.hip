// spin_stream_kernels.hip -- one whole sweep per launch for any L % 8 == 0,
// 2D or 3D, Ising or +-J (Sec. 3, Eq. 2; Sec. 4 for the glass).
//
// The lattice is streamed along its slowest axis ("planes": z in 3D, rows in
// 2D).  A workgroup owns the planes [z0, z0+H) (and in 3D the rows
// [y0, y0+TY) of them) and keeps a ring of 6 plane slices in LDS, spins
// packed 8 per word as nibbles (spin_nibble.h).  A 3D slice holds the rows
// y0-2 .. y0+TY+1 (slice row r <-> y = y0-2+r); a 2D slice is one row.  Each
// slice row has one pad word on each side holding the periodic neighbour
// word (word GPR-1 left of word 0, word 0 right of word GPR-1).  Plane
// k = z - z0 + 2 lives in slot k % 6.
//
// Step i = 0 .. H+2, with a = z0-1+i:
//   load plane a+2 into its slot (the slot of plane a-4, unused this step);
//   colour 0 on plane a (3D: slice rows 1..TY+2, i.e. the owned rows and a
//     one-row ring that colour 1 needs): reads planes a-1..a+1, writes a;
//   colour 1 on plane a-2 (owned rows only): reads planes a-3..a-1, writes
//     the finished words (both colours) to dst;
//   barrier.
// Colour-0 results stay in LDS and colour-1 results go to HBM, so the ring
// always holds colour-1 values from before the sweep, as colour 0 needs,
// and colour-0 values from this sweep, as colour 1 needs (the order of the
// canonical chain: all colour-0 sites of sweep t, then all colour-1 sites).
// In-place writes of plane a race with nobody: a colour-0 update reads only
// colour-1 nibbles of its neighbours, which the writes leave unchanged.
// Neighbouring strips recompute the colour-0 planes z0-1 and z0+H from the
// same data, so they agree bit for bit.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "spin_internal.h"
#include "spin_nibble.h"

namespace spin {

struct StreamArgs {
  RoundKeys keys;
  uint32_t bound[8];
  uint32_t never4;  // 4 * never_level
  uint32_t L;       // edge
  uint32_t GPR;     // words (8-site groups) per row = L / 8
  uint32_t t;       // sweep index
  uint32_t replica;
  uint32_t TY;      // 3D: rows per workgroup (divides L); 2D: 1
  uint32_t H;       // planes per strip
};

__device__ __forceinline__ uint32_t wrap_sub2(uint32_t v, uint32_t L) {  // (v - 2) mod L, v < 2L + 2
  uint32_t w = v + L - 2u;
  if (w >= L) w -= L;
  if (w >= L) w -= L;
  return w;
}

// Load plane z (global, int8) into ring slot `slot` as nibble words, with pads.
template <int D, int NT>
__device__ __forceinline__ void sg_load(const int8_t* __restrict__ src, uint32_t* slot, uint32_t z, uint32_t y0,
                                        const StreamArgs& a, uint32_t RP, uint32_t RW) {
  const uint32_t GPR = a.GPR, L = a.L;
  const uint32_t tot = RP * GPR;
  const uint32_t dr = NT / GPR, dg = NT - dr * GPR;
  uint32_t r = threadIdx.x / GPR, g = threadIdx.x - r * GPR;
  const uint2* s2 = reinterpret_cast<const uint2*>(src);
  for (uint32_t u = threadIdx.x; u < tot; u += NT) {
    const uint32_t y = (D == 3) ? wrap_sub2(y0 + r, L) : 0u;
    const uint32_t w = (D == 3) ? (z * L + y) * GPR + g : z * GPR + g;
    const uint2 b = s2[w];
    const uint32_t v = pack_nibbles(b.x, b.y);
    uint32_t* row = slot + r * RW;
    row[1 + g] = v;
    if (g == 0) row[GPR + 1] = v;
    if (g == GPR - 1) row[0] = v;
    g += dg;
    r += dr;
    if (g >= GPR) {
      g -= GPR;
      r += 1;
    }
  }
}

// Update the colour-C nibbles of word g of slice row r (slots pm, pc, pp hold
// planes z-1, z, z+1); returns the new word.
template <int D, bool EA, bool NEVER, uint32_t C>
__device__ __forceinline__ uint32_t sg_unit(const uint32_t* pm, const uint32_t* pc, const uint32_t* pp, uint32_t r,
                                            uint32_t g, uint32_t y, uint32_t z, const StreamArgs& a,
                                            const PhiloxUniform& U, const uint32_t* bound, gu32* Jn, uint32_t NW,
                                            uint32_t RW) {
  const uint32_t GPR = a.GPR, L = a.L;
  const uint32_t o = r * RW + 1 + g;
  const uint32_t c = pc[o];
  const uint32_t lw = pc[o - 1], rw = pc[o + 1];
  uint32_t nb[2 * D - 2];
  if (D == 3) {
    nb[0] = pc[o - RW];
    nb[1] = pc[o + RW];
    nb[2] = pm[o];
    nb[3] = pp[o];
  } else {
    nb[0] = pm[o];
    nb[1] = pp[o];
  }
  const uint32_t w = (D == 3) ? (z * L + y) * GPR + g : z * GPR + g;
  uint32_t jn[2 * D];
  if (EA) {
    const uint32_t wl = g ? w - 1u : w + GPR - 1u;
    const uint32_t jx = Jn[w];
    jn[0] = __builtin_amdgcn_alignbit(jx, Jn[wl], 28);
    jn[1] = jx;
    if (D == 3) {
      const uint32_t wym = y ? w - GPR : w + (L - 1u) * GPR;
      const uint32_t wzm = z ? w - L * GPR : w + (L - 1u) * L * GPR;
      jn[2] = Jn[NW + wym];
      jn[3] = Jn[NW + w];
      jn[4] = Jn[2 * NW + wzm];
      jn[5] = Jn[2 * NW + w];
    } else {
      const uint32_t wym = z ? w - GPR : w + (L - 1u) * GPR;
      jn[2] = Jn[NW + wym];
      jn[3] = Jn[NW + w];
    }
  }
  const uint32_t S = nib_unsat<D, EA>(c, lw, rw, nb, jn);
  uint32_t rnd[4];
  philox_lane(w, U, a.keys, rnd);
  const uint32_t p = (C + y + z) & 1u;
  return c ^ nib_flips<NEVER>(S, p, rnd, bound, a.never4);
}

template <int D, bool EA, bool NEVER, int NT>
__global__ __launch_bounds__(NT) void k_streamg(const int8_t* __restrict__ src, int8_t* __restrict__ dst,
                                                const uint32_t* __restrict__ Jraw, StreamArgs a) {
  extern __shared__ __align__(16) uint32_t lds[];
  uint32_t* bound = lds;  // first: constant-offset lookups
  uint32_t* ring = lds + 8;
  const uint32_t L = a.L, GPR = a.GPR;
  const uint32_t RW = GPR + 2;
  const uint32_t TY = (D == 3) ? a.TY : 1u;
  const uint32_t RP = (D == 3) ? TY + 4 : 1u;
  const uint32_t SB = RP * RW;
  const uint32_t NW = (D == 3) ? L * L * GPR : L * GPR;
  const uint32_t y0 = (D == 3) ? blockIdx.x * TY : 0u;
  const uint32_t z0 = blockIdx.y * a.H;
  const uint32_t H = (L - z0 < a.H) ? L - z0 : a.H;
  gu32* Jn = as_global(Jraw);
  if (threadIdx.x < 8) bound[threadIdx.x] = a.bound[threadIdx.x];
  const PhiloxUniform U0 = philox_uniform(a.t, a.replica, 0u, a.keys);
  const PhiloxUniform U1 = philox_uniform(a.t, a.replica, 1u, a.keys);
  for (uint32_t k = 0; k < 3; ++k) sg_load<D, NT>(src, ring + k * SB, wrap_sub2(z0 + k, L), y0, a, RP, RW);
  __syncthreads();
  // units: colour 0 on slice rows 1..TY+2 (3D) / row 0 (2D); colour 1 on rows 2..TY+1 / row 0
  const uint32_t U0n = (D == 3) ? (TY + 2) * GPR : GPR;
  const uint32_t U1n = (D == 3) ? TY * GPR : GPR;
  const uint32_t dr = NT / GPR, dg = NT - dr * GPR;
  const uint32_t r_first = threadIdx.x / GPR, g_first = threadIdx.x - r_first * GPR;
  uint32_t sa = 1;  // slot of plane a = z0 - 1 + i
  for (uint32_t i = 0; i < H + 3; ++i) {
    const uint32_t s_m3 = sa >= 3 ? sa - 3 : sa + 3;   // a-3
    const uint32_t s_m2 = sa >= 2 ? sa - 2 : sa + 4;   // a-2
    const uint32_t s_m1 = sa >= 1 ? sa - 1 : 5;        // a-1
    const uint32_t s_p1 = sa <= 4 ? sa + 1 : 0;        // a+1
    const uint32_t s_p2 = sa <= 3 ? sa + 2 : sa - 4;   // a+2
    if (i <= H) sg_load<D, NT>(src, ring + s_p2 * SB, wrap_sub2(z0 + i + 3, L), y0, a, RP, RW);
    if (i <= H + 1) {
      const uint32_t za = wrap_sub2(z0 + i + 1, L);
      const uint32_t* pm = ring + s_m1 * SB;
      uint32_t* pc = ring + sa * SB;
      const uint32_t* pp = ring + s_p1 * SB;
      uint32_t r = r_first, g = g_first;
      for (uint32_t u = threadIdx.x; u < U0n; u += NT) {
        const uint32_t rr = (D == 3) ? r + 1 : 0u;
        const uint32_t y = (D == 3) ? wrap_sub2(y0 + rr, L) : 0u;
        const uint32_t v = sg_unit<D, EA, NEVER, 0>(pm, pc, pp, rr, g, y, za, a, U0, bound, Jn, NW, RW);
        uint32_t* row = pc + rr * RW;
        row[1 + g] = v;
        if (g == 0) row[GPR + 1] = v;
        if (g == GPR - 1) row[0] = v;
        g += dg;
        r += dr;
        if (g >= GPR) {
          g -= GPR;
          r += 1;
        }
      }
    }
    if (i >= 3) {
      const uint32_t zb = z0 + i - 3u;
      const uint32_t* pm = ring + s_m3 * SB;
      const uint32_t* pc = ring + s_m2 * SB;
      const uint32_t* pp = ring + s_m1 * SB;
      uint2* d2 = reinterpret_cast<uint2*>(dst);
      uint32_t r = r_first, g = g_first;
      for (uint32_t u = threadIdx.x; u < U1n; u += NT) {
        const uint32_t rr = (D == 3) ? r + 2 : 0u;
        const uint32_t y = (D == 3) ? y0 + r : 0u;
        const uint32_t v = sg_unit<D, EA, NEVER, 1>(pm, pc, pp, rr, g, y, zb, a, U1, bound, Jn, NW, RW);
        const uint32_t w = (D == 3) ? (zb * L + y) * GPR + g : zb * GPR + g;
        uint2 b;
        unpack_nibbles(v, b.x, b.y);
        d2[w] = b;
        g += dg;
        r += dr;
        if (g >= GPR) {
          g -= GPR;
          r += 1;
        }
      }
    }
    __syncthreads();
    sa = sa == 5 ? 0 : sa + 1;
  }
}

// Supported: L % 8 == 0, L >= 16; 3D: TY in {4, 8, 16, 32} dividing L;
// H >= 1 (the last strip may be shorter); threads 256 or 512.
bool streamg_supported(const Lat& lat, const Tile& tile) {
  if (lat.L % 8 != 0 || lat.L < 16) return false;
  if (tile.threads != 256 && tile.threads != 512) return false;
  if (tile.z < 1 || (uint32_t)tile.z > lat.L) return false;
  if (lat.d == 3) {
    if (tile.y != 4 && tile.y != 8 && tile.y != 16 && tile.y != 32) return false;
    if (lat.L % (uint32_t)tile.y != 0) return false;
  }
  return streamg_lds_bytes(lat, tile) <= 150 * 1024;
}

size_t streamg_lds_bytes(const Lat& lat, const Tile& tile) {
  const size_t RW = lat.L / 8 + 2;
  const size_t RP = lat.d == 3 ? (size_t)tile.y + 4 : 1;
  return 32 + 6 * RP * RW * 4;
}

template <int D, bool EA, int NT>
static hipError_t go_streamg(dim3 grid, size_t lds, bool never, const int8_t* src, int8_t* dst, const uint32_t* Jn,
                             const StreamArgs& a, hipStream_t stream) {
  static bool attr = false;
  if (!attr) {
    hipError_t e = hipFuncSetAttribute((const void*)k_streamg<D, EA, true, NT>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, 150 * 1024);
    if (e == hipSuccess)
      e = hipFuncSetAttribute((const void*)k_streamg<D, EA, false, NT>, hipFuncAttributeMaxDynamicSharedMemorySize,
                              150 * 1024);
    if (e != hipSuccess) return e;
    attr = true;
  }
  if (never)
    hipLaunchKernelGGL((k_streamg<D, EA, true, NT>), grid, dim3(NT), lds, stream, src, dst, Jn, a);
  else
    hipLaunchKernelGGL((k_streamg<D, EA, false, NT>), grid, dim3(NT), lds, stream, src, dst, Jn, a);
  return hipGetLastError();
}

hipError_t launch_streamg(const Lat& lat, const uint32_t* Jn, const int8_t* src, int8_t* dst, uint32_t t,
                          const Accept& acc, const Tile& tile, hipStream_t stream) {
  if (!streamg_supported(lat, tile)) return hipErrorInvalidValue;
  const bool ea = lat.J != nullptr;
  if (ea && !Jn) return hipErrorInvalidValue;
  StreamArgs a;
  a.keys = lat.keys;
  for (int i = 0; i < 8; ++i) a.bound[i] = acc.bound[i];
  a.never4 = 4u * acc.never_level;
  a.L = lat.L;
  a.GPR = lat.L / 8;
  a.t = t;
  a.replica = lat.replica;
  a.TY = lat.d == 3 ? (uint32_t)tile.y : 1u;
  a.H = (uint32_t)tile.z;
  const dim3 grid(lat.d == 3 ? lat.L / a.TY : 1u, (lat.L + a.H - 1) / a.H);
  const size_t lds = streamg_lds_bytes(lat, tile);
  const bool never = acc.never_level > 0;
  if (lat.d == 2) {
    if (tile.threads == 256)
      return ea ? go_streamg<2, true, 256>(grid, lds, never, src, dst, Jn, a, stream)
                : go_streamg<2, false, 256>(grid, lds, never, src, dst, Jn, a, stream);
    return ea ? go_streamg<2, true, 512>(grid, lds, never, src, dst, Jn, a, stream)
              : go_streamg<2, false, 512>(grid, lds, never, src, dst, Jn, a, stream);
  }
  if (tile.threads == 256)
    return ea ? go_streamg<3, true, 256>(grid, lds, never, src, dst, Jn, a, stream)
              : go_streamg<3, false, 256>(grid, lds, never, src, dst, Jn, a, stream);
  return ea ? go_streamg<3, true, 512>(grid, lds, never, src, dst, Jn, a, stream)
            : go_streamg<3, false, 512>(grid, lds, never, src, dst, Jn, a, stream);
}

}  // namespace spin
