// spin_coarse_kernels.hip -- the paper's own schedule (Sec. 3, steps 1-7,
// with the generalized multi-hit of the paragraph after them), a mode with
// its own chain: tiles of edge T on a coarse checkerboard; one launch
// updates every tile of one parity, each workgroup one tile: it loads the
// tile and a one-site boundary layer into LDS, updates the tile's colour-0
// sites, then its colour-1 sites, k times, and writes the tile back.  Tiles
// of one parity are never neighbours and the boundary layer belongs to
// tiles of the other parity, which this launch does not write, so the
// update is in place and race-free.
//
// LDS holds spins as nibble words (spin_nibble.h): a tile row of T sites is
// T/8 words plus one pad word on each side (the whole neighbouring words,
// so that the boundary site sits in the pad's edge nibble); rows y0-1 ..
// y0+T (and in 3D planes z0-1 .. z0+T).  For the +-J glass the packed
// couplings of the same region are staged the same way, once per launch,
// and reused by all k hits.  Hit h of sweep t draws from Philox counter
// (s>>3, t*k + h, replica, colour), as the oracle's coarse mode does.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "spin_internal.h"
#include "spin_nibble.h"
#include "spin_packed.h"

namespace spin {

struct CoarseArgs {
  RoundKeys keys;
  uint32_t bound[8];
  uint32_t never4;   // 4 * never_level
  uint32_t L;
  uint32_t t;        // sweep index
  uint32_t k;        // hits per tile load
  uint32_t replica;
  uint32_t q;        // tile parity of this launch
};

// nib_flips with the bounds from the pair table (spin_packed.h): the active
// nibbles' counts 2u, shifted to 8u per byte, give the byte offsets of two
// 8-byte entries (sites 0 and 1, sites 2 and 3) in two operations where four
// extractions were; never8 = 8 never_level.
template <bool NEVER>
__device__ __forceinline__ uint32_t nib_flips_pair(uint32_t S, uint32_t p, const uint32_t r[4], const char* pair,
                                                   uint32_t never8) {
  const uint32_t T = ((S >> (4u * p)) & 0x0F0F0F0Fu) << 2;  // byte i: 8u of active nibble i
  const uint4 b = lookup_pair(T, pair);
  bool a0 = r[0] <= b.x, a1 = r[1] <= b.y, a2 = r[2] <= b.z, a3 = r[3] <= b.w;
  if (NEVER) {
    a0 = a0 && (T & 0xFFu) >= never8;
    a1 = a1 && __builtin_amdgcn_perm(0u, T, 0x0C0C0C01u) >= never8;
    a2 = a2 && __builtin_amdgcn_ubfe(T, 16u, 8u) >= never8;
    a3 = a3 && (T >> 24) >= never8;
  }
  return (xor3(a0 ? 0xEu : 0u, a1 ? 0xE00u : 0u, a2 ? 0xE0000u : 0u) ^ (a3 ? 0xE000000u : 0u)) << (4u * p);
}

__device__ __forceinline__ uint32_t wrap_m1(uint32_t v, uint32_t n) {  // (v - 1) mod n for v < 2n
  uint32_t w = v + n - 1u;
  return w >= n ? (w >= 2u * n ? w - 2u * n : w - n) : w;
}

template <int D, int T, bool EA, bool NEVER, int NT>
__global__ __launch_bounds__(NT) void k_coarse(int8_t* __restrict__ spins, const uint32_t* __restrict__ Jraw,
                                               CoarseArgs a) {
  constexpr uint32_t TW = T / 8;                     // words per tile row
  constexpr uint32_t RW = TW + 2;                    // words per LDS row
  constexpr uint32_t RR = T + 2;                     // LDS rows per plane
  constexpr uint32_t PL = (D == 3) ? T + 2 : 1;      // LDS planes
  constexpr uint32_t PW = RR * RW;                   // words per LDS plane
  constexpr uint32_t NWL = PL * PW;                  // words of the LDS block
  constexpr uint32_t U = (D == 3) ? T * T * TW : T * TW;  // units (tile words) per colour step
  // accept bounds: the pair table (8 KB) for 2D tiles of edge 32 and 64, the per-u table otherwise
  // (with the small workgroups of smaller tiles, or the 12 KB table of 3D, LDS would cost
  // workgroups per CU: 2D T = 16 lost 25 % at k = 1 with it)
  constexpr bool PAIR = D == 2 && T >= 32;
  __shared__ __align__(16) uint32_t bound[PAIR ? pair_words(4) : 8];
  __shared__ uint32_t sp[NWL];
  __shared__ uint32_t jl[EA ? D * NWL : 1];
  const uint32_t L = a.L, GPR = L / 8;
  const uint32_t NW = (D == 3) ? L * L * GPR : L * GPR;  // words of one direction of couplings
  // Workgroups are dealt to the 8 XCDs round-robin; renumber them so that each XCD takes a
  // contiguous run of tiles in (x, y, z) order: neighbouring tiles share the 128-byte lines of their
  // rows and their boundary rows, and then they share one L2.
  const uint32_t nbx = gridDim.x, nby = gridDim.y, nblk = gridDim.x * gridDim.y * gridDim.z;
  uint32_t blk = blockIdx.x + nbx * (blockIdx.y + nby * blockIdx.z);
  if ((nblk & 7u) == 0) blk = (blk & 7u) * (nblk >> 3) + (blk >> 3);
  const uint32_t bxh = blk % nbx, byz = blk / nbx;
  // tile coordinates: the launch covers the tiles with bx + by (+ bz) = q (mod 2)
  const uint32_t by = byz % nby, bz = (D == 3) ? byz / nby : 0u;
  const uint32_t bx = 2u * bxh + ((by + bz + a.q) & 1u);
  const uint32_t x0w = bx * TW, y0 = by * T, z0 = bz * T;  // first word column, row, plane
  if (PAIR)
    fill_pair<4>(bound, a.bound, threadIdx.x);
  else if (threadIdx.x < 8)
    bound[threadIdx.x] = a.bound[threadIdx.x];
  gu32* Jn = as_global(Jraw);
  // load the tile and its boundary layer
  for (uint32_t i = threadIdx.x; i < NWL; i += NT) {
    const uint32_t p = i / PW, rem = i - p * PW, r = rem / RW, wi = rem - r * RW;
    const uint32_t y = wrap_m1(y0 + r, L);
    const uint32_t z = (D == 3) ? wrap_m1(z0 + p, L) : 0u;
    const uint32_t xw = wrap_m1(x0w + wi, GPR);
    const uint32_t w = (D == 3) ? (z * L + y) * GPR + xw : y * GPR + xw;
    const uint2 b = reinterpret_cast<const uint2*>(spins)[w];
    sp[i] = pack_nibbles(b.x, b.y);
    if (EA) {
#pragma unroll
      for (int dir = 0; dir < D; ++dir) jl[dir * NWL + i] = Jn[dir * NW + w];
    }
  }
  __syncthreads();
  for (uint32_t h = 0; h < a.k; ++h) {
    const uint32_t hit = a.t * a.k + h;
#pragma unroll 1
    for (uint32_t c = 0; c < 2; ++c) {
      const PhiloxUniform Uph = philox_uniform(hit, a.replica, c, a.keys);
      for (uint32_t u = threadIdx.x; u < U; u += NT) {
        // unit u: tile row ry, plane rz, word column cw
        const uint32_t cw = u % TW, rows = u / TW;
        const uint32_t ry = (D == 3) ? rows % T : rows, rz = (D == 3) ? rows / T : 0u;
        const uint32_t o = ((D == 3) ? (rz + 1) * PW : 0u) + (ry + 1) * RW + 1 + cw;
        const uint32_t cv = sp[o];
        uint32_t nb[2 * D - 2];
        nb[0] = sp[o - RW];
        nb[1] = sp[o + RW];
        if (D == 3) {
          nb[2] = sp[o - PW];
          nb[3] = sp[o + PW];
        }
        uint32_t jn[2 * D];
        if (EA) {
          jn[0] = __builtin_amdgcn_alignbit(jl[o], jl[o - 1], 28);  // bond (x-1, x) of each site
          jn[1] = jl[o];
          jn[2] = jl[NWL + o - RW];
          jn[3] = jl[NWL + o];
          if (D == 3) {
            jn[4] = jl[2 * NWL + o - PW];
            jn[5] = jl[2 * NWL + o];
          }
        }
        const uint32_t S = nib_unsat<D, EA>(cv, sp[o - 1], sp[o + 1], nb, jn);
        const uint32_t y = y0 + ry, z = z0 + rz;
        const uint32_t w = (D == 3) ? (z * L + y) * GPR + x0w + cw : y * GPR + x0w + cw;
        uint32_t rnd[4];
        philox_lane(w, Uph, a.keys, rnd);
        const uint32_t p = (c + y + z) & 1u;
        sp[o] = cv ^ (PAIR ? nib_flips_pair<NEVER>(S, p, rnd, (const char*)bound, 2u * a.never4)
                           : nib_flips<NEVER>(S, p, rnd, bound, a.never4));
      }
      __syncthreads();
    }
  }
  // write the tile back
  for (uint32_t u = threadIdx.x; u < U; u += NT) {
    const uint32_t cw = u % TW, rows = u / TW;
    const uint32_t ry = (D == 3) ? rows % T : rows, rz = (D == 3) ? rows / T : 0u;
    const uint32_t o = ((D == 3) ? (rz + 1) * PW : 0u) + (ry + 1) * RW + 1 + cw;
    const uint32_t y = y0 + ry, z = z0 + rz;
    const uint32_t w = (D == 3) ? (z * L + y) * GPR + x0w + cw : y * GPR + x0w + cw;
    uint2 b;
    unpack_nibbles(sp[o], b.x, b.y);
    reinterpret_cast<uint2*>(spins)[w] = b;
  }
}

bool coarse_supported(const Lat& lat, int T) {
  if (lat.L % (uint32_t)T != 0 || (lat.L / (uint32_t)T) % 2 != 0) return false;
  if (lat.J != nullptr && (uint64_t)lat.d * lat.N / 8 >= ((uint64_t)1 << 32)) return false;
  if (lat.d == 2) return T == 8 || T == 16 || T == 32 || T == 64;
  return T == 8 || T == 16;
}

template <int D, int T, int NT>
static hipError_t go_coarse(const Lat& lat, const uint32_t* Jn, const CoarseArgs& a, bool never, hipStream_t stream) {
  const uint32_t B = lat.L / T;
  const dim3 grid(B / 2, B, D == 3 ? B : 1);
  const bool ea = lat.J != nullptr;
  if (ea && never) hipLaunchKernelGGL((k_coarse<D, T, true, true, NT>), grid, dim3(NT), 0, stream, lat.spins, Jn, a);
  if (ea && !never) hipLaunchKernelGGL((k_coarse<D, T, true, false, NT>), grid, dim3(NT), 0, stream, lat.spins, Jn, a);
  if (!ea && never) hipLaunchKernelGGL((k_coarse<D, T, false, true, NT>), grid, dim3(NT), 0, stream, lat.spins, Jn, a);
  if (!ea && !never)
    hipLaunchKernelGGL((k_coarse<D, T, false, false, NT>), grid, dim3(NT), 0, stream, lat.spins, Jn, a);
  return hipGetLastError();
}

hipError_t launch_coarse_phase(const Lat& lat, const uint32_t* Jn, uint32_t t, uint32_t k, uint32_t q,
                               const Accept& acc, int T, hipStream_t stream) {
  if (!coarse_supported(lat, T) || k < 1) return hipErrorInvalidValue;
  if (lat.J != nullptr && !Jn) return hipErrorInvalidValue;
  CoarseArgs a;
  a.keys = lat.keys;
  for (int i = 0; i < 8; ++i) a.bound[i] = acc.bound[i];
  a.never4 = 4u * acc.never_level;
  a.L = lat.L;
  a.t = t;
  a.k = k;
  a.replica = lat.replica;
  a.q = q;
  const bool never = acc.never_level > 0;
  if (lat.d == 2) {
    if (T == 8) return go_coarse<2, 8, 64>(lat, Jn, a, never, stream);
    if (T == 16) return go_coarse<2, 16, 64>(lat, Jn, a, never, stream);
    if (T == 32) return go_coarse<2, 32, 128>(lat, Jn, a, never, stream);
    return go_coarse<2, 64, 256>(lat, Jn, a, never, stream);
  }
  if (T == 8) return go_coarse<3, 8, 64>(lat, Jn, a, never, stream);
  return go_coarse<3, 16, 256>(lat, Jn, a, never, stream);
}

}  // namespace spin
