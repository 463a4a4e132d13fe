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

// Words of a plane slice each thread loads (slice words u = thread + NT*q).
constexpr int kFetch = 8;

// Load the slice of plane z (global, int8) into registers: word u of the
// slice is row u / GPR, column u % GPR.
template <int D, int NT>
__device__ __forceinline__ void sg_fetch(const int8_t* __restrict__ src, uint32_t z, uint32_t y0, const StreamArgs& a,
                                         uint32_t tot, uint2 (&v)[kFetch]) {
  const uint32_t GPR = a.GPR, L = a.L;
  const uint32_t dr = NT / GPR, dg = NT - dr * GPR;
  uint32_t r = threadIdx.x / GPR, g = threadIdx.x - r * GPR;
  const uint2* s2 = reinterpret_cast<const uint2*>(src);
#pragma unroll
  for (int q = 0; q < kFetch; ++q) {
    if (threadIdx.x + NT * q < tot) {
      const uint32_t y = (D == 3) ? wrap_sub2(y0 + r, L) : 0u;
      const uint32_t w = (D == 3) ? (z * L + y) * GPR + g : z * GPR + g;
      v[q] = s2[w];
    }
    g += dg;
    r += dr;
    if (g >= GPR) {
      g -= GPR;
      r += 1;
    }
  }
}

// Store fetched words into ring slot `slot` as nibble words, with the pads:
// word g of a slice row at OFF + g, word GPR-1 again at OFF - 1 and word 0 at
// OFF + GPR (OFF = 1; 2 in the word-pair form, so that pairs are 8-byte aligned).
template <int NT, uint32_t OFF>
__device__ __forceinline__ void sg_store(uint32_t* slot, const StreamArgs& a, uint32_t tot, uint32_t RW,
                                         const uint2 (&v)[kFetch]) {
  const uint32_t GPR = a.GPR;
  const uint32_t dr = NT / GPR, dg = NT - dr * GPR;
  uint32_t r = threadIdx.x / GPR, g = threadIdx.x - r * GPR;
#pragma unroll
  for (int q = 0; q < kFetch; ++q) {
    if (threadIdx.x + NT * q < tot) {
      const uint32_t x = pack_nibbles(v[q].x, v[q].y);
      uint32_t* row = slot + r * RW;
      row[OFF + g] = x;
      if (g == 0) row[OFF + GPR] = x;
      if (g == GPR - 1) row[OFF - 1] = x;
    }
    g += dg;
    r += dr;
    if (g >= GPR) {
      g -= GPR;
      r += 1;
    }
  }
}

// Couplings of the 2d bonds of word w (raw words: x at w and its left
// neighbour word, y at w and the row below, z at w and the plane below).
template <int D>
__device__ __forceinline__ void sg_jload(gu32* Jn, uint32_t NW, uint32_t w, uint32_t g, uint32_t y, uint32_t z,
                                         const StreamArgs& a, uint32_t (&j)[2 * D]) {
  const uint32_t GPR = a.GPR, L = a.L;
  const uint32_t wl = g ? w - 1u : w + GPR - 1u;
  j[0] = ldg_word(Jn, wl);
  j[1] = ldg_word(Jn, w);
  if (D == 3) {
    const uint32_t wym = y ? w - GPR : w + (L - 1u) * GPR;
    const uint32_t wzm = z ? w - L * GPR : w + (L - 1u) * L * GPR;
    j[2] = ldg_word(Jn, NW + wym);
    j[3] = ldg_word(Jn, NW + w);
    j[4] = ldg_word(Jn, 2 * NW + wzm);
    j[5] = ldg_word(Jn, 2 * NW + w);
  } else {
    const uint32_t wym = z ? w - GPR : w + (L - 1u) * GPR;
    j[2] = ldg_word(Jn, NW + wym);
    j[3] = ldg_word(Jn, NW + w);
  }
}

// Update the colour-C nibbles of word g of slice row r (slots pm, pc, pp hold
// planes z-1, z, z+1; w is the word's global index, jr its raw couplings);
// returns the new word.
template <int D, bool EA, bool NEVER, uint32_t C>
__device__ __forceinline__ uint32_t sg_unit(const uint32_t* pm, const uint32_t* pc, const uint32_t* pp, uint32_t r,
                                            uint32_t g, uint32_t y, uint32_t z, uint32_t w, const StreamArgs& a,
                                            const PhiloxUniform& U, const uint32_t* bound, uint32_t RW,
                                            const uint32_t (&jr)[2 * D]) {
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
  uint32_t jn[2 * D];
  if (EA) {
    jn[0] = __builtin_amdgcn_alignbit(jr[1], jr[0], 28);  // bond (x-1, x) of each site
    jn[1] = jr[1];
    jn[2] = jr[2];
    jn[3] = jr[3];
    if (D == 3) {
      jn[4] = jr[4];
      jn[5] = jr[5];
    }
  }
  const uint32_t S = nib_unsat<D, EA>(c, lw, rw, nb, jn);
  uint32_t rnd[4];
  philox_lane(w, U, a.keys, rnd);
  const uint32_t p = (C + y + z) & 1u;
  return c ^ nib_flips<NEVER>(S, p, rnd, bound, a.never4);
}

// The colour-C units of one step: slice rows RB0 + (u / GPR), words u % GPR,
// u = thread + NT*q < n.  Colour 0 writes back into slot pc (with pads),
// colour 1 writes the finished words to dst.  The couplings of the next unit
// are loaded while the current one is computed.
template <int D, bool EA, bool NEVER, int NT, uint32_t C>
__device__ __forceinline__ void sg_units(const uint32_t* pm, uint32_t* pc, const uint32_t* pp, uint32_t n, uint32_t y0,
                                         uint32_t z, const StreamArgs& a, const PhiloxUniform& U,
                                         const uint32_t* bound, uint32_t RW, gu32* Jn, uint32_t NW,
                                         int8_t* __restrict__ dst) {
  const uint32_t GPR = a.GPR, L = a.L;
  constexpr uint32_t RB0 = (D == 3) ? (C == 0 ? 1u : 2u) : 0u;  // first slice row
  const uint32_t dr = NT / GPR, dg = NT - dr * GPR;
  uint32_t r = threadIdx.x / GPR, g = threadIdx.x - r * GPR;
  // slice row rr -> y: colour 0 rows may wrap (y0 - 1, y0 + TY), colour 1 rows are owned
  auto ycoord = [&](uint32_t rr) -> uint32_t {
    if (D != 3) return 0u;
    return C == 0 ? wrap_sub2(y0 + rr, L) : y0 + rr - 2u;
  };
  auto word = [&](uint32_t y, uint32_t gg) -> uint32_t { return (D == 3) ? (z * L + y) * GPR + gg : z * GPR + gg; };
  uint32_t jc[2 * D] = {}, jx[2 * D] = {};
  if (EA && threadIdx.x < n) sg_jload<D>(Jn, NW, word(ycoord(r + RB0), g), g, ycoord(r + RB0), z, a, jc);
  for (uint32_t u = threadIdx.x; u < n; u += NT) {
    const uint32_t rr = r + RB0;
    const uint32_t y = ycoord(rr);
    const uint32_t w = word(y, g);
    uint32_t rn = r + dr, gn = g + dg;
    if (gn >= GPR) {
      gn -= GPR;
      rn += 1;
    }
    if (EA && u + NT < n) sg_jload<D>(Jn, NW, word(ycoord(rn + RB0), gn), gn, ycoord(rn + RB0), z, a, jx);
    const uint32_t v = sg_unit<D, EA, NEVER, C>(pm, pc, pp, rr, g, y, z, w, a, U, bound, RW, jc);
    if (C == 0) {
      uint32_t* row = pc + rr * RW;
      row[1 + g] = v;
      if (g == 0) row[GPR + 1] = v;
      if (g == GPR - 1) row[0] = v;
    } else {
      uint2 b;
      unpack_nibbles(v, b.x, b.y);
      reinterpret_cast<uint2*>(dst)[w] = b;
    }
    if (EA) {
#pragma unroll
      for (int k = 0; k < 2 * D; ++k) jc[k] = jx[k];
    }
    r = rn;
    g = gn;
  }
}

// Word-pair form (GPR even): thread units are pairs of adjacent words
// (g, g+1), g even.  A pair reads each neighbour row with one 8-byte LDS
// access and each coupling direction and side with one 8-byte load (3
// coupling loads per word instead of 6); the x neighbours and the x bond
// between the two words come from the pair itself; colour 1 stores the two
// finished words as one 16-byte store.
typedef uint32_t sg_u2 __attribute__((ext_vector_type(2)));

__device__ __forceinline__ uint2 ldg_pair(gu32* base, uint32_t i) {  // words i, i+1 (i even)
  const sg_u2 v = *reinterpret_cast<const __attribute__((address_space(1))) sg_u2*>(
      reinterpret_cast<gc8*>(base) + (uint64_t)(i << 2));
  return make_uint2(v.x, v.y);
}

// Couplings of the pair at words w, w+1: x at the pair and the word left of
// it, y at the pair and the row below, z at the pair and the plane below.
template <int D>
__device__ __forceinline__ void sg_jload2(gu32* Jn, uint32_t NW, uint32_t w, uint32_t g, uint32_t y, uint32_t z,
                                          const StreamArgs& a, uint32_t (&j)[4 * D + 1]) {
  const uint32_t GPR = a.GPR, L = a.L;
  const uint32_t wl = g ? w - 1u : w + GPR - 1u;
  j[0] = ldg_word(Jn, wl);
  const uint2 jx = ldg_pair(Jn, w);
  j[1] = jx.x;
  j[2] = jx.y;
  const uint32_t wym = (D == 3) ? (y ? w - GPR : w + (L - 1u) * GPR) : (z ? w - GPR : w + (L - 1u) * GPR);
  const uint2 jym = ldg_pair(Jn, NW + wym), jy = ldg_pair(Jn, NW + w);
  j[3] = jym.x;
  j[4] = jym.y;
  j[5] = jy.x;
  j[6] = jy.y;
  if (D == 3) {
    const uint32_t wzm = z ? w - L * GPR : w + (L - 1u) * L * GPR;
    const uint2 jzm = ldg_pair(Jn, 2 * NW + wzm), jz = ldg_pair(Jn, 2 * NW + w);
    j[7] = jzm.x;
    j[8] = jzm.y;
    j[9] = jz.x;
    j[10] = jz.y;
  }
}

// Update the colour-C nibbles of the pair at word g (even) of slice row r;
// returns the two new words.
template <int D, bool EA, bool NEVER, uint32_t C>
__device__ __forceinline__ uint2 sg_unit2(const uint32_t* pm, const uint32_t* pc, const uint32_t* pp, uint32_t r,
                                          uint32_t g, uint32_t y, uint32_t z, uint32_t w, const StreamArgs& a,
                                          const PhiloxUniform& U, const uint32_t* bound, uint32_t RW,
                                          const uint32_t (&jr)[4 * D + 1]) {
  const uint32_t o = r * RW + 2 + g;
  const uint2 c = *reinterpret_cast<const uint2*>(pc + o);
  const uint32_t lw = pc[o - 1], rw = pc[o + 2];
  uint2 nbp[2 * D - 2];
  if (D == 3) {
    nbp[0] = *reinterpret_cast<const uint2*>(pc + o - RW);
    nbp[1] = *reinterpret_cast<const uint2*>(pc + o + RW);
    nbp[2] = *reinterpret_cast<const uint2*>(pm + o);
    nbp[3] = *reinterpret_cast<const uint2*>(pp + o);
  } else {
    nbp[0] = *reinterpret_cast<const uint2*>(pm + o);
    nbp[1] = *reinterpret_cast<const uint2*>(pp + o);
  }
  uint32_t nb0[2 * D - 2], nb1[2 * D - 2], jn0[2 * D], jn1[2 * D];
#pragma unroll
  for (int k = 0; k < 2 * D - 2; ++k) {
    nb0[k] = nbp[k].x;
    nb1[k] = nbp[k].y;
  }
  if (EA) {
    jn0[0] = __builtin_amdgcn_alignbit(jr[1], jr[0], 28);  // bond (x-1, x) of each site
    jn0[1] = jr[1];
    jn1[0] = __builtin_amdgcn_alignbit(jr[2], jr[1], 28);
    jn1[1] = jr[2];
    jn0[2] = jr[3];
    jn1[2] = jr[4];
    jn0[3] = jr[5];
    jn1[3] = jr[6];
    if (D == 3) {
      jn0[4] = jr[7];
      jn1[4] = jr[8];
      jn0[5] = jr[9];
      jn1[5] = jr[10];
    }
  }
  const uint32_t S0 = nib_unsat<D, EA>(c.x, lw, c.y, nb0, jn0);
  const uint32_t S1 = nib_unsat<D, EA>(c.y, c.x, rw, nb1, jn1);
  uint32_t r0[4], r1[4];
  philox_lane(w, U, a.keys, r0);
  philox_lane(w + 1u, U, a.keys, r1);
  const uint32_t p = (C + y + z) & 1u;
  return make_uint2(c.x ^ nib_flips<NEVER>(S0, p, r0, bound, a.never4),
                    c.y ^ nib_flips<NEVER>(S1, p, r1, bound, a.never4));
}

// The colour-C pairs of one step: slice rows RB0 + u / (GPR/2), pairs
// u % (GPR/2), u = thread + NT*q < n (pairs).  As sg_units.
template <int D, bool EA, bool NEVER, int NT, uint32_t C>
__device__ __forceinline__ void sg_units2(const uint32_t* pm, uint32_t* pc, const uint32_t* pp, uint32_t n,
                                          uint32_t y0, uint32_t z, const StreamArgs& a, const PhiloxUniform& U,
                                          const uint32_t* bound, uint32_t RW, gu32* Jn, uint32_t NW,
                                          int8_t* __restrict__ dst) {
  const uint32_t GPR = a.GPR, L = a.L, PG = GPR / 2;
  constexpr uint32_t RB0 = (D == 3) ? (C == 0 ? 1u : 2u) : 0u;  // first slice row
  const uint32_t dr = NT / PG, dg = NT - dr * PG;
  uint32_t r = threadIdx.x / PG, q = threadIdx.x - r * PG;
  auto ycoord = [&](uint32_t rr) -> uint32_t {
    if (D != 3) return 0u;
    return C == 0 ? wrap_sub2(y0 + rr, L) : y0 + rr - 2u;
  };
  auto word = [&](uint32_t y, uint32_t gg) -> uint32_t { return (D == 3) ? (z * L + y) * GPR + gg : z * GPR + gg; };
  uint32_t jc[4 * D + 1] = {}, jx[4 * D + 1] = {};
  if (EA && threadIdx.x < n) sg_jload2<D>(Jn, NW, word(ycoord(r + RB0), 2 * q), 2 * q, ycoord(r + RB0), z, a, jc);
  for (uint32_t u = threadIdx.x; u < n; u += NT) {
    const uint32_t rr = r + RB0, g = 2 * q;
    const uint32_t y = ycoord(rr);
    const uint32_t w = word(y, g);
    uint32_t rn = r + dr, qn = q + dg;
    if (qn >= PG) {
      qn -= PG;
      rn += 1;
    }
    if (EA && u + NT < n) sg_jload2<D>(Jn, NW, word(ycoord(rn + RB0), 2 * qn), 2 * qn, ycoord(rn + RB0), z, a, jx);
    const uint2 v = sg_unit2<D, EA, NEVER, C>(pm, pc, pp, rr, g, y, z, w, a, U, bound, RW, jc);
    if (C == 0) {
      uint32_t* row = pc + rr * RW;
      *reinterpret_cast<uint2*>(row + 2 + g) = v;
      if (g == 0) row[2 + GPR] = v.x;
      if (g + 2 == GPR) row[1] = v.y;
    } else {
      uint4 b;
      unpack_nibbles(v.x, b.x, b.y);
      unpack_nibbles(v.y, b.z, b.w);
      reinterpret_cast<uint4*>(dst)[w >> 1] = b;
    }
    if (EA) {
#pragma unroll
      for (int k = 0; k < 4 * D + 1; ++k) jc[k] = jx[k];
    }
    r = rn;
    q = qn;
  }
}

template <int D, bool EA, bool NEVER, int NT, bool PAIR>
__global__ __launch_bounds__(NT) void k_streamg(const int8_t* __restrict__ src, int8_t* __restrict__ dst,
                                                const uint32_t* __restrict__ Jraw, StreamArgs a) {
  extern __shared__ __align__(16) uint32_t lds[];
  uint32_t* bound = lds;  // first: constant-offset lookups
  uint32_t* ring = lds + 8;
  const uint32_t L = a.L, GPR = a.GPR;
  constexpr uint32_t OFF = PAIR ? 2u : 1u;  // index of word 0 in a slice row
  const uint32_t RW = GPR + 2 * OFF;
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
  const uint32_t tot = RP * GPR;  // words of a plane slice
  uint2 nxt[kFetch];
  for (uint32_t k = 0; k < 3; ++k) {
    sg_fetch<D, NT>(src, wrap_sub2(z0 + k, L), y0, a, tot, nxt);
    sg_store<NT, OFF>(ring + k * SB, a, tot, RW, nxt);
  }
  __syncthreads();
  // units: colour 0 on slice rows 1..TY+2 (3D) / row 0 (2D); colour 1 on rows 2..TY+1 / row 0
  const uint32_t U0n = ((D == 3) ? (TY + 2) * GPR : GPR) / (PAIR ? 2u : 1u);
  const uint32_t U1n = ((D == 3) ? TY * GPR : GPR) / (PAIR ? 2u : 1u);
  uint32_t sa = 1;  // slot of plane a = z0 - 1 + i
  for (uint32_t i = 0; i < H + 3; ++i) {
    const uint32_t s_m3 = sa >= 3 ? sa - 3 : sa + 3;   // a-3
    const uint32_t s_m2 = sa >= 2 ? sa - 2 : sa + 4;   // a-2
    const uint32_t s_m1 = sa >= 1 ? sa - 1 : 5;        // a-1
    const uint32_t s_p1 = sa <= 4 ? sa + 1 : 0;        // a+1
    const uint32_t s_p2 = sa <= 3 ? sa + 2 : sa - 4;   // a+2
    // plane a+2: loads issued now, stored after the compute of this step
    if (i <= H) sg_fetch<D, NT>(src, wrap_sub2(z0 + i + 3, L), y0, a, tot, nxt);
    if (PAIR) {
      if (i <= H + 1)
        sg_units2<D, EA, NEVER, NT, 0>(ring + s_m1 * SB, ring + sa * SB, ring + s_p1 * SB, U0n, y0,
                                       wrap_sub2(z0 + i + 1, L), a, U0, bound, RW, Jn, NW, dst);
      if (i >= 3)
        sg_units2<D, EA, NEVER, NT, 1>(ring + s_m3 * SB, ring + s_m2 * SB, ring + s_m1 * SB, U1n, y0, z0 + i - 3u,
                                       a, U1, bound, RW, Jn, NW, dst);
    } else {
      if (i <= H + 1)
        sg_units<D, EA, NEVER, NT, 0>(ring + s_m1 * SB, ring + sa * SB, ring + s_p1 * SB, U0n, y0,
                                      wrap_sub2(z0 + i + 1, L), a, U0, bound, RW, Jn, NW, dst);
      if (i >= 3)
        sg_units<D, EA, NEVER, NT, 1>(ring + s_m3 * SB, ring + s_m2 * SB, ring + s_m1 * SB, U1n, y0, z0 + i - 3u, a,
                                      U1, bound, RW, Jn, NW, dst);
    }
    if (i <= H) sg_store<NT, OFF>(ring + s_p2 * SB, a, tot, RW, nxt);
    __syncthreads();
    sa = sa == 5 ? 0 : sa + 1;
  }
}

// Supported: L % 8 == 0, L >= 16; +-J: packed couplings (d*L^d/2 bytes) under 4 GiB;
// 3D: TY in {4, 8, 16, 32} dividing L;
// H >= 1 (the last strip may be shorter); threads 256 or 512.
bool streamg_supported(const Lat& lat, const Tile& tile) {
  if (lat.L % 8 != 0 || lat.L < 16) return false;
  if (lat.J != nullptr && (uint64_t)lat.d * lat.N / 2 >= ((uint64_t)1 << 32)) return false;  // 32-bit offsets (ldg_word)
  if (tile.threads != 256 && tile.threads != 512) return false;
  if (tile.z < 1 || (uint32_t)tile.z > lat.L) return false;
  if (lat.d == 3) {
    if (tile.y != 4 && tile.y != 8 && tile.y != 16 && tile.y != 32) return false;
    if (lat.L % (uint32_t)tile.y != 0) return false;
  }
  const uint32_t RP = lat.d == 3 ? (uint32_t)tile.y + 4 : 1u;
  if (RP * (lat.L / 8) > (uint32_t)kFetch * (uint32_t)tile.threads) return false;  // slice words per thread
  return streamg_lds_bytes(lat, tile) <= 150 * 1024;
}

size_t streamg_lds_bytes(const Lat& lat, const Tile& tile) {
  const size_t RW = lat.L / 8 + (lat.L % 16 == 0 ? 4 : 2);  // the word-pair form's rows have two pads more
  const size_t RP = lat.d == 3 ? (size_t)tile.y + 4 : 1;
  return 32 + 6 * RP * RW * 4;
}

template <int D, bool EA, int NT, bool PAIR>
static hipError_t go_streamg_p(dim3 grid, size_t lds, bool never, const int8_t* src, int8_t* dst, const uint32_t* Jn,
                               const StreamArgs& a, hipStream_t stream) {
  static bool attr = false;
  if (!attr) {
    hipError_t e = hipFuncSetAttribute((const void*)k_streamg<D, EA, true, NT, PAIR>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, 150 * 1024);
    if (e == hipSuccess)
      e = hipFuncSetAttribute((const void*)k_streamg<D, EA, false, NT, PAIR>,
                              hipFuncAttributeMaxDynamicSharedMemorySize, 150 * 1024);
    if (e != hipSuccess) return e;
    attr = true;
  }
  if (never)
    hipLaunchKernelGGL((k_streamg<D, EA, true, NT, PAIR>), grid, dim3(NT), lds, stream, src, dst, Jn, a);
  else
    hipLaunchKernelGGL((k_streamg<D, EA, false, NT, PAIR>), grid, dim3(NT), lds, stream, src, dst, Jn, a);
  return hipGetLastError();
}

// Rows of an even number of words (L % 16 == 0) run the word-pair form when
// its units still cover every thread (colour-1 pairs of a step >= threads);
// measured: 3D +-J L = 512 567 -> 647 attempts/ns, while with fewer pairs than
// threads (2D rows, 3D L <= 256) the halved parallelism lost up to 18 %.
template <int D, bool EA, int NT>
static hipError_t go_streamg(dim3 grid, size_t lds, bool never, const int8_t* src, int8_t* dst, const uint32_t* Jn,
                             const StreamArgs& a, hipStream_t stream) {
  if (a.GPR % 2 == 0 && a.TY * (a.GPR / 2) >= (uint32_t)NT)
    return go_streamg_p<D, EA, NT, true>(grid, lds, never, src, dst, Jn, a, stream);
  return go_streamg_p<D, EA, NT, false>(grid, lds, never, src, dst, Jn, a, stream);
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
