// spin_stream3d.hip -- 3D Ising, one whole sweep per launch, streamed over
// planes (the kernel of the L = 512 and 1024 lattices).
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "spin_device.h"
#include "spin_packed.h"
#include "spin_phase.h"

namespace spin {

// 3D Ising, one whole sweep, streaming over planes.  Rows are full x rows,
// L = 512 * G (lane l of a wave owns groups g = l + 64 j, j < G).  A
// workgroup of W waves owns the TY rows [y0, y0+TY) of the planes
// [z0, z0+H) and keeps a ring of 6 plane slices in LDS; a slice holds the
// rows y0-2 .. y0+TY+1 (row r <-> y = y0-2+r), each row with 16 wrap bytes
// on both sides.  Plane k of the strip (z = z0-2+k) lives in slot k % 6.
// Step i (i = 0..H+2), a = z0-1+i:
//   load plane a+2 (registers; stored to LDS at the end of the step);
//   colour 0 on plane a, rows y0-1 .. y0+TY (the tile rows and a one-row
//   ring that colour 1 needs): reads planes a-1..a+1, writes plane a;
//   colour 1 on plane a-2, rows y0 .. y0+TY-1: reads planes a-3..a-1,
//   writes dst;
//   barrier.
// The 2TY+2 row-units of a step are dealt to the waves round-robin.  The
// step loop is unrolled over the ring period (slots compile-time; with z0
// even the plane parities are too).
typedef uint32_t u32x2 __attribute__((ext_vector_type(2)));

// Rows move between HBM and registers by buffer instructions over the
// lattice's L^3 bytes (at most 2^30; third descriptor word 0x00020000, the
// raw-buffer format of the gfx9 family): the row offset (z L + y) L is a
// scalar operand and the thread's byte offset 8 (lane + 64 j) the vector
// operand, so no per-lane 64-bit address arithmetic remains.
template <int TY, int W, int G>
struct Stream3Ctx {
  static constexpr uint32_t L = 512u * G;
  static constexpr uint32_t GPR = L / 8;
  static constexpr uint32_t RB = L + 32;
  static constexpr uint32_t RP = TY + 4;
  static constexpr uint32_t PB = RP * RB;
  static constexpr int NT = 64 * W;
  static constexpr int RPW = (RP + W - 1) / W;  // plane rows loaded per wave
  __amdgpu_buffer_rsrc_t rsrc, rdst;
  int8_t* ring;
  const uint32_t* bound;
  const RoundKeys* keys;
  PhiloxUniform U0, U1;
  uint32_t never4, y0, z0, H, lane, wave;

  __device__ __forceinline__ void get_plane(uint32_t z, uint2 (&v)[RPW][G]) const {
#pragma unroll
    for (int q = 0; q < RPW; ++q) {
      const uint32_t rr = wave + W * q;
      if (rr < RP) {
        const uint32_t y = wrap_row(y0 + rr, 2u, L);
        const uint32_t roff = (z * L + y) * L;
#pragma unroll
        for (int j = 0; j < G; ++j) {
          const u32x2 w = __builtin_amdgcn_raw_buffer_load_b64(rsrc, 8u * (lane + 64 * j), roff, 0);
          v[q][j] = make_uint2(w.x, w.y);
        }
      }
    }
  }
  __device__ __forceinline__ void put_plane(uint32_t slot, const uint2 (&v)[RPW][G]) const {
#pragma unroll
    for (int q = 0; q < RPW; ++q) {
      const uint32_t rr = wave + W * q;
      if (rr < RP) {
        int8_t* row = ring + slot * PB + rr * RB;
#pragma unroll
        for (int j = 0; j < G; ++j) {
          const uint32_t g = lane + 64 * j;
          *reinterpret_cast<uint2*>(row + 16 + 8 * g) = v[q][j];
          if (g >= GPR - 2) *reinterpret_cast<uint2*>(row + 8 * (g - (GPR - 2))) = v[q][j];
          if (g < 2) *reinterpret_cast<uint2*>(row + 16 + L + 8 * g) = v[q][j];
        }
      }
    }
  }
};

// One 8-site group of row r (LDS slot PC, z-neighbour slots PM, PP) in colour C.
template <int TY, int W, int G, bool NEVER, uint32_t C, uint32_t PM, uint32_t PC, uint32_t PP>
__device__ __forceinline__ void stream3_group(const Stream3Ctx<TY, W, G>& c, uint32_t r, uint32_t y,
                                              uint32_t z, uint32_t g, uint32_t& o_lo,
                                              uint32_t& o_hi) {
  using X = Stream3Ctx<TY, W, G>;
  constexpr uint32_t L = X::L, GPR = X::GPR, RB = X::RB, PB = X::PB;
  const int8_t* row = c.ring + PC * PB + r * RB + 16;
  const int8_t* zm = c.ring + PM * PB + r * RB + 16;
  const int8_t* zp = c.ring + PP * PB + r * RB + 16;
  const uint2 cc = *reinterpret_cast<const uint2*>(row + 8 * g);
  const uint2 ym = *reinterpret_cast<const uint2*>(row - RB + 8 * g);
  const uint2 yp = *reinterpret_cast<const uint2*>(row + RB + 8 * g);
  const uint2 a2 = *reinterpret_cast<const uint2*>(zm + 8 * g);
  const uint2 b2 = *reinterpret_cast<const uint2*>(zp + 8 * g);
  const uint32_t lw = *reinterpret_cast<const uint32_t*>(row + 8 * g - 4);
  const uint32_t rw = *reinterpret_cast<const uint32_t*>(row + 8 * g + 8);
  uint32_t rnd[4];
  const uint32_t cbase = (z * L + y) * GPR;  // < 2^27 for L <= 1024
  philox_lane(cbase + g, C ? c.U1 : c.U0, *c.keys, rnd);
  const uint32_t o0[4] = {ym.x, yp.x, a2.x, b2.x}, o1[4] = {ym.y, yp.y, a2.y, b2.y};
  const uint32_t P = (C + y + z) & 1u;
  const uint32_t Sp = unsat_packed<4>(P, cc.x, cc.y, lw, rw, o0, o1);
  uint32_t c0 = cc.x, c1 = cc.y;
  apply_packed<NEVER>(P, c0, c1, Sp, rnd, c.bound, c.never4);
  o_lo = c0;
  o_hi = c1;
}

// Step i of the plane pipeline.  Wave w updates colour-0 rows 1 + w + W q
// (q < N0, rows 1..TY+2 of plane a) and colour-1 rows 2 + w + W q (q < N1,
// rows 2..TY+1 of plane a-2); rows past the end are computed on a valid row
// and not stored, so the compute is straight-line and the units interleave.
template <int TY, int W, int G, bool NEVER, uint32_t S>
__device__ __forceinline__ void stream3_step(const Stream3Ctx<TY, W, G>& c, uint32_t i) {
  using X = Stream3Ctx<TY, W, G>;
  constexpr uint32_t L = X::L, GPR = X::GPR, RB = X::RB, PB = X::PB;
  constexpr int N0 = (TY + 2 + W - 1) / W, N1 = (TY + W - 1) / W;
  const uint32_t H = c.H;
  if (i >= H + 3) return;
  uint2 nxt[X::RPW][G];
  const bool do_load = (i <= H);
  if (do_load) c.get_plane(wrap_row(c.z0 + i + 3, 2u, L), nxt);
  const bool col0 = (i <= H + 1), col1 = (i >= 3);
  const uint32_t za = wrap_row(c.z0 + i + 1, 2u, L);  // plane a = z0 - 1 + i
  const uint32_t zb = c.z0 + i - 3u;                   // plane a - 2
  uint32_t r0[N0], r1[N1], y0v[N0], y1v[N1];
#pragma unroll
  for (int q = 0; q < N0; ++q) {
    const uint32_t rr = 1u + c.wave + W * q;
    r0[q] = rr <= TY + 2u ? rr : TY + 2u;
    y0v[q] = wrap_row(c.y0 + r0[q], 2u, L);
  }
#pragma unroll
  for (int q = 0; q < N1; ++q) {
    const uint32_t rr = 2u + c.wave + W * q;
    r1[q] = rr <= TY + 1u ? rr : TY + 1u;
    y1v[q] = c.y0 + r1[q] - 2u;
  }
  uint32_t v0[N0][G][2], v1[N1][G][2];
#pragma unroll
  for (int j = 0; j < G; ++j) {
    const uint32_t g = c.lane + 64 * j;
#pragma unroll
    for (int q = 0; q < N0; ++q)
      stream3_group<TY, W, G, NEVER, 0, S % 6, (S + 1) % 6, (S + 2) % 6>(c, r0[q], y0v[q], za, g, v0[q][j][0], v0[q][j][1]);
#pragma unroll
    for (int q = 0; q < N1; ++q)
      stream3_group<TY, W, G, NEVER, 1, (S + 4) % 6, (S + 5) % 6, S % 6>(c, r1[q], y1v[q], zb, g, v1[q][j][0], v1[q][j][1]);
  }
  if (col0) {
#pragma unroll
    for (int q = 0; q < N0; ++q) {
      if (1u + c.wave + W * q > TY + 2u) break;
      int8_t* row = c.ring + ((S + 1) % 6) * PB + r0[q] * RB + 16;
#pragma unroll
      for (int j = 0; j < G; ++j) {
        const uint32_t g = c.lane + 64 * j;
        const uint2 v = make_uint2(v0[q][j][0], v0[q][j][1]);
        *reinterpret_cast<uint2*>(row + 8 * g) = v;
        if (g >= GPR - 2) *reinterpret_cast<uint2*>(row - 16 + 8 * (g - (GPR - 2))) = v;
        if (g < 2) *reinterpret_cast<uint2*>(row + L + 8 * g) = v;
      }
    }
  }
  if (col1) {
#pragma unroll
    for (int q = 0; q < N1; ++q) {
      if (2u + c.wave + W * q > TY + 1u) break;
      const uint32_t roff = (zb * L + y1v[q]) * L;
#pragma unroll
      for (int j = 0; j < G; ++j) {
        const u32x2 w = {v1[q][j][0], v1[q][j][1]};
        __builtin_amdgcn_raw_buffer_store_b64(w, c.rdst, 8u * (c.lane + 64 * j), roff, 0);
      }
    }
  }
  if (do_load) c.put_plane((S + 3) % 6, nxt);
  __syncthreads();
}

template <int TY, int W, int G, bool NEVER>
__global__ __launch_bounds__(64 * W) void k_stream3d(const int8_t* __restrict__ src,
                                                     int8_t* __restrict__ dst, PhaseArgs a,
                                                     uint32_t H) {
  using X = Stream3Ctx<TY, W, G>;
  __shared__ __align__(16) int8_t lds[32 + 6 * X::PB];
  X c;
  c.rsrc = __builtin_amdgcn_make_buffer_rsrc((void*)src, 0, (int)(X::L * X::L * X::L), 0x00020000);
  c.rdst = __builtin_amdgcn_make_buffer_rsrc((void*)dst, 0, (int)(X::L * X::L * X::L), 0x00020000);
  c.ring = lds + 32;
  c.bound = reinterpret_cast<const uint32_t*>(lds);
  c.keys = &a.keys;
  c.U0 = philox_uniform(a.t, a.replica, 0u, a.keys);
  c.U1 = philox_uniform(a.t, a.replica, 1u, a.keys);
  c.never4 = a.never4;
  c.y0 = blockIdx.x * TY;
  c.z0 = blockIdx.y * H;
  c.H = H;
  c.lane = threadIdx.x & 63;
  c.wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  if (threadIdx.x < 8) reinterpret_cast<uint32_t*>(lds)[threadIdx.x] = a.bound[threadIdx.x];
  for (uint32_t k = 0; k < 3; ++k) {
    uint2 v[X::RPW][G];
    c.get_plane(wrap_row(c.z0 + k, 2u, X::L), v);
    c.put_plane(k, v);
  }
  __syncthreads();
  const uint32_t steps = H + 3;
  for (uint32_t i0 = 0; i0 < steps; i0 += 6) {
    stream3_step<TY, W, G, NEVER, 0>(c, i0 + 0);
    stream3_step<TY, W, G, NEVER, 1>(c, i0 + 1);
    stream3_step<TY, W, G, NEVER, 2>(c, i0 + 2);
    stream3_step<TY, W, G, NEVER, 3>(c, i0 + 3);
    stream3_step<TY, W, G, NEVER, 4>(c, i0 + 4);
    stream3_step<TY, W, G, NEVER, 5>(c, i0 + 5);
  }
}

// ---------------------------------------------------------------------------
// 3D Ising, L = 512, one whole sweep per launch, streamed over planes with
// each row's z column held in registers (k_stream3r).
//
// A workgroup owns the TY rows [y0, y0+TY) of the planes [z0, z0+H) and has
// W = TY/2 + 1 waves.  Rows of the slab are numbered r = 0..TY+3 (y = y0-2+r):
// wave w keeps rows r = 2w+1 and 2w+2 for the whole launch, so rows 2..TY+1
// are the owned rows, 1 and TY+2 a one-row ring whose colour 0 is recomputed
// here (colour 1 of the owned edge rows needs it), and 0 and TY+3 (loaded by
// the first and last wave) the halo that colour 0 of the ring reads.  Lane l
// holds the 8-site group x = 8l of each of its rows (a row is 512 bytes).
// Step i = 0..H+1, a = z0-1+i:
//   load plane a+2 of the wave's rows into registers;
//   colour 0 on plane a: z neighbours from the registers (plane a-1 after
//     its colour 0 -- whose colour-1 bytes are the old ones -- and plane
//     a+1 as loaded), y neighbours from the wave's other row (registers)
//     and from LDS, x neighbours across the group edge by a wavefront
//     rotate (DPP), so no row needs wrap bytes;
//   colour 1 on plane a-1 (i >= 2, owned rows only): z neighbours a-2 and a
//     after colour 0 (registers), y neighbours as above from the LDS copy
//     of plane a-1 after colour 0; the result goes to dst;
//   barrier.
// LDS holds three plane slices of TY+4 rows in a ring by step: slot i%3
// gets plane a as loaded at the end of step i-1, is read for colour 0 in
// step i and overwritten in place with the colour-0 results (only colour-0
// bytes change, and colour 0 reads only colour-1 bytes of its neighbours,
// so the concurrent reads of other waves see the same values either way);
// step i+1 reads it for colour 1; step i+2 overwrites it with plane a+3.
// Every cross-wave read therefore happens one step after its write.
// With MEAS the launch also counts E and M of its result: every bond joins a
// colour-0 and a colour-1 site, so the unsatisfied bonds are the sum over
// the owned colour-1 sites of their count after the update -- the count the
// update computed against final colour-0 neighbours, or 2d minus it where
// the site flipped -- and M from the owned sites' final bytes.
typedef uint32_t u32x2r __attribute__((ext_vector_type(2)));

template <uint32_t LL, int TY>
struct Col3Ctx {
  static constexpr uint32_t L = LL;
  static constexpr uint32_t GPR = LL / 8;        // groups per row (<= 64)
  static constexpr uint32_t RP = TY + 4;         // rows of a slice
  static constexpr uint32_t PB = RP * L;         // bytes of a slice
  static constexpr int W = TY / 2 + 1;
  static constexpr uint32_t PW = (pair_words(6) + 15u) & ~15u;  // pair table words, rounded to 64 bytes
  __amdgpu_buffer_rsrc_t rsrc, rdst;
  int8_t* ring;
  const char* pair;
  const RoundKeys* keys;
  PhiloxUniform U0, U1;
  uint32_t never8, y0, z0, H, lane, wave;
  uint32_t cnt;       // 1 on the first copy of a row in the wavefront (the one that counts E/M), else 0
  uint32_t yrow[2];   // y of the wave's two rows
  uint32_t yhalo;     // y of the halo row the edge wave loads
};

// x neighbour dword of a parity-split group for active parity P: P = 0 needs
// the odd half of the group to the left (lane - 1; its byte 3 is the site
// left of the group), P = 1 the even half of the group to the right (lane + 1;
// its byte 0); a row is one wavefront, so the rotates wrap x periodically.
template <uint32_t P>
__device__ __forceinline__ uint32_t xnb(uint2 c) {
  if (P == 0) return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)c.y, 0x13C, 0xF, 0xF, false);  // wave_ror:1
  return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)c.x, 0x134, 0xF, 0xF, false);             // wave_rol:1
}

// One colour unit of a parity-split group c (x: even bytes, y: odd bytes,
// split_group) with active parity P: y neighbours ym, yp, z neighbours zm,
// zp (split); Philox counter base + lane, with mbase = philox_base(base).
// Returns the new group; with MEAS adds 4 x the unsatisfied bonds of the
// active sites after the update to acc.  The active half and the neighbours'
// halves of the same parity need no gathering; the bounds come from the pair
// table (8u per packed byte), read before the Philox rounds so that the LDS
// reads are in flight during them.
template <uint32_t P, bool NEVER, bool MEAS>
__device__ __forceinline__ uint2 col3_unit(uint2 c, uint2 ym, uint2 yp, uint2 zm, uint2 zp, uint32_t lane,
                                           uint64_t mbase, const PhiloxUniform& U, const RoundKeys& K,
                                           const char* pair, uint32_t never8, uint32_t& acc) {
  const uint32_t A = P ? c.y : c.x, I = P ? c.x : c.y;
  const uint32_t N = __builtin_amdgcn_perm(I, xnb<P>(c), P ? 0x00070605u : 0x06050403u);
  const uint32_t S = ((A ^ I) & kSignBit8) + ((A ^ N) & kSignBit8) + ((A ^ (P ? ym.y : ym.x)) & kSignBit8) +
                     ((A ^ (P ? yp.y : yp.x)) & kSignBit8) + ((A ^ (P ? zm.y : zm.x)) & kSignBit8) +
                     ((A ^ (P ? zp.y : zp.x)) & kSignBit8);
  const uint4 b = lookup_pair(S, pair);
  uint32_t rnd[4];
  philox_lane_split(lane, mbase, U, K, rnd);
  const uint32_t An = MEAS ? apply_split_count<NEVER, 3>(A, S, b, rnd, never8, acc)
                           : apply_split<NEVER>(A, S, b, rnd, never8);
  return P ? make_uint2(c.x, An) : make_uint2(An, c.y);
}

// Register state of one wave: its two rows' z columns and, on the edge
// waves, the halo row's.
struct Col3Regs {
  uint2 xa[2];    // plane a as loaded (colour-0 centre)
  uint2 xa1[2];   // plane a+1 as loaded
  uint2 ya1[2];   // plane a-1 after colour 0
  uint2 ya2[2];   // plane a-2 after colour 0
  uint2 xh1;      // halo row, plane a+1 as loaded
  uint32_t sA, sB, sN;  // ring slots of planes a, a-1, a+1
};

template <uint32_t LL, int TY>
__device__ __forceinline__ uint2 col3_load(const Col3Ctx<LL, TY>& c, uint32_t z, uint32_t y) {
  constexpr uint32_t L = Col3Ctx<LL, TY>::L;
  const u32x2r v = __builtin_amdgcn_raw_buffer_load_b64(c.rsrc, 8u * c.lane, (z * L + y) * L, 0);
  return split_group(v.x, v.y);
}

// Step i of the pipeline (Q = i & 1; C1: colour 1 runs, i.e. i >= 2).  Row j
// of the wave has y parity (1 + j) & 1 and plane a = z0-1+i parity (i+1) & 1
// (z0 is even), so the active parity of row j is (Q + j) & 1 in both colours.
template <uint32_t LL, int TY, int EDGE, bool NEVER, bool MEAS, uint32_t Q, bool C1>
__device__ __forceinline__ void col3_step(const Col3Ctx<LL, TY>& c, Col3Regs& R, uint32_t i, int8_t* base,
                                          uint32_t& unsat4, uint32_t& neg) {
  using X = Col3Ctx<LL, TY>;
  constexpr uint32_t L = X::L, PB = X::PB, GPR = X::GPR;
  constexpr bool OWN0 = EDGE != 1, OWN1 = EDGE != 2;  // row j is owned (not the ring)
  constexpr uint32_t P0 = Q, P1 = Q ^ 1u;             // active parity of rows 0 and 1
  // load plane a+2 (the last step reloads plane z0+H+1, which nothing reads, so that the load is
  // unconditional)
  const uint32_t zl = wrap_row(c.z0 + 1u + (i <= c.H ? i : c.H), 0u, L);
  uint2 xa2[2], xh2 = make_uint2(0, 0);
#pragma unroll
  for (int j = 0; j < 2; ++j) xa2[j] = col3_load(c, zl, c.yrow[j]);
  if (EDGE) xh2 = col3_load(c, zl, c.yhalo);
  const uint32_t a = wrap_row(c.z0 + i, 1u, L);
  int8_t* pA = base + R.sA * PB;
  int8_t* pB = base + R.sB * PB;
  int8_t* pN = base + R.sN * PB;
  uint32_t none = 0;
  // colour 0 on plane a: y neighbours rows 2w (LDS) and 2w+3 (LDS), the wave's other row (registers)
  const uint2 up0 = *reinterpret_cast<const uint2*>(pA);
  const uint2 dn1 = *reinterpret_cast<const uint2*>(pA + 3 * L);
  uint2 ya0[2];
  ya0[0] = col3_unit<P0, NEVER, false>(R.xa[0], up0, R.xa[1], R.ya1[0], R.xa1[0], c.lane,
                                       philox_base((a * L + c.yrow[0]) * GPR), c.U0, *c.keys, c.pair, c.never8,
                                       none);
  ya0[1] = col3_unit<P1, NEVER, false>(R.xa[1], R.xa[0], dn1, R.ya1[1], R.xa1[1], c.lane,
                                       philox_base((a * L + c.yrow[1]) * GPR), c.U0, *c.keys, c.pair, c.never8,
                                       none);
  *reinterpret_cast<uint2*>(pA + L) = ya0[0];
  *reinterpret_cast<uint2*>(pA + 2 * L) = ya0[1];
  // colour 1 on plane b = a-1 (owned rows)
  uint2 fin[2];
  const uint32_t b = wrap_row(a, 1u, L);
  if (C1) {
    const uint2 upB = *reinterpret_cast<const uint2*>(pB);
    const uint2 dnB = *reinterpret_cast<const uint2*>(pB + 3 * L);
    uint32_t add = 0;
    if (OWN0)
      fin[0] = col3_unit<P0, NEVER, MEAS>(R.ya1[0], upB, R.ya1[1], R.ya2[0], ya0[0], c.lane,
                                          philox_base((b * L + c.yrow[0]) * GPR), c.U1, *c.keys, c.pair, c.never8,
                                          add);
    if (OWN1)
      fin[1] = col3_unit<P1, NEVER, MEAS>(R.ya1[1], R.ya1[0], dnB, R.ya2[1], ya0[1], c.lane,
                                          philox_base((b * L + c.yrow[1]) * GPR), c.U1, *c.keys, c.pair, c.never8,
                                          add);
    if (MEAS) {
      // only the first copy of the row in the wavefront counts
      unsat4 += c.cnt * add;
      if (OWN0) neg += c.cnt * (__popc(fin[0].x & 0x80808080u) + __popc(fin[0].y & 0x80808080u));
      if (OWN1) neg += c.cnt * (__popc(fin[1].x & 0x80808080u) + __popc(fin[1].y & 0x80808080u));
    }
  }
  // plane a+1 as loaded, for colour 0 of the next step
  *reinterpret_cast<uint2*>(pN + L) = R.xa1[0];
  *reinterpret_cast<uint2*>(pN + 2 * L) = R.xa1[1];
  if (EDGE == 1) *reinterpret_cast<uint2*>(pN) = R.xh1;
  if (EDGE == 2) *reinterpret_cast<uint2*>(pN + 3 * L) = R.xh1;
  if (C1) {
    if (OWN0) {
      const uint2 o = join_group(fin[0]);
      const u32x2r w = {o.x, o.y};
      __builtin_amdgcn_raw_buffer_store_b64(w, c.rdst, 8u * c.lane, (b * L + c.yrow[0]) * L, 0);
    }
    if (OWN1) {
      const uint2 o = join_group(fin[1]);
      const u32x2r w = {o.x, o.y};
      __builtin_amdgcn_raw_buffer_store_b64(w, c.rdst, 8u * c.lane, (b * L + c.yrow[1]) * L, 0);
    }
  }
#pragma unroll
  for (int j = 0; j < 2; ++j) {
    R.ya2[j] = R.ya1[j];
    R.ya1[j] = ya0[j];
    R.xa[j] = R.xa1[j];
    R.xa1[j] = xa2[j];
  }
  R.xh1 = xh2;
  const uint32_t t = R.sB;
  R.sB = R.sA;
  R.sA = R.sN;
  R.sN = t;
  __syncthreads();
}

template <uint32_t LL, int TY, int EDGE, bool NEVER, bool MEAS>
__device__ __forceinline__ void col3_run(const Col3Ctx<LL, TY>& c, uint32_t& unsat4, uint32_t& neg) {
  using X = Col3Ctx<LL, TY>;
  constexpr uint32_t L = X::L;
  // LDS address of (slot 0, row 2w, this lane's group); rows 2w .. 2w+3 of a slot sit at +0 .. +3L
  int8_t* base = c.ring + 2u * c.wave * L + 8u * c.lane;
  Col3Regs R;
  // prologue: planes z0-2 (its colour-1 bytes are the z-1 neighbours of step 0), z0-1 and z0
  const uint32_t zm2 = wrap_row(c.z0, 2u, L), zm1 = wrap_row(c.z0, 1u, L);
#pragma unroll
  for (int j = 0; j < 2; ++j) {
    R.ya1[j] = col3_load(c, zm2, c.yrow[j]);
    R.xa[j] = col3_load(c, zm1, c.yrow[j]);
    R.xa1[j] = col3_load(c, c.z0, c.yrow[j]);
    R.ya2[j] = make_uint2(0, 0);
  }
  uint2 xh = make_uint2(0, 0);
  R.xh1 = make_uint2(0, 0);
  if (EDGE) {
    xh = col3_load(c, zm1, c.yhalo);
    R.xh1 = col3_load(c, c.z0, c.yhalo);
  }
  *reinterpret_cast<uint2*>(base + L) = R.xa[0];
  *reinterpret_cast<uint2*>(base + 2 * L) = R.xa[1];
  if (EDGE == 1) *reinterpret_cast<uint2*>(base) = xh;
  if (EDGE == 2) *reinterpret_cast<uint2*>(base + 3 * L) = xh;
  R.sA = 0;
  R.sB = 2;
  R.sN = 1;
  __syncthreads();
  // steps 0 and 1 (planes z0-1 and z0 for colour 0; no owned plane for colour 1 yet), then pairs
  col3_step<LL, TY, EDGE, NEVER, MEAS, 0, false>(c, R, 0u, base, unsat4, neg);
  col3_step<LL, TY, EDGE, NEVER, MEAS, 1, false>(c, R, 1u, base, unsat4, neg);
  const uint32_t steps = c.H + 2;
  for (uint32_t i0 = 2; i0 < steps; i0 += 2) {
    col3_step<LL, TY, EDGE, NEVER, MEAS, 0, true>(c, R, i0, base, unsat4, neg);
    col3_step<LL, TY, EDGE, NEVER, MEAS, 1, true>(c, R, i0 + 1u, base, unsat4, neg);
  }
}

template <uint32_t LL, int TY, bool NEVER, bool MEAS>
__global__ __launch_bounds__(64 * (TY / 2 + 1)) void k_stream3r(const int8_t* __restrict__ src,
                                                                int8_t* __restrict__ dst, PhaseArgs a,
                                                                uint32_t H, Record rec) {
  using X = Col3Ctx<LL, TY>;
  constexpr uint32_t L = X::L;
  constexpr int W = X::W;
  __shared__ __align__(16) int8_t lds[4 * X::PW + 3 * X::PB];
  X c;
  c.rsrc = __builtin_amdgcn_make_buffer_rsrc((void*)src, 0, (int)(L * L * L), 0x00020000);
  c.rdst = __builtin_amdgcn_make_buffer_rsrc((void*)dst, 0, (int)(L * L * L), 0x00020000);
  c.ring = lds + 4 * X::PW;
  c.pair = (const char*)lds;
  c.keys = &a.keys;
  c.U0 = philox_uniform(a.t, a.replica, 0u, a.keys);
  c.U1 = philox_uniform(a.t, a.replica, 1u, a.keys);
  c.never8 = 2u * a.never4;
  // workgroups are dealt to the 8 XCDs round-robin; give each XCD a contiguous run of tiles (all slabs
  // of its strips), so that the halo rows of neighbouring slabs are read from the same L2
  const uint32_t nslab = L / TY;
  const uint32_t nblk = gridDim.x;
  const uint32_t b = blockIdx.x;
  const uint32_t tile = (nblk % 8u == 0u) ? (b % 8u) * (nblk / 8u) + b / 8u : b;
  c.y0 = (tile % nslab) * TY;
  c.z0 = (tile / nslab) * H;
  c.H = H;
  // a row has GPR <= 64 groups: with GPR < 64 the wavefront holds 64 / GPR copies of its rows, lane l
  // working on group l mod GPR; the copies load, compute and store the same values, the wavefront
  // rotates give every lane its periodic x neighbour, and only the first copy counts E and M
  c.lane = threadIdx.x & (X::GPR - 1u);
  c.cnt = (threadIdx.x & 63u) < X::GPR ? 1u : 0u;
  c.wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
#pragma unroll
  for (int j = 0; j < 2; ++j) c.yrow[j] = wrap_row(c.y0 + 2u * c.wave + 1u + j, 2u, L);
  c.yhalo = (c.wave == 0) ? wrap_row(c.y0, 2u, L) : wrap_row(c.y0 + TY + 3u, 2u, L);
  fill_pair<6>(reinterpret_cast<uint32_t*>(lds), a.bound, threadIdx.x);
  keys_resident(a.keys);
  uint32_t unsat4 = 0, neg = 0;
  if (c.wave == 0)
    col3_run<LL, TY, 1, NEVER, MEAS>(c, unsat4, neg);
  else if (c.wave == (uint32_t)(W - 1))
    col3_run<LL, TY, 2, NEVER, MEAS>(c, unsat4, neg);
  else
    col3_run<LL, TY, 0, NEVER, MEAS>(c, unsat4, neg);
  if (MEAS) {
    __shared__ int64_t red[W];
    record_block<64 * W>((int64_t)(unsat4 >> 2), (int64_t)neg, rec, red);
  }
}

// Register-column kernel (k_stream3r): L = 128, 256 or 512, tile.y = TY in
// {8, 16} with TY/2 + 1 waves (320 or 576 threads), tile.z = H even.
static bool col3_shape(const Lat& lat, const Tile& tile) {
  if (lat.J != nullptr || lat.d != 3 || (uint32_t)tile.x != lat.L) return false;
  if (lat.L != 128 && lat.L != 256 && lat.L != 512) return false;
  const bool ok = (tile.y == 16 && tile.threads == 576) || (tile.y == 8 && tile.threads == 320);
  return ok && tile.z >= 2 && tile.z % 2 == 0 && lat.L % (uint32_t)tile.z == 0;
}

// 3D streaming shapes: tile.x == L == 512*G, tile.y = TY, tile.z = H, threads = 64*W
// (k_stream3d), or the register-column shapes above.
bool stream3d_shape(const Lat& lat, const Tile& tile) {
  if (col3_shape(lat, tile)) return true;
  if (lat.J != nullptr || lat.d != 3) return false;
  if ((uint32_t)tile.x != lat.L || (lat.L != 512 && lat.L != 1024)) return false;
  const bool ok_shape = (tile.y == 8 && (tile.threads == 640 || tile.threads == 320)) ||
                        (tile.y == 16 && (tile.threads == 576 || tile.threads == 384)) ||
                        (tile.y == 32 && tile.threads == 704 && lat.L == 512);
  return ok_shape && lat.L % (uint32_t)tile.y == 0 && tile.z >= 4 && tile.z % 2 == 0 &&
         lat.L % (uint32_t)tile.z == 0;
}

uint32_t stream3d_record_parts(const Lat& lat, const Tile& tile) {
  if (!col3_shape(lat, tile)) return 0;
  return (lat.L / (uint32_t)tile.y) * (lat.L / (uint32_t)tile.z);
}

template <uint32_t LL, int TY>
static hipError_t gocol3(const Lat& lat, const int8_t* src, int8_t* dst, const PhaseArgs& a, bool never,
                         uint32_t H, const Record* rec, hipStream_t stream) {
  dim3 grid((lat.L / TY) * (lat.L / H));
  dim3 block(64 * (TY / 2 + 1));
  const Record r = rec ? *rec : Record{nullptr};
  if (rec) {
    if (never)
      hipLaunchKernelGGL((k_stream3r<LL, TY, true, true>), grid, block, 0, stream, src, dst, a, H, r);
    else
      hipLaunchKernelGGL((k_stream3r<LL, TY, false, true>), grid, block, 0, stream, src, dst, a, H, r);
  } else {
    if (never)
      hipLaunchKernelGGL((k_stream3r<LL, TY, true, false>), grid, block, 0, stream, src, dst, a, H, r);
    else
      hipLaunchKernelGGL((k_stream3r<LL, TY, false, false>), grid, block, 0, stream, src, dst, a, H, r);
  }
  return hipGetLastError();
}

template <int TY, int W, int G>
static hipError_t gostream3(const Lat& lat, const int8_t* src, int8_t* dst, const PhaseArgs& a,
                            bool never, uint32_t H, hipStream_t stream) {
  dim3 grid(lat.L / TY, lat.L / H);
  if (never)
    hipLaunchKernelGGL((k_stream3d<TY, W, G, true>), grid, dim3(64 * W), 0, stream, src, dst, a, H);
  else
    hipLaunchKernelGGL((k_stream3d<TY, W, G, false>), grid, dim3(64 * W), 0, stream, src, dst, a, H);
  return hipGetLastError();
}

hipError_t launch_stream3d(const Lat& lat, const int8_t* src, int8_t* dst, const PhaseArgs& a, bool never,
                           const Tile& tile, const Record* rec, bool* measured, hipStream_t stream) {
  if (measured) *measured = false;
  if (!stream3d_shape(lat, tile)) return hipErrorInvalidValue;
  const uint32_t H = (uint32_t)tile.z;
  if (col3_shape(lat, tile)) {
    if (measured) *measured = (rec != nullptr);
    if (lat.L == 512) return tile.y == 16 ? gocol3<512, 16>(lat, src, dst, a, never, H, rec, stream)
                                          : gocol3<512, 8>(lat, src, dst, a, never, H, rec, stream);
    if (lat.L == 256) return tile.y == 16 ? gocol3<256, 16>(lat, src, dst, a, never, H, rec, stream)
                                          : gocol3<256, 8>(lat, src, dst, a, never, H, rec, stream);
    return tile.y == 16 ? gocol3<128, 16>(lat, src, dst, a, never, H, rec, stream)
                        : gocol3<128, 8>(lat, src, dst, a, never, H, rec, stream);
  }
  if (lat.L == 512) {
    if (tile.y == 8 && tile.threads == 640) return gostream3<8, 10, 1>(lat, src, dst, a, never, H, stream);
    if (tile.y == 16) return gostream3<16, 6, 1>(lat, src, dst, a, never, H, stream);
    return gostream3<32, 11, 1>(lat, src, dst, a, never, H, stream);
  }
  if (tile.y == 8 && tile.threads == 640) return gostream3<8, 10, 2>(lat, src, dst, a, never, H, stream);
  if (tile.y == 8) return gostream3<8, 5, 2>(lat, src, dst, a, never, H, stream);
  if (tile.y == 16 && tile.threads == 576) return gostream3<16, 9, 2>(lat, src, dst, a, never, H, stream);
  return gostream3<16, 6, 2>(lat, src, dst, a, never, H, stream);
}

}  // namespace spin
