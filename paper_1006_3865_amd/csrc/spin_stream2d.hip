// spin_stream2d.hip -- 2D Ising, one whole sweep per launch, streamed over
// full-width rows (the kernel of the L = 4096 .. 16384 lattices).
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "spin_device.h"
#include "spin_packed.h"
#include "spin_phase.h"

namespace spin {

// 2D Ising, one whole sweep, streaming over full-width rows.  L = 8 * NT * G:
// thread l owns the groups g = l + NT*j (j < G) of every row (x = 8g).  A
// workgroup owns the strip of H rows [y0, y0+H) (H even) and keeps a ring of 8
// rows in LDS (row k of the strip, k = y - (y0-2), lives in slot k & 7; a
// row's bytes sit at [16, 16+L) with x = L-16..L-1 copied to [0,16) and
// x = 0..15 to [16+L, 32+L)).  Step i (i = 0..H+2), with a = y0-1+i:
//   load row a+2 into registers (stored to LDS at the end of the step; the
//     last two steps reload row y0+H+1 into slots no longer read);
//   colour 0 on row a (i <= H+1): reads rows a-1..a+1, writes row a in LDS;
//   colour 1 on row a-2 (i >= 3): reads rows a-3..a-1, writes dst;
//   barrier.
// Row a's colour-1 bytes are still the old ones when colour 0 reads them
// (colour 1 reaches row a two steps later), and colour 1 on row a-2 reads
// colour-0 bytes finished one or more steps earlier.  The step loop is
// unrolled over the ring period so that ring slots and row parities (y0 is
// even) are compile-time constants.
// Rows move between HBM and registers by buffer instructions: a descriptor
// over the lattice's L*L bytes (third word 0x00020000, the raw-buffer format
// of the gfx9 family), the row offset y*L as a scalar operand and the
// thread's byte offset 8*(t + NT*j) as the vector operand, so no per-lane
// 64-bit address arithmetic remains.
typedef uint32_t u32x2 __attribute__((ext_vector_type(2)));

template <int NT, int G>
struct StreamCtx {
  static constexpr uint32_t L = 8u * NT * G;
  static constexpr uint32_t GPR = L / 8;
  static constexpr uint32_t RBS = L + 32;
  __amdgpu_buffer_rsrc_t rsrc, rdst;
  int8_t* ring;
  const uint32_t* bound;
  const RoundKeys* keys;
  PhiloxUniform U0, U1;
  uint32_t never4, y0, H, t;

  __device__ __forceinline__ void get_row(uint32_t y, uint2 (&v)[G]) const {
#pragma unroll
    for (int j = 0; j < G; ++j) {
      const u32x2 w = __builtin_amdgcn_raw_buffer_load_b64(rsrc, 8u * (t + NT * j), y * L, 0);
      v[j] = make_uint2(w.x, w.y);
    }
  }
  __device__ __forceinline__ void put_out(uint32_t y, const uint2 (&v)[G]) const {
#pragma unroll
    for (int j = 0; j < G; ++j) {
      const u32x2 w = {v[j].x, v[j].y};
      __builtin_amdgcn_raw_buffer_store_b64(w, rdst, 8u * (t + NT * j), y * L, 0);
    }
  }
  __device__ __forceinline__ void put_row(uint32_t slot, const uint2 (&v)[G]) const {
    int8_t* row = ring + slot * RBS;
#pragma unroll
    for (int j = 0; j < G; ++j) {
      const uint32_t g = t + NT * j;
      *reinterpret_cast<uint2*>(row + 16 + 8 * g) = v[j];
      if (g >= GPR - 2) *reinterpret_cast<uint2*>(row + 8 * (g - (GPR - 2))) = v[j];
      if (g < 2) *reinterpret_cast<uint2*>(row + 16 + L + 8 * g) = v[j];
    }
  }
};

template <int NT, int G, bool NEVER, bool MEAS, uint32_t S>
__device__ __forceinline__ void stream_step(const StreamCtx<NT, G>& c, uint32_t i, int& unsat,
                                            int& neg) {
  using C = StreamCtx<NT, G>;
  constexpr uint32_t L = C::L, GPR = C::GPR, RBS = C::RBS;
  const uint32_t H = c.H, y0 = c.y0, t = c.t;
  if (i >= H + 3) return;
  // Row k = i + 3 of the strip for steps i <= H; the two steps after that
  // fetch row H + 3 again (an L2 hit) into ring slots no step reads any more
  // (slot (i + 3) & 7 holds row i - 5; colour 1 reads rows i - 2 .. i and the
  // closing count reads row H + 1), so that the load and its LDS store are
  // unconditional and the load never waits on the previous step's stores.
  uint2 nxt[G];
  c.get_row(wrap_row(y0 + (i <= H ? i : H) + 3, 2u, L), nxt);
  if (i <= H + 1) {
    // colour 0 on row a = y0 - 1 + i (strip row k = i + 1); parity of a is (i+1) & 1
    const uint32_t y = wrap_row(y0 + i + 1, 2u, L);
    int8_t* row = c.ring + ((S + 1) & 7) * RBS + 16;
    const int8_t* up = c.ring + (S & 7) * RBS + 16;
    const int8_t* dn = c.ring + ((S + 2) & 7) * RBS + 16;
#pragma unroll
    for (int j = 0; j < G; ++j) {
      const uint32_t g = t + NT * j;
      const uint2 cc = *reinterpret_cast<const uint2*>(row + 8 * g);
      const uint2 u2 = *reinterpret_cast<const uint2*>(up + 8 * g);
      const uint2 d2 = *reinterpret_cast<const uint2*>(dn + 8 * g);
      const uint32_t lw = *reinterpret_cast<const uint32_t*>(row + 8 * g - 4);
      const uint32_t rw = *reinterpret_cast<const uint32_t*>(row + 8 * g + 8);
      uint32_t rnd[4];
      philox_lane(y * GPR + g, c.U0, *c.keys, rnd);
      const uint32_t o0[2] = {u2.x, d2.x}, o1[2] = {u2.y, d2.y};
      const uint32_t Sp = unsat_packed<2>((S + 1) & 1, cc.x, cc.y, lw, rw, o0, o1);
      uint32_t c0 = cc.x, c1 = cc.y;
      apply_packed<NEVER>((S + 1) & 1, c0, c1, Sp, rnd, c.bound, c.never4);
      *reinterpret_cast<uint2*>(row + 8 * g) = make_uint2(c0, c1);
      if (g >= GPR - 2) *reinterpret_cast<uint2*>(row - 16 + 8 * (g - (GPR - 2))) = make_uint2(c0, c1);
      if (g < 2) *reinterpret_cast<uint2*>(row + L + 8 * g) = make_uint2(c0, c1);
    }
  }
  // colour 1 on row b = y0 + i - 3 (strip row k = i - 1); parity of (1 + b) is i & 1.
  // Its results go to dst after the LDS store of the loaded row below, so that
  // the wait for that load does not include these stores.
  uint2 res[G];
  const bool col1 = (i >= 3);
  if (col1) {
    const uint32_t y = y0 + i - 3u;
    int8_t* row = c.ring + ((S + 7) & 7) * RBS + 16;
    const int8_t* up = c.ring + ((S + 6) & 7) * RBS + 16;
    const int8_t* dn = c.ring + (S & 7) * RBS + 16;
#pragma unroll
    for (int j = 0; j < G; ++j) {
      const uint32_t g = t + NT * j;
      const uint2 cc = *reinterpret_cast<const uint2*>(row + 8 * g);
      const uint2 u2 = *reinterpret_cast<const uint2*>(up + 8 * g);
      const uint2 d2 = *reinterpret_cast<const uint2*>(dn + 8 * g);
      const uint32_t lw = *reinterpret_cast<const uint32_t*>(row + 8 * g - 4);
      const uint32_t rw = *reinterpret_cast<const uint32_t*>(row + 8 * g + 8);
      uint32_t rnd[4];
      philox_lane(y * GPR + g, c.U1, *c.keys, rnd);
      const uint32_t o0[2] = {u2.x, d2.x}, o1[2] = {u2.y, d2.y};
      const uint32_t Sp = unsat_packed<2>(S & 1, cc.x, cc.y, lw, rw, o0, o1);
      uint32_t c0 = cc.x, c1 = cc.y;
      apply_packed<NEVER>(S & 1, c0, c1, Sp, rnd, c.bound, c.never4);
      res[j] = make_uint2(c0, c1);
      if (MEAS) {
        // E and M of the swept lattice, counted on final values:
        //  - row b's negative spins;
        //  - bonds (b-1, b): row b-1 in LDS is final when b > y0 (written by the
        //    previous step); for b == y0 it is the ring row y0-1 whose colour-0
        //    bytes only are final, so only bonds whose row-b end is colour 1
        //    are counted (the strip above counts the others);
        //  - for the last row, bonds to the ring row y0+H, same rule;
        //  - horizontal bonds of row b-1 (final in LDS);
        // and row b's final bytes go to LDS for the next step.
        constexpr uint32_t kMsb = 0x80808080u;
        constexpr uint32_t kCol1 = (S & 1) ? 0x80008000u : 0x00800080u;  // colour-1 bytes of row b
        *reinterpret_cast<uint2*>(row + 8 * g) = make_uint2(c0, c1);
        if (g >= GPR - 2) *reinterpret_cast<uint2*>(row - 16 + 8 * (g - (GPR - 2))) = make_uint2(c0, c1);
        if (g < 2) *reinterpret_cast<uint2*>(row + L + 8 * g) = make_uint2(c0, c1);
        neg += __popc(c0 & kMsb) + __popc(c1 & kMsb);
        const uint32_t vm = (i == 3) ? kCol1 : kMsb;
        unsat += __popc((c0 ^ u2.x) & vm) + __popc((c1 ^ u2.y) & vm);
        if (i == H + 2) unsat += __popc((c0 ^ d2.x) & kCol1) + __popc((c1 ^ d2.y) & kCol1);
        if (i >= 4) {
          const uint32_t nx = *reinterpret_cast<const uint32_t*>(up + 8 * g + 8);
          unsat += __popc((u2.x ^ __builtin_amdgcn_alignbyte(u2.y, u2.x, 1)) & kMsb) +
                   __popc((u2.y ^ __builtin_amdgcn_alignbyte(nx, u2.y, 1)) & kMsb);
        }
      }
    }
  }
  c.put_row((S + 3) & 7, nxt);
  if (col1) c.put_out(y0 + i - 3u, res);
  __syncthreads();
}

template <int NT, int G, bool NEVER, bool MEAS>
__global__ __launch_bounds__(NT) void k_stream2d(const int8_t* __restrict__ src,
                                                 int8_t* __restrict__ dst, PhaseArgs a,
                                                 uint32_t H, Record rec) {
  using C = StreamCtx<NT, G>;
  // one LDS block: the bound table at byte 0 (a lookup address is just 4u),
  // then the 8-row ring
  __shared__ __align__(16) int8_t lds[32 + 8 * C::RBS];
  C c;
  c.rsrc = __builtin_amdgcn_make_buffer_rsrc((void*)src, 0, (int)(C::L * C::L), 0x00020000);
  c.rdst = __builtin_amdgcn_make_buffer_rsrc((void*)dst, 0, (int)(C::L * C::L), 0x00020000);
  c.ring = lds + 32;
  c.bound = reinterpret_cast<const uint32_t*>(lds);
  c.keys = &a.keys;
  c.U0 = philox_uniform(a.t, a.replica, 0u, a.keys);
  c.U1 = philox_uniform(a.t, a.replica, 1u, a.keys);
  c.never4 = a.never4;
  c.y0 = blockIdx.x * H;
  c.H = H;
  c.t = threadIdx.x;
  if (threadIdx.x < 8) reinterpret_cast<uint32_t*>(lds)[threadIdx.x] = a.bound[threadIdx.x];
  // prologue: rows k = 0, 1, 2 (y0-2, y0-1, y0)
  for (uint32_t k = 0; k < 3; ++k) {
    uint2 v[G];
    c.get_row(wrap_row(c.y0 + k, 2u, C::L), v);
    c.put_row(k, v);
  }
  __syncthreads();
  const uint32_t steps = H + 3;
  int unsat = 0, neg = 0;
  for (uint32_t i0 = 0; i0 < steps; i0 += 8) {
    stream_step<NT, G, NEVER, MEAS, 0>(c, i0 + 0, unsat, neg);
    stream_step<NT, G, NEVER, MEAS, 1>(c, i0 + 1, unsat, neg);
    stream_step<NT, G, NEVER, MEAS, 2>(c, i0 + 2, unsat, neg);
    stream_step<NT, G, NEVER, MEAS, 3>(c, i0 + 3, unsat, neg);
    stream_step<NT, G, NEVER, MEAS, 4>(c, i0 + 4, unsat, neg);
    stream_step<NT, G, NEVER, MEAS, 5>(c, i0 + 5, unsat, neg);
    stream_step<NT, G, NEVER, MEAS, 6>(c, i0 + 6, unsat, neg);
    stream_step<NT, G, NEVER, MEAS, 7>(c, i0 + 7, unsat, neg);
  }
  if (MEAS) {
    // horizontal bonds of the strip's last row (final in LDS, strip row k = H + 1)
    const int8_t* last = c.ring + ((H + 1) & 7) * C::RBS + 16;
#pragma unroll
    for (int j = 0; j < G; ++j) {
      const uint32_t g = c.t + NT * j;
      const uint2 v = *reinterpret_cast<const uint2*>(last + 8 * g);
      const uint32_t nx = *reinterpret_cast<const uint32_t*>(last + 8 * g + 8);
      unsat += __popc((v.x ^ __builtin_amdgcn_alignbyte(v.y, v.x, 1)) & 0x80808080u) +
               __popc((v.y ^ __builtin_amdgcn_alignbyte(nx, v.y, 1)) & 0x80808080u);
    }
    __shared__ int64_t red[NT / 64];
    record_block<NT>(unsat, neg, rec, red);
  }
}

// ---------------------------------------------------------------------------
// 2D Ising, one whole sweep per launch, with each thread's column of groups
// held in registers (k_stream2c).  L = 8 * NT * G; thread t owns the groups
// g = t + NT*j (j < G) of every row of the strip [y0, y0+H), so the 64 lanes
// of a wave hold one 512-site segment of each row (segment s = wave + W*j, W
// = NT/64 waves, NS = L/512 segments per row).  Row k of the strip (y =
// y0-2+k) lives in register slot k & 7.  Step i = 0..H+4, a = y0-1+i:
//   load row a+2 (and each lane's edge word, below);
//   colour 0 on row a (i <= H+1): y neighbours rows a-1 (after its colour 0)
//     and a+1 (as loaded) from registers, x neighbours by a wavefront rotate;
//   colour 1 on row b = a-4 (i >= 5): rows b-1..b+1 after colour 0 from
//     registers; the group goes to dst.
// The only data that crosses waves is the x neighbour at a segment's ends.
// Colour 0 reads it as loaded: every lane loads one more word with its row,
// lane 0 the word left of its segment, lane 63 the word right of it (the
// others a word of their own group).  Colour 1 needs the neighbouring
// segment's colour-0 result: after colour 0 on a row, lane 0 of each
// segment puts its even half (byte 0: the segment's first site) and lane 63
// its odd half (byte 3: its last site) into an LDS ring of 8 rows, and
// colour 1 reads them 4 steps later.  A barrier after every 4th
// step orders each such write before its read and each read before the slot
// is written again (written in step k-1 for row k, read in step k+3,
// rewritten in step k+7).  No spin row goes through LDS.  The two edge
// writes are made by every lane, the other lanes into 64 words of their own
// after the slot's edge words, so that no branch on the lane is taken.
// Groups are held parity-split (split_group: even bytes, odd bytes), so a
// colour unit's active sites and their row neighbours need no gathering.
// Accept bounds come from the pair table (8u per packed byte, spin_packed.h),
// and the first Philox product takes the row's part of the counter as a
// scalar addend.
template <int NT, int G>
struct Col2Ctx {
  static constexpr uint32_t L = 8u * NT * G;
  static constexpr uint32_t GPR = L / 8;
  static constexpr uint32_t W = NT / 64;
  static constexpr uint32_t NS = W * G;  // segments per row
  static constexpr uint32_t SW = 2 * NS + 64;  // words per ring slot: [segment NS][lo, hi], then 64 spare
  static constexpr uint32_t PW = (pair_words(4) + 15u) & ~15u;  // pair table words, rounded to 64 bytes
  __amdgpu_buffer_rsrc_t rsrc, rdst;
  uint32_t* edge;                        // LDS: [slot 8][SW]
  const char* pair;
  const RoundKeys* keys;
  PhiloxUniform U0, U1;
  uint32_t never8, y0, H, t, lane;
  uint32_t eoff[G];                      // byte offset in a row of this lane's edge word
  uint32_t lnb[G], rnb[G];               // LDS word of the left segment's high word, the right one's low word
  uint32_t wlo[G], whi[G];               // LDS words the lane's low and high results go to (spare unless lane 0 / 63)
};

// One colour unit of a parity-split group c (x: even bytes, y: odd bytes)
// with active parity P: y neighbours up, dn (split), x neighbour dword nb
// (natural layout: its byte 3 is the site left of the group for P = 0, its
// byte 0 the site right of it for P = 1); Philox counter base + v with mbase
// = philox_base(base).  The other half of the group holds the neighbours on
// one side, moved by one byte with nb's boundary byte shifted in those on
// the other.  The bounds are read before the Philox rounds so that their LDS
// reads are in flight during them.  With MEAS adds 4 x the unsatisfied bonds
// of the active sites after the update to acc.
template <uint32_t P, bool NEVER, bool MEAS>
__device__ __forceinline__ uint2 col2_unit(uint2 c, uint2 up, uint2 dn, uint32_t nb, uint32_t v, uint64_t mbase,
                                           const PhiloxUniform& U, const RoundKeys& K, const char* pair,
                                           uint32_t never8, uint32_t& acc) {
  const uint32_t A = P ? c.y : c.x, I = P ? c.x : c.y;
  const uint32_t N = __builtin_amdgcn_perm(I, nb, P ? 0x00070605u : 0x06050403u);
  const uint32_t S = ((A ^ I) & kSignBit8) + ((A ^ N) & kSignBit8) + ((A ^ (P ? up.y : up.x)) & kSignBit8) +
                     ((A ^ (P ? dn.y : dn.x)) & kSignBit8);
  const uint4 b = lookup_pair(S, pair);
  uint32_t rnd[4];
  philox_lane_split(v, mbase, U, K, rnd);
  const uint32_t An = MEAS ? apply_split_count<NEVER, 2>(A, S, b, rnd, never8, acc)
                           : apply_split<NEVER>(A, S, b, rnd, never8);
  return P ? make_uint2(c.x, An) : make_uint2(An, c.y);
}

// x neighbour dword for active parity P (P = 0: the high dword of the group to
// the left; P = 1: the low dword of the group to the right) from the
// adjacent lane, or at the segment's end (lane 0 / lane 63) the value given:
// a wavefront shift by one lane (wave_shr:1 / wave_shl:1) with bound_ctrl off
// leaves the lane that has no source lane with the old value, `end`.
template <uint32_t P>
__device__ __forceinline__ uint32_t col2_xnb(uint2 c, uint32_t end) {
  if (P == 0) return (uint32_t)__builtin_amdgcn_update_dpp((int)end, (int)c.y, 0x138, 0xF, 0xF, false);
  return (uint32_t)__builtin_amdgcn_update_dpp((int)end, (int)c.x, 0x130, 0xF, 0xF, false);
}

template <int NT, int G, bool NEVER, bool MEAS, uint32_t S>
__device__ __forceinline__ void col2_step(const Col2Ctx<NT, G>& c, uint2 (&R)[8][G], uint32_t (&E)[8][G],
                                          uint32_t i, uint32_t& unsat4, uint32_t& neg) {
  using C = Col2Ctx<NT, G>;
  constexpr uint32_t L = C::L, GPR = C::GPR;
  if (i >= c.H + 5) return;
  // row a+2 = strip row i+3 (steps after i = H reload row H+3, which nothing reads)
  const uint32_t yl = wrap_row(c.y0 + (i <= c.H ? i : c.H) + 3u, 2u, L);
#pragma unroll
  for (int j = 0; j < G; ++j) {
    const u32x2 w = __builtin_amdgcn_raw_buffer_load_b64(c.rsrc, 8u * (c.t + NT * j), yl * L, 0);
    R[(S + 3) & 7][j] = split_group(w.x, w.y);
    E[(S + 3) & 7][j] = __builtin_amdgcn_raw_buffer_load_b32(c.rsrc, c.eoff[j], yl * L, 0);
  }
  if (i <= c.H + 1) {
    // colour 0 on row a (strip row i+1, register slot S+1); a has the parity of i+1
    constexpr uint32_t P = (S + 1u) & 1u;
    const uint32_t y = wrap_row(c.y0 + i + 1u, 2u, L);
    uint32_t* slot = c.edge + ((S + 1u) & 7u) * C::SW;
#pragma unroll
    for (int j = 0; j < G; ++j) {
      const uint2 cc = R[(S + 1) & 7][j];
      const uint32_t nb = col2_xnb<P>(cc, E[(S + 1) & 7][j]);
      uint32_t none = 0;
      const uint2 n = col2_unit<P, NEVER, false>(cc, R[S & 7][j], R[(S + 2) & 7][j], nb, c.t,
                                                 philox_base(y * GPR + NT * j), c.U0, *c.keys, c.pair, c.never8,
                                                 none);
      R[(S + 1) & 7][j] = n;
      slot[c.wlo[j]] = n.x;
      slot[c.whi[j]] = n.y;
    }
  }
  if (i >= 5) {
    // colour 1 on row b (strip row i-3, register slot S+5); 1 + b has the parity of i
    constexpr uint32_t P = S & 1u;
    const uint32_t y = c.y0 + i - 5u;
    const uint32_t* slot = c.edge + ((S + 5u) & 7u) * C::SW;
#pragma unroll
    for (int j = 0; j < G; ++j) {
      const uint2 cc = R[(S + 5) & 7][j];
      const uint32_t nb = col2_xnb<P>(cc, slot[P == 0 ? c.lnb[j] : c.rnb[j]]);
      const uint2 n = col2_unit<P, NEVER, MEAS>(cc, R[(S + 4) & 7][j], R[(S + 6) & 7][j], nb, c.t,
                                                philox_base(y * GPR + NT * j), c.U1, *c.keys, c.pair, c.never8,
                                                unsat4);
      // the group is final: count its negative spins
      if (MEAS) neg += __popc(n.x & 0x80808080u) + __popc(n.y & 0x80808080u);
      R[(S + 5) & 7][j] = n;
      const uint2 o = join_group(n);
      const u32x2 w = {o.x, o.y};
      __builtin_amdgcn_raw_buffer_store_b64(w, c.rdst, 8u * (c.t + NT * j), y * L, 0);
    }
  }
  if ((S & 3u) == 3u) __syncthreads();
}

template <int NT, int G, bool NEVER, bool MEAS>
__global__ __launch_bounds__(NT) void k_stream2c(const int8_t* __restrict__ src, int8_t* __restrict__ dst,
                                                 PhaseArgs a, uint32_t H, Record rec) {
  using C = Col2Ctx<NT, G>;
  constexpr uint32_t L = C::L, NS = C::NS;
  __shared__ __align__(16) uint32_t lds[C::PW + 8 * C::SW];
  C c;
  c.rsrc = __builtin_amdgcn_make_buffer_rsrc((void*)src, 0, (int)(L * L), 0x00020000);
  c.rdst = __builtin_amdgcn_make_buffer_rsrc((void*)dst, 0, (int)(L * L), 0x00020000);
  c.pair = (const char*)lds;
  c.edge = lds + C::PW;
  c.keys = &a.keys;
  c.U0 = philox_uniform(a.t, a.replica, 0u, a.keys);
  c.U1 = philox_uniform(a.t, a.replica, 1u, a.keys);
  c.never8 = 2u * a.never4;
  c.y0 = blockIdx.x * H;
  c.H = H;
  c.t = threadIdx.x;
  c.lane = threadIdx.x & 63u;
  const uint32_t wave = threadIdx.x >> 6;
#pragma unroll
  for (int j = 0; j < G; ++j) {
    const uint32_t g = c.t + NT * j, s = wave + C::W * j;
    c.eoff[j] = c.lane == 0 ? (g ? 8u * g - 4u : L - 4u) : (c.lane == 63 ? (8u * (g + 1u)) % L : 8u * g);
    c.wlo[j] = c.lane == 0 ? 2u * s : 2u * NS + c.lane;
    c.whi[j] = c.lane == 63 ? 2u * s + 1u : 2u * NS + c.lane;
    c.lnb[j] = 2u * ((s + NS - 1u) % NS) + 1u;
    c.rnb[j] = 2u * ((s + 1u) % NS);
  }
  fill_pair<4>(lds, a.bound, threadIdx.x);
  keys_resident(a.keys);
  uint2 R[8][G];
  uint32_t E[8][G];
  // prologue: strip rows 0, 1, 2 (y0-2, y0-1, y0)
#pragma unroll
  for (uint32_t k = 0; k < 3; ++k) {
    const uint32_t y = wrap_row(c.y0 + k, 2u, L);
#pragma unroll
    for (int j = 0; j < G; ++j) {
      const u32x2 w = __builtin_amdgcn_raw_buffer_load_b64(c.rsrc, 8u * (c.t + NT * j), y * L, 0);
      R[k][j] = split_group(w.x, w.y);
      E[k][j] = __builtin_amdgcn_raw_buffer_load_b32(c.rsrc, c.eoff[j], y * L, 0);
    }
  }
#pragma unroll
  for (int k = 3; k < 8; ++k)
#pragma unroll
    for (int j = 0; j < G; ++j) {
      R[k][j] = make_uint2(0u, 0u);
      E[k][j] = 0u;
    }
  __syncthreads();
  // with MEAS: 4 x the unsatisfied bonds of the strip's colour-1 sites after their update (every
  // bond joins a colour-0 and a colour-1 site, and the colour-0 sites are final by then) and the
  // negative spins of its final groups
  uint32_t unsat4 = 0, neg = 0;
  const uint32_t steps = H + 5;
  for (uint32_t i0 = 0; i0 < steps; i0 += 8) {
    col2_step<NT, G, NEVER, MEAS, 0>(c, R, E, i0 + 0, unsat4, neg);
    col2_step<NT, G, NEVER, MEAS, 1>(c, R, E, i0 + 1, unsat4, neg);
    col2_step<NT, G, NEVER, MEAS, 2>(c, R, E, i0 + 2, unsat4, neg);
    col2_step<NT, G, NEVER, MEAS, 3>(c, R, E, i0 + 3, unsat4, neg);
    col2_step<NT, G, NEVER, MEAS, 4>(c, R, E, i0 + 4, unsat4, neg);
    col2_step<NT, G, NEVER, MEAS, 5>(c, R, E, i0 + 5, unsat4, neg);
    col2_step<NT, G, NEVER, MEAS, 6>(c, R, E, i0 + 6, unsat4, neg);
    col2_step<NT, G, NEVER, MEAS, 7>(c, R, E, i0 + 7, unsat4, neg);
  }
  if (MEAS) {
    __shared__ int64_t red[NT / 64];
    record_block<NT>((int64_t)(unsat4 >> 2), (int64_t)neg, rec, red);
  }
}

// Streaming variants: tile.x == L (full rows), tile.y = strip height H,
// tile.threads = NT with L = 8 * NT * G.
bool stream2d_shape(uint32_t L, int threads, int* G) {
  if (threads != 256 && threads != 512 && threads != 1024) return false;
  if (L % (8u * (uint32_t)threads) != 0) return false;
  const uint32_t g = L / (8u * (uint32_t)threads);
  if (g != 1 && g != 2) return false;
  if (threads == 256 && g != 2) return false;  // instantiated: (1024,1) (1024,2) (512,1) (512,2) (256,2)
  *G = (int)g;
  return true;
}

template <int NT, int G>
static hipError_t gostream(const Lat& lat, const int8_t* src, int8_t* dst, const PhaseArgs& a,
                           bool never, uint32_t H, const Record* rec, hipStream_t stream) {
  dim3 grid(lat.L / H);
  const Record r = rec ? *rec : Record{nullptr};
  if (rec) {
    if (never)
      hipLaunchKernelGGL((k_stream2d<NT, G, true, true>), grid, dim3(NT), 0, stream, src, dst, a, H, r);
    else
      hipLaunchKernelGGL((k_stream2d<NT, G, false, true>), grid, dim3(NT), 0, stream, src, dst, a, H, r);
  } else {
    if (never)
      hipLaunchKernelGGL((k_stream2d<NT, G, true, false>), grid, dim3(NT), 0, stream, src, dst, a, H, r);
    else
      hipLaunchKernelGGL((k_stream2d<NT, G, false, false>), grid, dim3(NT), 0, stream, src, dst, a, H, r);
  }
  return hipGetLastError();
}

template <int NT, int G>
static hipError_t gocol2(const Lat& lat, const int8_t* src, int8_t* dst, const PhaseArgs& a, bool never,
                         uint32_t H, const Record* rec, hipStream_t stream) {
  dim3 grid(lat.L / H);
  const Record r = rec ? *rec : Record{nullptr};
  if (rec) {
    if (never)
      hipLaunchKernelGGL((k_stream2c<NT, G, true, true>), grid, dim3(NT), 0, stream, src, dst, a, H, r);
    else
      hipLaunchKernelGGL((k_stream2c<NT, G, false, true>), grid, dim3(NT), 0, stream, src, dst, a, H, r);
  } else {
    if (never)
      hipLaunchKernelGGL((k_stream2c<NT, G, true, false>), grid, dim3(NT), 0, stream, src, dst, a, H, r);
    else
      hipLaunchKernelGGL((k_stream2c<NT, G, false, false>), grid, dim3(NT), 0, stream, src, dst, a, H, r);
  }
  return hipGetLastError();
}

hipError_t launch_stream2c(const Lat& lat, const int8_t* src, int8_t* dst, const PhaseArgs& a, bool never,
                           uint32_t H, const Record* rec, int threads, int G, hipStream_t stream) {
  if (threads == 1024 && G == 1) return gocol2<1024, 1>(lat, src, dst, a, never, H, rec, stream);
  if (threads == 1024 && G == 2) return gocol2<1024, 2>(lat, src, dst, a, never, H, rec, stream);
  if (threads == 512 && G == 1) return gocol2<512, 1>(lat, src, dst, a, never, H, rec, stream);
  if (threads == 512 && G == 2) return gocol2<512, 2>(lat, src, dst, a, never, H, rec, stream);
  if (threads == 256 && G == 2) return gocol2<256, 2>(lat, src, dst, a, never, H, rec, stream);
  return hipErrorInvalidValue;
}

hipError_t launch_stream2d(const Lat& lat, const int8_t* src, int8_t* dst, const PhaseArgs& a, bool never,
                           uint32_t H, const Record* rec, int threads, int G, hipStream_t stream) {
  if (threads == 1024 && G == 1) return gostream<1024, 1>(lat, src, dst, a, never, H, rec, stream);
  if (threads == 1024 && G == 2) return gostream<1024, 2>(lat, src, dst, a, never, H, rec, stream);
  if (threads == 512 && G == 1) return gostream<512, 1>(lat, src, dst, a, never, H, rec, stream);
  if (threads == 512 && G == 2) return gostream<512, 2>(lat, src, dst, a, never, H, rec, stream);
  if (threads == 256 && G == 2) return gostream<256, 2>(lat, src, dst, a, never, H, rec, stream);
  return hipErrorInvalidValue;
}

}  // namespace spin
