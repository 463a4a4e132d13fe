// spin_batch_kernels.hip -- many lattices per launch (disorder realisations x
// temperatures, Sec. 4, last paragraph).
//
// A persistent kernel takes tasks (one lattice, n sweeps) from a queue; the
// workgroup holding a task keeps the whole lattice in LDS for all n sweeps and
// writes it back at the end.  In LDS the spins are packed 8 per 32-bit word:
// site 8w+j is nibble j of word w, +1 = 0x1, -1 = 0xF (the low nibble of the
// int8 value), so bits 1..3 of a nibble carry the sign.  (a ^ b) & 0x2 per
// nibble marks an unsatisfied bond (with a coupling nibble in the XOR for the
// +-J glass), the sum over the 2d neighbours is 2u per nibble (u <= 6), and
// a flip XORs the nibble with 0xE.  The Metropolis decision is the same
// bound lookup as in the single-lattice kernels.  The chain is unchanged:
// same Philox counters (group s>>3 = word index), same tables, same order.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "spin_batch.h"
#include "spin_device.h"

namespace spin {

// Philox4x32-10 as philox_lane computes it, with round 3 left in the loop of
// the later rounds: c3 after round 2 is recovered from the folded word
// (x4 = c3 ^ k1[2]) on the scalar unit.  Same words; this kernel waits on
// its texture path rather than on VALU issue, and measured this form 3 %
// faster than the folded one, whose changed schedule costs it more than the
// operation it saves.
__device__ __forceinline__ void philox_lane_unfolded(uint32_t c0, const PhiloxUniform& U, const RoundKeys& K,
                                                     uint32_t r[4]) {
  const uint64_t p0 = (uint64_t)kPhiloxM0 * c0;
  const uint32_t a2 = (uint32_t)(p0 >> 32) ^ U.x1;
  const uint32_t a3 = (uint32_t)p0;
  const uint64_t p1 = (uint64_t)kPhiloxM1 * a2;
  uint32_t d0 = (uint32_t)(p1 >> 32) ^ U.x2;
  uint32_t d1 = (uint32_t)p1;
  uint32_t d2 = a3 ^ U.x3;
  uint32_t d3 = U.x4 ^ K.k1[2];
#pragma unroll
  for (int i = 2; i < 10; ++i) {
    const uint64_t q0 = (uint64_t)kPhiloxM0 * d0;
    const uint64_t q1 = (uint64_t)kPhiloxM1 * d2;
    const uint32_t n0 = xor3((uint32_t)(q1 >> 32), d1, K.k0[i]);
    const uint32_t n2 = xor3((uint32_t)(q0 >> 32), d3, K.k1[i]);
    d1 = (uint32_t)q1;
    d3 = (uint32_t)q0;
    d0 = n0;
    d2 = n2;
  }
  r[0] = d0; r[1] = d1; r[2] = d2; r[3] = d3;
}

// ---------------------------------------------------------------- couplings

// Generate couplings (Philox rule of spin.h) directly in nibble form:
// word w of direction dir holds J[dir][8w .. 8w+7].
__global__ void k_couplings_nibble(uint32_t* __restrict__ Jn, uint32_t nwords, uint32_t d,
                                   RoundKeys K, uint32_t realisation) {
  for (uint32_t dir = 0; dir < d; ++dir)
    for (uint32_t w = blockIdx.x * blockDim.x + threadIdx.x; w < nwords; w += gridDim.x * blockDim.x) {
      uint32_t v = 0;
#pragma unroll
      for (uint32_t h = 0; h < 2; ++h) {
        uint32_t r[4];
        philox(2 * w + h, dir, realisation, 3u, K, r);
#pragma unroll
        for (int j = 0; j < 4; ++j) v |= ((r[j] >> 31) ? 0xFu : 0x1u) << (4 * (4 * h + j));
      }
      Jn[(size_t)dir * nwords + w] = v;
    }
}

// Pack int8 couplings [dir][site] into nibble words.
__global__ void k_pack_nibbles(const int8_t* __restrict__ src, uint32_t* __restrict__ dst, uint32_t nwords) {
  for (uint32_t w = blockIdx.x * blockDim.x + threadIdx.x; w < nwords; w += gridDim.x * blockDim.x) {
    const uint2 b = reinterpret_cast<const uint2*>(src)[w];
    dst[w] = pack_nibbles(b.x, b.y);
  }
}

hipError_t launch_couplings_nibble(uint32_t* Jn, uint64_t N, uint32_t d, uint64_t cseed,
                                   uint32_t realisation, hipStream_t stream) {
  const uint32_t nwords = (uint32_t)(N / 8);
  const uint32_t blocks = (nwords + 255) / 256 < 4096 ? (nwords + 255) / 256 : 4096;
  hipLaunchKernelGGL(k_couplings_nibble, dim3(blocks ? blocks : 1), dim3(256), 0, stream, Jn, nwords, d,
                     make_round_keys(cseed), realisation);
  return hipGetLastError();
}

hipError_t launch_pack_nibbles(const int8_t* src, uint32_t* dst, uint64_t nbytes, hipStream_t stream) {
  const uint32_t nwords = (uint32_t)(nbytes / 8);
  const uint32_t blocks = (nwords + 255) / 256 < 4096 ? (nwords + 255) / 256 : 4096;
  hipLaunchKernelGGL(k_pack_nibbles, dim3(blocks ? blocks : 1), dim3(256), 0, stream, src, dst, nwords);
  return hipGetLastError();
}

// --------------------------------------------------------- batch kernel

__global__ void k_zero_u32(uint32_t* p, uint32_t n) {
  for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) p[i] = 0;
}

// E = -d N + 2 (unsatisfied bonds), M = N - 2 (negative spins) of the LDS
// lattice into Cl.E[rec], Cl.M[rec].
template <int D, bool EA, int NT>
__device__ void batch_record(const BatchLattice& B, const BatchCall& Cl, const uint32_t* sp, int64_t* red,
                             uint32_t rec) {
  const uint32_t L = B.L, LG = L / 8, R = (D == 3) ? L * L : L, NW = R * LG, PS = L * LG;
  const uint32_t* Jx = B.Jn;
  const uint32_t* Jy = EA ? B.Jn + NW : nullptr;
  const uint32_t* Jz = EA ? B.Jn + 2 * NW : nullptr;
  int64_t unsat = 0, neg = 0;
  for (uint32_t w = threadIdx.x; w < NW; w += NT) {
    const uint32_t c = sp[w];
    const uint32_t x = w % LG, row = w / LG, y = row % L, z = row / L;
    neg += __popc(c & 0x88888888u);
    const uint32_t rwd = sp[(x + 1 < LG) ? w + 1 : w - (LG - 1)];
    const uint32_t Rx = __builtin_amdgcn_alignbit(rwd, c, 4);
    const uint32_t yp = sp[(y + 1 < L) ? w + LG : w - (L - 1) * LG];
    unsat += __popc(xor3(c, Rx, EA ? Jx[w] : 0u) & 0x88888888u);
    unsat += __popc(xor3(c, yp, EA ? Jy[w] : 0u) & 0x88888888u);
    if (D == 3) {
      const uint32_t zp = sp[(z + 1 < L) ? w + PS : w - (L - 1) * PS];
      unsat += __popc(xor3(c, zp, EA ? Jz[w] : 0u) & 0x88888888u);
    }
  }
  const int64_t su = block_sum<NT>(unsat, red);
  const int64_t sn = block_sum<NT>(neg, red);
  if (threadIdx.x == 0) {
    const int64_t N = (int64_t)NW * 8;
    Cl.E[rec] = -(int64_t)D * N + 2 * su;
    Cl.M[rec] = N - 2 * sn;
  }
}

// Wavefront-uniform copies of a task's parameters.  The descriptors are read
// from global memory by every lane; readfirstlane tells the compiler the
// values are the same in all lanes, so they live in scalar registers and the
// coupling loads below take a scalar base with 32-bit lane offsets.
__device__ __forceinline__ uint32_t uni(uint32_t v) { return __builtin_amdgcn_readfirstlane(v); }

template <class T>
__device__ __forceinline__ T* uni_ptr(T* p) {
  const uint64_t v = (uint64_t)p;
  return (T*)(((uint64_t)uni((uint32_t)(v >> 32)) << 32) | uni((uint32_t)v));
}

__device__ __forceinline__ BatchLattice uniform_lattice(const BatchLattice& B) {
  BatchLattice u;
  u.spins = uni_ptr(B.spins);
  u.Jn = uni_ptr(B.Jn);
  u.L = uni(B.L);
  u.d = uni(B.d);
  u.replica = uni(B.replica);
  u.t = uni(B.t);
#pragma unroll
  for (int i = 0; i < 10; ++i) {
    u.keys.k0[i] = uni(B.keys.k0[i]);
    u.keys.k1[i] = uni(B.keys.k1[i]);
  }
  return u;
}

__device__ __forceinline__ BatchCall uniform_call(const BatchCall& C) {
  BatchCall u;
  u.n = uni(C.n);
  u.every = uni(C.every);
  u.never4 = uni(C.never4);
#pragma unroll
  for (int i = 0; i < 8; ++i) u.bound[i] = uni(C.bound[i]);
  u.E = uni_ptr(C.E);
  u.M = uni_ptr(C.M);
  return u;
}

// Per-thread geometry of a task: thread -> (word column xg, first row); rows
// advance by RI = NT / LG per iteration.
struct BatchGeo {
  uint32_t L, LG, R, NW, PS, RI, xg, r_first, dy, dz, wl, wr, ym_wrap, zm_wrap;
};

// One colour phase over the thread's rows.  YFIX: RI is a multiple of L, so
// every row the thread visits has the same y: its y-neighbour offsets are
// fixed, and the parity of the active sites steps by dz per row.
template <int D, bool EA, bool NEVER, bool YFIX>
__device__ __forceinline__ void batch_colour(uint32_t* sp, const uint32_t* bound, __amdgpu_buffer_rsrc_t rj,
                                             const BatchGeo& g, const PhiloxUniform& U, const RoundKeys& K,
                                             uint32_t colour, uint32_t nev) {
  const uint32_t L = g.L, LG = g.LG, PS = g.PS, NW = g.NW;
  uint32_t y = g.r_first % L, z = g.r_first / L;
  const uint32_t ymo = y ? 0u - LG : g.ym_wrap;               // used when YFIX
  const uint32_t ypo = (y + 1 < L) ? LG : 0u - g.ym_wrap;
  uint32_t p = (colour + y + z) & 1u;
  const uint32_t pstep = g.dz & 1u;
  const uint32_t wstep = g.RI * LG;
  uint32_t w = g.r_first * LG + g.xg;
  for (uint32_t row = g.r_first; row < g.R; row += g.RI, w += wstep) {
    const uint32_t c = sp[w];
    const uint32_t lw = sp[w + g.wl], rw = sp[w + g.wr];
    const uint32_t wym = w + (YFIX ? ymo : (y ? 0u - LG : g.ym_wrap));
    const uint32_t wyp = w + (YFIX ? ypo : ((y + 1 < L) ? LG : 0u - g.ym_wrap));
    uint32_t nb[2 * D - 2];
    uint32_t jn[2 * D];
    nb[0] = sp[wym];
    nb[1] = sp[wyp];
    uint32_t wzm = 0;
    if (D == 3) {
      // planes z-1 and z+1, periodic: w -/+ PS wrapped into [0, NW) by an unsigned minimum (the
      // out-of-range candidate has wrapped past 2^32 or is at least NW), no per-lane select
      const uint32_t m = w - PS, q = w + PS;
      wzm = __builtin_elementwise_min(m, m + NW);
      const uint32_t wzp = __builtin_elementwise_min(q, q - NW);
      nb[2] = sp[wzm];
      nb[3] = sp[wzp];
    }
    if (EA) {
      const uint32_t jx = __builtin_amdgcn_raw_buffer_load_b32(rj, 4u * w, 0, 0);
      const uint32_t jxl = __builtin_amdgcn_raw_buffer_load_b32(rj, 4u * (w + g.wl), 0, 0);
      jn[0] = __builtin_amdgcn_alignbit(jx, jxl, 28);  // bond (x-1, x)
      jn[1] = jx;                                      // bond (x, x+1)
      jn[2] = __builtin_amdgcn_raw_buffer_load_b32(rj, 4u * wym, 4u * NW, 0);
      jn[3] = __builtin_amdgcn_raw_buffer_load_b32(rj, 4u * w, 4u * NW, 0);
      if (D == 3) {
        jn[4] = __builtin_amdgcn_raw_buffer_load_b32(rj, 4u * wzm, 8u * NW, 0);
        jn[5] = __builtin_amdgcn_raw_buffer_load_b32(rj, 4u * w, 8u * NW, 0);
      }
    }
    const uint32_t S = nib_unsat<D, EA>(c, lw, rw, nb, jn);
    uint32_t rnd[4];
    philox_lane_unfolded(w, U, K, rnd);
    sp[w] = c ^ nib_flips<NEVER>(S, p, rnd, bound, nev);
    if (YFIX) {
      z += g.dz;
      p ^= pstep;
    } else {
      y += g.dy;
      z += g.dz;
      if (y >= L) {
        y -= L;
        z += 1;
      }
      p = (colour + y + z) & 1u;
    }
  }
}

// The same phase with two adjacent words per thread (rows of an even number
// of words): the pair is one 8-byte LDS access per neighbour row and one
// 8-byte coupling load per direction and side, so a word costs 3 coupling
// loads instead of 6 and 4.5 LDS reads instead of 7 (the coupling loads
// through the vector memory path, not the ALU, set this kernel's pace).  The
// x neighbours and the x bond between the two words come from the pair
// itself.  g describes the pair columns: xg the pair, wl / wr the offsets of
// the words left of the first and right of the second word.
template <int D, bool EA, bool NEVER, bool YFIX>
__device__ __forceinline__ void batch_colour2(uint32_t* sp, const uint32_t* bound, __amdgpu_buffer_rsrc_t rj,
                                              const BatchGeo& g, const PhiloxUniform& U, const RoundKeys& K,
                                              uint32_t colour, uint32_t nev) {
  const uint32_t L = g.L, LG = g.LG, PS = g.PS, NW = g.NW;
  uint32_t y = g.r_first % L, z = g.r_first / L;
  const uint32_t ymo = y ? 0u - LG : g.ym_wrap;               // used when YFIX
  const uint32_t ypo = (y + 1 < L) ? LG : 0u - g.ym_wrap;
  uint32_t p = (colour + y + z) & 1u;
  const uint32_t pstep = g.dz & 1u;
  const uint32_t wstep = g.RI * LG;
  uint32_t w = g.r_first * LG + 2u * g.xg;
  for (uint32_t row = g.r_first; row < g.R; row += g.RI, w += wstep) {
    const uint2 c = *reinterpret_cast<const uint2*>(sp + w);
    const uint32_t lw = sp[w + g.wl], rw = sp[w + g.wr];
    const uint32_t wym = w + (YFIX ? ymo : (y ? 0u - LG : g.ym_wrap));
    const uint32_t wyp = w + (YFIX ? ypo : ((y + 1 < L) ? LG : 0u - g.ym_wrap));
    uint2 nbp[2 * D - 2];
    nbp[0] = *reinterpret_cast<const uint2*>(sp + wym);
    nbp[1] = *reinterpret_cast<const uint2*>(sp + wyp);
    uint32_t wzm = 0;
    if (D == 3) {
      const uint32_t m = w - PS, q = w + PS;
      wzm = __builtin_elementwise_min(m, m + NW);
      const uint32_t wzp = __builtin_elementwise_min(q, q - NW);
      nbp[2] = *reinterpret_cast<const uint2*>(sp + wzm);
      nbp[3] = *reinterpret_cast<const uint2*>(sp + wzp);
    }
    uint32_t nb0[2 * D - 2], nb1[2 * D - 2], jn0[2 * D], jn1[2 * D];
#pragma unroll
    for (int k = 0; k < 2 * D - 2; ++k) {
      nb0[k] = nbp[k].x;
      nb1[k] = nbp[k].y;
    }
    if (EA) {
      typedef uint32_t u2v __attribute__((ext_vector_type(2)));
      const u2v jx = __builtin_amdgcn_raw_buffer_load_b64(rj, 4u * w, 0, 0);
      const uint32_t jxl = __builtin_amdgcn_raw_buffer_load_b32(rj, 4u * (w + g.wl), 0, 0);
      const u2v jy = __builtin_amdgcn_raw_buffer_load_b64(rj, 4u * w, 4u * NW, 0);
      const u2v jym = __builtin_amdgcn_raw_buffer_load_b64(rj, 4u * wym, 4u * NW, 0);
      jn0[0] = __builtin_amdgcn_alignbit(jx.x, jxl, 28);   // bond (x-1, x)
      jn0[1] = jx.x;                                       // bond (x, x+1)
      jn1[0] = __builtin_amdgcn_alignbit(jx.y, jx.x, 28);
      jn1[1] = jx.y;
      jn0[2] = jym.x;
      jn0[3] = jy.x;
      jn1[2] = jym.y;
      jn1[3] = jy.y;
      if (D == 3) {
        const u2v jz = __builtin_amdgcn_raw_buffer_load_b64(rj, 4u * w, 8u * NW, 0);
        const u2v jzm = __builtin_amdgcn_raw_buffer_load_b64(rj, 4u * wzm, 8u * NW, 0);
        jn0[4] = jzm.x;
        jn0[5] = jz.x;
        jn1[4] = jzm.y;
        jn1[5] = jz.y;
      }
    }
    const uint32_t S0 = nib_unsat<D, EA>(c.x, lw, c.y, nb0, jn0);
    const uint32_t S1 = nib_unsat<D, EA>(c.y, c.x, rw, nb1, jn1);
    uint32_t r0[4], r1[4];
    philox_lane_unfolded(w, U, K, r0);
    philox_lane_unfolded(w + 1u, U, K, r1);
    *reinterpret_cast<uint2*>(sp + w) =
        make_uint2(c.x ^ nib_flips<NEVER>(S0, p, r0, bound, nev), c.y ^ nib_flips<NEVER>(S1, p, r1, bound, nev));
    if (YFIX) {
      z += g.dz;
      p ^= pstep;
    } else {
      y += g.dy;
      z += g.dz;
      if (y >= L) {
        y -= L;
        z += 1;
      }
      p = (colour + y + z) & 1u;
    }
  }
}

// n sweeps of lattice B (uniform parameters) in LDS, NEVER: the table has
// classes with T == 0.
template <int D, bool EA, int NT, bool NEVER>
__device__ __forceinline__ void batch_sweeps(const BatchLattice& B, const BatchCall& Cl, uint32_t* sp,
                                             const uint32_t* bound, int64_t* red) {
  BatchGeo g;
  g.L = B.L;
  g.LG = g.L / 8;                                  // words per row
  g.R = (D == 3) ? g.L * g.L : g.L;                // rows
  g.NW = g.R * g.LG;                               // words
  g.PS = g.L * g.LG;                               // words per plane (3D)
  const uint32_t tid = threadIdx.x;
  g.RI = NT / g.LG;                                // rows per iteration (>= 1: L <= 8192)
  // rows of a fixed y per thread (a multiple of L rows per iteration) when that keeps at least 4/5
  // of the threads busy (L = 48 at 1024 threads: 144 of 170 rows, L = 24 at 256: 72 of 85)
  if (g.RI > g.L && g.RI % g.L != 0 && 5u * (g.RI - g.RI % g.L) >= 4u * g.RI) g.RI -= g.RI % g.L;
  const bool active = tid < g.RI * g.LG;           // active threads
  g.xg = tid % g.LG;
  g.r_first = tid / g.LG;
  g.dz = g.RI / g.L;                               // row step in (y, z)
  g.dy = g.RI % g.L;
  g.wl = g.xg ? 0u - 1u : g.LG - 1u;               // offset to the word on the left
  g.wr = (g.xg + 1 < g.LG) ? 1u : 0u - (g.LG - 1u);
  g.ym_wrap = (g.L - 1) * g.LG;
  g.zm_wrap = (g.L - 1) * g.PS;
  const bool yfix = g.dy == 0;
  // rows of an even number of words: pairs of words per thread (batch_colour2)
  const bool pair = (g.LG & 1u) == 0;
  BatchGeo g2 = g;
  if (pair) {
    const uint32_t PG = g.LG / 2;                  // pairs per row
    g2.RI = NT / PG;
    if (g2.RI > g.L && g2.RI % g.L != 0 && 5u * (g2.RI - g2.RI % g.L) >= 4u * g2.RI) g2.RI -= g2.RI % g.L;
    g2.xg = tid % PG;
    g2.r_first = tid / PG;
    g2.dz = g2.RI / g.L;
    g2.dy = g2.RI % g.L;
    g2.wl = g2.xg ? 0u - 1u : g.LG - 1u;            // word left of the pair's first word
    g2.wr = (g2.xg + 1 < PG) ? 2u : 2u - g.LG;      // word right of its second word
  }
  const bool active2 = pair && tid < g2.RI * (g.LG / 2);
  const bool yfix2 = g2.dy == 0;
  // couplings by buffer loads: one descriptor over the d arrays of NW words, byte offsets per lane
  const __amdgpu_buffer_rsrc_t rj =
      __builtin_amdgcn_make_buffer_rsrc((void*)B.Jn, 0, (int)(4u * D * g.NW), 0x00020000);
  const uint32_t nev = NEVER ? Cl.never4 : 0u;
  uint32_t rec = 0;
  for (uint32_t i = 0; i < Cl.n; ++i) {
    const uint32_t t = B.t + i;
#pragma unroll 1
    for (uint32_t colour = 0; colour < 2; ++colour) {
      const PhiloxUniform U = philox_uniform(t, B.replica, colour, B.keys);
      if (pair) {
        if (active2) {
          if (yfix2)
            batch_colour2<D, EA, NEVER, true>(sp, bound, rj, g2, U, B.keys, colour, nev);
          else
            batch_colour2<D, EA, NEVER, false>(sp, bound, rj, g2, U, B.keys, colour, nev);
        }
      } else if (active) {
        if (yfix)
          batch_colour<D, EA, NEVER, true>(sp, bound, rj, g, U, B.keys, colour, nev);
        else
          batch_colour<D, EA, NEVER, false>(sp, bound, rj, g, U, B.keys, colour, nev);
      }
      __syncthreads();
    }
    if (Cl.every && (i + 1) % Cl.every == 0) {
      batch_record<D, EA, NT>(B, Cl, sp, red, rec);
      ++rec;
    }
  }
}

// One task: lattice B, sweeps B.t .. B.t+n-1, all in LDS.  n == 0 with
// every > 0 records the current state once.
template <int D, bool EA, int NT>
__device__ void batch_task(const BatchLattice& Bg, const BatchCall& Cg, uint32_t* sp, uint32_t* bound,
                           int64_t* red) {
  const BatchLattice B = uniform_lattice(Bg);
  const BatchCall Cl = uniform_call(Cg);
  const uint32_t L = B.L;
  const uint32_t R = (D == 3) ? L * L : L;
  const uint32_t NW = R * (L / 8);
  const uint32_t tid = threadIdx.x;
  // pack the lattice into LDS
  for (uint32_t w = tid; w < NW; w += NT) {
    const uint2 b = reinterpret_cast<const uint2*>(B.spins)[w];
    sp[w] = pack_nibbles(b.x, b.y);
  }
  if (tid < 8) bound[tid] = Cl.bound[tid];
  __syncthreads();
  if (Cl.never4)
    batch_sweeps<D, EA, NT, true>(B, Cl, sp, bound, red);
  else
    batch_sweeps<D, EA, NT, false>(B, Cl, sp, bound, red);
  if (Cl.n == 0 && Cl.every) batch_record<D, EA, NT>(B, Cl, sp, red, 0);
  for (uint32_t w = tid; w < NW; w += NT) {
    uint2 b;
    unpack_nibbles(sp[w], b.x, b.y);
    reinterpret_cast<uint2*>(B.spins)[w] = b;
  }
}

template <int D, bool EA, int NT>
__global__ __launch_bounds__(NT) void k_batch(BatchLattice* lats, const BatchCall* calls,
                                              const uint32_t* order, uint32_t ntasks, uint32_t* next) {
  __shared__ uint32_t bound[8];   // static LDS first: lookups use a constant base
  __shared__ int64_t red[16];
  __shared__ uint32_t task;
  extern __shared__ __align__(16) uint32_t lds[];
  uint32_t* sp = lds;
  // Termination: the queue fetch, both barriers, the readfirstlane of the
  // task index and the exit test sit at this one loop level, and no branch
  // at this level depends on per-lane data: the fetch and the counter store
  // are made by all of wave 0 (a wave-uniform condition; lane 0 adds 1, the
  // other lanes 0, and every lane stores lane 0's result), the task body ends
  // with a barrier.  So every wave reads the same k and leaves on the same
  // iteration.  A lane-dependent branch here (thread 0 alone fetching) let
  // the compiler move the fetch into an outer loop and the barriers into a
  // nested one whose exit is per lane, so that lanes re-read a stale index
  // and the loop never ended.
  const uint32_t wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const uint32_t lane = threadIdx.x & 63u;
  for (;;) {
    if (wave == 0) {
      const uint32_t got = atomicAdd(next, lane == 0 ? 1u : 0u);
      task = __builtin_amdgcn_readlane(got, 0);
    }
    __syncthreads();
    const uint32_t k = __builtin_amdgcn_readfirstlane(task);  // uniform: scalar loads below
    __syncthreads();
    if (k >= ntasks) break;
    const uint32_t li = __builtin_amdgcn_readfirstlane(order[k]);
    const BatchCall Cl = calls[li];
    const BatchLattice B = lats[li];
    batch_task<D, EA, NT>(B, Cl, sp, bound, red);
    if (wave == 0) lats[li].t = __builtin_amdgcn_readfirstlane(B.t + Cl.n);
    __syncthreads();
  }
}

size_t batch_lds_bytes(uint32_t L, uint32_t d) {
  const uint64_t N = (d == 3) ? (uint64_t)L * L * L : (uint64_t)L * L;
  return N / 2;
}

template <int NT>
static hipError_t set_batch_attrs() {
  const void* ks[4] = {(const void*)k_batch<2, false, NT>, (const void*)k_batch<2, true, NT>,
                       (const void*)k_batch<3, false, NT>, (const void*)k_batch<3, true, NT>};
  for (const void* k : ks) {
    hipError_t e = hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)kBatchMaxLds);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

template <int NT>
static void go_batch(uint32_t d, bool ea, dim3 grid, size_t lds, hipStream_t stream, BatchLattice* lats,
                     const BatchCall* calls, const uint32_t* order, uint32_t ntasks, uint32_t* counter) {
  if (d == 2 && !ea) hipLaunchKernelGGL((k_batch<2, false, NT>), grid, dim3(NT), lds, stream, lats, calls, order, ntasks, counter);
  if (d == 2 && ea) hipLaunchKernelGGL((k_batch<2, true, NT>), grid, dim3(NT), lds, stream, lats, calls, order, ntasks, counter);
  if (d == 3 && !ea) hipLaunchKernelGGL((k_batch<3, false, NT>), grid, dim3(NT), lds, stream, lats, calls, order, ntasks, counter);
  if (d == 3 && ea) hipLaunchKernelGGL((k_batch<3, true, NT>), grid, dim3(NT), lds, stream, lats, calls, order, ntasks, counter);
}

hipError_t launch_batch(uint32_t d, bool ea, uint32_t nt, BatchLattice* lats, const BatchCall* calls,
                        const uint32_t* order, uint32_t ntasks, uint32_t* counter, size_t lds_bytes,
                        uint32_t grid, hipStream_t stream) {
  static bool attr = false;
  if (!attr) {
    hipError_t e = set_batch_attrs<256>();
    if (e == hipSuccess) e = set_batch_attrs<512>();
    if (e == hipSuccess) e = set_batch_attrs<576>();
    if (e == hipSuccess) e = set_batch_attrs<1024>();
    if (e != hipSuccess) return e;
    attr = true;
  }
  hipLaunchKernelGGL(k_zero_u32, dim3(1), dim3(64), 0, stream, counter, 1u);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  if (nt == 256) go_batch<256>(d, ea, dim3(grid), lds_bytes, stream, lats, calls, order, ntasks, counter);
  else if (nt == 512) go_batch<512>(d, ea, dim3(grid), lds_bytes, stream, lats, calls, order, ntasks, counter);
  else if (nt == 576) go_batch<576>(d, ea, dim3(grid), lds_bytes, stream, lats, calls, order, ntasks, counter);
  else if (nt == 1024) go_batch<1024>(d, ea, dim3(grid), lds_bytes, stream, lats, calls, order, ntasks, counter);
  else return hipErrorInvalidValue;
  return hipGetLastError();
}

__global__ void k_store_single(BatchSingle* blk, BatchLattice lat, BatchCall call) {
  if (threadIdx.x == 0) {
    blk->lat = lat;
    blk->call = call;
    blk->order = 0;
  }
}

hipError_t launch_batch_single(BatchSingle* blk, const BatchLattice& lat, const BatchCall& call, uint32_t nt,
                               hipStream_t stream) {
  hipLaunchKernelGGL(k_store_single, dim3(1), dim3(64), 0, stream, blk, lat, call);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  return launch_batch(lat.d, lat.Jn != nullptr, nt, &blk->lat, &blk->call, &blk->order, 1, &blk->counter,
                      batch_lds_bytes(lat.L, lat.d), 1, stream);
}

}  // namespace spin
