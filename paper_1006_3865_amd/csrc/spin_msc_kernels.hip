// spin_msc_kernels.hip -- multi-spin-coded +-J glass (Sec. 4, last paragraph:
// many disorder realisations at once, combined with multi-spin coding): 32
// systems share the lattice, bit b of every word belongs to system b.
//
// spins: one uint32 per site, bit set = spin -1.  couplings: one uint32 per
// direction and site ([dir][site]), bit set = J -1 for the bond (s, s+e_dir).
// A bond is unsatisfied in system b iff bit b of s_i ^ s_j ^ J is set.  An
// update of site s counts its unsatisfied bonds u (0..2d) in every bit at
// once with a bit-sliced adder (full adders: sum = xor3, carry = majority,
// one v_bitop3 each), then accepts system b iff r < T at k_b = 2d - 2u_b,
// i.e. iff u_b >= u*(r), where u*(r) = #{u < d : r >= T at k = 2d - 2u} is
// one scalar per site (T grows as u grows, and is 2^32 for u >= d).  r is
// the site's shared draw: word
// (s>>1)&3 of Philox counter (s>>3, t, p0, 4 + colour), the chain of the
// oracle's multi-spin-coded mode.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "spin_device.h"
#include "spin_internal.h"
#include "spin_msc.h"

namespace spin {

__device__ __forceinline__ uint32_t maj3(uint32_t a, uint32_t b, uint32_t c) {
  return __builtin_amdgcn_bitop3_b32(a, b, c, 0xE8);
}

// Hot start: bit b of word s is set iff system b's spin is -1, i.e. iff
// bit 31 of word s&3 of Philox(seed, (s>>2, 0, p0 + b, 2)) is clear.
__global__ void k_msc_init(uint32_t* __restrict__ S, uint64_t nquads, RoundKeys K, uint32_t p0) {
  for (uint64_t q = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; q < nquads; q += (uint64_t)gridDim.x * blockDim.x) {
    uint32_t w[4] = {0, 0, 0, 0};
    for (uint32_t b = 0; b < 32; ++b) {
      uint32_t r[4];
      philox((uint32_t)q, 0u, p0 + b, 2u, K, r);
#pragma unroll
      for (int j = 0; j < 4; ++j) w[j] |= ((r[j] >> 31) ^ 1u) << b;
    }
    reinterpret_cast<uint4*>(S)[q] = make_uint4(w[0], w[1], w[2], w[3]);
  }
}

// Device layout of the couplings: J[dir * N + jidx(dir, s)].  The x bonds
// (dir 0) are in site order; the y and z bonds (dir 1, 2) keep each row of L
// words split by x parity, the L/2 even-x words first, then the odd-x ones,
// so that the four same-colour sites of an 8-site group find their y and z
// bonds in 16 contiguous bytes.
__device__ __forceinline__ uint64_t msc_split(uint64_t s, uint32_t L) {
  const uint32_t x = (uint32_t)(s % L);
  return s - x + (x & 1u) * (L / 2) + (x >> 1);
}

// Couplings: bit b of the word of bond (dir, s) is set iff bit 31 of word
// s&3 of Philox(cseed, (s>>2, dir, r0 + b, 3)) is set (J = -1).
__global__ void k_msc_couplings(uint32_t* __restrict__ J, uint64_t nquads, uint32_t L, uint32_t d, RoundKeys K,
                                uint32_t r0) {
  const uint64_t N = nquads * 4;
  for (uint32_t dir = 0; dir < d; ++dir)
    for (uint64_t q = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; q < nquads;
         q += (uint64_t)gridDim.x * blockDim.x) {
      uint32_t w[4] = {0, 0, 0, 0};
      for (uint32_t b = 0; b < 32; ++b) {
        uint32_t r[4];
        philox((uint32_t)q, dir, r0 + b, 3u, K, r);
#pragma unroll
        for (int j = 0; j < 4; ++j) w[j] |= (r[j] >> 31) << b;
      }
      if (dir == 0) {
        reinterpret_cast<uint4*>(J)[q] = make_uint4(w[0], w[1], w[2], w[3]);
      } else {  // sites 4q .. 4q+3 start at an even x of one row (L % 8 == 0)
        const uint64_t e = (uint64_t)dir * N + msc_split(4 * q, L);
        reinterpret_cast<uint2*>(J + e)[0] = make_uint2(w[0], w[2]);
        reinterpret_cast<uint2*>(J + e + L / 2)[0] = make_uint2(w[1], w[3]);
      }
    }
}

__device__ __forceinline__ void load4(const uint32_t* p, uint32_t (&v)[4]) {
  const uint4 a = reinterpret_cast<const uint4*>(p)[0];
  v[0] = a.x; v[1] = a.y; v[2] = a.z; v[3] = a.w;
}

__device__ __forceinline__ void load8(const uint32_t* p, uint32_t (&v)[8]) {
  const uint4 a = reinterpret_cast<const uint4*>(p)[0];
  const uint4 b = reinterpret_cast<const uint4*>(p)[1];
  v[0] = a.x; v[1] = a.y; v[2] = a.z; v[3] = a.w;
  v[4] = b.x; v[5] = b.y; v[6] = b.z; v[7] = b.w;
}

// Mask of the systems whose unsatisfied count u (bit-sliced u2 u1 u0) is at least us.
__device__ __forceinline__ uint32_t at_least(uint32_t u0, uint32_t u1, uint32_t u2, uint32_t us) {
  uint32_t m = 0xFFFFFFFFu;                         // us == 0
  m = us >= 1 ? (u0 | u1 | u2) : m;
  m = us >= 2 ? (u1 | u2) : m;
  m = us >= 3 ? (u2 | (u1 & u0)) : m;
  return m;
}

// The four colour-P sites of an 8-site group (words c[]; neighbours: lw, rw
// the sites left and right of the group, ym/yp rows y-1/y+1 and zm/zp planes
// z-1/z+1 at the same x); jb[i]: the couplings of active site i = 0..3
// (site 2i + P) in the order -x, +x, -y, +y (, -z, +z); r: the shared draws.
template <int D, int P>
__device__ __forceinline__ void msc_update8(uint32_t (&c)[8], uint32_t lw, uint32_t rw, const uint32_t (&ym)[8],
                                            const uint32_t (&yp)[8], const uint32_t (&zm)[8], const uint32_t (&zp)[8],
                                            const uint32_t (&jb)[4][2 * D], const uint32_t (&r)[4],
                                            const MscArgs& a) {
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int j = 2 * i + P;
    const uint32_t left = j ? c[j - 1] : lw;
    const uint32_t right = j < 7 ? c[j + 1] : rw;
    const uint32_t s = c[j];
    // unsatisfied bits of the 2d bonds
    const uint32_t b0 = xor3(s, left, jb[i][0]), b1 = xor3(s, right, jb[i][1]);
    const uint32_t b2 = xor3(s, ym[j], jb[i][2]), b3 = xor3(s, yp[j], jb[i][3]);
    uint32_t u0, u1, u2;
    if (D == 3) {
      const uint32_t b4 = xor3(s, zm[j], jb[i][4]), b5 = xor3(s, zp[j], jb[i][5]);
      const uint32_t s1 = xor3(b0, b1, b2), c1 = maj3(b0, b1, b2);
      const uint32_t s2 = xor3(b3, b4, b5), c2 = maj3(b3, b4, b5);
      u0 = s1 ^ s2;
      const uint32_t t = s1 & s2;
      u1 = xor3(c1, c2, t);
      u2 = maj3(c1, c2, t);
    } else {
      const uint32_t s1 = xor3(b0, b1, b2), c1 = maj3(b0, b1, b2);
      u0 = s1 ^ b3;
      const uint32_t t = s1 & b3;
      u1 = c1 ^ t;
      u2 = c1 & t;
    }
    // u*(r): thresholds of u = 0 .. d-1 at or below r
    const uint64_t ri = r[i];
    uint32_t us = (ri >= a.thr[0] ? 1u : 0u) + (ri >= a.thr[1] ? 1u : 0u);
    if (D == 3) us += ri >= a.thr[2] ? 1u : 0u;
    c[j] = s ^ at_least(u0, u1, u2, us);
  }
}

// Couplings of the active sites of group g in colour c: J6 holds, per group
// and colour, 4 x 2d words (site i's bonds -x, +x, -y, +y(, -z, +z)).
template <int D>
__device__ __forceinline__ void load_bonds(const uint32_t* __restrict__ J6, uint64_t g, uint32_t c,
                                           uint32_t (&jb)[4][2 * D]) {
  const uint4* p = reinterpret_cast<const uint4*>(J6 + (g * 2 + c) * (8 * D));
  uint32_t w[8 * D];
#pragma unroll
  for (int q = 0; q < 2 * D; ++q) {
    const uint4 v = p[q];
    w[4 * q] = v.x;
    w[4 * q + 1] = v.y;
    w[4 * q + 2] = v.z;
    w[4 * q + 3] = v.w;
  }
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int k = 0; k < 2 * D; ++k) jb[i][k] = w[i * 2 * D + k];
}

// The couplings of the four active sites of a group in the order of
// msc_update8: x bonds from the group's x-bond words jx (jl: the word left of
// the group), y and z bonds from the parity-P halves jy/jym (rows y, y-1) and
// jz/jzm (planes z, z-1), word i for site 2i + P.
template <int D, int P>
__device__ __forceinline__ void bonds_split(const uint32_t (&jx)[8], uint32_t jl, const uint32_t (&jy)[4],
                                            const uint32_t (&jym)[4], const uint32_t (&jz)[4],
                                            const uint32_t (&jzm)[4], uint32_t (&jb)[4][2 * D]) {
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int j = 2 * i + P;
    jb[i][0] = j ? jx[j - 1] : jl;
    jb[i][1] = jx[j];
    jb[i][2] = jym[i];
    jb[i][3] = jy[i];
    if (D == 3) {
      jb[i][4] = jzm[i];
      jb[i][5] = jz[i];
    }
  }
}

// Build J6 from the [dir][site] couplings: thread = (group, colour).
template <int D>
__global__ void k_msc_bonds(const uint32_t* __restrict__ J, uint32_t* __restrict__ J6, uint32_t L, uint64_t N) {
  const uint32_t GPR = L / 8;
  const uint64_t row = L, plane = (uint64_t)L * L;
  for (uint64_t q = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; q < N / 4; q += (uint64_t)gridDim.x * blockDim.x) {
    const uint64_t g = q >> 1;
    const uint32_t c = (uint32_t)(q & 1);
    const uint64_t rowi = g / GPR;
    const uint32_t x0 = (uint32_t)(g - rowi * GPR) * 8u;
    const uint32_t y = (uint32_t)(rowi % L), z = (D == 3) ? (uint32_t)(rowi / L) : 0u;
    const uint32_t P = (c + y + z) & 1u;
    uint32_t* out = J6 + q * (8 * D);
    for (uint32_t i = 0; i < 4; ++i) {
      const uint32_t x = x0 + 2 * i + P;
      const uint64_t s = g * 8 + 2 * i + P;
      const uint64_t sxm = x ? s - 1 : s + L - 1;
      const uint64_t sym = y ? s - row : s + (L - 1) * row;
      out[i * 2 * D + 0] = J[sxm];
      out[i * 2 * D + 1] = J[s];
      out[i * 2 * D + 2] = J[N + msc_split(sym, L)];
      out[i * 2 * D + 3] = J[N + msc_split(s, L)];
      if (D == 3) {
        const uint64_t szm = z ? s - plane : s + (L - 1) * plane;
        out[i * 2 * D + 4] = J[2 * N + msc_split(szm, L)];
        out[i * 2 * D + 5] = J[2 * N + msc_split(s, L)];
      }
    }
  }
}

// One colour phase: thread = 8-site group g (sites 8g .. 8g+7 of one row);
// its four sites of colour c (offset P = (c + y + z) & 1 inside the group).
template <int D, int P>
__device__ __forceinline__ void msc_group(uint32_t* __restrict__ S, const uint32_t* __restrict__ J6,
                                          const MscArgs& a, uint64_t s0, uint32_t x0, uint32_t y, uint32_t z,
                                          const uint32_t (&r)[4]) {
  const uint32_t L = a.L;
  const uint64_t row = (uint64_t)L, plane = (uint64_t)L * L;
  uint32_t c[8], ym[8], yp[8], zm[8], zp[8];
  load8(S + s0, c);
  load8(S + (y ? s0 - row : s0 + (L - 1) * row), ym);
  load8(S + ((y + 1 < L) ? s0 + row : s0 - (L - 1) * row), yp);
  if (D == 3) {
    load8(S + (z ? s0 - plane : s0 + (L - 1) * plane), zm);
    load8(S + ((z + 1 < L) ? s0 + plane : s0 - (L - 1) * plane), zp);
  }
  uint32_t jb[4][2 * D];
  load_bonds<D>(J6, s0 >> 3, a.colour, jb);
  const uint64_t sl = x0 ? s0 - 1 : s0 + L - 1;     // site left of the group
  const uint64_t sr = (x0 + 8 < L) ? s0 + 8 : s0 + 8 - L;
  msc_update8<D, P>(c, S[sl], S[sr], ym, yp, zm, zp, jb, r, a);
  reinterpret_cast<uint4*>(S + s0)[0] = make_uint4(c[0], c[1], c[2], c[3]);
  reinterpret_cast<uint4*>(S + s0)[1] = make_uint4(c[4], c[5], c[6], c[7]);
}

template <int D>
__global__ __launch_bounds__(256) void k_msc_phase(uint32_t* __restrict__ S, const uint32_t* __restrict__ J6,
                                                   MscArgs a) {
  const uint32_t L = a.L, GPR = L / 8;
  const PhiloxUniform U = philox_uniform(a.t, a.p0, 4u + a.colour, a.keys);
  for (uint64_t g = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; g < a.N / 8;
       g += (uint64_t)gridDim.x * blockDim.x) {
    const uint64_t rowi = g / GPR;
    const uint32_t x0 = (uint32_t)(g - rowi * GPR) * 8u;
    const uint32_t y = (uint32_t)(rowi % L), z = (D == 3) ? (uint32_t)(rowi / L) : 0u;
    uint32_t r[4];
    philox_lane((uint32_t)g, U, a.keys, r);
    if (((a.colour + y + z) & 1u) == 0)
      msc_group<D, 0>(S, J6, a, g * 8, x0, y, z, r);
    else
      msc_group<D, 1>(S, J6, a, g * 8, x0, y, z, r);
  }
}

// ------------------------------------------------------------ streaming
// One whole sweep per launch, streamed over planes (z in 3D, rows in 2D)
// like the general streaming kernel: a workgroup owns planes [z0, z0+H), in
// 3D rows [y0, y0+TY), and sites [x0, x0+XW) of each row, and keeps a ring
// of 6 plane slices of site words in LDS.  A slice row holds the 8-site
// groups x0/8-2 .. x0/8+XW/8+1 (two neighbouring groups on each side,
// periodic); 3D slices hold rows y0-2 .. y0+TY+1.  A slice row keeps words
// 0-3 of its groups in its first half and words 4-7 in its second, so that
// neighbouring lanes touch neighbouring 16 bytes.  Step i, plane a =
// z0-1+i: fetch plane a+2 into registers; colour 0 on plane a over slice
// rows 1..TY+2 and groups 1..XW/8+2 (the owned part and a one-group /
// one-row ring that colour 1 needs), written back into the ring; colour 1
// on plane a-2 over the owned rows and groups, written to dst with both
// colours; store the fetched plane; barrier.  Couplings come from HBM.
constexpr int kMscFetch = 4;  // slice groups per thread
// A register vector: copies of uint4 structs are lowered to memcpy and left in scratch.
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ uint32_t msc_wrap2(uint32_t v, uint32_t L) {  // (v - 2) mod L, v < 2L + 2
  uint32_t w = v + L - 2u;
  if (w >= L) w -= L;
  if (w >= L) w -= L;
  return w;
}

struct MscGeom {
  uint32_t L, GPR;   // edge, groups per row
  uint32_t SG;       // groups per slice row (XW/8 + 4)
  uint32_t RW;       // words per slice row (8 * SG)
  uint32_t HW;       // offset of the second half of a slice row (4 * SG)
  uint32_t gx0;      // first owned group column (x0 / 8)
};

template <int D, int NT>
__device__ __forceinline__ void msc_fetch(const uint32_t* __restrict__ src, uint32_t z, uint32_t y0, const MscGeom& G,
                                          uint32_t tot, u32x4 (&v)[2 * kMscFetch]) {
#pragma unroll
  for (int q = 0; q < kMscFetch; ++q) {
    const uint32_t u = threadIdx.x + NT * q;
    if (u < tot) {
      const uint32_t r = u / G.SG, k = u - r * G.SG;
      const uint32_t y = (D == 3) ? msc_wrap2(y0 + r, G.L) : 0u;
      const uint32_t gx = msc_wrap2(G.gx0 + k, G.GPR);
      const uint64_t s0 = ((D == 3) ? ((uint64_t)z * G.L + y) * G.L : (uint64_t)z * G.L) + 8u * gx;
      v[2 * q] = reinterpret_cast<const u32x4*>(src + s0)[0];
      v[2 * q + 1] = reinterpret_cast<const u32x4*>(src + s0)[1];
    }
  }
}

template <int NT>
__device__ __forceinline__ void msc_put(uint32_t* slot, const MscGeom& G, uint32_t tot,
                                        const u32x4 (&v)[2 * kMscFetch]) {
#pragma unroll
  for (int q = 0; q < kMscFetch; ++q) {
    const uint32_t u = threadIdx.x + NT * q;
    if (u < tot) {
      const uint32_t r = u / G.SG, k = u - r * G.SG;
      uint32_t* p = slot + r * G.RW + 4 * k;
      *reinterpret_cast<u32x4*>(p) = v[2 * q];
      *reinterpret_cast<u32x4*>(p + G.HW) = v[2 * q + 1];
    }
  }
}

// The 8 words of a slice group: words 0-3 at p, words 4-7 at p + hw.
__device__ __forceinline__ void lds8(const uint32_t* p, uint32_t hw, uint32_t (&v)[8]) {
  const u32x4 a = *reinterpret_cast<const u32x4*>(p);
  const u32x4 b = *reinterpret_cast<const u32x4*>(p + hw);
  v[0] = a.x; v[1] = a.y; v[2] = a.z; v[3] = a.w;
  v[4] = b.x; v[5] = b.y; v[6] = b.z; v[7] = b.w;
}

// Colour-C groups of one step: slice rows RB0 + u / NG, slice groups KB0 + u % NG.
template <int D, int NT, uint32_t C>
__device__ __forceinline__ void msc_units(const uint32_t* pm, uint32_t* pc, const uint32_t* pp, uint32_t n,
                                          uint32_t NG, uint32_t y0, uint32_t z, const MscGeom& G, const MscArgs& a,
                                          const PhiloxUniform& U, const uint32_t* __restrict__ J,
                                          uint32_t* __restrict__ dst) {
  const uint32_t L = G.L, RW = G.RW, HW = G.HW;
  constexpr uint32_t RB0 = (D == 3) ? (C == 0 ? 1u : 2u) : 0u;
  constexpr uint32_t KB0 = C == 0 ? 1u : 2u;
  for (uint32_t u = threadIdx.x; u < n; u += NT) {
    const uint32_t rr = u / NG, kk = u - rr * NG;
    const uint32_t r = rr + RB0, k = kk + KB0;
    const uint32_t y = (D == 3) ? (C == 0 ? msc_wrap2(y0 + r, L) : y0 + r - 2u) : z;
    const uint32_t zz = (D == 3) ? z : 0u;
    const uint32_t gx = msc_wrap2(G.gx0 + k, G.GPR);
    const uint64_t rowbase = (D == 3) ? ((uint64_t)zz * L + y) * L : (uint64_t)y * L;
    const uint64_t s0 = rowbase + 8u * gx;
    const uint32_t o = r * RW + 4 * k;
    uint32_t c[8], ym[8], yp[8], zm[8], zp[8];
    lds8(pc + o, HW, c);
    if (D == 3) {
      lds8(pc + o - RW, HW, ym);
      lds8(pc + o + RW, HW, yp);
      lds8(pm + o, HW, zm);
      lds8(pp + o, HW, zp);
    } else {
      lds8(pm + o, HW, ym);
      lds8(pp + o, HW, yp);
    }
    const uint32_t lw = pc[o + HW - 1], rw = pc[o + 4];  // word 7 of group k-1, word 0 of group k+1
    // couplings from HBM: the group's 8 x-bond words and the one left of it; the y and z bonds of
    // the four active sites (x parity P) from the parity-P halves of rows y and y-1 (planes z, z-1)
    const uint64_t N = a.N, plane = (uint64_t)L * L;
    const uint64_t sl = gx ? s0 - 1 : s0 + L - 1;
    const uint32_t P = (C + y + zz) & 1u;
    const uint64_t hoff = (uint64_t)P * (L / 2) + 4u * gx;
    const uint64_t rym = y ? rowbase - L : rowbase + (uint64_t)(L - 1) * L;  // start of row y-1
    uint32_t jx[8], jy[4], jym[4], jz[4], jzm[4];
    load8(J + s0, jx);
    load4(J + N + rowbase + hoff, jy);
    load4(J + N + rym + hoff, jym);
    if (D == 3) {
      const uint64_t rzm = zz ? rowbase - plane : rowbase + (uint64_t)(L - 1) * plane;  // row y of plane z-1
      load4(J + 2 * N + rowbase + hoff, jz);
      load4(J + 2 * N + rzm + hoff, jzm);
    }
    const uint32_t jl = J[sl];
    uint32_t rnd[4];
    philox_lane((uint32_t)(s0 >> 3), U, a.keys, rnd);
    uint32_t jb[4][2 * D];
    if (P == 0) {
      bonds_split<D, 0>(jx, jl, jy, jym, jz, jzm, jb);
      msc_update8<D, 0>(c, lw, rw, ym, yp, zm, zp, jb, rnd, a);
    } else {
      bonds_split<D, 1>(jx, jl, jy, jym, jz, jzm, jb);
      msc_update8<D, 1>(c, lw, rw, ym, yp, zm, zp, jb, rnd, a);
    }
    const u32x4 lo = {c[0], c[1], c[2], c[3]}, hi = {c[4], c[5], c[6], c[7]};
    if (C == 0) {
      *reinterpret_cast<u32x4*>(pc + o) = lo;
      *reinterpret_cast<u32x4*>(pc + o + HW) = hi;
    } else {
      reinterpret_cast<u32x4*>(dst + s0)[0] = lo;
      reinterpret_cast<u32x4*>(dst + s0)[1] = hi;
    }
  }
}

template <int D, int NT>
__global__ __launch_bounds__(NT) void k_msc_stream(const uint32_t* __restrict__ src, uint32_t* __restrict__ dst,
                                                   const uint32_t* __restrict__ J, MscArgs a, uint32_t TYa,
                                                   uint32_t Ha, uint32_t XW) {
  extern __shared__ __align__(16) uint32_t ring[];
  MscGeom G;
  G.L = a.L;
  G.GPR = a.L / 8;
  G.SG = XW / 8 + 4;
  G.RW = 8 * G.SG;
  G.HW = 4 * G.SG;
  const uint32_t L = a.L;
  const uint32_t TY = (D == 3) ? TYa : 1u;
  const uint32_t RP = (D == 3) ? TY + 4 : 1u;
  const uint32_t SB = RP * G.RW;
  const uint32_t nseg = L / XW;
  const uint32_t gx = (D == 3) ? (L / TY) * nseg : nseg;
  uint32_t blk = blockIdx.x;
  if ((gridDim.x & 7u) == 0) blk = (blk & 7u) * (gridDim.x >> 3) + (blk >> 3);
  const uint32_t bx = blk % gx, by = blk / gx;
  const uint32_t seg = bx % nseg;
  G.gx0 = seg * (XW / 8);
  const uint32_t y0 = (D == 3) ? (bx / nseg) * TY : 0u;
  const uint32_t z0 = by * Ha;
  const uint32_t H = (L - z0 < Ha) ? L - z0 : Ha;
  const PhiloxUniform U0 = philox_uniform(a.t, a.p0, 4u, a.keys);
  const PhiloxUniform U1 = philox_uniform(a.t, a.p0, 5u, a.keys);
  const uint32_t tot = RP * G.SG;
  u32x4 nxt[2 * kMscFetch];
  for (uint32_t k = 0; k < 3; ++k) {
    msc_fetch<D, NT>(src, msc_wrap2(z0 + k, L), y0, G, tot, nxt);
    msc_put<NT>(ring + k * SB, G, tot, nxt);
  }
  __syncthreads();
  const uint32_t NG0 = XW / 8 + 2, NG1 = XW / 8;            // groups per row of colour 0 / colour 1 units
  const uint32_t U0n = ((D == 3) ? TY + 2 : 1u) * NG0;
  const uint32_t U1n = ((D == 3) ? TY : 1u) * NG1;
  uint32_t sa = 1;
  for (uint32_t i = 0; i < H + 3; ++i) {
    const uint32_t s_m3 = sa >= 3 ? sa - 3 : sa + 3;
    const uint32_t s_m2 = sa >= 2 ? sa - 2 : sa + 4;
    const uint32_t s_m1 = sa >= 1 ? sa - 1 : 5;
    const uint32_t s_p1 = sa <= 4 ? sa + 1 : 0;
    const uint32_t s_p2 = sa <= 3 ? sa + 2 : sa - 4;
    if (i <= H) msc_fetch<D, NT>(src, msc_wrap2(z0 + i + 3, L), y0, G, tot, nxt);
    if (i <= H + 1)
      msc_units<D, NT, 0>(ring + s_m1 * SB, ring + sa * SB, ring + s_p1 * SB, U0n, NG0, y0, msc_wrap2(z0 + i + 1, L),
                          G, a, U0, J, dst);
    if (i >= 3)
      msc_units<D, NT, 1>(ring + s_m3 * SB, ring + s_m2 * SB, ring + s_m1 * SB, U1n, NG1, y0, z0 + i - 3u, G, a, U1, J,
                          dst);
    if (i <= H) msc_put<NT>(ring + s_p2 * SB, G, tot, nxt);
    __syncthreads();
    sa = sa == 5 ? 0 : sa + 1;
  }
}

constexpr size_t kMscMaxLds = 160 * 1024;  // all of a CU's LDS

size_t msc_stream_lds(uint32_t L, uint32_t d, uint32_t TY, uint32_t XW) {
  (void)L;
  const size_t RP = d == 3 ? TY + 4 : 1;
  return 6 * RP * (XW + 32) * 4;
}

bool msc_stream_supported(uint32_t L, uint32_t d, uint32_t TY, uint32_t H, uint32_t NT, uint32_t XW) {
  if (L % 8 != 0 || L < 16 || H < 1 || H > L) return false;
  if (NT != 256 && NT != 512) return false;
  if (XW < 8 || XW % 8 != 0 || L % XW != 0) return false;
  if (d == 3 && (TY == 0 || L % TY != 0 || TY > 32)) return false;
  const uint32_t RP = d == 3 ? TY + 4 : 1;
  if (RP * (XW / 8 + 4) > (uint32_t)kMscFetch * NT) return false;
  return msc_stream_lds(L, d, TY, XW) <= kMscMaxLds;
}

template <int D, int NT>
static hipError_t go_msc_stream(const uint32_t* src, uint32_t* dst, const uint32_t* J, const MscArgs& a,
                                uint32_t TY, uint32_t H, uint32_t XW, hipStream_t stream) {
  static bool attr = false;
  if (!attr) {
    hipError_t e = hipFuncSetAttribute((const void*)k_msc_stream<D, NT>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                       (int)kMscMaxLds);
    if (e != hipSuccess) return e;
    attr = true;
  }
  const uint32_t nseg = a.L / XW;
  const dim3 grid((D == 3 ? (a.L / TY) * nseg : nseg) * ((a.L + H - 1) / H));
  hipLaunchKernelGGL((k_msc_stream<D, NT>), grid, dim3(NT), msc_stream_lds(a.L, D, TY, XW), stream, src, dst, J, a,
                     TY, H, XW);
  return hipGetLastError();
}

hipError_t launch_msc_stream(const uint32_t* src, uint32_t* dst, const uint32_t* J, const MscArgs& a, uint32_t d,
                             uint32_t TY, uint32_t H, uint32_t NT, uint32_t XW, hipStream_t stream) {
  if (!msc_stream_supported(a.L, d, TY, H, NT, XW)) return hipErrorInvalidValue;
  if (d == 3) return NT == 256 ? go_msc_stream<3, 256>(src, dst, J, a, TY, H, XW, stream)
                               : go_msc_stream<3, 512>(src, dst, J, a, TY, H, XW, stream);
  return NT == 256 ? go_msc_stream<2, 256>(src, dst, J, a, TY, H, XW, stream)
                   : go_msc_stream<2, 512>(src, dst, J, a, TY, H, XW, stream);
}

// ------------------------------------------------------------ register columns
// 3D, L = 512: one whole sweep per launch with each row's z column in
// registers, and every coupling word read from HBM once per sweep (the plane
// streaming kernel above reads the couplings of a site once per colour).
//
// A workgroup owns the TY rows [y0, y0+TY) of the planes [z0, z0+H) and has
// TY + 2 waves; wave w keeps slab row r = w + 1 (y = y0 - 2 + r) for the
// whole launch: rows 2..TY+1 are owned, 1 and TY+2 a ring whose colour 0 is
// recomputed here (colour 1 of the owned edge rows needs it), and 0 and TY+3
// a halo that the ring's colour 0 reads.  Lane l holds the group of sites
// x = 8l .. 8l+7 of its row (a 512-site row is one wavefront).
// Step i = 0..H+1 with a = z0-1+i, b = a-1.  Both colour units of a step
// have active sites of x parity P = (y + a) & 1 (colour 0 on plane a,
// colour 1 on plane b):
//   write plane a+1's spins as loaded (the parity-P words: colour-1 sites,
//     which the neighbouring rows' colour 0 reads in step i+1) and y bonds
//     (all words) into LDS slot N;
//   issue the loads of plane a+2's spins and y bonds and plane a+1's x and z
//     bonds (registers; used in step i+1);
//   colour 0 on plane a: z neighbours plane b after its colour 0 (its
//     colour-1 words still the old ones) and plane a+1 as loaded, from
//     registers; y neighbours and y bonds from slot A; x neighbours and the
//     x bond left of the group by a wavefront rotate; the new parity-P words
//     go into slot A (the other rows read the other half of it in this step);
//   colour 1 on plane b (owned rows, i >= 2): z neighbours plane b-1 and
//     plane a after colour 0 (registers), y neighbours and bonds from slot B
//     (plane b after colour 0, written in step i-1); the group goes to dst;
//   barrier.
// Register lifetimes: an x-bond word serves colour 0 of its plane in one
// step and colour 1 of the same plane in the next; a z-bond word (bond to the
// plane above) serves its plane's colour-0 unit and the next plane's
// colour-1 unit for one parity half, and the next plane's colour-0 and its
// own plane's colour-1 unit for the other, over three steps.  LDS rows keep
// the parity split of the y and z bonds in HBM (even-x words, then odd-x
// words), so the four active words of a group are 16 contiguous bytes.
typedef uint32_t v4u __attribute__((ext_vector_type(4)));

namespace col {

struct G8 {  // one group, natural site order: words 0-3 in lo, 4-7 in hi
  v4u lo, hi;
};
struct H8 {  // one group's y or z bonds, split by parity: h[0] even x, h[1] odd x
  v4u h[2];
};

template <uint32_t P>
__device__ __forceinline__ v4u half(const G8& g) {
  return v4u{g.lo[P], g.lo[2 + P], g.hi[P], g.hi[2 + P]};
}

__device__ __forceinline__ G8 ld_group(__amdgpu_buffer_rsrc_t r, uint32_t row, uint32_t lane) {
  G8 g;
  g.lo = __builtin_amdgcn_raw_buffer_load_b128(r, 32u * lane, row, 0);
  g.hi = __builtin_amdgcn_raw_buffer_load_b128(r, 32u * lane + 16u, row, 0);
  return g;
}

template <uint32_t L>
__device__ __forceinline__ H8 ld_split(__amdgpu_buffer_rsrc_t r, uint32_t row, uint32_t lane) {
  H8 g;
  g.h[0] = __builtin_amdgcn_raw_buffer_load_b128(r, 16u * lane, row, 0);
  g.h[1] = __builtin_amdgcn_raw_buffer_load_b128(r, 2u * L + 16u * lane, row, 0);  // the odd-x half
  return g;
}

__device__ __forceinline__ uint32_t ror1(uint32_t v) {  // lane l gets lane l-1's value (periodic)
  return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x13C, 0xF, 0xF, false);
}
__device__ __forceinline__ uint32_t rol1(uint32_t v) {  // lane l gets lane l+1's value (periodic)
  return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x134, 0xF, 0xF, false);
}

// One colour unit on the active sites j = 2i + P of group g: nb is the x
// neighbour outside the group (P = 0: word 7 of the group to the left; P = 1:
// word 0 of the group to the right), jx the group's x bonds and jl the x
// bond left of the group (P = 0 only); ym, yp, zm, zp the active sites'
// neighbours and jym, jy, jzm, jz their y and z bonds, word i for site 2i+P;
// r the shared draws.  Same bit-sliced count and acceptance as msc_update8.
template <uint32_t P>
__device__ __forceinline__ void unit(G8& g, uint32_t nb, const G8& jx, uint32_t jl, v4u ym, v4u yp, v4u zm, v4u zp,
                                     v4u jym, v4u jy, v4u jzm, v4u jz, const uint32_t (&r)[4],
                                     const uint64_t (&thr)[3]) {
  uint32_t w[8] = {g.lo.x, g.lo.y, g.lo.z, g.lo.w, g.hi.x, g.hi.y, g.hi.z, g.hi.w};
  const uint32_t x[8] = {jx.lo.x, jx.lo.y, jx.lo.z, jx.lo.w, jx.hi.x, jx.hi.y, jx.hi.z, jx.hi.w};
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int j = 2 * i + (int)P;
    const uint32_t s = w[j];
    const uint32_t left = j ? w[j - 1] : nb;
    const uint32_t right = j < 7 ? w[j + 1] : nb;
    const uint32_t b0 = xor3(s, left, j ? x[j - 1] : jl), b1 = xor3(s, right, x[j]);
    const uint32_t b2 = xor3(s, ym[i], jym[i]), b3 = xor3(s, yp[i], jy[i]);
    const uint32_t b4 = xor3(s, zm[i], jzm[i]), b5 = xor3(s, zp[i], jz[i]);
    const uint32_t s1 = xor3(b0, b1, b2), c1 = maj3(b0, b1, b2);
    const uint32_t s2 = xor3(b3, b4, b5), c2 = maj3(b3, b4, b5);
    const uint32_t u0 = s1 ^ s2, t = s1 & s2;
    const uint32_t u1 = xor3(c1, c2, t), u2 = maj3(c1, c2, t);
    const uint64_t ri = r[i];
    const uint32_t us = (ri >= thr[0] ? 1u : 0u) + (ri >= thr[1] ? 1u : 0u) + (ri >= thr[2] ? 1u : 0u);
    w[j] = s ^ at_least(u0, u1, u2, us);
  }
  g.lo = v4u{w[0], w[1], w[2], w[3]};
  g.hi = v4u{w[4], w[5], w[6], w[7]};
}

// Roles of the waves: row r, its parity, whether it is owned, and which halo
// row it loads (TOP: spins of row 0; JH: y bonds of row 0; BOT: spins of row TY+3).
enum { TOP = 0, JH = 1, BOT = 2, ODD = 3, EVEN = 4 };

template <int ROLE>
struct Role {
  static constexpr uint32_t RP = (ROLE == TOP || ROLE == ODD) ? 1u : 0u;
  static constexpr bool OWN = ROLE != TOP && ROLE != BOT;
};

struct Ctx {
  __amdgpu_buffer_rsrc_t src, dst, jx, jy, jz;
  uint32_t* ls;  // spin slices: 3 x (TY+4) rows
  uint32_t* lj;  // y-bond slices: 3 x (TY+3) rows
  const RoundKeys* keys;
  PhiloxUniform U0, U1;
  uint64_t thr[3];
  uint32_t z0, H, lane, r, y, yh;  // yh: the halo row this wave loads (TOP, JH: row 0; BOT: row TY+3)
};

struct Regs {
  G8 s2, s1, sa, sb;  // spins: plane a+2 (in flight), a+1 as loaded, a as loaded, b after colour 0
  v4u sbb;            // plane b-1 after colour 0, this step's active half
  H8 jy1;             // y bonds of plane a+1 (written to LDS at the start of the step), then of a+2
  G8 jxn, jxa, jxb;   // x bonds of planes a+1 (in flight), a, b
  H8 jzn, jza, jzb;   // z bonds of planes a+1 (in flight), a, b
  v4u jzbb;           // z bonds of plane b-1, this step's active half
  G8 hs;              // halo spins (TOP, BOT): plane a+1, then a+2
  H8 hj;              // halo y bonds (JH): plane a+1, then a+2
  uint32_t sA, sB, sN;  // LDS slots of planes a, b, a+1
};

template <uint32_t L>
__device__ __forceinline__ uint32_t row_off(uint32_t z, uint32_t y) { return (z * L + y) * L * 4u; }

template <uint32_t L, int TY, int ROLE, uint32_t Q, bool C1>
__device__ __forceinline__ void step(const Ctx& c, Regs& R, uint32_t i) {
  using RL = Role<ROLE>;
  constexpr uint32_t RW = L, HW = L / 2, GPR = L / 8;  // words per LDS row and parity half, groups per row
  constexpr uint32_t SS = (TY + 4) * RW, JS = (TY + 3) * RW;  // words per spin / y-bond slice
  constexpr uint32_t P = (RL::RP + Q + 1u) & 1u;
  const uint32_t lane = c.lane, r = c.r, y = c.y;
  const uint32_t a = (c.z0 + i + L - 1u) & (L - 1u);
  const uint32_t b = (a + L - 1u) & (L - 1u);
  const uint32_t ic = i <= c.H ? i : c.H;  // loads past the strip's needs reload a plane already read
  const uint32_t zs = (c.z0 + 1u + ic) & (L - 1u), zx = (c.z0 + ic) & (L - 1u);
  // plane a+1 into slot N (free since the last barrier: it held plane b-1)
  {
    uint32_t* sN = c.ls + R.sN * SS;
    uint32_t* jN = c.lj + R.sN * JS;
    *reinterpret_cast<v4u*>(sN + r * RW + P * HW + 4u * lane) = half<P>(R.s1);
    *reinterpret_cast<v4u*>(jN + r * RW + 4u * lane) = R.jy1.h[0];
    *reinterpret_cast<v4u*>(jN + r * RW + HW + 4u * lane) = R.jy1.h[1];
    if (ROLE == TOP) {
      constexpr uint32_t PH = (0u + Q + 1u) & 1u;
      *reinterpret_cast<v4u*>(sN + PH * HW + 4u * lane) = half<PH>(R.hs);
    }
    if (ROLE == BOT) {
      constexpr uint32_t PH = ((uint32_t)TY + 3u + Q + 1u) & 1u;
      *reinterpret_cast<v4u*>(sN + (TY + 3) * RW + PH * HW + 4u * lane) = half<PH>(R.hs);
    }
    if (ROLE == JH) {
      *reinterpret_cast<v4u*>(jN + 4u * lane) = R.hj.h[0];
      *reinterpret_cast<v4u*>(jN + HW + 4u * lane) = R.hj.h[1];
    }
  }
  // loads for the next step
  R.s2 = ld_group(c.src, row_off<L>(zs, y), lane);
  R.jy1 = ld_split<L>(c.jy, row_off<L>(zs, y), lane);
  R.jxn = ld_group(c.jx, row_off<L>(zx, y), lane);
  R.jzn = ld_split<L>(c.jz, row_off<L>(zx, y), lane);
  if (ROLE == TOP || ROLE == BOT) R.hs = ld_group(c.src, row_off<L>(zs, c.yh), lane);
  if (ROLE == JH) R.hj = ld_split<L>(c.jy, row_off<L>(zs, c.yh), lane);
  // colour 0 on plane a
  const uint32_t* sA = c.ls + R.sA * SS;
  const uint32_t* jA = c.lj + R.sA * JS;
  const uint32_t o = P * HW + 4u * lane;
  uint32_t rnd[4];
  philox_lane((a * L + y) * GPR + lane, c.U0, *c.keys, rnd);
  G8 na = R.sa;
  {
    const v4u ym = *reinterpret_cast<const v4u*>(sA + (r - 1) * RW + o);
    const v4u yp = *reinterpret_cast<const v4u*>(sA + (r + 1) * RW + o);
    const v4u jy = *reinterpret_cast<const v4u*>(jA + r * RW + o);
    const v4u jym = *reinterpret_cast<const v4u*>(jA + (r - 1) * RW + o);
    const uint32_t nb = P == 0 ? ror1(R.sa.hi.w) : rol1(R.sa.lo.x);
    const uint32_t jl = P == 0 ? ror1(R.jxa.hi.w) : 0u;
    unit<P>(na, nb, R.jxa, jl, ym, yp, half<P>(R.sb), half<P>(R.s1), jym, jy, R.jzb.h[P], R.jza.h[P], rnd, c.thr);
    *reinterpret_cast<v4u*>(c.ls + R.sA * SS + r * RW + o) = half<P>(na);
  }
  // colour 1 on plane b
  if (C1 && RL::OWN) {
    const uint32_t* sB = c.ls + R.sB * SS;
    const uint32_t* jB = c.lj + R.sB * JS;
    philox_lane((b * L + y) * GPR + lane, c.U1, *c.keys, rnd);
    const v4u ym = *reinterpret_cast<const v4u*>(sB + (r - 1) * RW + o);
    const v4u yp = *reinterpret_cast<const v4u*>(sB + (r + 1) * RW + o);
    const v4u jy = *reinterpret_cast<const v4u*>(jB + r * RW + o);
    const v4u jym = *reinterpret_cast<const v4u*>(jB + (r - 1) * RW + o);
    const uint32_t nb = P == 0 ? ror1(R.sb.hi.w) : rol1(R.sb.lo.x);
    const uint32_t jl = P == 0 ? ror1(R.jxb.hi.w) : 0u;
    G8 nbk = R.sb;
    unit<P>(nbk, nb, R.jxb, jl, ym, yp, R.sbb, half<P>(na), jym, jy, R.jzbb, R.jzb.h[P], rnd, c.thr);
    __builtin_amdgcn_raw_buffer_store_b128(nbk.lo, c.dst, 32u * lane, row_off<L>(b, y), 0);
    __builtin_amdgcn_raw_buffer_store_b128(nbk.hi, c.dst, 32u * lane + 16u, row_off<L>(b, y), 0);
  }
  // the next step's registers (its active half is 1 - P)
  R.sbb = half<P ^ 1u>(R.sb);
  R.sb = na;
  R.sa = R.s1;
  R.s1 = R.s2;
  R.jxb = R.jxa;
  R.jxa = R.jxn;
  R.jzbb = R.jzb.h[P ^ 1u];
  R.jzb = R.jza;
  R.jza = R.jzn;
  const uint32_t t = R.sB;
  R.sB = R.sA;
  R.sA = R.sN;
  R.sN = t;
  __syncthreads();
}

template <uint32_t L, int TY, int ROLE>
__device__ __forceinline__ void run(const Ctx& c) {
  using RL = Role<ROLE>;
  constexpr uint32_t RW = L, HW = L / 2;
  constexpr uint32_t SS = (TY + 4) * RW, JS = (TY + 3) * RW;
  const uint32_t lane = c.lane, r = c.r, y = c.y;
  const uint32_t zm2 = (c.z0 + L - 2u) & (L - 1u), zm1 = (c.z0 + L - 1u) & (L - 1u);
  Regs R;
  // prologue: plane z0-1 into slot 0 (spins half P(r, step -1) = r & 1, all y bonds); registers for step 0
  R.sb = ld_group(c.src, row_off<L>(zm2, y), lane);
  R.sa = ld_group(c.src, row_off<L>(zm1, y), lane);
  R.s1 = ld_group(c.src, row_off<L>(c.z0, y), lane);
  R.jxa = ld_group(c.jx, row_off<L>(zm1, y), lane);
  R.jza = ld_split<L>(c.jz, row_off<L>(zm1, y), lane);
  R.jzb = ld_split<L>(c.jz, row_off<L>(zm2, y), lane);
  const H8 jy0 = ld_split<L>(c.jy, row_off<L>(zm1, y), lane);
  R.jy1 = ld_split<L>(c.jy, row_off<L>(c.z0, y), lane);
  R.jxb = R.jxa;
  R.sbb = v4u{0u, 0u, 0u, 0u};
  R.jzbb = v4u{0u, 0u, 0u, 0u};
  R.hs.lo = R.hs.hi = v4u{0u, 0u, 0u, 0u};
  R.hj.h[0] = R.hj.h[1] = v4u{0u, 0u, 0u, 0u};
  if (RL::RP)
    *reinterpret_cast<v4u*>(c.ls + r * RW + HW + 4u * lane) = half<1>(R.sa);
  else
    *reinterpret_cast<v4u*>(c.ls + r * RW + 4u * lane) = half<0>(R.sa);
  *reinterpret_cast<v4u*>(c.lj + r * RW + 4u * lane) = jy0.h[0];
  *reinterpret_cast<v4u*>(c.lj + r * RW + HW + 4u * lane) = jy0.h[1];
  if (ROLE == TOP) {  // row 0: half 0
    const G8 h = ld_group(c.src, row_off<L>(zm1, c.yh), lane);
    *reinterpret_cast<v4u*>(c.ls + 4u * lane) = half<0>(h);
    R.hs = ld_group(c.src, row_off<L>(c.z0, c.yh), lane);
  }
  if (ROLE == BOT) {  // row TY+3: half (TY+3) & 1 = 1
    const G8 h = ld_group(c.src, row_off<L>(zm1, c.yh), lane);
    *reinterpret_cast<v4u*>(c.ls + (TY + 3) * RW + HW + 4u * lane) = half<1>(h);
    R.hs = ld_group(c.src, row_off<L>(c.z0, c.yh), lane);
  }
  if (ROLE == JH) {
    const H8 h = ld_split<L>(c.jy, row_off<L>(zm1, c.yh), lane);
    *reinterpret_cast<v4u*>(c.lj + 4u * lane) = h.h[0];
    *reinterpret_cast<v4u*>(c.lj + HW + 4u * lane) = h.h[1];
    R.hj = ld_split<L>(c.jy, row_off<L>(c.z0, c.yh), lane);
  }
  (void)SS;
  (void)JS;
  R.sA = 0;
  R.sN = 1;
  R.sB = 2;
  __syncthreads();
  step<L, TY, ROLE, 0, false>(c, R, 0u);
  step<L, TY, ROLE, 1, false>(c, R, 1u);
  for (uint32_t i0 = 2; i0 < c.H + 2u; i0 += 2) {
    step<L, TY, ROLE, 0, true>(c, R, i0);
    step<L, TY, ROLE, 1, true>(c, R, i0 + 1u);
  }
}

}  // namespace col

template <uint32_t L, int TY>
__global__ __launch_bounds__(64 * (TY + 2)) void k_msc_col(const uint32_t* __restrict__ src,
                                                           uint32_t* __restrict__ dst,
                                                           const uint32_t* __restrict__ J, MscArgs a,
                                                           uint32_t H) {
  using namespace col;
  extern __shared__ __align__(16) uint32_t lds[];
  constexpr uint32_t Nw = L * L * L;
  constexpr uint32_t RW = L, GPR = L / 8;
  Ctx c;
  c.src = __builtin_amdgcn_make_buffer_rsrc((void*)src, 0, (int)(Nw * 4u), 0x00020000);
  c.dst = __builtin_amdgcn_make_buffer_rsrc((void*)dst, 0, (int)(Nw * 4u), 0x00020000);
  c.jx = __builtin_amdgcn_make_buffer_rsrc((void*)J, 0, (int)(Nw * 4u), 0x00020000);
  c.jy = __builtin_amdgcn_make_buffer_rsrc((void*)(J + Nw), 0, (int)(Nw * 4u), 0x00020000);
  c.jz = __builtin_amdgcn_make_buffer_rsrc((void*)(J + 2u * (size_t)Nw), 0, (int)(Nw * 4u), 0x00020000);
  c.ls = lds;
  c.lj = lds + 3u * (TY + 4) * RW;
  c.keys = &a.keys;
  c.U0 = philox_uniform(a.t, a.p0, 4u, a.keys);
  c.U1 = philox_uniform(a.t, a.p0, 5u, a.keys);
  c.thr[0] = a.thr[0];
  c.thr[1] = a.thr[1];
  c.thr[2] = a.thr[2];
  // workgroups are dealt to the 8 XCDs round-robin; give each XCD a contiguous run of tiles (the slabs of
  // one strip side by side), so that the halo rows of neighbouring slabs are read through the same L2
  const uint32_t nslab = L / TY, nblk = gridDim.x, bk = blockIdx.x;
  const uint32_t tile = (nblk % 8u == 0u) ? (bk % 8u) * (nblk / 8u) + bk / 8u : bk;
  const uint32_t y0 = (tile % nslab) * TY;
  c.z0 = (tile / nslab) * H;
  c.H = H;
  // a row has GPR <= 64 groups: with GPR < 64 the wavefront holds 64 / GPR copies of the row, lane l
  // working on group l mod GPR; the copies load, compute and store the same values, and the
  // wavefront rotates give every lane its periodic neighbour within the row
  c.lane = threadIdx.x & (GPR - 1u);
  const uint32_t wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  c.r = wave + 1u;
  c.y = (y0 + L - 2u + c.r) & (L - 1u);
  c.yh = (wave == (uint32_t)TY + 1u) ? (y0 + TY + 1u) & (L - 1u) : (y0 + L - 2u) & (L - 1u);
  if (wave == 0)
    run<L, TY, TOP>(c);
  else if (wave == 1)
    run<L, TY, JH>(c);
  else if (wave == (uint32_t)TY + 1u)
    run<L, TY, BOT>(c);
  else if (c.r & 1u)
    run<L, TY, ODD>(c);
  else
    run<L, TY, EVEN>(c);
}

size_t msc_col_lds(uint32_t TY, uint32_t L) { return (size_t)(3 * (TY + 4) + 3 * (TY + 3)) * L * 4; }

bool msc_col_supported(uint32_t L, uint32_t d, uint32_t TY, uint32_t H) {
  return d == 3 && (L == 128 || L == 256 || L == 512) && (TY == 4 || TY == 8) && H >= 2 && H % 2 == 0 &&
         L % H == 0;
}

template <uint32_t L, int TY>
static hipError_t go_msc_col(const uint32_t* src, uint32_t* dst, const uint32_t* J, const MscArgs& a, uint32_t H,
                             hipStream_t stream) {
  static bool attr = false;
  if (!attr) {
    hipError_t e = hipFuncSetAttribute((const void*)k_msc_col<L, TY>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                       (int)msc_col_lds(TY, L));
    if (e != hipSuccess) return e;
    attr = true;
  }
  const dim3 grid((L / TY) * (L / H));
  hipLaunchKernelGGL((k_msc_col<L, TY>), grid, dim3(64 * (TY + 2)), msc_col_lds(TY, L), stream, src, dst, J, a, H);
  return hipGetLastError();
}

hipError_t launch_msc_col(const uint32_t* src, uint32_t* dst, const uint32_t* J, const MscArgs& a, uint32_t d,
                          uint32_t TY, uint32_t H, hipStream_t stream) {
  if (!msc_col_supported(a.L, d, TY, H)) return hipErrorInvalidValue;
  if (a.L == 512) return TY == 8 ? go_msc_col<512, 8>(src, dst, J, a, H, stream) : go_msc_col<512, 4>(src, dst, J, a, H, stream);
  if (a.L == 256) return TY == 8 ? go_msc_col<256, 8>(src, dst, J, a, H, stream) : go_msc_col<256, 4>(src, dst, J, a, H, stream);
  return TY == 8 ? go_msc_col<128, 8>(src, dst, J, a, H, stream) : go_msc_col<128, 4>(src, dst, J, a, H, stream);
}

// E and M of the 32 systems: per workgroup, counts of unsatisfied bonds and
// of negative spins for every bit into part[wg*64 + bit] (unsat) and
// part[wg*64 + 32 + bit] (negative); k_msc_finalize sums the workgroups.
template <int D>
__global__ __launch_bounds__(256) void k_msc_count(const uint32_t* __restrict__ S, const uint32_t* __restrict__ J,
                                                   uint32_t L, uint64_t N, int64_t* __restrict__ part) {
  __shared__ int64_t red[64];
  if (threadIdx.x < 64) red[threadIdx.x] = 0;
  __syncthreads();
  uint32_t cu[32], cn[32];
#pragma unroll
  for (int b = 0; b < 32; ++b) cu[b] = cn[b] = 0;
  const uint64_t row = L, plane = (uint64_t)L * L;
  for (uint64_t s = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; s < N; s += (uint64_t)gridDim.x * blockDim.x) {
    const uint32_t x = (uint32_t)(s % L), y = (uint32_t)((s / L) % L), z = (D == 3) ? (uint32_t)(s / plane) : 0u;
    const uint32_t v = S[s];
    const uint32_t bx = v ^ S[x + 1 < L ? s + 1 : s + 1 - L] ^ J[s];
    const uint64_t sj = msc_split(s, L);
    const uint32_t by = v ^ S[y + 1 < L ? s + row : s - (L - 1) * row] ^ J[N + sj];
    uint32_t bz = 0;
    if (D == 3) bz = v ^ S[z + 1 < L ? s + plane : s - (L - 1) * plane] ^ J[2 * N + sj];
#pragma unroll
    for (int b = 0; b < 32; ++b) {
      cu[b] += ((bx >> b) & 1u) + ((by >> b) & 1u) + ((bz >> b) & 1u);
      cn[b] += (v >> b) & 1u;
    }
  }
#pragma unroll
  for (int b = 0; b < 32; ++b) {
    atomicAdd((unsigned long long*)&red[b], (unsigned long long)cu[b]);
    atomicAdd((unsigned long long*)&red[32 + b], (unsigned long long)cn[b]);
  }
  __syncthreads();
  if (threadIdx.x < 64) part[(uint64_t)blockIdx.x * 64 + threadIdx.x] = red[threadIdx.x];
}

__global__ void k_msc_finalize(const int64_t* __restrict__ part, uint32_t nparts, int64_t nb, int64_t N,
                               int64_t* __restrict__ E, int64_t* __restrict__ M) {
  const uint32_t b = threadIdx.x;
  if (b >= 32) return;
  int64_t u = 0, n = 0;
  for (uint32_t w = 0; w < nparts; ++w) {
    u += part[(uint64_t)w * 64 + b];
    n += part[(uint64_t)w * 64 + 32 + b];
  }
  E[b] = -nb + 2 * u;
  M[b] = N - 2 * n;
}

static unsigned blocks_for(uint64_t work, unsigned cap) {
  uint64_t b = (work + 255) / 256;
  return (unsigned)(b < cap ? (b ? b : 1) : cap);
}

hipError_t launch_msc_init(uint32_t* S, uint64_t N, uint64_t seed, uint32_t p0, hipStream_t stream) {
  hipLaunchKernelGGL(k_msc_init, dim3(blocks_for(N / 4, 8192)), dim3(256), 0, stream, S, N / 4, make_round_keys(seed),
                     p0);
  return hipGetLastError();
}

hipError_t launch_msc_couplings(uint32_t* J, uint64_t N, uint32_t L, uint32_t d, uint64_t cseed, uint32_t r0,
                                hipStream_t stream) {
  hipLaunchKernelGGL(k_msc_couplings, dim3(blocks_for(N / 4, 8192)), dim3(256), 0, stream, J, N / 4, L, d,
                     make_round_keys(cseed), r0);
  return hipGetLastError();
}

hipError_t launch_msc_bonds(const uint32_t* J, uint32_t* J6, uint32_t L, uint32_t d, uint64_t N, hipStream_t stream) {
  if (d == 3)
    hipLaunchKernelGGL(k_msc_bonds<3>, dim3(blocks_for(N / 4, 8192)), dim3(256), 0, stream, J, J6, L, N);
  else
    hipLaunchKernelGGL(k_msc_bonds<2>, dim3(blocks_for(N / 4, 8192)), dim3(256), 0, stream, J, J6, L, N);
  return hipGetLastError();
}

hipError_t launch_msc_phase(uint32_t* S, const uint32_t* J6, const MscArgs& a, uint32_t d, hipStream_t stream) {
  const unsigned blocks = blocks_for(a.N / 8, 1u << 20);
  if (d == 3)
    hipLaunchKernelGGL(k_msc_phase<3>, dim3(blocks), dim3(256), 0, stream, S, J6, a);
  else
    hipLaunchKernelGGL(k_msc_phase<2>, dim3(blocks), dim3(256), 0, stream, S, J6, a);
  return hipGetLastError();
}

uint32_t msc_count_parts(uint64_t N) { return blocks_for(N, 2048); }

hipError_t launch_msc_measure(const uint32_t* S, const uint32_t* J, uint32_t L, uint32_t d, uint64_t N, int64_t* part,
                              int64_t* E, int64_t* M, hipStream_t stream) {
  const unsigned blocks = msc_count_parts(N);
  if (d == 3)
    hipLaunchKernelGGL(k_msc_count<3>, dim3(blocks), dim3(256), 0, stream, S, J, L, N, part);
  else
    hipLaunchKernelGGL(k_msc_count<2>, dim3(blocks), dim3(256), 0, stream, S, J, L, N, part);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_msc_finalize, dim3(1), dim3(64), 0, stream, part, blocks, (int64_t)d * (int64_t)N, (int64_t)N,
                     E, M);
  return hipGetLastError();
}

}  // namespace spin
