// spin_kernels.hip -- gfx950 kernels of the checkerboard Metropolis path.
//
// Families (all produce the same bits; the chain is stated in include/spin.h):
//   generic   one colour phase, per site, global memory, any even L;
//   resident  whole lattice in one workgroup's LDS, many sweeps per launch
//             (small lattices: one launch per call);
//   tiled     one colour phase, an LDS tile plus a one-site halo, updated in
//             place, 8-site groups processed four sites per register (2D/3D
//             Ising, L % 8 == 0);
//   fused     2D Ising, a whole sweep per launch: tile plus a two-site halo,
//             colour 0 on the tile and its one-site ring, barrier, colour 1
//             on the tile, written to the other buffer of a ping-pong pair.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "spin_device.h"
#include "spin_internal.h"

namespace spin {

// ============================================================ hot start etc.

__global__ void k_init_spins(int8_t* __restrict__ spins, uint64_t nquads, RoundKeys K,
                             uint32_t replica) {
  for (uint64_t q = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; q < nquads;
       q += (uint64_t)gridDim.x * blockDim.x) {
    uint32_t r[4];
    philox((uint32_t)q, 0u, replica, 2u, K, r);
    uint32_t v = 0;
#pragma unroll
    for (int j = 0; j < 4; ++j) v |= ((r[j] >> 31) ? 0x01u : 0xFFu) << (8 * j);
    reinterpret_cast<uint32_t*>(spins)[q] = v;
  }
}

__global__ void k_couplings(int8_t* __restrict__ J, uint64_t nquads, uint32_t d, RoundKeys K,
                            uint32_t realisation) {
  for (uint32_t dir = 0; dir < d; ++dir)
    for (uint64_t q = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; q < nquads;
         q += (uint64_t)gridDim.x * blockDim.x) {
      uint32_t r[4];
      philox((uint32_t)q, dir, realisation, 3u, K, r);
      uint32_t v = 0;
#pragma unroll
      for (int j = 0; j < 4; ++j) v |= ((r[j] >> 31) ? 0xFFu : 0x01u) << (8 * j);
      reinterpret_cast<uint32_t*>(J)[dir * nquads + q] = v;
    }
}

__global__ void k_zero(int64_t* p, uint64_t n) {
  for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < n;
       i += (uint64_t)gridDim.x * blockDim.x)
    p[i] = 0;
}

static unsigned grid_for(uint64_t work, int threads, unsigned cap = 65536) {
  uint64_t g = (work + threads - 1) / threads;
  if (g < 1) g = 1;
  if (g > cap) g = cap;
  return (unsigned)g;
}

hipError_t launch_init_spins(const Lat& lat, hipStream_t stream) {
  const uint64_t nq = lat.N / 4;
  hipLaunchKernelGGL(k_init_spins, dim3(grid_for(nq, 256)), dim3(256), 0, stream, lat.spins, nq,
                     lat.keys, lat.replica);
  return hipGetLastError();
}

hipError_t launch_couplings(int8_t* J, uint32_t L, uint32_t d, uint64_t N, uint64_t cseed,
                            uint32_t realisation, hipStream_t stream) {
  (void)L;
  const uint64_t nq = N / 4;
  hipLaunchKernelGGL(k_couplings, dim3(grid_for(nq, 256)), dim3(256), 0, stream, J, nq, d,
                     make_round_keys(cseed), realisation);
  return hipGetLastError();
}

hipError_t launch_zero(int64_t* p, uint64_t n, hipStream_t stream) {
  hipLaunchKernelGGL(k_zero, dim3(grid_for(n, 256, 1024)), dim3(256), 0, stream, p, n);
  return hipGetLastError();
}

// ================================================================ geometry

// (v - back) mod L for 0 <= v < L + 2L and back <= L: the coordinate `back`
// sites before v, wrapped periodically.
__device__ __forceinline__ uint32_t wrap_row(uint32_t v, uint32_t back, uint32_t L) {
  uint32_t w = v + L - back;  // in [0, 3L)
  if (w >= L) w -= L;
  if (w >= L) w -= L;
  return w;
}

// Coordinates and wrapped neighbours of site s (generic paths).
struct Site {
  uint32_t x, y, z;
};

__device__ __forceinline__ Site site_coords(uint64_t s, uint32_t L, uint32_t d) {
  Site c;
  c.x = (uint32_t)(s % L);
  const uint64_t q = s / L;
  c.y = (uint32_t)(q % L);
  c.z = (d == 3) ? (uint32_t)(q / L) : 0u;
  return c;
}

// Neighbour of s one step along +dir / -dir; coordinate cd along dir,
// stride st = L^dir.
__device__ __forceinline__ uint64_t nb_plus(uint64_t s, uint32_t cd, uint32_t L, uint64_t st) {
  return (cd + 1 == L) ? s - (uint64_t)(L - 1) * st : s + st;
}
__device__ __forceinline__ uint64_t nb_minus(uint64_t s, uint32_t cd, uint32_t L, uint64_t st) {
  return (cd == 0) ? s + (uint64_t)(L - 1) * st : s - st;
}

// k = s_i * h_i for site s in spin array sp (LDS or global).
__device__ __forceinline__ int local_k(const int8_t* sp, const int8_t* __restrict__ J, uint64_t s,
                                       uint32_t L, uint32_t d, uint64_t N) {
  const Site c = site_coords(s, L, d);
  const uint32_t cd[3] = {c.x, c.y, c.z};
  int h = 0;
  uint64_t st = 1;
  for (uint32_t dir = 0; dir < d; ++dir) {
    const uint64_t up = nb_plus(s, cd[dir], L, st);
    const uint64_t dn = nb_minus(s, cd[dir], L, st);
    const int jf = J ? (int)J[dir * N + s] : 1;
    const int jb = J ? (int)J[dir * N + dn] : 1;
    h += jf * (int)sp[up] + jb * (int)sp[dn];
    st *= L;
  }
  return (int)sp[s] * h;
}

// One 8-site group g in colour `colour` of sweep t: every active site of the
// group is decided with its own Philox word and flipped in place.
__device__ __forceinline__ void generic_group(int8_t* sp, const int8_t* __restrict__ J,
                                              uint32_t L, uint32_t d, uint64_t N, uint64_t g,
                                              uint32_t t, uint32_t colour, uint32_t replica,
                                              const RoundKeys& K, const uint64_t* T) {
  uint32_t r[4];
  philox((uint32_t)g, t, replica, colour, K, r);
  const int z = 2 * (int)d;
  for (int j = 0; j < 8; ++j) {
    const uint64_t s = g * 8 + j;
    if (s >= N) break;
    const Site c = site_coords(s, L, d);
    if (((c.x + c.y + c.z) & 1u) != colour) continue;
    const int k = local_k(sp, J, s, L, d, N);
    if ((uint64_t)r[(s >> 1) & 3] < T[(k + z) / 2]) sp[s] = (int8_t)(-sp[s]);
  }
}

// ============================================================ measurement

// E and M of a lattice: per site (generic) when L % 4 != 0, per 4-site dword
// otherwise; each workgroup adds its partial sums into *E, *M.
template <int NT>
__global__ __launch_bounds__(NT) void k_measure_sites(const int8_t* __restrict__ sp,
                                                      const int8_t* __restrict__ J, uint32_t L,
                                                      uint32_t d, uint64_t N, Record rec) {
  __shared__ int64_t red[NT / 64];
  int64_t unsat = 0, neg = 0;
  for (uint64_t s = blockIdx.x * (uint64_t)NT + threadIdx.x; s < N; s += (uint64_t)gridDim.x * NT) {
    const Site c = site_coords(s, L, d);
    const uint32_t cd[3] = {c.x, c.y, c.z};
    uint64_t st = 1;
    const int si = sp[s];
    neg += (si < 0);
    for (uint32_t dir = 0; dir < d; ++dir) {
      const uint64_t up = nb_plus(s, cd[dir], L, st);
      unsat += ((J ? J[dir * N + s] : 1) * si * sp[up] < 0);
      st *= L;
    }
  }
  record_block<NT>(unsat, neg, rec, red);
}

// Row-structured version (L % 16 == 0): each workgroup takes RPB lattice rows
// (a row = L sites along x at fixed y, z); a thread takes 16 sites of a row,
// counts negative spins and unsatisfied +x/+y/+z bonds from sign bits, with
// 32-bit index arithmetic (rows < 2^32, bytes per row < 2^17).
template <int NT>
__global__ __launch_bounds__(NT) void k_measure_rows(const int8_t* __restrict__ sp,
                                                     const int8_t* __restrict__ J, uint32_t L,
                                                     uint32_t d, uint64_t N, uint32_t nrows,
                                                     uint32_t rpb, Record rec) {
  __shared__ int64_t red[NT / 64];
  const uint32_t msb = 0x80808080u;
  const uint32_t cpr = L / 16;
  int64_t unsat = 0, neg = 0;
  const uint32_t row_end = min(nrows, (blockIdx.x + 1) * rpb);
  for (uint32_t row = blockIdx.x * rpb; row < row_end; ++row) {
    const uint32_t y = row % L;
    const uint32_t z = row / L;  // 0 in 2D
    const uint64_t base = (uint64_t)row * L;
    const uint64_t below = base + ((y + 1 == L) ? -(int64_t)(L - 1) * L : (int64_t)L);
    const uint64_t plane = (uint64_t)L * L;
    const uint64_t behind = (d == 3) ? (base + ((z + 1 == L) ? -(int64_t)(L - 1) * plane : (int64_t)plane)) : 0;
    for (uint32_t cx = threadIdx.x; cx < cpr; cx += NT) {
      const uint32_t x = 16 * cx;
      const uint4 c = *reinterpret_cast<const uint4*>(sp + base + x);
      const uint32_t nx = *reinterpret_cast<const uint32_t*>(sp + base + ((x + 16 == L) ? 0 : x + 16));
      const uint4 dy = *reinterpret_cast<const uint4*>(sp + below + x);
      const uint32_t cw[4] = {c.x, c.y, c.z, c.w};
      const uint32_t yw[4] = {dy.x, dy.y, dy.z, dy.w};
      const uint32_t rw[4] = {__builtin_amdgcn_alignbyte(c.y, c.x, 1), __builtin_amdgcn_alignbyte(c.z, c.y, 1),
                              __builtin_amdgcn_alignbyte(c.w, c.z, 1), __builtin_amdgcn_alignbyte(nx, c.w, 1)};
      uint4 jx = make_uint4(0, 0, 0, 0), jy = jx, jz = jx;
      if (J) {
        jx = *reinterpret_cast<const uint4*>(J + base + x);
        jy = *reinterpret_cast<const uint4*>(J + N + base + x);
        if (d == 3) jz = *reinterpret_cast<const uint4*>(J + 2 * N + base + x);
      }
      const uint32_t jxw[4] = {jx.x, jx.y, jx.z, jx.w}, jyw[4] = {jy.x, jy.y, jy.z, jy.w};
      const uint32_t jzw[4] = {jz.x, jz.y, jz.z, jz.w};
      uint4 dz = make_uint4(0, 0, 0, 0);
      if (d == 3) dz = *reinterpret_cast<const uint4*>(sp + behind + x);
      const uint32_t zw[4] = {dz.x, dz.y, dz.z, dz.w};
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        neg += __popc(cw[k] & msb);
        unsat += __popc(xor3(cw[k], rw[k], jxw[k]) & msb);
        unsat += __popc(xor3(cw[k], yw[k], jyw[k]) & msb);
        if (d == 3) unsat += __popc(xor3(cw[k], zw[k], jzw[k]) & msb);
      }
    }
  }
  record_block<NT>(unsat, neg, rec, red);
}

static uint32_t measure_rows_per_block(const Lat& lat) {
  const uint32_t nrows = (uint32_t)(lat.N / lat.L);
  uint32_t rpb = (nrows + 2047) / 2048;  // about 2048 workgroups, whole rows each
  return rpb < 1 ? 1 : rpb;
}

uint32_t measure_parts(const Lat& lat) {
  if (lat.L % 16 == 0) {
    const uint32_t nrows = (uint32_t)(lat.N / lat.L);
    const uint32_t rpb = measure_rows_per_block(lat);
    return (nrows + rpb - 1) / rpb;
  }
  return grid_for(lat.N, 256, 4096);
}

hipError_t launch_measure(const Lat& lat, const Record& rec, hipStream_t stream) {
  constexpr int NT = 256;
  if (lat.L % 16 == 0) {
    const uint32_t nrows = (uint32_t)(lat.N / lat.L);
    const uint32_t rpb = measure_rows_per_block(lat);
    hipLaunchKernelGGL(k_measure_rows<NT>, dim3(measure_parts(lat)), dim3(NT), 0, stream,
                       (const int8_t*)lat.spins, lat.J, lat.L, lat.d, lat.N, nrows, rpb, rec);
    return hipGetLastError();
  }
  hipLaunchKernelGGL(k_measure_sites<NT>, dim3(measure_parts(lat)), dim3(NT), 0, stream,
                     (const int8_t*)lat.spins, lat.J, lat.L, lat.d, lat.N, rec);
  return hipGetLastError();
}

// One workgroup per record: sum the partial counts, write E and M.
__global__ __launch_bounds__(256) void k_finalize(const int64_t* __restrict__ part, uint32_t stride,
                                                  uint32_t nparts, int64_t* E, int64_t* M,
                                                  int64_t e0, int64_t m0) {
  __shared__ int64_t red[4];
  const int64_t* p = part + (uint64_t)blockIdx.x * stride * 2;
  int64_t u = 0, n = 0;
  for (uint32_t i = threadIdx.x; i < nparts; i += 256) {
    u += p[2 * i];
    n += p[2 * i + 1];
  }
  const int64_t su = block_sum<256>(u, red);
  const int64_t sn = block_sum<256>(n, red);
  if (threadIdx.x == 0) {
    E[blockIdx.x] = e0 + 2 * su;
    M[blockIdx.x] = m0 - 2 * sn;
  }
}

hipError_t launch_finalize(const int64_t* part, uint32_t stride, uint32_t nparts, uint32_t nrec,
                           int64_t* E, int64_t* M, int64_t e0, int64_t m0, hipStream_t stream) {
  if (nrec == 0) return hipSuccess;
  hipLaunchKernelGGL(k_finalize, dim3(nrec), dim3(256), 0, stream, part, stride, nparts, E, M, e0, m0);
  return hipGetLastError();
}

// ========================================================= generic phase

__global__ __launch_bounds__(256) void k_generic_phase(Lat lat, uint32_t t, uint32_t colour,
                                                       Accept acc) {
  __shared__ uint64_t T[8];
  if (threadIdx.x < 8) T[threadIdx.x] = acc.T[threadIdx.x];
  __syncthreads();
  const uint64_t ngroups = (lat.N + 7) / 8;
  for (uint64_t g = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; g < ngroups;
       g += (uint64_t)gridDim.x * blockDim.x)
    generic_group(lat.spins, lat.J, lat.L, lat.d, lat.N, g, t, colour, lat.replica, lat.keys, T);
}

hipError_t launch_generic_phase(const Lat& lat, uint32_t t, uint32_t colour, const Accept& acc,
                                hipStream_t stream) {
  const uint64_t ngroups = (lat.N + 7) / 8;
  hipLaunchKernelGGL(k_generic_phase, dim3(grid_for(ngroups, 256)), dim3(256), 0, stream, lat, t,
                     colour, acc);
  return hipGetLastError();
}

// ============================================================ resident

// One workgroup holds the whole lattice in LDS and runs n sweeps; records
// (E, M) after every every-th sweep into E[i], M[i].
__global__ void k_resident(Lat lat, uint32_t t0, int n, Accept acc, int every, int64_t* E,
                           int64_t* M) {
  extern __shared__ __align__(16) int8_t lds[];
  __shared__ uint64_t T[8];
  __shared__ int64_t red[32];
  const int NT = blockDim.x;
  if (threadIdx.x < 8) T[threadIdx.x] = acc.T[threadIdx.x];
  const uint64_t N = lat.N;
  for (uint64_t q = threadIdx.x; q < N / 4; q += NT)
    reinterpret_cast<uint32_t*>(lds)[q] = reinterpret_cast<const uint32_t*>(lat.spins)[q];
  __syncthreads();
  const uint64_t ngroups = (N + 7) / 8;
  int rec = 0;
  for (int i = 0; i < n; ++i) {
    const uint32_t t = t0 + (uint32_t)i;
    for (uint32_t colour = 0; colour < 2; ++colour) {
      for (uint64_t g = threadIdx.x; g < ngroups; g += NT)
        generic_group(lds, lat.J, lat.L, lat.d, N, g, t, colour, lat.replica, lat.keys, T);
      __syncthreads();
    }
    if (every > 0 && (i + 1) % every == 0) {
      int64_t e = 0, m = 0;
      for (uint64_t s = threadIdx.x; s < N; s += NT) {
        const Site c = site_coords(s, lat.L, lat.d);
        const uint32_t cd[3] = {c.x, c.y, c.z};
        uint64_t st = 1;
        const int si = lds[s];
        m += si;
        for (uint32_t dir = 0; dir < lat.d; ++dir) {
          const uint64_t up = nb_plus(s, cd[dir], lat.L, st);
          e -= (int64_t)(lat.J ? lat.J[dir * N + s] : 1) * si * lds[up];
          st *= lat.L;
        }
      }
      // block reduction for a runtime thread count (<= 1024)
      e = wave_sum(e);
      m = wave_sum(m);
      const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
      if (lane == 0) {
        red[wid] = e;
        red[16 + wid] = m;
      }
      __syncthreads();
      if (threadIdx.x == 0) {
        int64_t se = 0, sm = 0;
        for (int w = 0; w < NT / 64; ++w) {
          se += red[w];
          sm += red[16 + w];
        }
        E[rec] = se;
        M[rec] = sm;
      }
      __syncthreads();
      ++rec;
    }
  }
  for (uint64_t q = threadIdx.x; q < N / 4; q += NT)
    reinterpret_cast<uint32_t*>(lat.spins)[q] = reinterpret_cast<const uint32_t*>(lds)[q];
}

size_t resident_lds_bytes(const Lat& lat) { return (size_t)lat.N; }

hipError_t launch_resident(const Lat& lat, uint32_t t0, int n, const Accept& acc, int every,
                           int64_t* E, int64_t* M, int threads, hipStream_t stream) {
  const size_t bytes = resident_lds_bytes(lat);
  static bool attr_set = false;
  if (!attr_set) {
    hipError_t e = hipFuncSetAttribute((const void*)k_resident,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, 150 * 1024);
    if (e != hipSuccess) return e;
    attr_set = true;
  }
  if (threads <= 0) threads = 512;
  hipLaunchKernelGGL(k_resident, dim3(1), dim3(threads), bytes, stream, lat, t0, n, acc, every, E,
                     M);
  return hipGetLastError();
}

// =============================================================== tiled

// Kernel arguments of the register-parallel phase kernels.
struct PhaseArgs {
  RoundKeys keys;
  uint32_t bound[8];
  uint32_t never4;  // 4 * never_level
  uint32_t L;
  uint32_t t;
  uint32_t colour;
  uint32_t replica;
};

static PhaseArgs phase_args(const Lat& lat, uint32_t t, uint32_t colour, const Accept& acc) {
  PhaseArgs a;
  a.keys = lat.keys;
  for (int i = 0; i < 8; ++i) a.bound[i] = acc.bound[i];
  a.never4 = 4u * acc.never_level;
  a.L = lat.L;
  a.t = t;
  a.colour = colour;
  a.replica = lat.replica;
  return a;
}

// 2D colour phase.  LDS row (TW+32 bytes): byte q <-> x = x0 - 16 + q, so the
// tile occupies bytes [16, 16+TW), its halo dwords [12,16) and [16+TW, 20+TW).
// LDS row r <-> y = y0 - 1 + r, r in [0, TH+2).
template <int TW, int TH, int NT, bool NEVER>
__global__ __launch_bounds__(NT) void k_tiled2d(int8_t* __restrict__ spins, PhaseArgs a) {
  constexpr int RB = TW + 32;
  constexpr int GPR = TW / 8;
  __shared__ __align__(16) int8_t tile[(TH + 2) * RB];
  __shared__ uint32_t bound[8];
  if (threadIdx.x < 8) bound[threadIdx.x] = a.bound[threadIdx.x];
  const uint32_t L = a.L;
  const uint32_t x0 = blockIdx.x * TW, y0 = blockIdx.y * TH;
  // tile interior, 16 bytes per load
  for (int i = threadIdx.x; i < (TH + 2) * (TW / 16); i += NT) {
    const int r = i / (TW / 16), q = i - r * (TW / 16);
    const uint32_t y = wrap_row(y0 + r, 1u, L);
    const uint4 v = *reinterpret_cast<const uint4*>(spins + (uint64_t)y * L + x0 + 16 * q);
    *reinterpret_cast<uint4*>(tile + r * RB + 16 + 16 * q) = v;
  }
  // halo dwords left and right
  for (int i = threadIdx.x; i < 2 * (TH + 2); i += NT) {
    const int r = i >> 1, side = i & 1;
    const uint32_t y = wrap_row(y0 + r, 1u, L);
    const uint32_t x = side ? ((x0 + TW == L) ? 0u : x0 + TW) : ((x0 == 0) ? L - 4 : x0 - 4);
    *reinterpret_cast<uint32_t*>(tile + r * RB + (side ? 16 + TW : 12)) =
        *reinterpret_cast<const uint32_t*>(spins + (uint64_t)y * L + x);
  }
  __syncthreads();
  for (int u = threadIdx.x; u < GPR * TH; u += NT) {
    const int r = u / GPR + 1, g = u - (r - 1) * GPR;
    const int8_t* row = tile + r * RB + 16 + 8 * g;
    const uint2 c = *reinterpret_cast<const uint2*>(row);
    const uint2 up = *reinterpret_cast<const uint2*>(row - RB);
    const uint2 dn = *reinterpret_cast<const uint2*>(row + RB);
    const uint32_t lw = *reinterpret_cast<const uint32_t*>(row - 4);
    const uint32_t rw = *reinterpret_cast<const uint32_t*>(row + 8);
    const uint32_t y = y0 + r - 1, x = x0 + 8 * g;
    const uint64_t s = (uint64_t)y * L + x;
    uint32_t rnd[4];
    philox((uint32_t)(s >> 3), a.t, a.replica, a.colour, a.keys, rnd);
    const uint32_t o0[2] = {up.x, dn.x}, o1[2] = {up.y, dn.y};
    uint32_t S0, S1;
    unsat_ising<2>(c.x, c.y, lw, rw, o0, o1, S0, S1);
    uint32_t c0 = c.x, c1 = c.y;
    apply_group<NEVER>(c0, c1, S0, S1, (a.colour + y) & 1u, rnd, bound, a.never4);
    *reinterpret_cast<uint2*>(spins + s) = make_uint2(c0, c1);
  }
}

// 3D colour phase.  LDS rows indexed (zz, yy), zz in [0, TZ+2) <-> z = z0-1+zz,
// yy in [0, TH+2) <-> y = y0-1+yy; row layout as in 2D.
template <int TW, int TH, int TZ, int NT, bool NEVER>
__global__ __launch_bounds__(NT) void k_tiled3d(int8_t* __restrict__ spins, PhaseArgs a) {
  constexpr int RB = TW + 32;
  constexpr int GPR = TW / 8;
  constexpr int RY = TH + 2;
  __shared__ __align__(16) int8_t tile[(TZ + 2) * RY * RB];
  __shared__ uint32_t bound[8];
  if (threadIdx.x < 8) bound[threadIdx.x] = a.bound[threadIdx.x];
  const uint32_t L = a.L;
  const uint64_t plane = (uint64_t)L * L;
  const uint32_t x0 = blockIdx.x * TW, y0 = blockIdx.y * TH, z0 = blockIdx.z * TZ;
  for (int i = threadIdx.x; i < (TZ + 2) * RY * (TW / 16); i += NT) {
    const int rr = i / (TW / 16), q = i - rr * (TW / 16);
    const int zz = rr / RY, yy = rr - zz * RY;
    const uint32_t y = wrap_row(y0 + yy, 1u, L);
    const uint32_t z = wrap_row(z0 + zz, 1u, L);
    const uint4 v =
        *reinterpret_cast<const uint4*>(spins + z * plane + (uint64_t)y * L + x0 + 16 * q);
    *reinterpret_cast<uint4*>(tile + rr * RB + 16 + 16 * q) = v;
  }
  for (int i = threadIdx.x; i < 2 * (TZ + 2) * RY; i += NT) {
    const int rr = i >> 1, side = i & 1;
    const int zz = rr / RY, yy = rr - zz * RY;
    const uint32_t y = wrap_row(y0 + yy, 1u, L);
    const uint32_t z = wrap_row(z0 + zz, 1u, L);
    const uint32_t x = side ? ((x0 + TW == L) ? 0u : x0 + TW) : ((x0 == 0) ? L - 4 : x0 - 4);
    *reinterpret_cast<uint32_t*>(tile + rr * RB + (side ? 16 + TW : 12)) =
        *reinterpret_cast<const uint32_t*>(spins + z * plane + (uint64_t)y * L + x);
  }
  __syncthreads();
  for (int u = threadIdx.x; u < GPR * TH * TZ; u += NT) {
    const int rr0 = u / GPR, g = u - rr0 * GPR;
    const int zi = rr0 / TH, yi = rr0 - zi * TH;  // interior coordinates
    const int rr = (zi + 1) * RY + (yi + 1);
    const int8_t* row = tile + rr * RB + 16 + 8 * g;
    const uint2 c = *reinterpret_cast<const uint2*>(row);
    const uint2 yu = *reinterpret_cast<const uint2*>(row - RB);
    const uint2 yd = *reinterpret_cast<const uint2*>(row + RB);
    const uint2 zu = *reinterpret_cast<const uint2*>(row - RY * RB);
    const uint2 zd = *reinterpret_cast<const uint2*>(row + RY * RB);
    const uint32_t lw = *reinterpret_cast<const uint32_t*>(row - 4);
    const uint32_t rw = *reinterpret_cast<const uint32_t*>(row + 8);
    const uint32_t y = y0 + yi, z = z0 + zi, x = x0 + 8 * g;
    const uint64_t s = z * plane + (uint64_t)y * L + x;
    uint32_t rnd[4];
    philox((uint32_t)(s >> 3), a.t, a.replica, a.colour, a.keys, rnd);
    const uint32_t o0[4] = {yu.x, yd.x, zu.x, zd.x}, o1[4] = {yu.y, yd.y, zu.y, zd.y};
    uint32_t S0, S1;
    unsat_ising<4>(c.x, c.y, lw, rw, o0, o1, S0, S1);
    uint32_t c0 = c.x, c1 = c.y;
    apply_group<NEVER>(c0, c1, S0, S1, (a.colour + y + z) & 1u, rnd, bound, a.never4);
    *reinterpret_cast<uint2*>(spins + s) = make_uint2(c0, c1);
  }
}

// Supported tile shapes (compile-time instantiations).
struct Tiled2DShape {
  int tw, th, nt;
};
struct Tiled3DShape {
  int tw, th, tz, nt;
};

bool tiled_supported(const Lat& lat, const Tile& tile) {
  if (lat.J != nullptr) return false;
  if (lat.L % 8 != 0) return false;
  if (lat.L % tile.x != 0 || lat.L % tile.y != 0) return false;
  if (lat.d == 3 && lat.L % tile.z != 0) return false;
  if (lat.d == 2) {
    return (tile.x == 256 && tile.y == 32 && tile.threads == 256) ||
           (tile.x == 128 && tile.y == 16 && tile.threads == 256) ||
           (tile.x == 512 && tile.y == 32 && tile.threads == 512) ||
           (tile.x == 64 && tile.y == 8 && tile.threads == 64) ||
           (tile.x == 16 && tile.y == 8 && tile.threads == 64);
  }
  return (tile.x == 64 && tile.y == 8 && tile.z == 8 && tile.threads == 256) ||
         (tile.x == 32 && tile.y == 8 && tile.z == 4 && tile.threads == 128) ||
         (tile.x == 128 && tile.y == 8 && tile.z == 4 && tile.threads == 256) ||
         (tile.x == 16 && tile.y == 4 && tile.z == 4 && tile.threads == 64);
}

template <int TW, int TH, int NT>
static hipError_t go2d(const Lat& lat, const PhaseArgs& a, bool never, hipStream_t stream) {
  dim3 grid(lat.L / TW, lat.L / TH);
  if (never)
    hipLaunchKernelGGL((k_tiled2d<TW, TH, NT, true>), grid, dim3(NT), 0, stream, lat.spins, a);
  else
    hipLaunchKernelGGL((k_tiled2d<TW, TH, NT, false>), grid, dim3(NT), 0, stream, lat.spins, a);
  return hipGetLastError();
}

template <int TW, int TH, int TZ, int NT>
static hipError_t go3d(const Lat& lat, const PhaseArgs& a, bool never, hipStream_t stream) {
  dim3 grid(lat.L / TW, lat.L / TH, lat.L / TZ);
  if (never)
    hipLaunchKernelGGL((k_tiled3d<TW, TH, TZ, NT, true>), grid, dim3(NT), 0, stream, lat.spins, a);
  else
    hipLaunchKernelGGL((k_tiled3d<TW, TH, TZ, NT, false>), grid, dim3(NT), 0, stream, lat.spins, a);
  return hipGetLastError();
}

hipError_t launch_tiled_phase(const Lat& lat, uint32_t t, uint32_t colour, const Accept& acc,
                              const Tile& tile, hipStream_t stream) {
  if (!tiled_supported(lat, tile)) return hipErrorInvalidValue;
  const PhaseArgs a = phase_args(lat, t, colour, acc);
  const bool never = acc.never_level > 0;
  if (lat.d == 2) {
    if (tile.x == 256 && tile.y == 32) return go2d<256, 32, 256>(lat, a, never, stream);
    if (tile.x == 128 && tile.y == 16) return go2d<128, 16, 256>(lat, a, never, stream);
    if (tile.x == 512 && tile.y == 32) return go2d<512, 32, 512>(lat, a, never, stream);
    if (tile.x == 64 && tile.y == 8) return go2d<64, 8, 64>(lat, a, never, stream);
    return go2d<16, 8, 64>(lat, a, never, stream);
  }
  if (tile.x == 64 && tile.y == 8 && tile.z == 8) return go3d<64, 8, 8, 256>(lat, a, never, stream);
  if (tile.x == 32 && tile.y == 8 && tile.z == 4) return go3d<32, 8, 4, 128>(lat, a, never, stream);
  if (tile.x == 128 && tile.y == 8 && tile.z == 4) return go3d<128, 8, 4, 256>(lat, a, never, stream);
  return go3d<16, 4, 4, 64>(lat, a, never, stream);
}

// ================================================================ fused

// 2D Ising, one whole sweep.  LDS row (TW+32 bytes): byte q <-> x = x0-16+q;
// LDS row r in [0, TH+4) <-> y = y0-2+r.  LDS group j (bytes [8j, 8j+8)):
// tile groups j in [2, TW/8+2), halo groups j = 1 and j = TW/8+2.
template <int TW, int TH, int NT, bool NEVER>
__global__ __launch_bounds__(NT) void k_fused2d(const int8_t* __restrict__ src,
                                               int8_t* __restrict__ dst, PhaseArgs a) {
  constexpr int RB = TW + 32;
  constexpr int GPR = TW / 8;
  constexpr int RT = TH + 4;
  __shared__ __align__(16) int8_t tile[RT * RB];
  __shared__ uint32_t bound[8];
  if (threadIdx.x < 8) bound[threadIdx.x] = a.bound[threadIdx.x];
  const uint32_t L = a.L;
  const uint32_t x0 = blockIdx.x * TW, y0 = blockIdx.y * TH;
  // rows: every 16-byte chunk of [x0-16, x0+TW+16)
  constexpr int CPR = TW / 16 + 2;
  for (int i = threadIdx.x; i < RT * CPR; i += NT) {
    const int r = i / CPR, q = i - r * CPR;
    const uint32_t y = wrap_row(y0 + r, 2u, L);
    const uint32_t x = wrap_row(x0 + 16 * q, 16u, L);
    *reinterpret_cast<uint4*>(tile + r * RB + 16 * q) =
        *reinterpret_cast<const uint4*>(src + (uint64_t)y * L + x);
  }
  __syncthreads();
  // colour 0 on the tile rows plus the ring: units are (row r, LDS group j)
  //   rows 2..TH+1: groups 1..GPR+2 ; rows 1 and TH+2: groups 2..GPR+1
  {
    constexpr int WIDE = GPR + 2;
    constexpr int NU = TH * WIDE + 2 * GPR;
    for (int u = threadIdx.x; u < NU; u += NT) {
      int r, j;
      if (u < TH * WIDE) {
        r = u / WIDE + 2;
        j = u - (r - 2) * WIDE + 1;
      } else {
        const int v = u - TH * WIDE;
        r = (v < GPR) ? 1 : TH + 2;
        j = (v < GPR ? v : v - GPR) + 2;
      }
      int8_t* row = tile + r * RB + 8 * j;
      const uint2 c = *reinterpret_cast<const uint2*>(row);
      const uint2 up = *reinterpret_cast<const uint2*>(row - RB);
      const uint2 dn = *reinterpret_cast<const uint2*>(row + RB);
      const uint32_t lw = *reinterpret_cast<const uint32_t*>(row - 4);
      const uint32_t rw = *reinterpret_cast<const uint32_t*>(row + 8);
      const uint32_t y = wrap_row(y0 + r, 2u, L);
      const uint32_t x = wrap_row(x0 + 8 * j, 16u, L);
      const uint64_t s = (uint64_t)y * L + x;
      uint32_t rnd[4];
      philox((uint32_t)(s >> 3), a.t, a.replica, 0u, a.keys, rnd);
      const uint32_t o0[2] = {up.x, dn.x}, o1[2] = {up.y, dn.y};
      uint32_t S0, S1;
      unsat_ising<2>(c.x, c.y, lw, rw, o0, o1, S0, S1);
      uint32_t c0 = c.x, c1 = c.y;
      apply_group<NEVER>(c0, c1, S0, S1, y & 1u, rnd, bound, a.never4);
      *reinterpret_cast<uint2*>(row) = make_uint2(c0, c1);
    }
  }
  __syncthreads();
  for (int u = threadIdx.x; u < GPR * TH; u += NT) {
    const int r = u / GPR + 2, g = u - (r - 2) * GPR;
    const int8_t* row = tile + r * RB + 16 + 8 * g;
    const uint2 c = *reinterpret_cast<const uint2*>(row);
    const uint2 up = *reinterpret_cast<const uint2*>(row - RB);
    const uint2 dn = *reinterpret_cast<const uint2*>(row + RB);
    const uint32_t lw = *reinterpret_cast<const uint32_t*>(row - 4);
    const uint32_t rw = *reinterpret_cast<const uint32_t*>(row + 8);
    const uint32_t y = y0 + r - 2, x = x0 + 8 * g;
    const uint64_t s = (uint64_t)y * L + x;
    uint32_t rnd[4];
    philox((uint32_t)(s >> 3), a.t, a.replica, 1u, a.keys, rnd);
    const uint32_t o0[2] = {up.x, dn.x}, o1[2] = {up.y, dn.y};
    uint32_t S0, S1;
    unsat_ising<2>(c.x, c.y, lw, rw, o0, o1, S0, S1);
    uint32_t c0 = c.x, c1 = c.y;
    apply_group<NEVER>(c0, c1, S0, S1, (1u + y) & 1u, rnd, bound, a.never4);
    *reinterpret_cast<uint2*>(dst + s) = make_uint2(c0, c1);
  }
}

// 2D Ising, one whole sweep, tile 512 bytes wide (one 64-lane wave per row:
// lane l owns the group at x = x0 + 8l) and TH rows.  Everything that depends
// on the row only (parity of the active bytes, flip constants, addresses,
// counter base) is wave-uniform.  LDS layout as in k_fused2d with TW = 512.
// Phase 0: colour 0 on LDS rows 1..TH+2 (tile columns), plus the two halo
// groups (x0-8, x0+512) on rows 2..TH+1; phase 1: colour 1 on rows 2..TH+1.
template <int TH, bool NEVER>
__global__ __launch_bounds__(256) void k_fused2d_w(const int8_t* __restrict__ src,
                                                   int8_t* __restrict__ dst, PhaseArgs a) {
  constexpr int TW = 512;
  constexpr int RB = TW + 32;
  constexpr int GPR = TW / 8;
  constexpr int RT = TH + 4;
  constexpr int CPR = TW / 16 + 2;
  __shared__ __align__(16) int8_t tile[RT * RB];
  __shared__ uint32_t bound[8];
  if (threadIdx.x < 8) bound[threadIdx.x] = a.bound[threadIdx.x];
  const uint32_t L = a.L;
  const uint32_t x0 = blockIdx.x * TW, y0 = blockIdx.y * TH;
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  for (int i = threadIdx.x; i < RT * CPR; i += 256) {
    const int r = i / CPR, q = i - r * CPR;
    const uint32_t y = wrap_row(y0 + r, 2u, L);
    const uint32_t x = wrap_row(x0 + 16 * q, 16u, L);
    *reinterpret_cast<uint4*>(tile + r * RB + 16 * q) =
        *reinterpret_cast<const uint4*>(src + (uint64_t)y * L + x);
  }
  __syncthreads();
  const uint32_t gq = (x0 >> 3) + (uint32_t)lane;  // counter word of this lane's group, minus row part
  const uint32_t Lg = L >> 3;                      // groups per lattice row
  const PhiloxUniform U0 = philox_uniform(a.t, a.replica, 0u, a.keys);
  const PhiloxUniform U1 = philox_uniform(a.t, a.replica, 1u, a.keys);
  // ---- phase 0: colour 0, tile columns, LDS rows 1..TH+2 (wave-strided)
  {
    const int r_first = 1 + wave;
    const uint32_t p = (y0 + (uint32_t)r_first) & 1u;  // parity of y = y0 + r - 2
#pragma unroll 2
    for (int r = r_first; r <= TH + 2; r += 4) {
      int8_t* row = tile + r * RB + 16 + 8 * lane;
      const uint2 c = *reinterpret_cast<const uint2*>(row);
      const uint2 up = *reinterpret_cast<const uint2*>(row - RB);
      const uint2 dn = *reinterpret_cast<const uint2*>(row + RB);
      const uint32_t lw = *reinterpret_cast<const uint32_t*>(row - 4);
      const uint32_t rw = *reinterpret_cast<const uint32_t*>(row + 8);
      const uint32_t y = wrap_row(y0 + (uint32_t)r, 2u, L);
      uint32_t rnd[4];
      philox_lane(y * Lg + gq, U0, a.keys, rnd);
      const uint32_t o0[2] = {up.x, dn.x}, o1[2] = {up.y, dn.y};
      uint32_t S0, S1;
      unsat_ising<2>(c.x, c.y, lw, rw, o0, o1, S0, S1);
      uint32_t c0 = c.x, c1 = c.y;
      apply_group<NEVER>(c0, c1, S0, S1, p, rnd, bound, a.never4);
      *reinterpret_cast<uint2*>(row) = make_uint2(c0, c1);
    }
  }
  // ---- phase 0: the halo groups left (LDS group 1) and right (group GPR+2) of rows 2..TH+1
  for (int u = threadIdx.x; u < 2 * TH; u += 256) {
    const int r = 2 + (u >> 1), side = u & 1;
    const int j = side ? GPR + 2 : 1;
    int8_t* row = tile + r * RB + 8 * j;
    const uint2 c = *reinterpret_cast<const uint2*>(row);
    const uint2 up = *reinterpret_cast<const uint2*>(row - RB);
    const uint2 dn = *reinterpret_cast<const uint2*>(row + RB);
    const uint32_t lw = *reinterpret_cast<const uint32_t*>(row - 4);
    const uint32_t rw = *reinterpret_cast<const uint32_t*>(row + 8);
    const uint32_t y = y0 + (uint32_t)r - 2u;
    const uint32_t x = wrap_row(x0 + 8 * j, 16u, L);
    uint32_t rnd[4];
    philox_lane(y * Lg + (x >> 3), U0, a.keys, rnd);
    const uint32_t o0[2] = {up.x, dn.x}, o1[2] = {up.y, dn.y};
    uint32_t S0, S1;
    unsat_ising<2>(c.x, c.y, lw, rw, o0, o1, S0, S1);
    uint32_t c0 = c.x, c1 = c.y;
    apply_group<NEVER>(c0, c1, S0, S1, y & 1u, rnd, bound, a.never4);
    *reinterpret_cast<uint2*>(row) = make_uint2(c0, c1);
  }
  __syncthreads();
  // ---- phase 1: colour 1 on the tile rows, written to dst
  {
    const int r_first = 2 + wave;
    const uint32_t p = (y0 + (uint32_t)r_first + 1u) & 1u;  // parity of (1 + y), y = y0 + r - 2
    int8_t* out = dst + (uint64_t)(y0 + (uint32_t)r_first - 2u) * L + x0 + 8 * lane;
#pragma unroll 2
    for (int r = r_first; r <= TH + 1; r += 4) {
      const int8_t* row = tile + r * RB + 16 + 8 * lane;
      const uint2 c = *reinterpret_cast<const uint2*>(row);
      const uint2 up = *reinterpret_cast<const uint2*>(row - RB);
      const uint2 dn = *reinterpret_cast<const uint2*>(row + RB);
      const uint32_t lw = *reinterpret_cast<const uint32_t*>(row - 4);
      const uint32_t rw = *reinterpret_cast<const uint32_t*>(row + 8);
      const uint32_t y = y0 + (uint32_t)r - 2u;
      uint32_t rnd[4];
      philox_lane(y * Lg + gq, U1, a.keys, rnd);
      const uint32_t o0[2] = {up.x, dn.x}, o1[2] = {up.y, dn.y};
      uint32_t S0, S1;
      unsat_ising<2>(c.x, c.y, lw, rw, o0, o1, S0, S1);
      uint32_t c0 = c.x, c1 = c.y;
      apply_group<NEVER>(c0, c1, S0, S1, p, rnd, bound, a.never4);
      *reinterpret_cast<uint2*>(out) = make_uint2(c0, c1);
      out += 4 * (uint64_t)L;
    }
  }
}

// 2D Ising, one whole sweep, streaming over full-width rows.  L = 8 * NT * G:
// thread l owns the groups g = l + NT*j (j < G) of every row (x = 8g).  A
// workgroup owns the strip of H rows [y0, y0+H) (H even) and keeps a ring of 8
// rows in LDS (row k of the strip, k = y - (y0-2), lives in slot k & 7; a
// row's bytes sit at [16, 16+L) with x = L-16..L-1 copied to [0,16) and
// x = 0..15 to [16+L, 32+L)).  Step i (i = 0..H+2), with a = y0-1+i:
//   load row a+2 into registers (stored to LDS at the end of the step);
//   colour 0 on row a (i <= H+1): reads rows a-1..a+1, writes row a in LDS;
//   colour 1 on row a-2 (i >= 3): reads rows a-3..a-1, writes dst;
//   barrier.
// Row a's colour-1 bytes are still the old ones when colour 0 reads them
// (colour 1 reaches row a two steps later), and colour 1 on row a-2 reads
// colour-0 bytes finished one or more steps earlier.  The step loop is
// unrolled over the ring period so that ring slots and row parities (y0 is
// even) are compile-time constants.
template <int NT, int G>
struct StreamCtx {
  static constexpr uint32_t L = 8u * NT * G;
  static constexpr uint32_t GPR = L / 8;
  static constexpr uint32_t RBS = L + 32;
  const int8_t* __restrict__ src;
  int8_t* __restrict__ dst;
  int8_t* ring;
  const uint32_t* bound;
  const RoundKeys* keys;
  PhiloxUniform U0, U1;
  uint32_t never4, y0, H, t;

  __device__ __forceinline__ void get_row(uint32_t y, uint2 (&v)[G]) const {
    const int8_t* rowp = src + (uint64_t)y * L;
#pragma unroll
    for (int j = 0; j < G; ++j) v[j] = *reinterpret_cast<const uint2*>(rowp + 8 * (t + NT * j));
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
  uint2 nxt[G];
  const bool do_load = (i <= H);
  if (do_load) c.get_row(wrap_row(y0 + i + 3, 2u, L), nxt);
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
      uint32_t S0, S1;
      unsat_ising<2>(cc.x, cc.y, lw, rw, o0, o1, S0, S1);
      uint32_t c0 = cc.x, c1 = cc.y;
      apply_group_p<(S + 1) & 1, NEVER>(c0, c1, S0, S1, rnd, c.bound, c.never4);
      *reinterpret_cast<uint2*>(row + 8 * g) = make_uint2(c0, c1);
      if (g >= GPR - 2) *reinterpret_cast<uint2*>(row - 16 + 8 * (g - (GPR - 2))) = make_uint2(c0, c1);
      if (g < 2) *reinterpret_cast<uint2*>(row + L + 8 * g) = make_uint2(c0, c1);
    }
  }
  if (i >= 3) {
    // colour 1 on row b = y0 + i - 3 (strip row k = i - 1); parity of (1 + b) is i & 1
    const uint32_t y = y0 + i - 3u;
    int8_t* row = c.ring + ((S + 7) & 7) * RBS + 16;
    const int8_t* up = c.ring + ((S + 6) & 7) * RBS + 16;
    const int8_t* dn = c.ring + (S & 7) * RBS + 16;
    int8_t* out = c.dst + (uint64_t)y * L;
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
      uint32_t S0, S1;
      unsat_ising<2>(cc.x, cc.y, lw, rw, o0, o1, S0, S1);
      uint32_t c0 = cc.x, c1 = cc.y;
      apply_group_p<S & 1, NEVER>(c0, c1, S0, S1, rnd, c.bound, c.never4);
      *reinterpret_cast<uint2*>(out + 8 * g) = make_uint2(c0, c1);
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
  if (do_load) c.put_row((S + 3) & 7, nxt);
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
  c.src = src;
  c.dst = dst;
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
template <int TY, int W, int G>
struct Stream3Ctx {
  static constexpr uint32_t L = 512u * G;
  static constexpr uint32_t GPR = L / 8;
  static constexpr uint32_t RB = L + 32;
  static constexpr uint32_t RP = TY + 4;
  static constexpr uint32_t PB = RP * RB;
  static constexpr int NT = 64 * W;
  static constexpr int RPW = (RP + W - 1) / W;  // plane rows loaded per wave
  const int8_t* __restrict__ src;
  int8_t* __restrict__ dst;
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
        const int8_t* rowp = src + ((uint64_t)z * L + y) * L;
#pragma unroll
        for (int j = 0; j < G; ++j) v[q][j] = *reinterpret_cast<const uint2*>(rowp + 8 * (lane + 64 * j));
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
  constexpr uint32_t L = X::L, RB = X::RB, PB = X::PB;
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
  const uint32_t cbase = (uint32_t)((((uint64_t)z * L + y) * L) >> 3);
  philox_lane(cbase + g, C ? c.U1 : c.U0, *c.keys, rnd);
  const uint32_t o0[4] = {ym.x, yp.x, a2.x, b2.x}, o1[4] = {ym.y, yp.y, a2.y, b2.y};
  uint32_t S0, S1;
  unsat_ising<4>(cc.x, cc.y, lw, rw, o0, o1, S0, S1);
  uint32_t c0 = cc.x, c1 = cc.y;
  apply_group<NEVER>(c0, c1, S0, S1, (C + y + z) & 1u, rnd, c.bound, c.never4);
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
      int8_t* out = c.dst + ((uint64_t)zb * L + y1v[q]) * L;
#pragma unroll
      for (int j = 0; j < G; ++j) {
        const uint32_t g = c.lane + 64 * j;
        *reinterpret_cast<uint2*>(out + 8 * g) = make_uint2(v1[q][j][0], v1[q][j][1]);
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
  c.src = src;
  c.dst = dst;
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

// Streaming variants: tile.x == L (full rows), tile.y = strip height H,
// tile.threads = NT with L = 8 * NT * G.
static bool stream_shape(uint32_t L, int threads, int* G) {
  if (threads != 256 && threads != 512 && threads != 1024) return false;
  if (L % (8u * (uint32_t)threads) != 0) return false;
  const uint32_t g = L / (8u * (uint32_t)threads);
  if (g != 1 && g != 2) return false;
  if (threads == 256 && g != 2) return false;  // instantiated: (1024,1) (1024,2) (512,1) (512,2) (256,2)
  *G = (int)g;
  return true;
}

// 3D streaming shapes: tile.x == L == 512*G, tile.y = TY, tile.z = H, threads = 64*W.
static bool stream3_shape(const Lat& lat, const Tile& tile) {
  if (lat.J != nullptr || lat.d != 3) return false;
  if ((uint32_t)tile.x != lat.L || (lat.L != 512 && lat.L != 1024)) return false;
  const bool ok_shape = (tile.y == 8 && (tile.threads == 640 || tile.threads == 320)) ||
                        (tile.y == 16 && (tile.threads == 576 || tile.threads == 384)) ||
                        (tile.y == 32 && tile.threads == 704 && lat.L == 512);
  return ok_shape && lat.L % (uint32_t)tile.y == 0 && tile.z >= 4 && tile.z % 2 == 0 &&
         lat.L % (uint32_t)tile.z == 0;
}

bool fused_supported(const Lat& lat, const Tile& tile) {
  if (lat.d == 3) return stream3_shape(lat, tile);
  if (lat.J != nullptr || lat.d != 2) return false;
  if ((uint32_t)tile.x == lat.L && tile.x >= 4096) {
    int G;
    return stream_shape(lat.L, tile.threads, &G) && tile.y >= 4 && tile.y % 2 == 0 &&
           lat.L % (uint32_t)tile.y == 0 && (uint32_t)tile.y <= lat.L;
  }
  if (lat.L % 16 != 0 || lat.L < 32) return false;
  if (lat.L % tile.x != 0 || lat.L % tile.y != 0) return false;
  return (tile.x == 256 && tile.y == 32 && tile.threads == 256) ||
         (tile.x == 512 && tile.y == 32 && tile.threads == 512) ||
         (tile.x == 128 && tile.y == 16 && tile.threads == 256) ||
         (tile.x == 16 && tile.y == 8 && tile.threads == 64) ||
         (tile.x == 512 && (tile.y == 16 || tile.y == 32 || tile.y == 64) && tile.threads == 256);
}

template <int TH>
static hipError_t gofused_w(const Lat& lat, const int8_t* src, int8_t* dst, const PhaseArgs& a,
                            bool never, hipStream_t stream) {
  dim3 grid(lat.L / 512, lat.L / TH);
  if (never)
    hipLaunchKernelGGL((k_fused2d_w<TH, true>), grid, dim3(256), 0, stream, src, dst, a);
  else
    hipLaunchKernelGGL((k_fused2d_w<TH, false>), grid, dim3(256), 0, stream, src, dst, a);
  return hipGetLastError();
}

template <int TW, int TH, int NT>
static hipError_t gofused(const Lat& lat, const int8_t* src, int8_t* dst, const PhaseArgs& a,
                          bool never, hipStream_t stream) {
  dim3 grid(lat.L / TW, lat.L / TH);
  if (never)
    hipLaunchKernelGGL((k_fused2d<TW, TH, NT, true>), grid, dim3(NT), 0, stream, src, dst, a);
  else
    hipLaunchKernelGGL((k_fused2d<TW, TH, NT, false>), grid, dim3(NT), 0, stream, src, dst, a);
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

uint32_t fused_record_parts(const Lat& lat, const Tile& tile) {
  if (!fused_supported(lat, tile)) return 0;
  if (lat.d == 2 && (uint32_t)tile.x == lat.L && tile.x >= 4096) return lat.L / (uint32_t)tile.y;
  return 0;
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

hipError_t launch_fused_sweep(const Lat& lat, const int8_t* src, int8_t* dst, uint32_t t,
                              const Accept& acc, const Tile& tile, const Record* rec,
                              bool* measured, hipStream_t stream) {
  if (measured) *measured = false;
  if (!fused_supported(lat, tile)) return hipErrorInvalidValue;
  const PhaseArgs a = phase_args(lat, t, 0u, acc);
  const bool never = acc.never_level > 0;
  if (lat.d == 3) {
    const uint32_t H = (uint32_t)tile.z;
    if (lat.L == 512) {
      if (tile.y == 8 && tile.threads == 640) return gostream3<8, 10, 1>(lat, src, dst, a, never, H, stream);
      if (tile.y == 8) return gostream3<8, 5, 1>(lat, src, dst, a, never, H, stream);
      if (tile.y == 16 && tile.threads == 576) return gostream3<16, 9, 1>(lat, src, dst, a, never, H, stream);
      if (tile.y == 16) return gostream3<16, 6, 1>(lat, src, dst, a, never, H, stream);
      return gostream3<32, 11, 1>(lat, src, dst, a, never, H, stream);
    }
    if (tile.y == 8 && tile.threads == 640) return gostream3<8, 10, 2>(lat, src, dst, a, never, H, stream);
    if (tile.y == 8) return gostream3<8, 5, 2>(lat, src, dst, a, never, H, stream);
    if (tile.y == 16 && tile.threads == 576) return gostream3<16, 9, 2>(lat, src, dst, a, never, H, stream);
    return gostream3<16, 6, 2>(lat, src, dst, a, never, H, stream);
  }
  if ((uint32_t)tile.x == lat.L && tile.x >= 4096) {
    int G = 0;
    stream_shape(lat.L, tile.threads, &G);
    const uint32_t H = (uint32_t)tile.y;
    if (measured) *measured = (rec != nullptr);
    if (tile.threads == 1024 && G == 1) return gostream<1024, 1>(lat, src, dst, a, never, H, rec, stream);
    if (tile.threads == 1024 && G == 2) return gostream<1024, 2>(lat, src, dst, a, never, H, rec, stream);
    if (tile.threads == 512 && G == 1) return gostream<512, 1>(lat, src, dst, a, never, H, rec, stream);
    if (tile.threads == 512 && G == 2) return gostream<512, 2>(lat, src, dst, a, never, H, rec, stream);
    return gostream<256, 2>(lat, src, dst, a, never, H, rec, stream);
  }
  if (tile.x == 512 && tile.threads == 256) {
    if (tile.y == 16) return gofused_w<16>(lat, src, dst, a, never, stream);
    if (tile.y == 32) return gofused_w<32>(lat, src, dst, a, never, stream);
    return gofused_w<64>(lat, src, dst, a, never, stream);
  }
  if (tile.x == 256) return gofused<256, 32, 256>(lat, src, dst, a, never, stream);
  if (tile.x == 512) return gofused<512, 32, 512>(lat, src, dst, a, never, stream);
  if (tile.x == 128) return gofused<128, 16, 256>(lat, src, dst, a, never, stream);
  return gofused<16, 8, 64>(lat, src, dst, a, never, stream);
}

}  // namespace spin
