// spin_kernels.hip -- gfx950 kernels of the checkerboard Metropolis path.
//
// Families (all produce the same bits; the chain is stated in include/spin.h):
//   generic   one colour phase, per site, global memory, any even L;
//   resident  whole lattice in one workgroup's LDS, many sweeps per launch
//             (small lattices: one launch per call);
//   tiled     one colour phase, an LDS tile plus a one-site halo, updated in
//             place, 8-site groups processed four sites per register (2D/3D
//             Ising, L % 8 == 0);
//   fused     Ising, a whole sweep per launch, written to the other buffer of
//             a ping-pong pair: 2D tiles plus a two-site halo (colour 0 on
//             the tile and its one-site ring, barrier, colour 1 on the tile)
//             here; the row- and plane-streaming kernels of the large 2D and
//             3D lattices in spin_stream2d.hip and spin_stream3d.hip.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "spin_device.h"
#include "spin_internal.h"
#include "spin_phase.h"

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
// (a row = L sites along x at fixed y, z), cut into 16-site chunks that its
// threads take in turn across rows (so short rows still occupy every
// thread); a thread counts negative spins and unsatisfied +x/+y/+z bonds of
// its chunk from sign bits, with 32-bit index arithmetic (rows < 2^32, bytes
// per row < 2^17, chunks per workgroup < 2^32).
template <int NT>
__global__ __launch_bounds__(NT) void k_measure_rows(const int8_t* __restrict__ sp,
                                                     const int8_t* __restrict__ J, uint32_t L,
                                                     uint32_t d, uint64_t N, uint32_t nrows,
                                                     uint32_t rpb, Record rec) {
  __shared__ int64_t red[NT / 64];
  const uint32_t msb = 0x80808080u;
  const uint32_t cpr = L / 16;
  int64_t unsat = 0, neg = 0;
  const uint32_t row0 = blockIdx.x * rpb;
  const uint32_t row_end = min(nrows, row0 + rpb);
  const uint32_t chunks = (row_end - row0) * cpr;
  for (uint32_t k = threadIdx.x; k < chunks; k += NT) {
    const uint32_t rk = k / cpr;
    const uint32_t row = row0 + rk;
    const uint32_t cx = k - rk * cpr;
    const uint32_t y = row % L;
    const uint32_t z = row / L;  // 0 in 2D
    const uint64_t base = (uint64_t)row * L;
    const uint64_t below = base + ((y + 1 == L) ? -(int64_t)(L - 1) * L : (int64_t)L);
    const uint64_t plane = (uint64_t)L * L;
    const uint64_t behind = (d == 3) ? (base + ((z + 1 == L) ? -(int64_t)(L - 1) * plane : (int64_t)plane)) : 0;
    {
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
      for (int w = 0; w < 4; ++w) {
        neg += __popc(cw[w] & msb);
        unsat += __popc(xor3(cw[w], rw[w], jxw[w]) & msb);
        unsat += __popc(xor3(cw[w], yw[w], jyw[w]) & msb);
        if (d == 3) unsat += __popc(xor3(cw[w], zw[w], jzw[w]) & msb);
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



bool fused_supported(const Lat& lat, const Tile& tile) {
  if (lat.d == 3) return stream3d_shape(lat, tile);
  if (lat.J != nullptr || lat.d != 2) return false;
  if ((uint32_t)tile.x == lat.L && tile.x >= 4096) {  // row streaming; tile.z == 1: register columns
    int G;
    return stream2d_shape(lat.L, tile.threads, &G) && tile.y >= 4 && tile.y % 2 == 0 &&
           lat.L % (uint32_t)tile.y == 0 && (uint32_t)tile.y <= lat.L && (tile.z == 0 || tile.z == 1);
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


uint32_t fused_record_parts(const Lat& lat, const Tile& tile) {
  if (!fused_supported(lat, tile)) return 0;
  if (lat.d == 2 && (uint32_t)tile.x == lat.L && tile.x >= 4096) return lat.L / (uint32_t)tile.y;
  if (lat.d == 3) return stream3d_record_parts(lat, tile);
  return 0;
}


hipError_t launch_fused_sweep(const Lat& lat, const int8_t* src, int8_t* dst, uint32_t t,
                              const Accept& acc, const Tile& tile, const Record* rec,
                              bool* measured, hipStream_t stream) {
  if (measured) *measured = false;
  if (!fused_supported(lat, tile)) return hipErrorInvalidValue;
  const PhaseArgs a = phase_args(lat, t, 0u, acc);
  const bool never = acc.never_level > 0;
  if (lat.d == 3) return launch_stream3d(lat, src, dst, a, never, tile, rec, measured, stream);
  if ((uint32_t)tile.x == lat.L && tile.x >= 4096) {
    int G = 0;
    stream2d_shape(lat.L, tile.threads, &G);
    // both forms count E/M inside the sweep when asked, into one partial per workgroup (L / tile.y)
    if (measured) *measured = (rec != nullptr);
    if (tile.z == 1) return launch_stream2c(lat, src, dst, a, never, (uint32_t)tile.y, rec, tile.threads, G, stream);
    return launch_stream2d(lat, src, dst, a, never, (uint32_t)tile.y, rec, tile.threads, G, stream);
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
