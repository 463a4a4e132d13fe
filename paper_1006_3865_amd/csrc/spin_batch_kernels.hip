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

// One task: lattice B, sweeps B.t .. B.t+n-1, all in LDS.  n == 0 with
// every > 0 records the current state once.
template <int D, bool EA, int NT>
__device__ void batch_task(const BatchLattice& B, const BatchCall& Cl, uint32_t* sp, uint32_t* bound,
                           int64_t* red) {
  const uint32_t L = B.L;
  const uint32_t LG = L / 8;                       // words per row
  const uint32_t R = (D == 3) ? L * L : L;         // rows
  const uint32_t NW = R * LG;                      // words
  const uint32_t PS = L * LG;                      // words per plane (3D)
  const uint32_t tid = threadIdx.x;
  // pack the lattice into LDS
  for (uint32_t w = tid; w < NW; w += NT) {
    const uint2 b = reinterpret_cast<const uint2*>(B.spins)[w];
    sp[w] = pack_nibbles(b.x, b.y);
  }
  if (tid < 8) bound[tid] = Cl.bound[tid];
  __syncthreads();
  // thread -> (word column xg, first row); rows advance by RI per iteration
  const uint32_t RI = NT / LG;                      // rows per iteration (>= 1: L <= 8192)
  const uint32_t NTa = RI * LG;                     // active threads
  const bool active = tid < NTa;
  const uint32_t xg = tid % LG;
  const uint32_t r_first = tid / LG;
  const uint32_t dz = RI / L, dy = RI % L;          // row step in (y, z)
  gu32* Jx = as_global(B.Jn);
  gu32* Jy = Jx + NW;
  gu32* Jz = Jx + 2 * NW;
  const uint32_t wl = xg ? 0u - 1u : LG - 1u;       // offset to the word on the left
  const uint32_t wr = (xg + 1 < LG) ? 1u : 0u - (LG - 1u);
  uint32_t rec = 0;
  for (uint32_t i = 0; i < Cl.n; ++i) {
    const uint32_t t = B.t + i;
#pragma unroll 1
    for (uint32_t colour = 0; colour < 2; ++colour) {
      const PhiloxUniform U = philox_uniform(t, B.replica, colour, B.keys);
      if (active) {
        uint32_t y = r_first % L, z = r_first / L;
        for (uint32_t row = r_first; row < R; row += RI) {
          const uint32_t w = row * LG + xg;
          const uint32_t c = sp[w];
          const uint32_t lw = sp[w + wl], rw = sp[w + wr];
          const uint32_t wym = y ? w - LG : w + (L - 1) * LG;
          const uint32_t wyp = (y + 1 < L) ? w + LG : w - (L - 1) * LG;
          uint32_t nb[2 * D - 2];
          uint32_t jn[2 * D];
          nb[0] = sp[wym];
          nb[1] = sp[wyp];
          uint32_t wzm = 0;
          if (D == 3) {
            wzm = z ? w - PS : w + (L - 1) * PS;
            const uint32_t wzp = (z + 1 < L) ? w + PS : w - (L - 1) * PS;
            nb[2] = sp[wzm];
            nb[3] = sp[wzp];
          }
          if (EA) {
            jn[0] = __builtin_amdgcn_alignbit(Jx[w], Jx[w + wl], 28);  // bond (x-1, x)
            jn[1] = Jx[w];                                              // bond (x, x+1)
            jn[2] = Jy[wym];
            jn[3] = Jy[w];
            if (D == 3) {
              jn[4] = Jz[wzm];
              jn[5] = Jz[w];
            }
          }
          const uint32_t S = nib_unsat<D, EA>(c, lw, rw, nb, jn);
          uint32_t rnd[4];
          philox_lane(w, U, B.keys, rnd);
          const uint32_t p = (colour + y + z) & 1u;
          const uint32_t f = Cl.never4 ? nib_flips<true>(S, p, rnd, bound, Cl.never4)
                                       : nib_flips<false>(S, p, rnd, bound, 0);
          sp[w] = c ^ f;
          y += dy;
          z += dz;
          if (y >= L) {
            y -= L;
            z += 1;
          }
        }
      }
      __syncthreads();
    }
    if (Cl.every && (i + 1) % Cl.every == 0) {
      batch_record<D, EA, NT>(B, Cl, sp, red, rec);
      ++rec;
    }
  }
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
  // Termination: the queue fetch (thread 0's atomic), both barriers, the
  // readfirstlane of the task index and the exit test sit at this one loop
  // level and nothing before the exit test branches on per-lane data, so
  // every wave reads the same k and leaves on the same iteration.  Moving the
  // fetch or a barrier into a nested loop or a lane-dependent branch breaks
  // that: a wave can then re-read a stale index and never reach k >= ntasks.
  for (;;) {
    if (threadIdx.x == 0) task = atomicAdd(next, 1u);
    __syncthreads();
    const uint32_t k = __builtin_amdgcn_readfirstlane(task);  // uniform: scalar loads below
    __syncthreads();
    if (k >= ntasks) break;
    const uint32_t li = __builtin_amdgcn_readfirstlane(order[k]);
    const BatchCall Cl = calls[li];
    const BatchLattice B = lats[li];
    batch_task<D, EA, NT>(B, Cl, sp, bound, red);
    if (threadIdx.x == 0) lats[li].t = B.t + Cl.n;
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
    if (e == hipSuccess) e = set_batch_attrs<1024>();
    if (e != hipSuccess) return e;
    attr = true;
  }
  hipLaunchKernelGGL(k_zero_u32, dim3(1), dim3(64), 0, stream, counter, 1u);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  if (nt == 256) go_batch<256>(d, ea, dim3(grid), lds_bytes, stream, lats, calls, order, ntasks, counter);
  else if (nt == 512) go_batch<512>(d, ea, dim3(grid), lds_bytes, stream, lats, calls, order, ntasks, counter);
  else go_batch<1024>(d, ea, dim3(grid), lds_bytes, stream, lats, calls, order, ntasks, counter);
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
