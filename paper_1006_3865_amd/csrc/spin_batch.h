// spin_batch.h -- types and launchers of the batched (many-lattice) path.
// Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "spin_internal.h"
#include "spin_nibble.h"

namespace spin {

// Largest dynamic LDS block of the batch kernel (spins packed 2 per byte).
constexpr size_t kBatchMaxLds = 150 * 1024;  // plus 208 bytes of static LDS

// Device-resident state of one lattice of a batch.
struct BatchLattice {
  int8_t* spins;        // int8 [N] in HBM (read at task start, written at task end)
  const uint32_t* Jn;   // couplings, nibble words [dir][N/8], or nullptr (Ising)
  uint32_t L;
  uint32_t d;
  uint32_t replica;
  uint32_t t;           // absolute index of the next sweep (advanced by the kernel)
  RoundKeys keys;
};

// Per-call parameters of one lattice.
struct BatchCall {
  uint32_t n;           // sweeps this call
  uint32_t every;       // record cadence (0: none)
  uint32_t never4;      // 4 * never_level of the acceptance table
  uint32_t bound[8];    // acceptance bounds by unsatisfied-bond count
  int64_t* E;           // n/every records (device) or nullptr
  int64_t* M;
};

// Device block of a lone lattice swept by the batch kernel as a one-task launch.
struct BatchSingle {
  BatchLattice lat;
  BatchCall call;
  uint32_t order;       // 0: the only task
  uint32_t counter;     // task queue of the launch
};

size_t batch_lds_bytes(uint32_t L, uint32_t d);

// Shapes the batch kernel holds in one workgroup's LDS.
inline bool batch_fits(uint32_t L, uint32_t d) {
  return L >= 8 && L % 8 == 0 && batch_lds_bytes(L, d) <= kBatchMaxLds;
}

// Workgroup size of the batch kernel for a lattice of edge L in d dimensions:
// 256, 512 or 1024 threads by size (L^d/8 nibble words up to 2048, 8192,
// more).  Sizes shared by many shapes keep them in one persistent launch.
inline uint32_t batch_threads_for(uint32_t L, uint32_t d) {
  const uint64_t nwords = (d == 3 ? (uint64_t)L * L * L : (uint64_t)L * L) / 8;
  return nwords <= 2048 ? 256u : (nwords <= 8192 ? 512u : 1024u);
}

// Workgroup sizes the batch kernel is built for (576 = 9 wavefronts: rows of a
// fixed y for L = 24 and 48 with every thread busy; a choice of the autotuner
// or the caller).
inline bool batch_threads_ok(uint32_t nt) { return nt == 256 || nt == 512 || nt == 576 || nt == 1024; }

// Write lat and call into blk (a device BatchSingle) and sweep the lattice as
// one task (nt threads, LDS for the whole lattice), all on `stream`.
hipError_t launch_batch_single(BatchSingle* blk, const BatchLattice& lat, const BatchCall& call, uint32_t nt,
                               hipStream_t stream);
// One persistent launch over ntasks tasks (lattices order[0..ntasks) with
// their calls) of one class (d, model), nt threads per workgroup; counter is
// a device word the launch zeroes and uses as the task queue.
hipError_t launch_batch(uint32_t d, bool ea, uint32_t nt, BatchLattice* lats, const BatchCall* calls,
                        const uint32_t* order, uint32_t ntasks, uint32_t* counter, size_t lds_bytes,
                        uint32_t grid, hipStream_t stream);
hipError_t launch_couplings_nibble(uint32_t* Jn, uint64_t N, uint32_t d, uint64_t cseed,
                                   uint32_t realisation, hipStream_t stream);
hipError_t launch_pack_nibbles(const int8_t* src, uint32_t* dst, uint64_t nbytes, hipStream_t stream);

}  // namespace spin
