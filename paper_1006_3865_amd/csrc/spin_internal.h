// spin_internal.h -- types shared by the host runtime and the kernels, and
// the launch functions the runtime calls.  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <vector>

namespace spin {

// Philox4x32-10 round keys: key (k0, k1) plus i times the Weyl constants
// (0x9E3779B9, 0xBB67AE85) for round i, precomputed on the host.
struct RoundKeys {
  uint32_t k0[10];
  uint32_t k1[10];
};

// Acceptance data for one (beta, d): the 64-bit table of Eq. 2 and the
// 32-bit bounds indexed by u = number of unsatisfied bonds (see spin_device.h).
struct Accept {
  uint64_t T[8];       // T[(k+z)/2], z+1 entries
  uint32_t bound[8];   // bound[u], z+1 entries
  uint32_t never_level;  // classes u < never_level have T == 0
};

// Everything one colour phase (or a resident run) of one lattice needs.
struct Lat {
  int8_t* spins;
  const int8_t* J;     // [dir][site] or nullptr (Ising)
  uint32_t L;
  uint32_t d;
  uint64_t N;
  uint32_t replica;
  RoundKeys keys;
};

// Every device allocation of the library goes through these two: the hook
// (torch's caching allocator, spin_set_allocator) when given, else
// hipMalloc / hipFree.  They keep the count of live blocks and apply the
// injected allocation failure of spin_debug_fault_alloc (or the environment
// variable SPIN_FAULT_ALLOC), so that out-of-memory paths can be forced.
void* device_alloc(size_t bytes, void* (*hook)(size_t, void*) = nullptr, void* ctx = nullptr);
void device_free(void* p, void (*hook)(void*, void*) = nullptr, void* ctx = nullptr);

// Persisted tuning records (spin_autotune, spin_batch_autotune): one line per
// record, "<kind> <arch> <fields...>", in the file named by SPIN_TUNE_CACHE
// (default $HOME/.cache/spin-gfx950/tune.txt; empty: not persisted).  Records
// of other GPU architectures are ignored; for a key the last record wins.
const char* device_arch();  // "gfx950": the current device's architecture
std::vector<std::vector<long long>> tune_cache_read(const char* kind);  // fields after <arch>
void tune_cache_append(const char* kind, const std::vector<long long>& fields);

RoundKeys make_round_keys(uint64_t seed);
Accept make_accept(double beta, int d);
// Record msg as the calling thread's spin_last_error(); returns code.
int set_error(int code, const char* msg);

// Kernel tile shapes (bytes along x, rows along y, planes along z, threads).
struct Tile {
  int x, y, z, threads;
};

// Where one (E, M) record goes: every workgroup of the kernel that counts it
// stores its partial counts (unsatisfied bonds, negative spins) in
// part[2*wg], part[2*wg + 1]; launch_finalize later turns them into
// E = -d*N + 2*sum(unsat) and M = N - 2*sum(neg).  No atomics.
struct Record {
  int64_t* part;
};

// Number of partial slots (workgroups) a record of this lattice uses when it
// is counted by the measure kernel, or by the fused kernel with this tile.
uint32_t measure_parts(const Lat& lat);
uint32_t fused_record_parts(const Lat& lat, const Tile& tile);  // 0: the kernel cannot count
// nrec records, record r's partials at part + r*stride*2 (nparts used), into
// E[r], M[r] (device arrays).
hipError_t launch_finalize(const int64_t* part, uint32_t stride, uint32_t nparts, uint32_t nrec,
                           int64_t* E, int64_t* M, int64_t e0, int64_t m0, hipStream_t stream);

// ---- launchers (all asynchronous on `stream`, return the launch status) ----
hipError_t launch_init_spins(const Lat& lat, hipStream_t stream);
hipError_t launch_couplings(int8_t* J, uint32_t L, uint32_t d, uint64_t N, uint64_t cseed,
                            uint32_t realisation, hipStream_t stream);
hipError_t launch_zero(int64_t* p, uint64_t n, hipStream_t stream);
// Partial E/M counts of the lattice into rec (measure_parts(lat) slots).
hipError_t launch_measure(const Lat& lat, const Record& rec, hipStream_t stream);

// One colour phase with the per-site generic kernel, any even L.
hipError_t launch_generic_phase(const Lat& lat, uint32_t t, uint32_t colour, const Accept& acc,
                                hipStream_t stream);
// n sweeps with the whole lattice in one workgroup's LDS; E/M written to
// E[i], M[i] after every every-th sweep (every == 0: no records).
size_t resident_lds_bytes(const Lat& lat);
hipError_t launch_resident(const Lat& lat, uint32_t t0, int n, const Accept& acc, int every,
                           int64_t* E, int64_t* M, int threads, hipStream_t stream);
// One colour phase, LDS tile + one-site halo, in place; Ising, L % 8 == 0.
bool tiled_supported(const Lat& lat, const Tile& tile);
hipError_t launch_tiled_phase(const Lat& lat, uint32_t t, uint32_t colour, const Accept& acc,
                              const Tile& tile, hipStream_t stream);
// One whole sweep of a 2D Ising lattice from `src` into `dst` (ping-pong).
// With rec != nullptr the sweep also records E, M of its result if the
// kernel can (returns true in *measured), else the caller measures.
// The coarse-tile schedule with multi-hit: tile edge T (2D: 8, 16, 32, 64;
// 3D: 8, 16; L/T even), k hits, tiles of parity q; in place.  Jn: packed
// couplings (EA) or nullptr.
bool coarse_supported(const Lat& lat, int T);
hipError_t launch_coarse_phase(const Lat& lat, const uint32_t* Jn, uint32_t t, uint32_t k, uint32_t q,
                               const Accept& acc, int T, hipStream_t stream);

// General streaming sweep (both colours, any L % 8 == 0, L >= 16, both
// models): tile.y = rows per workgroup (3D), tile.z = planes per strip,
// tile.threads = 256 or 512.  Jn: nibble-packed couplings (EA) or nullptr.
bool streamg_supported(const Lat& lat, const Tile& tile);
size_t streamg_lds_bytes(const Lat& lat, const Tile& tile);
hipError_t launch_streamg(const Lat& lat, const uint32_t* Jn, const int8_t* src, int8_t* dst, uint32_t t,
                          const Accept& acc, const Tile& tile, hipStream_t stream);
bool fused_supported(const Lat& lat, const Tile& tile);
hipError_t launch_fused_sweep(const Lat& lat, const int8_t* src, int8_t* dst, uint32_t t,
                              const Accept& acc, const Tile& tile, const Record* rec,
                              bool* measured, hipStream_t stream);

}  // namespace spin

struct spin_lattice;
namespace spin {
// E, M of a handle's current state into device int64s (asynchronous).
int record_device(spin_lattice* h, int64_t* E, int64_t* M);

// Device scratch of one sweep call supplied by the caller instead of the
// handle's own buffers: record partials (part_slots int64) and the one-task
// block of the LDS-resident path (single_bytes() bytes).
struct CallScratch {
  int64_t* part;
  size_t part_slots;
  void* single;
};
size_t single_bytes();
// spin_sweep_record_device on fixed scratch: allocates nothing, never
// synchronises; buffers the handle lacks are an SPIN_ESTATE error.
int sweep_record_fixed(spin_lattice* h, int n, double beta, int every, int64_t* E, int64_t* M,
                       const CallScratch& fx);
}  // namespace spin
