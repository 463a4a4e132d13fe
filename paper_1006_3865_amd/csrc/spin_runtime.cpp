// spin_runtime.cpp -- host side of the C ABI declared in include/spin.h:
// argument checks, device memory, the FP64 threshold table, kernel choice
// and the per-sweep launch sequence.
#include <hip/hip_runtime.h>

#include <sys/stat.h>

#include <atomic>
#include <cstdlib>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <tuple>
#include <vector>

#include "spin.h"
#include "spin_batch.h"
#include "spin_internal.h"
#include "spin_lcg.h"

namespace spin {

RoundKeys make_round_keys(uint64_t seed) {
  RoundKeys K;
  uint32_t k0 = (uint32_t)(seed & 0xffffffffu), k1 = (uint32_t)(seed >> 32);
  for (int i = 0; i < 10; ++i) {
    K.k0[i] = k0;
    K.k1[i] = k1;
    k0 += 0x9E3779B9u;
    k1 += 0xBB67AE85u;
  }
  return K;
}

// Eq. 2 of the paper, exact in integers: accept iff r < T with
// T = floor(2^32 exp(-beta dE)), dE = 2k, evaluated in IEEE double.
Accept make_accept(double beta, int d) {
  Accept a;
  std::memset(&a, 0, sizeof(a));
  const int z = 2 * d;
  for (int k = -z; k <= z; k += 2) {
    uint64_t T;
    if (k <= 0) {
      T = (uint64_t)1 << 32;
    } else {
      const double dE = (double)(2 * k);
      T = (uint64_t)std::floor(std::ldexp(std::exp(-(beta * dE)), 32));
    }
    a.T[(k + z) / 2] = T;
  }
  // u = unsatisfied bonds, k = z - 2u, table index z - u
  a.never_level = 0;
  for (int u = 0; u <= z; ++u) {
    const uint64_t T = a.T[z - u];
    a.bound[u] = (T == 0) ? 0u : (uint32_t)(T - 1);
    if (T == 0) a.never_level = (uint32_t)(u + 1);
  }
  return a;
}

}  // namespace spin

using namespace spin;

// ------------------------------------------------------------------ errors

static thread_local std::string g_error;
static thread_local int g_status = SPIN_OK;

static int fail(int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  std::vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_error = buf;
  g_status = code;
  return code;
}

int spin::set_error(int code, const char* msg) {
  g_error = msg;
  g_status = code;
  return code;
}

static int hip_fail(hipError_t e, const char* what) {
  return fail(SPIN_EDEVICE, "%s: %s", what, hipGetErrorString(e));
}

// --------------------------------------------------------------- allocator

static void* (*g_alloc)(size_t, void*) = nullptr;
static void (*g_release)(void*, void*) = nullptr;
static void* g_ctx = nullptr;

// Injected allocation failure: -2 = the environment not read yet, -1 = off,
// k >= 0 = k more allocations succeed, the next one fails (then off).
static std::atomic<int64_t> g_fault_after{-2};
static std::atomic<int64_t> g_live_blocks{0};

static bool injected_failure() {
  int64_t v = g_fault_after.load();
  if (v == -2) {
    const char* env = std::getenv("SPIN_FAULT_ALLOC");
    int64_t k = -1;
    if (env && *env) {
      char* end = nullptr;
      const long long x = std::strtoll(env, &end, 10);
      if (end && *end == 0 && x >= 0) k = (int64_t)x;
    }
    g_fault_after.compare_exchange_strong(v, k);
    v = g_fault_after.load();
  }
  while (v >= 0) {
    if (g_fault_after.compare_exchange_weak(v, v == 0 ? -1 : v - 1)) return v == 0;
  }
  return false;
}

void* spin::device_alloc(size_t bytes, void* (*hook)(size_t, void*), void* ctx) {
  if (bytes == 0) bytes = 16;
  if (injected_failure()) return nullptr;
  void* p = nullptr;
  if (hook) {
    p = hook(bytes, ctx);
  } else if (hipMalloc(&p, bytes) != hipSuccess) {
    (void)hipGetLastError();
    p = nullptr;
  }
  if (p) ++g_live_blocks;
  return p;
}

void spin::device_free(void* p, void (*hook)(void*, void*), void* ctx) {
  if (!p) return;
  if (hook)
    hook(p, ctx);
  else
    (void)hipFree(p);
  --g_live_blocks;
}

// --------------------------------------------------------------- tuning cache

static std::mutex g_cache_mu;

static std::string tune_cache_path() {
  const char* env = std::getenv("SPIN_TUNE_CACHE");
  if (env) return std::string(env);
  const char* home = std::getenv("HOME");
  if (!home || !*home) return std::string();
  return std::string(home) + "/.cache/spin-gfx950/tune.txt";
}

const char* spin::device_arch() {
  static thread_local char arch[64] = {0};
  int dev = 0;
  hipDeviceProp_t prop;
  if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess) {
    (void)hipGetLastError();
    std::snprintf(arch, sizeof(arch), "unknown");
    return arch;
  }
  size_t k = 0;
  while (k + 1 < sizeof(arch) && prop.gcnArchName[k] && prop.gcnArchName[k] != ':') {
    arch[k] = prop.gcnArchName[k];
    ++k;
  }
  arch[k] = 0;
  return arch;
}

std::vector<std::vector<long long>> spin::tune_cache_read(const char* kind) {
  std::vector<std::vector<long long>> out;
  const std::string path = tune_cache_path();
  if (path.empty()) return out;
  const std::string arch = device_arch();
  std::lock_guard<std::mutex> lk(g_cache_mu);
  FILE* f = std::fopen(path.c_str(), "r");
  if (!f) return out;
  char line[512];
  while (std::fgets(line, sizeof(line), f)) {
    char k[32], a[64];
    int used = 0;
    if (std::sscanf(line, "%31s %63s%n", k, a, &used) != 2) continue;
    if (std::strcmp(k, kind) != 0 || arch != a) continue;
    std::vector<long long> v;
    const char* p = line + used;
    long long x;
    int m = 0;
    while (std::sscanf(p, "%lld%n", &x, &m) == 1) {
      v.push_back(x);
      p += m;
    }
    out.push_back(v);
  }
  std::fclose(f);
  return out;
}

void spin::tune_cache_append(const char* kind, const std::vector<long long>& fields) {
  const std::string path = tune_cache_path();
  if (path.empty()) return;
  const std::string arch = device_arch();
  std::lock_guard<std::mutex> lk(g_cache_mu);
  const size_t slash = path.rfind('/');
  if (slash != std::string::npos && slash > 0) {
    // create the directory chain (best effort)
    std::string dir = path.substr(0, slash);
    for (size_t i = 1; i <= dir.size(); ++i)
      if (i == dir.size() || dir[i] == '/') (void)mkdir(dir.substr(0, i).c_str(), 0755);
  }
  FILE* f = std::fopen(path.c_str(), "a");
  if (!f) return;
  std::fprintf(f, "%s %s", kind, arch.c_str());
  for (long long x : fields) std::fprintf(f, " %lld", x);
  std::fprintf(f, "\n");
  std::fclose(f);
}

struct Allocator {
  void* (*alloc)(size_t, void*);
  void (*release)(void*, void*);
  void* ctx;

  void* get(size_t bytes) const { return device_alloc(bytes, alloc, ctx); }
  void put(void* p) const { device_free(p, release, ctx); }
};

// ------------------------------------------------------------------ handle

struct spin_lattice {
  int model;
  int L;
  int d;
  uint64_t N;
  int8_t* buf[2];
  int cur;
  int8_t* J;
  int64_t* em;       // 2 int64: spin_measure's output
  int64_t* part;     // partial counts of records (grown on demand)
  size_t part_slots; // capacity in int64
  uint64_t seed;
  uint32_t replica;
  uint64_t t;
  hipStream_t stream;
  int kernel;  // requested family
  Tile tile;   // requested shape (0 = default)
  Allocator mem;
  int schedule;         // spin_schedule
  int coarse_tile;      // SPIN_SCHEDULE_COARSE: tile edge T
  int hits;             // SPIN_SCHEDULE_COARSE: k
  BatchSingle* single;  // one-task block of the LDS-resident batch kernel (allocated on first use)
  uint32_t* jn;         // EA couplings as nibble words for that kernel (packed on first use)
  int rng;              // spin_rng
  uint64_t* lcg;        // LCG modes: one generator state per 8-site group
};

static const uint64_t kMaxSweepIndex = (uint64_t)1 << 32;
static const uint64_t kResidentMaxSites = 150 * 1024;   // LDS budget of the resident kernel
static const uint64_t kResidentAutoSites = 32768;       // auto choice for a lone lattice

static Lat lat_of(const spin_lattice* h) {
  Lat l;
  l.spins = h->buf[h->cur];
  l.J = h->J;
  l.L = (uint32_t)h->L;
  l.d = (uint32_t)h->d;
  l.N = h->N;
  l.replica = h->replica;
  l.keys = make_round_keys(h->seed);
  return l;
}

static int check_shape(int model, int L, int d) {
  if (model != SPIN_ISING && model != SPIN_EA_PMJ) return fail(SPIN_EINVAL, "model must be 0 (Ising) or 1 (EA +-J)");
  if (d != 2 && d != 3) return fail(SPIN_EINVAL, "d must be 2 or 3 (got %d)", d);
  if (L < 4 || (L % 2) != 0) return fail(SPIN_EINVAL, "L must be even and >= 4 (got %d)", L);
  uint64_t N = 1;
  for (int i = 0; i < d; ++i) N *= (uint64_t)L;
  if (N / 8 >= ((uint64_t)1 << 32)) return fail(SPIN_EINVAL, "L^d/8 must be < 2^32");
  return SPIN_OK;
}

static void destroy(spin_lattice* h) {
  if (!h) return;
  (void)hipStreamSynchronize(h->stream);
  h->mem.put(h->buf[0]);
  h->mem.put(h->buf[1]);
  h->mem.put(h->J);
  h->mem.put(h->em);
  h->mem.put(h->part);
  h->mem.put(h->single);
  h->mem.put(h->jn);
  h->mem.put(h->lcg);
  delete h;
}

// Workgroup size when the RESIDENT family runs on the nibble batch kernel
// (L % 8 == 0 and the packed lattice fits LDS), else 0 (the per-site kernel).
// A requested size of 256, 512, 576 or 1024 is used; none (0) picks by
// lattice shape; any other requested size selects the per-site kernel.
static uint32_t single_threads(const spin_lattice* h, const Tile& tile) {
  if (!batch_fits((uint32_t)h->L, (uint32_t)h->d)) return 0;
  const int req = tile.threads;
  if (req == 0) return batch_threads_for((uint32_t)h->L, (uint32_t)h->d);
  if (req > 0 && batch_threads_ok((uint32_t)req)) return (uint32_t)req;
  return 0;
}

// Choices of spin_autotune, per (model, L, d), used by the AUTO family.
struct Tuned {
  int kernel;
  Tile tile;
};
static std::mutex g_tune_mu;
static std::map<std::tuple<int, int, int>, Tuned> g_tuned;

static bool g_tuned_loaded = false;

// Records "lattice <arch> model L d kernel x y z threads": the persisted choices of spin_autotune.
static void load_tuned_locked() {
  if (g_tuned_loaded) return;
  g_tuned_loaded = true;
  for (const auto& v : tune_cache_read("lattice"))
    if (v.size() >= 8)
      g_tuned[std::make_tuple((int)v[0], (int)v[1], (int)v[2])] =
          Tuned{(int)v[3], Tile{(int)v[4], (int)v[5], (int)v[6], (int)v[7]}};
}

static bool tuned_choice(const spin_lattice* h, Tuned* out) {
  std::lock_guard<std::mutex> lk(g_tune_mu);
  load_tuned_locked();
  auto it = g_tuned.find(std::make_tuple(h->model, h->L, h->d));
  if (it == g_tuned.end()) return false;
  *out = it->second;
  return true;
}

static Tile default_tile(const spin_lattice* h, int kernel) {
  Tile t = h->tile;
  const int L = h->L;
  if (kernel == SPIN_KERNEL_STREAM) {  // each field: the request if given, else the default
    Tile d = h->d == 3 ? Tile{L, 8, L >= 8 ? 8 : L, 512} : Tile{L, 1, 8, 512};
    if (h->d == 3) {
      // 3D defaults from measured rates (Ising and +-J alike): rows per slab, planes per strip and
      // threads by lattice size
      Tile m = L >= 384   ? Tile{L, 16, L >= 512 ? 16 : 8, 256}
               : L >= 256 ? Tile{L, 16, 8, 512}
               : L >= 192 ? Tile{L, 8, 4, 256}
                          : Tile{L, 16, 4, 512};
      if (L % m.y != 0) m.y = 8;
      if (streamg_supported(lat_of(h), m)) d = m;
    }
    if (t.y && h->d == 3) d.y = t.y;
    if (t.z) d.z = t.z;
    if (t.threads) d.threads = t.threads;
    return d;
  }
  if (t.x && t.y && t.threads && (h->d == 2 || t.z)) return t;
  if (kernel == SPIN_KERNEL_FUSED) {
    // 3D Ising: the register-column plane streaming at L = 512 and 256 (measured at 256: 654 attempts/ns
    // against 534 for the general streaming kernel), the slab kernel at 1024
    if (h->d == 3) return L == 512 ? Tile{512, 16, 32, 576} : (L == 256 ? Tile{256, 16, 8, 576} : Tile{L, 8, 64, 640});
    // 2D full rows: the register-column form of the row-streaming kernel (measured 6-15 % faster)
    if (L == 8192) return Tile{8192, 16, 1, 1024};
    if (L == 16384) return Tile{16384, 32, 1, 1024};
    if (L == 4096) return Tile{4096, 8, 1, 512};
    if (L % 512 == 0 && L >= 1024) return Tile{512, 16, 0, 256};
    if (L % 256 == 0) return Tile{256, 32, 0, 256};
    if (L % 128 == 0) return Tile{128, 16, 0, 256};
    return Tile{16, 8, 0, 64};
  }
  if (kernel == SPIN_KERNEL_TILED) {
    if (h->d == 2) {
      if (L % 256 == 0) return Tile{256, 32, 0, 256};
      if (L % 128 == 0) return Tile{128, 16, 0, 256};
      if (L % 64 == 0) return Tile{64, 8, 0, 64};
      return Tile{16, 8, 0, 64};
    }
    if (L % 64 == 0) return Tile{64, 8, 8, 256};
    if (L % 32 == 0) return Tile{32, 8, 4, 128};
    return Tile{16, 4, 4, 64};
  }
  if (kernel == SPIN_KERNEL_RESIDENT) return Tile{0, 0, 0, t.threads};
  return Tile{0, 0, 0, 256};
}

static bool family_ok(const spin_lattice* h, int kernel, const Tile& tile) {
  const Lat l = lat_of(h);
  switch (kernel) {
    case SPIN_KERNEL_GENERIC: return true;
    case SPIN_KERNEL_RESIDENT:
      if (tile.threads != 0 && (tile.threads < 64 || tile.threads > 1024 || tile.threads % 64 != 0)) return false;
      return single_threads(h, tile) != 0 || h->N <= kResidentMaxSites;
    case SPIN_KERNEL_TILED: return tiled_supported(l, tile);
    case SPIN_KERNEL_FUSED: return fused_supported(l, tile);
    case SPIN_KERNEL_STREAM: return streamg_supported(l, tile);
    default: return false;
  }
}

// Family and tile that the next sweep uses.
static int resolve(const spin_lattice* h, Tile* tile) {
  if (h->kernel != SPIN_KERNEL_AUTO) {
    *tile = default_tile(h, h->kernel);
    return h->kernel;
  }
  Tuned tc;
  if (tuned_choice(h, &tc) && family_ok(h, tc.kernel, tc.tile)) {
    *tile = tc.tile;
    return tc.kernel;
  }
  if (h->N <= kResidentAutoSites) {
    *tile = default_tile(h, SPIN_KERNEL_RESIDENT);
    return SPIN_KERNEL_RESIDENT;
  }
  // 3D lattices from L = 160 up stream faster than they tile (measured); below that, tiles win
  const bool stream_first = h->d == 3 && h->L >= 160;
  const int order[3] = {SPIN_KERNEL_FUSED, stream_first ? SPIN_KERNEL_STREAM : SPIN_KERNEL_TILED,
                        stream_first ? SPIN_KERNEL_TILED : SPIN_KERNEL_STREAM};
  for (int k : order) {
    Tile t = default_tile(h, k);
    if (family_ok(h, k, t)) {
      *tile = t;
      return k;
    }
  }
  *tile = default_tile(h, SPIN_KERNEL_GENERIC);
  return SPIN_KERNEL_GENERIC;
}

// Make room for nrec records of `parts` slots each.
static int reserve_parts(spin_lattice* h, uint32_t nrec, uint32_t parts) {
  const size_t need = (size_t)nrec * parts * 2;
  if (need <= h->part_slots) return SPIN_OK;
  (void)hipStreamSynchronize(h->stream);
  h->mem.put(h->part);
  h->part = (int64_t*)h->mem.get(need * sizeof(int64_t));
  h->part_slots = h->part ? need : 0;
  if (!h->part) return fail(SPIN_ENOMEM, "record buffer allocation failed");
  return SPIN_OK;
}

// Partial-count slots for nrec records of `parts` slots each: the caller's fixed
// scratch (no allocation; too small is an error) or the handle's own buffer.
static int take_parts(spin_lattice* h, const CallScratch* fx, uint32_t nrec, uint32_t parts, int64_t** out) {
  *out = nullptr;
  if (nrec == 0) return SPIN_OK;
  if (fx) {
    const size_t need = (size_t)nrec * parts * 2;
    if (need > fx->part_slots)
      return fail(SPIN_EINVAL,
                  "%u records of this lattice need %llu bytes of record scratch, more than the %llu bytes "
                  "the allocation-free call has (record fewer per call)",
                  nrec, (unsigned long long)(need * sizeof(int64_t)),
                  (unsigned long long)(fx->part_slots * sizeof(int64_t)));
    *out = fx->part;
    return SPIN_OK;
  }
  if (int rc = reserve_parts(h, nrec, parts)) return rc;
  *out = h->part;
  return SPIN_OK;
}

static int64_t e_offset(const spin_lattice* h) { return -(int64_t)h->d * (int64_t)h->N; }

static int check_beta(double beta) {
  if (std::isnan(beta) || beta < 0) return fail(SPIN_EINVAL, "beta must be >= 0 or +inf (got %g)", beta);
  return SPIN_OK;
}

// Nibble-packed couplings (EA) for the kernels that read them, packed on first use.
static int ensure_jn(spin_lattice* h, const CallScratch* fx = nullptr) {
  if (h->model != SPIN_EA_PMJ || h->jn) return SPIN_OK;
  if (fx) return fail(SPIN_ESTATE, "the packed couplings of this lattice are not allocated yet");
  const uint64_t nbytes = (uint64_t)h->d * h->N;
  h->jn = (uint32_t*)h->mem.get(nbytes / 2);
  if (!h->jn) return fail(SPIN_ENOMEM, "allocation of the packed couplings failed");
  hipError_t e = launch_pack_nibbles(h->J, h->jn, nbytes, h->stream);
  if (e != hipSuccess) return hip_fail(e, "coupling packing launch");
  return SPIN_OK;
}

// n sweeps of the whole lattice in one workgroup's LDS (the batch kernel with
// one task); records (every > 0) go straight to dE, dM.
static int run_single(spin_lattice* h, int n, const Accept& acc, int every, int64_t* dE, int64_t* dM,
                      uint32_t nt, const CallScratch* fx) {
  if (!fx && !h->single) {
    h->single = (BatchSingle*)h->mem.get(sizeof(BatchSingle));
    if (!h->single) return fail(SPIN_ENOMEM, "allocation of the one-task block failed");
  }
  BatchSingle* blk = fx ? (BatchSingle*)fx->single : h->single;
  if (int rc = ensure_jn(h, fx)) return rc;
  BatchLattice bl;
  bl.spins = h->buf[h->cur];
  bl.Jn = h->jn;
  bl.L = (uint32_t)h->L;
  bl.d = (uint32_t)h->d;
  bl.replica = h->replica;
  bl.t = (uint32_t)h->t;
  bl.keys = make_round_keys(h->seed);
  BatchCall c;
  c.n = (uint32_t)n;
  c.every = every > 0 && n >= every ? (uint32_t)every : 0u;
  c.never4 = 4u * acc.never_level;
  for (int k = 0; k < 8; ++k) c.bound[k] = acc.bound[k];
  c.E = c.every ? dE : nullptr;
  c.M = c.every ? dM : nullptr;
  hipError_t e = launch_batch_single(blk, bl, c, nt, h->stream);
  if (e != hipSuccess) return hip_fail(e, "resident sweep launch");
  return SPIN_OK;
}

// n sweeps of the coarse-tile schedule (two launches each, one per tile
// parity), records by the measurement kernel.
static int run_coarse(spin_lattice* h, int n, const Accept& acc, int every, int64_t* dE, int64_t* dM,
                      const CallScratch* fx) {
  if ((h->t + (uint64_t)n) * (uint64_t)h->hits > kMaxSweepIndex)
    return fail(SPIN_EINVAL, "sweep index times hits would exceed 2^32");
  if (int rc = ensure_jn(h, fx)) return rc;
  const uint32_t nrec = every > 0 ? (uint32_t)(n / every) : 0;
  const uint32_t parts = measure_parts(lat_of(h));
  int64_t* part = nullptr;
  if (int rc = take_parts(h, fx, nrec, parts, &part)) return rc;
  hipError_t e = hipSuccess;
  uint32_t rec = 0;
  for (int i = 0; i < n; ++i) {
    const Lat l = lat_of(h);
    const uint32_t t = (uint32_t)(h->t + (uint64_t)i);
    for (uint32_t q = 0; q < 2 && e == hipSuccess; ++q)
      e = launch_coarse_phase(l, h->jn, t, (uint32_t)h->hits, q, acc, h->coarse_tile, h->stream);
    if (e != hipSuccess) return hip_fail(e, "coarse phase launch");
    if (every > 0 && (i + 1) % every == 0) {
      e = launch_measure(l, Record{part + (size_t)rec * parts * 2}, h->stream);
      if (e != hipSuccess) return hip_fail(e, "measure launch");
      ++rec;
    }
  }
  if (nrec > 0) {
    e = launch_finalize(part, parts, parts, nrec, dE, dM, e_offset(h), (int64_t)h->N, h->stream);
    if (e != hipSuccess) return hip_fail(e, "record finalize launch");
  }
  h->t += (uint64_t)n;
  return SPIN_OK;
}

// The canonical chain with LCG draws (spin_set_rng): two colour phases per sweep, records as for the
// coarse mode.
static int run_lcg(spin_lattice* h, int n, const Accept& acc, int every, int64_t* dE, int64_t* dM,
                   const CallScratch* fx) {
  const uint32_t nrec = every > 0 ? (uint32_t)(n / every) : 0;
  const uint32_t parts = measure_parts(lat_of(h));
  int64_t* part = nullptr;
  if (int rc = take_parts(h, fx, nrec, parts, &part)) return rc;
  LcgArgs a;
  for (int i = 0; i < 8; ++i) a.T[i] = acc.T[i];
  a.N = h->N;
  a.L = (uint32_t)h->L;
  a.mode = (uint32_t)h->rng;
  hipError_t e = hipSuccess;
  uint32_t rec = 0;
  for (int i = 0; i < n; ++i) {
    for (uint32_t c = 0; c < 2 && e == hipSuccess; ++c) {
      a.colour = c;
      e = launch_lcg_phase(h->buf[h->cur], h->lcg, (uint32_t)h->d, a, h->stream);
    }
    if (e != hipSuccess) return hip_fail(e, "LCG phase launch");
    if (every > 0 && (i + 1) % every == 0) {
      e = launch_measure(lat_of(h), Record{part + (size_t)rec * parts * 2}, h->stream);
      if (e != hipSuccess) return hip_fail(e, "measure launch");
      ++rec;
    }
  }
  if (nrec > 0) {
    e = launch_finalize(part, parts, parts, nrec, dE, dM, e_offset(h), (int64_t)h->N, h->stream);
    if (e != hipSuccess) return hip_fail(e, "record finalize launch");
  }
  h->t += (uint64_t)n;
  return SPIN_OK;
}

// Enqueue n sweeps; if every > 0 write records into device arrays dE, dM.
static int run_sweeps(spin_lattice* h, int n, double beta, int every, int64_t* dE, int64_t* dM,
                      const CallScratch* fx = nullptr) {
  if (!h) return fail(SPIN_EINVAL, "NULL handle");
  if (n < 0) return fail(SPIN_EINVAL, "n must be >= 0");
  if (int rc = check_beta(beta)) return rc;
  if (h->t + (uint64_t)n > kMaxSweepIndex) return fail(SPIN_EINVAL, "sweep index would exceed 2^32");
  if (n == 0) return SPIN_OK;
  const Accept acc = make_accept(beta, h->d);
  if (h->rng != SPIN_RNG_PHILOX) return run_lcg(h, n, acc, every, dE, dM, fx);
  if (h->schedule == SPIN_SCHEDULE_COARSE) return run_coarse(h, n, acc, every, dE, dM, fx);
  Tile tile;
  const int kernel = resolve(h, &tile);
  hipError_t e = hipSuccess;
  if (kernel == SPIN_KERNEL_RESIDENT && single_threads(h, tile)) {
    if (int rc = run_single(h, n, acc, every, dE, dM, single_threads(h, tile), fx)) return rc;
    h->t += (uint64_t)n;
    return SPIN_OK;
  }
  if (kernel == SPIN_KERNEL_RESIDENT) {
    const Lat l = lat_of(h);
    e = launch_resident(l, (uint32_t)h->t, n, acc, every, dE, dM, tile.threads, h->stream);
    if (e != hipSuccess) return hip_fail(e, "resident sweep launch");
    h->t += (uint64_t)n;
    return SPIN_OK;
  }
  if (kernel == SPIN_KERNEL_STREAM)
    if (int rc = ensure_jn(h, fx)) return rc;
  if ((kernel == SPIN_KERNEL_FUSED || kernel == SPIN_KERNEL_STREAM) && !h->buf[1]) {
    if (fx) return fail(SPIN_ESTATE, "the second spin buffer of this lattice is not allocated yet");
    h->buf[1] = (int8_t*)h->mem.get(h->N);
    if (!h->buf[1]) return fail(SPIN_ENOMEM, "allocation of the second spin buffer failed");
  }
  // records: partial counts per workgroup, reduced by one kernel at the end
  const uint32_t nrec = every > 0 ? (uint32_t)(n / every) : 0;
  const uint32_t fparts = (kernel == SPIN_KERNEL_FUSED) ? fused_record_parts(lat_of(h), tile) : 0;
  const uint32_t parts = fparts ? fparts : measure_parts(lat_of(h));
  int64_t* part = nullptr;
  if (int rc = take_parts(h, fx, nrec, parts, &part)) return rc;
  int rec = 0;
  for (int i = 0; i < n; ++i) {
    const uint32_t t = (uint32_t)(h->t + (uint64_t)i);
    Lat l = lat_of(h);
    const bool record_now = every > 0 && (i + 1) % every == 0;
    const Record r = Record{record_now ? part + (size_t)rec * parts * 2 : nullptr};
    bool measured = false;
    if (kernel == SPIN_KERNEL_FUSED) {
      e = launch_fused_sweep(l, h->buf[h->cur], h->buf[1 - h->cur], t, acc, tile,
                             record_now ? &r : nullptr, &measured, h->stream);
      if (e != hipSuccess) return hip_fail(e, "fused sweep launch");
      h->cur = 1 - h->cur;
    } else if (kernel == SPIN_KERNEL_STREAM) {
      e = launch_streamg(l, h->jn, h->buf[h->cur], h->buf[1 - h->cur], t, acc, tile, h->stream);
      if (e != hipSuccess) return hip_fail(e, "stream sweep launch");
      h->cur = 1 - h->cur;
    } else {
      for (uint32_t c = 0; c < 2; ++c) {
        e = (kernel == SPIN_KERNEL_TILED) ? launch_tiled_phase(l, t, c, acc, tile, h->stream)
                                          : launch_generic_phase(l, t, c, acc, h->stream);
        if (e != hipSuccess) return hip_fail(e, "colour phase launch");
      }
    }
    if (record_now) {
      if (!measured) {
        e = launch_measure(lat_of(h), r, h->stream);
        if (e != hipSuccess) return hip_fail(e, "measure launch");
      }
      ++rec;
    }
  }
  if (nrec > 0) {
    e = launch_finalize(part, parts, parts, nrec, dE, dM, e_offset(h), (int64_t)h->N, h->stream);
    if (e != hipSuccess) return hip_fail(e, "record finalize launch");
  }
  h->t += (uint64_t)n;
  return SPIN_OK;
}

size_t spin::single_bytes() { return sizeof(BatchSingle); }

int spin::sweep_record_fixed(spin_lattice* h, int n, double beta, int every, int64_t* E, int64_t* M,
                             const CallScratch& fx) {
  if (!h) return fail(SPIN_EINVAL, "NULL handle");
  if (every < 1) return fail(SPIN_EINVAL, "every must be >= 1");
  if (n / every > 0 && (!E || !M)) return fail(SPIN_EINVAL, "NULL record arrays");
  return run_sweeps(h, n, beta, every, E, M, &fx);
}

// Allocate what the handle's next sweep needs (the second spin buffer of the
// ping-pong kernels, the packed couplings), so that sweeping later allocates
// nothing.
static int prepare_buffers(spin_lattice* h) {
  if (h->rng != SPIN_RNG_PHILOX) return SPIN_OK;
  if (h->schedule == SPIN_SCHEDULE_COARSE) return ensure_jn(h);
  Tile tile;
  const int kernel = resolve(h, &tile);
  if ((kernel == SPIN_KERNEL_RESIDENT && single_threads(h, tile)) || kernel == SPIN_KERNEL_STREAM)
    if (int rc = ensure_jn(h)) return rc;
  if ((kernel == SPIN_KERNEL_FUSED || kernel == SPIN_KERNEL_STREAM) && !h->buf[1]) {
    h->buf[1] = (int8_t*)h->mem.get(h->N);
    if (!h->buf[1]) return fail(SPIN_ENOMEM, "allocation of the second spin buffer failed");
  }
  return SPIN_OK;
}

// E, M of the current state into device int64 E, M (asynchronous).
int spin::record_device(spin_lattice* h, int64_t* E, int64_t* M) {
  if (!h || !E || !M) return fail(SPIN_EINVAL, "NULL argument");
  const uint32_t parts = measure_parts(lat_of(h));
  if (int rc = reserve_parts(h, 1, parts)) return rc;
  hipError_t e = launch_measure(lat_of(h), Record{h->part}, h->stream);
  if (e == hipSuccess) e = launch_finalize(h->part, parts, parts, 1, E, M, e_offset(h), (int64_t)h->N, h->stream);
  if (e != hipSuccess) return hip_fail(e, "record");
  return SPIN_OK;
}

// Candidate (family, tile) pairs for a shape; family_ok filters them.
static std::vector<Tuned> tune_candidates(const spin_lattice* h) {
  std::vector<Tuned> c;
  const int L = h->L;
  for (int th : {256, 512, 1024}) c.push_back({SPIN_KERNEL_RESIDENT, Tile{0, 0, 0, th}});
  c.push_back({SPIN_KERNEL_RESIDENT, Tile{0, 0, 0, 512 + 64}});  // the per-site resident kernel
  if (h->d == 2) {
    for (int th : {256, 512, 1024})
      for (int H : {8, 16, 32}) c.push_back({SPIN_KERNEL_FUSED, Tile{L, H, 0, th}});
    const int f2[7][3] = {{256, 32, 256}, {512, 32, 512}, {128, 16, 256}, {16, 8, 64},
                          {512, 16, 256}, {512, 32, 256}, {512, 64, 256}};
    for (auto& f : f2) c.push_back({SPIN_KERNEL_FUSED, Tile{f[0], f[1], 0, f[2]}});
    const int t2[5][3] = {{256, 32, 256}, {128, 16, 256}, {512, 32, 512}, {64, 8, 64}, {16, 8, 64}};
    for (auto& f : t2) c.push_back({SPIN_KERNEL_TILED, Tile{f[0], f[1], 0, f[2]}});
    for (int th : {256, 512})
      for (int H : {4, 8, 16, 32}) c.push_back({SPIN_KERNEL_STREAM, Tile{L, 1, H, th}});
  } else {
    const int f3[5][2] = {{8, 640}, {8, 320}, {16, 576}, {16, 384}, {32, 704}};
    for (auto& f : f3)
      for (int H : {8, 16, 32, 64}) c.push_back({SPIN_KERNEL_FUSED, Tile{L, f[0], H, f[1]}});
    const int t3[4][4] = {{64, 8, 8, 256}, {32, 8, 4, 128}, {128, 8, 4, 256}, {16, 4, 4, 64}};
    for (auto& f : t3) c.push_back({SPIN_KERNEL_TILED, Tile{f[0], f[1], f[2], f[3]}});
    for (int th : {256, 512})
      for (int TY : {4, 8, 16, 32})
        for (int H : {4, 8, 16, 32}) c.push_back({SPIN_KERNEL_STREAM, Tile{L, TY, H, th}});
  }
  c.push_back({SPIN_KERNEL_GENERIC, Tile{0, 0, 0, 256}});
  return c;
}

// ------------------------------------------------------------------ C ABI

extern "C" {

const char* spin_last_error(void) { return g_error.c_str(); }

int spin_last_status(void) { return g_status; }

const char* spin_version(void) { return "spin-gfx950 0.1"; }

int spin_debug_fault_alloc(int64_t after) {
  if (after < -1) return fail(SPIN_EINVAL, "after must be >= -1");
  g_fault_after.store(after);
  return SPIN_OK;
}

int64_t spin_debug_live_allocations(void) { return g_live_blocks.load(); }

void spin_set_allocator(void* (*alloc)(size_t, void*), void (*release)(void*, void*), void* ctx) {
  g_alloc = alloc;
  g_release = release;
  g_ctx = ctx;
}

int spin_threshold_table(double beta, int d, uint64_t* T) {
  if (d != 2 && d != 3) return fail(SPIN_EINVAL, "d must be 2 or 3");
  if (!T) return fail(SPIN_EINVAL, "NULL output");
  if (int rc = check_beta(beta)) return rc;
  const Accept a = make_accept(beta, d);
  for (int i = 0; i <= 2 * d; ++i) T[i] = a.T[i];
  return SPIN_OK;
}

spin_lattice* spin_create_config(const spin_config* cfg) {
  if (!cfg) {
    fail(SPIN_EINVAL, "NULL config");
    return nullptr;
  }
  if (check_shape(cfg->model, cfg->L, cfg->d) != SPIN_OK) return nullptr;
  uint64_t N = 1;
  for (int i = 0; i < cfg->d; ++i) N *= (uint64_t)cfg->L;
  if (cfg->model == SPIN_ISING && cfg->couplings) {
    fail(SPIN_EINVAL, "couplings must be NULL for the Ising model");
    return nullptr;
  }
  if (cfg->model == SPIN_EA_PMJ && cfg->couplings) {
    for (uint64_t i = 0; i < (uint64_t)cfg->d * N; ++i)
      if (cfg->couplings[i] != 1 && cfg->couplings[i] != -1) {
        fail(SPIN_EINVAL, "coupling %llu is %d, must be +-1", (unsigned long long)i, (int)cfg->couplings[i]);
        return nullptr;
      }
  }
  spin_lattice* h = new spin_lattice();
  h->model = cfg->model;
  h->L = cfg->L;
  h->d = cfg->d;
  h->N = N;
  h->buf[0] = h->buf[1] = nullptr;
  h->single = nullptr;
  h->jn = nullptr;
  h->rng = SPIN_RNG_PHILOX;
  h->lcg = nullptr;
  h->schedule = SPIN_SCHEDULE_CHECKERBOARD;
  h->coarse_tile = 0;
  h->hits = 1;
  h->cur = 0;
  h->J = nullptr;
  h->em = nullptr;
  h->seed = cfg->seed;
  h->replica = cfg->replica;
  h->t = 0;
  h->stream = (hipStream_t)cfg->stream;
  h->kernel = SPIN_KERNEL_AUTO;
  h->tile = Tile{0, 0, 0, 0};
  h->mem = Allocator{g_alloc, g_release, g_ctx};
  h->part = nullptr;
  h->part_slots = 0;
  h->buf[0] = (int8_t*)h->mem.get(N);
  h->em = (int64_t*)h->mem.get(2 * sizeof(int64_t));
  if (!h->buf[0] || !h->em) {
    fail(SPIN_ENOMEM, "device allocation of %llu bytes failed", (unsigned long long)N);
    destroy(h);
    return nullptr;
  }
  hipError_t e = hipSuccess;
  if (h->model == SPIN_EA_PMJ) {
    h->J = (int8_t*)h->mem.get((size_t)cfg->d * N);
    if (!h->J) {
      fail(SPIN_ENOMEM, "device allocation of couplings failed");
      destroy(h);
      return nullptr;
    }
    if (cfg->couplings) {
      e = hipMemcpyAsync(h->J, cfg->couplings, (size_t)cfg->d * N, hipMemcpyHostToDevice, h->stream);
      if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
    } else {
      e = launch_couplings(h->J, (uint32_t)h->L, (uint32_t)h->d, N, cfg->coupling_seed,
                           cfg->realisation, h->stream);
    }
    if (e != hipSuccess) {
      hip_fail(e, "couplings");
      destroy(h);
      return nullptr;
    }
  }
  e = launch_init_spins(lat_of(h), h->stream);
  if (e != hipSuccess) {
    hip_fail(e, "hot start");
    destroy(h);
    return nullptr;
  }
  if (prepare_buffers(h) != SPIN_OK) {
    destroy(h);
    return nullptr;
  }
  return h;
}

spin_lattice* spin_create(int model, int L, int d, const int8_t* couplings, uint64_t seed) {
  spin_config c;
  std::memset(&c, 0, sizeof(c));
  c.model = model;
  c.L = L;
  c.d = d;
  c.couplings = couplings;
  c.seed = seed;
  if (model == SPIN_EA_PMJ && !couplings) {
    fail(SPIN_EINVAL, "EA model needs couplings (use spin_create_config to generate them)");
    return nullptr;
  }
  return spin_create_config(&c);
}

void spin_free(spin_lattice* h) { destroy(h); }

int spin_sweep(spin_lattice* h, int n, double beta) { return run_sweeps(h, n, beta, 0, nullptr, nullptr); }

int spin_sweep_record_device(spin_lattice* h, int n, double beta, int every, int64_t* E, int64_t* M) {
  if (every < 1) return fail(SPIN_EINVAL, "every must be >= 1");
  if (n / every > 0 && (!E || !M)) return fail(SPIN_EINVAL, "NULL record arrays");
  return run_sweeps(h, n, beta, every, E, M);
}

int spin_sweep_record(spin_lattice* h, int n, double beta, int every, int64_t* E, int64_t* M) {
  if (!h) return fail(SPIN_EINVAL, "NULL handle");
  if (every < 1) return fail(SPIN_EINVAL, "every must be >= 1");
  if (n < 0) return fail(SPIN_EINVAL, "n must be >= 0");
  const int nrec = n / every;
  if (nrec > 0 && (!E || !M)) return fail(SPIN_EINVAL, "NULL record arrays");
  int64_t* d = nullptr;
  if (nrec > 0) {
    d = (int64_t*)h->mem.get(2 * sizeof(int64_t) * (size_t)nrec);
    if (!d) return fail(SPIN_ENOMEM, "record buffer allocation failed");
  }
  int rc = run_sweeps(h, n, beta, every, d, d ? d + nrec : nullptr);
  if (rc == SPIN_OK && nrec > 0) {
    hipError_t e = hipMemcpyAsync(E, d, sizeof(int64_t) * nrec, hipMemcpyDeviceToHost, h->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(M, d + nrec, sizeof(int64_t) * nrec, hipMemcpyDeviceToHost, h->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
    if (e != hipSuccess) rc = hip_fail(e, "record copy");
  } else if (rc == SPIN_OK) {
    hipError_t e = hipStreamSynchronize(h->stream);
    if (e != hipSuccess) rc = hip_fail(e, "synchronize");
  }
  if (d) {
    (void)hipStreamSynchronize(h->stream);
    h->mem.put(d);
  }
  return rc;
}

int spin_measure(spin_lattice* h, int64_t* E, int64_t* M) {
  if (!h || !E || !M) return fail(SPIN_EINVAL, "NULL argument");
  const uint32_t parts = measure_parts(lat_of(h));
  if (int rc = reserve_parts(h, 1, parts)) return rc;
  hipError_t e = launch_measure(lat_of(h), Record{h->part}, h->stream);
  if (e == hipSuccess)
    e = launch_finalize(h->part, parts, parts, 1, h->em, h->em + 1, e_offset(h), (int64_t)h->N, h->stream);
  int64_t v[2];
  if (e == hipSuccess) e = hipMemcpyAsync(v, h->em, sizeof(v), hipMemcpyDeviceToHost, h->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
  if (e != hipSuccess) return hip_fail(e, "measure");
  *E = v[0];
  *M = v[1];
  return SPIN_OK;
}

int spin_get_spins(const spin_lattice* h, int8_t* out, size_t n) {
  if (!h || !out) return fail(SPIN_EINVAL, "NULL argument");
  if (n != h->N) return fail(SPIN_EINVAL, "n must equal L^d = %llu", (unsigned long long)h->N);
  hipError_t e = hipMemcpyAsync(out, h->buf[h->cur], n, hipMemcpyDeviceToHost, h->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
  if (e != hipSuccess) return hip_fail(e, "get spins");
  return SPIN_OK;
}

int spin_set_spins(spin_lattice* h, const int8_t* in, size_t n) {
  if (!h || !in) return fail(SPIN_EINVAL, "NULL argument");
  if (n != h->N) return fail(SPIN_EINVAL, "n must equal L^d = %llu", (unsigned long long)h->N);
  for (size_t i = 0; i < n; ++i)
    if (in[i] != 1 && in[i] != -1) return fail(SPIN_EINVAL, "spin %zu is %d, must be +-1", i, (int)in[i]);
  hipError_t e = hipMemcpyAsync(h->buf[h->cur], in, n, hipMemcpyHostToDevice, h->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
  if (e != hipSuccess) return hip_fail(e, "set spins");
  return SPIN_OK;
}

int spin_get_couplings(const spin_lattice* h, int8_t* out, size_t n) {
  if (!h || !out) return fail(SPIN_EINVAL, "NULL argument");
  if (!h->J) return fail(SPIN_ESTATE, "the Ising model has no couplings");
  if (n != (size_t)h->d * h->N) return fail(SPIN_EINVAL, "n must equal d*L^d");
  hipError_t e = hipMemcpyAsync(out, h->J, n, hipMemcpyDeviceToHost, h->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
  if (e != hipSuccess) return hip_fail(e, "get couplings");
  return SPIN_OK;
}

uint64_t spin_sweeps_done(const spin_lattice* h) { return h ? h->t : 0; }

int spin_set_sweeps_done(spin_lattice* h, uint64_t t) {
  if (!h) return fail(SPIN_EINVAL, "NULL handle");
  if (t > kMaxSweepIndex) return fail(SPIN_EINVAL, "sweep index must be <= 2^32");
  h->t = t;
  return SPIN_OK;
}

int spin_set_replica(spin_lattice* h, uint32_t replica) {
  if (!h) return fail(SPIN_EINVAL, "NULL handle");
  if (h->rng != SPIN_RNG_PHILOX)
    return fail(SPIN_ESTATE, "the LCG draw modes seed their generators from the replica when the mode is set");
  h->replica = replica;
  return SPIN_OK;
}

int spin_set_stream(spin_lattice* h, void* stream) {
  if (!h) return fail(SPIN_EINVAL, "NULL handle");
  h->stream = (hipStream_t)stream;
  return SPIN_OK;
}

int spin_set_kernel(spin_lattice* h, int kernel, int tile_x, int tile_y, int tile_z, int threads) {
  if (!h) return fail(SPIN_EINVAL, "NULL handle");
  if (kernel < SPIN_KERNEL_AUTO || kernel > SPIN_KERNEL_STREAM) return fail(SPIN_EINVAL, "unknown kernel family %d", kernel);
  const int old_kernel = h->kernel;
  const Tile old_tile = h->tile;
  h->kernel = kernel;
  h->tile = Tile{tile_x, tile_y, tile_z, threads};
  if (kernel != SPIN_KERNEL_AUTO) {
    const Tile t = default_tile(h, kernel);
    if (!family_ok(h, kernel, t)) {
      h->kernel = old_kernel;
      h->tile = old_tile;
      return fail(SPIN_EINVAL, "kernel family %d with tile (%d,%d,%d,%d) cannot run L=%d d=%d model=%d",
                  kernel, t.x, t.y, t.z, t.threads, h->L, h->d, h->model);
    }
  }
  return prepare_buffers(h);
}

int spin_autotune(spin_lattice* h, double beta, int sweeps) {
  if (!h) return fail(SPIN_EINVAL, "NULL handle");
  if (int rc = check_beta(beta)) return rc;
  if (sweeps < 1 || sweeps > 1000) return fail(SPIN_EINVAL, "sweeps must be in 1..1000");
  hipError_t e = hipStreamSynchronize(h->stream);
  if (e != hipSuccess) return hip_fail(e, "autotune");
  spin_config c;
  std::memset(&c, 0, sizeof(c));
  c.model = h->model;
  c.L = h->L;
  c.d = h->d;
  c.coupling_seed = 1;
  c.seed = h->seed;
  c.replica = h->replica;
  c.stream = h->stream;
  spin_lattice* s = spin_create_config(&c);
  if (!s) return SPIN_ENOMEM;
  hipEvent_t e0, e1;
  if (hipEventCreate(&e0) != hipSuccess) {
    destroy(s);
    return hip_fail(hipGetLastError(), "autotune event");
  }
  if (hipEventCreate(&e1) != hipSuccess) {
    (void)hipEventDestroy(e0);
    destroy(s);
    return hip_fail(hipGetLastError(), "autotune event");
  }
  float best_ms = 1e30f;
  Tuned best{SPIN_KERNEL_GENERIC, Tile{0, 0, 0, 256}};
  for (const Tuned& cand : tune_candidates(h)) {
    s->kernel = cand.kernel;
    s->tile = cand.tile;
    if (!family_ok(s, cand.kernel, default_tile(s, cand.kernel))) continue;
    if (run_sweeps(s, 1, beta, 0, nullptr, nullptr) != SPIN_OK) continue;
    if (hipEventRecord(e0, s->stream) != hipSuccess) continue;
    if (run_sweeps(s, sweeps, beta, 0, nullptr, nullptr) != SPIN_OK) continue;
    float ms = 0;
    if (hipEventRecord(e1, s->stream) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
        hipEventElapsedTime(&ms, e0, e1) != hipSuccess)
      continue;
    if (ms < best_ms) {
      best_ms = ms;
      best = Tuned{cand.kernel, default_tile(s, cand.kernel)};
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  destroy(s);
  g_error.clear();
  g_status = SPIN_OK;
  {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    load_tuned_locked();
    g_tuned[std::make_tuple(h->model, h->L, h->d)] = best;
  }
  tune_cache_append("lattice", {h->model, h->L, h->d, best.kernel, best.tile.x, best.tile.y, best.tile.z,
                                best.tile.threads});
  h->kernel = best.kernel;
  h->tile = best.tile;
  if (int rc = prepare_buffers(h)) return rc;
  return best.kernel;
}

int spin_set_schedule(spin_lattice* h, int schedule, int tile, int hits) {
  if (!h) return fail(SPIN_EINVAL, "NULL handle");
  if (schedule == SPIN_SCHEDULE_CHECKERBOARD) {
    h->schedule = schedule;
    h->coarse_tile = 0;
    h->hits = 1;
    return SPIN_OK;
  }
  if (schedule != SPIN_SCHEDULE_COARSE) return fail(SPIN_EINVAL, "unknown schedule %d", schedule);
  if (h->rng != SPIN_RNG_PHILOX) return fail(SPIN_EINVAL, "the coarse schedule draws from Philox only");
  if (hits < 1) return fail(SPIN_EINVAL, "hits must be >= 1 (got %d)", hits);
  if (!coarse_supported(lat_of(h), tile))
    return fail(SPIN_EINVAL, "coarse tile %d cannot run L=%d d=%d (2D: 8, 16, 32, 64; 3D: 8, 16; L/T even)", tile,
                h->L, h->d);
  if ((h->t + 1) * (uint64_t)hits > kMaxSweepIndex) return fail(SPIN_EINVAL, "sweep index times hits past 2^32");
  h->schedule = schedule;
  h->coarse_tile = tile;
  h->hits = hits;
  return prepare_buffers(h);
}

int spin_set_rng(spin_lattice* h, int rng) {
  if (!h) return fail(SPIN_EINVAL, "NULL handle");
  if (rng == SPIN_RNG_PHILOX) {
    h->rng = rng;
    return SPIN_OK;
  }
  if (rng != SPIN_RNG_LCG32_ARRAY && rng != SPIN_RNG_LCG32_DISJOINT && rng != SPIN_RNG_LCG64_DISJOINT)
    return fail(SPIN_EINVAL, "unknown RNG mode %d", rng);
  if (h->J) return fail(SPIN_EINVAL, "the LCG modes run the Ising model only");
  if (h->L % 8 != 0) return fail(SPIN_EINVAL, "the LCG modes need L %% 8 == 0 (got %d)", h->L);
  if (h->schedule != SPIN_SCHEDULE_CHECKERBOARD) return fail(SPIN_EINVAL, "the LCG modes run the checkerboard chain");
  if (!h->lcg) {
    h->lcg = (uint64_t*)h->mem.get(h->N / 8 * sizeof(uint64_t));
    if (!h->lcg) return fail(SPIN_ENOMEM, "LCG state allocation failed");
  }
  hipError_t e = launch_lcg_init(h->lcg, h->N / 8, (uint32_t)rng, h->seed, h->replica, h->stream);
  if (e != hipSuccess) return hip_fail(e, "LCG init launch");
  h->rng = rng;
  return SPIN_OK;
}

int spin_get_rng_state(const spin_lattice* h, uint64_t* out, size_t n) {
  if (!h) return fail(SPIN_EINVAL, "NULL handle");
  if (h->rng == SPIN_RNG_PHILOX || !h->lcg) return fail(SPIN_ESTATE, "no generator state: the RNG is Philox");
  if (n != h->N / 8) return fail(SPIN_EINVAL, "n must equal L^d / 8");
  hipError_t e = hipMemcpyAsync(out, h->lcg, n * sizeof(uint64_t), hipMemcpyDeviceToHost, h->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
  if (e != hipSuccess) return hip_fail(e, "LCG state copy");
  return SPIN_OK;
}

int spin_get_kernel(const spin_lattice* h) {
  if (!h) return fail(SPIN_EINVAL, "NULL handle");
  Tile t;
  return resolve(h, &t);
}

int spin_get_tile(const spin_lattice* h, int* tile_x, int* tile_y, int* tile_z, int* threads) {
  if (!h) return fail(SPIN_EINVAL, "NULL handle");
  Tile t;
  resolve(h, &t);
  if (tile_x) *tile_x = t.x;
  if (tile_y) *tile_y = t.y;
  if (tile_z) *tile_z = t.z;
  if (threads) *threads = t.threads;
  return SPIN_OK;
}

int spin_synchronize(spin_lattice* h) {
  if (!h) return fail(SPIN_EINVAL, "NULL handle");
  hipError_t e = hipStreamSynchronize(h->stream);
  if (e != hipSuccess) return hip_fail(e, "synchronize");
  return SPIN_OK;
}

const int8_t* spin_device_spins(const spin_lattice* h) {
  if (!h) {
    fail(SPIN_EINVAL, "NULL handle");
    return nullptr;
  }
  return h->buf[h->cur];
}

}  // extern "C"
