// spin_batch.cpp -- C ABI of the batched path (include/spin.h, spin_batch_*):
// a pool of lattices (disorder realisations x temperatures, or the jobs of a
// serving loop) advanced together.  Members whose spins fit one workgroup's
// LDS are swept by one persistent launch per class of (dimension, model,
// workgroup size); larger members are advanced by the single-lattice kernels
// on the same stream in the same call.  Members can be added and removed
// between calls; their slots are reused.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <set>
#include <string>
#include <tuple>
#include <vector>

#include "spin.h"
#include "spin_batch.h"
#include "spin_internal.h"

using namespace spin;

static int bfail(int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  std::vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  return set_error(code, buf);
}

static int hfail(hipError_t e, const char* what) {
  return bfail(SPIN_EDEVICE, "%s: %s", what, hipGetErrorString(e));
}

namespace {

template <class T>
bool dmalloc(T** p, size_t bytes) {
  *p = (T*)device_alloc(bytes);
  return *p != nullptr;
}

// Device memory of the members: 256-byte blocks carved from 32 MiB chunks,
// with one free list per block size, so that thousands of small lattices
// (and a serving loop that admits and retires them) do not each cost a
// hipMalloc.  Memory goes back to the device when the batch is freed.
class Slab {
 public:
  static constexpr size_t kChunk = (size_t)32 << 20;

  void* get(size_t bytes) {
    bytes = (bytes + 255) / 256 * 256;
    if (bytes == 0) bytes = 256;
    if (bytes > kChunk / 8) {
      void* p;
      if (!dmalloc(&p, bytes)) return nullptr;
      direct_.insert(p);
      return p;
    }
    auto& fl = free_[bytes];
    if (!fl.empty()) {
      void* p = fl.back();
      fl.pop_back();
      return p;
    }
    if (left_ < bytes) {
      char* c;
      if (!dmalloc(&c, kChunk)) return nullptr;
      chunks_.push_back(c);
      cur_ = c;
      left_ = kChunk;
    }
    void* p = cur_;
    cur_ += bytes;
    left_ -= bytes;
    return p;
  }

  void put(void* p, size_t bytes) {
    if (!p) return;
    auto it = direct_.find(p);
    if (it != direct_.end()) {
      device_free(p);
      direct_.erase(it);
      return;
    }
    bytes = (bytes + 255) / 256 * 256;
    if (bytes == 0) bytes = 256;
    free_[bytes].push_back(p);
  }

  void release() {
    for (char* c : chunks_) device_free(c);
    for (void* p : direct_) device_free(p);
    chunks_.clear();
    direct_.clear();
    free_.clear();
    cur_ = nullptr;
    left_ = 0;
  }

 private:
  std::vector<char*> chunks_;
  std::set<void*> direct_;
  std::map<size_t, std::vector<void*>> free_;
  char* cur_ = nullptr;
  size_t left_ = 0;
};

typedef std::tuple<uint64_t, uint32_t, int, int> CouplingKey;  // seed, realisation, L, d

struct Member {
  bool active = false;
  int L = 0, d = 0, model = 0;
  uint64_t N = 0;
  uint64_t t = 0;                // sweep counter of a resident member (host mirror)
  bool resident = false;         // swept by the persistent batch kernel
  int8_t* spins = nullptr;       // resident: slab block of N bytes
  uint32_t* jn = nullptr;        // resident EA: nibble couplings, d*N/2 bytes
  bool jn_shared = false;        // jn belongs to the shared map under `key`
  CouplingKey key;
  spin_lattice* big = nullptr;   // not resident: a single-lattice handle
  int aux = 0;                   // not resident: index of its stream
};

struct Shared {
  uint32_t* jn;
  int refs;
};

struct Class {
  uint32_t d;
  bool ea;
  uint32_t nt;                   // threads per workgroup
  size_t lds;                    // dynamic LDS of the launch (largest member of the class)
  std::vector<uint32_t> members;
  uint32_t per_cu;               // planned workgroups per CU (smallest over the planned members), 0: none
  bool unplanned;                // some member has no plan
};

size_t rec_count(int n, int every) { return every > 0 ? (n > 0 ? (size_t)(n / every) : 1) : 0; }

// Launch plan of the persistent kernel for one lattice shape (d, model, L):
// workgroup size and workgroups per CU, chosen by spin_batch_autotune (or
// read back from the tuning cache).  Shapes without a plan use the static
// rule: threads by lattice size (batch_threads_for), workgroups per CU as
// many as threads and LDS allow.
struct Plan {
  uint32_t nt;
  uint32_t per_cu;
};
std::mutex g_plan_mu;
std::map<std::tuple<int, int, int>, Plan> g_plan;
bool g_plan_loaded = false;

// Records "batch <arch> d model L threads per_cu ns_per_sweep".
void load_plans_locked() {
  if (g_plan_loaded) return;
  g_plan_loaded = true;
  for (const auto& v : tune_cache_read("batch"))
    if (v.size() >= 5 && batch_threads_ok((uint32_t)v[3]) && v[4] >= 1 && v[4] <= 8)
      g_plan[std::make_tuple((int)v[0], (int)v[1], (int)v[2])] = Plan{(uint32_t)v[3], (uint32_t)v[4]};
}

bool plan_for(int d, int model, int L, Plan* out) {
  std::lock_guard<std::mutex> lk(g_plan_mu);
  load_plans_locked();
  auto it = g_plan.find(std::make_tuple(d, model, L));
  if (it == g_plan.end()) return false;
  *out = it->second;
  return true;
}

// Workgroups of nt threads with `lds` bytes of dynamic LDS that one CU holds.
uint32_t max_per_cu(uint32_t nt, size_t lds) {
  const uint32_t by_threads = 2048u / nt;
  const uint32_t by_lds = (uint32_t)((160 * 1024 - 256) / std::max<size_t>(lds, 1));
  return std::max<uint32_t>(1, std::min(by_threads, by_lds));
}

}  // namespace

struct spin_batch {
  std::vector<Member> m;
  std::vector<int> free_slots;
  std::map<CouplingKey, Shared> shared;
  Slab slab;
  size_t cap = 0;                     // slots the per-slot arrays hold
  BatchLattice* d_lats = nullptr;
  BatchLattice* h_lats = nullptr;     // pinned staging, one entry per slot
  BatchCall* d_calls = nullptr;
  BatchCall* h_calls = nullptr;       // pinned
  uint32_t* d_order = nullptr;
  uint32_t* h_order = nullptr;        // pinned
  hipEvent_t uploaded = nullptr;      // the last upload of h_calls / h_order has been read
  uint32_t* d_counters = nullptr;     // one queue counter per class
  int64_t* d_rec = nullptr;
  size_t rec_cap = 0;
  hipStream_t stream = nullptr;
  // Larger members run on these streams (members round-robin), forked from
  // `stream` at the start of a call and joined back at its end, so that they
  // overlap each other and the persistent launch.
  static constexpr int kAux = 4;
  hipStream_t aux[kAux] = {};
  hipEvent_t fork = nullptr;
  hipEvent_t joined[kAux] = {};
  int next_aux = 0;
  int num_cu = 256;
  int wgs_override = 0;               // 0: by occupancy
  uint32_t force_nt = 0;              // autotuner's scratch pools: this launch shape for every class
  uint32_t force_per_cu = 0;
  // The tables of the last upload (a call that repeats them uploads nothing, which is what lets
  // a call be captured into a graph) and whether a call has been captured: then any replay may
  // have advanced the resident members' device sweep counters, and the host mirrors are read
  // back from the device whenever they are needed.
  std::vector<BatchCall> last_calls;
  std::vector<uint32_t> last_order;
  bool t_stale = false;
};

// Whether work enqueued on the pool's stream is being captured into a graph.
static bool capturing(const spin_batch* b) {
  if (!b->stream) return false;  // the null stream is never captured here
  hipStreamCaptureStatus st = hipStreamCaptureStatusNone;
  if (hipStreamIsCapturing(b->stream, &st) != hipSuccess) {
    (void)hipGetLastError();
    return false;
  }
  return st == hipStreamCaptureStatusActive;
}

// Bring the host mirrors of the resident members' sweep counters up to the
// device copies (a pool with a captured call: graph replays advance them
// without the host's knowledge).  Synchronises.
static int refresh_counters(spin_batch* b) {
  if (!b->t_stale) return SPIN_OK;
  const size_t S = b->m.size();
  std::vector<BatchLattice> tmp(S);
  hipError_t e = S ? hipMemcpyAsync(tmp.data(), b->d_lats, sizeof(BatchLattice) * S, hipMemcpyDeviceToHost, b->stream)
                   : hipSuccess;
  if (e == hipSuccess) e = hipStreamSynchronize(b->stream);
  if (e != hipSuccess) return hfail(e, "batch counter refresh");
  for (size_t i = 0; i < S; ++i)
    if (b->m[i].active && b->m[i].resident) b->m[i].t = tmp[i].t;
  return SPIN_OK;
}

static void free_member(spin_batch* b, Member& mb) {
  if (mb.big) spin_free(mb.big);
  if (mb.spins) b->slab.put(mb.spins, mb.N);
  if (mb.jn) {
    const size_t jbytes = (size_t)mb.d * mb.N / 2;
    if (mb.jn_shared) {
      auto it = b->shared.find(mb.key);
      if (it != b->shared.end() && --it->second.refs == 0) {
        b->slab.put(it->second.jn, jbytes);
        b->shared.erase(it);
      }
    } else {
      b->slab.put(mb.jn, jbytes);
    }
  }
  mb = Member();
}

static void batch_destroy(spin_batch* b) {
  if (!b) return;
  (void)hipStreamSynchronize(b->stream);
  for (Member& mb : b->m)
    if (mb.active || mb.big) free_member(b, mb);
  b->slab.release();
  device_free(b->d_lats);
  device_free(b->d_calls);
  device_free(b->d_order);
  device_free(b->d_counters);
  device_free(b->d_rec);
  if (b->h_lats) (void)hipHostFree(b->h_lats);
  if (b->h_calls) (void)hipHostFree(b->h_calls);
  if (b->h_order) (void)hipHostFree(b->h_order);
  if (b->uploaded) (void)hipEventDestroy(b->uploaded);
  if (b->fork) (void)hipEventDestroy(b->fork);
  for (int k = 0; k < spin_batch::kAux; ++k) {
    if (b->joined[k]) (void)hipEventDestroy(b->joined[k]);
    if (b->aux[k]) {
      (void)hipStreamSynchronize(b->aux[k]);
      (void)hipStreamDestroy(b->aux[k]);
    }
  }
  delete b;
}

// Make the per-slot device and pinned arrays hold at least n slots.
static int ensure_capacity(spin_batch* b, size_t n) {
  if (n <= b->cap) return SPIN_OK;
  const size_t cap = std::max<size_t>({n, 2 * b->cap, 64});
  hipError_t e = hipStreamSynchronize(b->stream);
  if (e != hipSuccess) return hfail(e, "batch grow");
  BatchLattice* d_lats = nullptr;
  BatchCall* d_calls = nullptr;
  uint32_t* d_order = nullptr;
  BatchLattice* h_lats = nullptr;
  BatchCall* h_calls = nullptr;
  uint32_t* h_order = nullptr;
  bool ok = dmalloc(&d_lats, sizeof(BatchLattice) * cap) && dmalloc(&d_calls, sizeof(BatchCall) * cap) &&
            dmalloc(&d_order, sizeof(uint32_t) * cap);
  ok = ok && hipHostMalloc((void**)&h_lats, sizeof(BatchLattice) * cap, hipHostMallocDefault) == hipSuccess;
  ok = ok && hipHostMalloc((void**)&h_calls, sizeof(BatchCall) * cap, hipHostMallocDefault) == hipSuccess;
  ok = ok && hipHostMalloc((void**)&h_order, sizeof(uint32_t) * cap, hipHostMallocDefault) == hipSuccess;
  if (ok && b->cap) {
    e = hipMemcpyAsync(d_lats, b->d_lats, sizeof(BatchLattice) * b->cap, hipMemcpyDeviceToDevice, b->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(b->stream);
    ok = e == hipSuccess;
  }
  if (!ok) {
    (void)hipGetLastError();
    device_free(d_lats);
    device_free(d_calls);
    device_free(d_order);
    if (h_lats) (void)hipHostFree(h_lats);
    if (h_calls) (void)hipHostFree(h_calls);
    if (h_order) (void)hipHostFree(h_order);
    return bfail(SPIN_ENOMEM, "batch slot arrays (%zu slots)", cap);
  }
  device_free(b->d_lats);
  device_free(b->d_calls);
  device_free(b->d_order);
  if (b->h_lats) (void)hipHostFree(b->h_lats);
  if (b->h_calls) (void)hipHostFree(b->h_calls);
  if (b->h_order) (void)hipHostFree(b->h_order);
  b->d_lats = d_lats;
  b->d_calls = d_calls;
  b->d_order = d_order;
  b->h_lats = h_lats;
  b->h_calls = h_calls;
  b->h_order = h_order;
  b->cap = cap;
  b->last_calls.clear();  // the new device tables hold nothing yet
  b->last_order.clear();
  return SPIN_OK;
}

static int check_desc(const spin_desc& s) {
  if (s.model != SPIN_ISING && s.model != SPIN_EA_PMJ) return bfail(SPIN_EINVAL, "model must be 0 or 1");
  if (s.d != 2 && s.d != 3) return bfail(SPIN_EINVAL, "d must be 2 or 3 (got %d)", s.d);
  if (s.L < 4 || s.L % 2 != 0) return bfail(SPIN_EINVAL, "L must be even and >= 4 (got %d)", s.L);
  uint64_t N = 1;
  for (int k = 0; k < s.d; ++k) N *= (uint64_t)s.L;
  if (N / 8 >= ((uint64_t)1 << 32)) return bfail(SPIN_EINVAL, "L^d/8 must be < 2^32");
  if (s.model == SPIN_ISING && s.couplings) return bfail(SPIN_EINVAL, "couplings must be NULL for the Ising model");
  if (s.couplings)
    for (uint64_t k = 0; k < (uint64_t)s.d * N; ++k)
      if (s.couplings[k] != 1 && s.couplings[k] != -1)
        return bfail(SPIN_EINVAL, "coupling %llu is not +-1", (unsigned long long)k);
  return SPIN_OK;
}

// Set up a member in slot `slot` (already sized); the device copy of a
// resident member's BatchLattice is uploaded from h_lats[slot] when `upload`.
static int init_member(spin_batch* b, int slot, const spin_desc& s, bool upload) {
  Member& mb = b->m[slot];
  mb = Member();
  mb.L = s.L;
  mb.d = s.d;
  mb.model = s.model;
  mb.N = 1;
  for (int k = 0; k < s.d; ++k) mb.N *= (uint64_t)s.L;
  mb.resident = batch_fits((uint32_t)s.L, (uint32_t)s.d);
  if (!mb.resident) {
    spin_config c;
    std::memset(&c, 0, sizeof(c));
    c.model = s.model;
    c.L = s.L;
    c.d = s.d;
    c.couplings = s.couplings;
    c.coupling_seed = s.coupling_seed;
    c.realisation = s.realisation;
    c.seed = s.seed;
    c.replica = s.replica;
    mb.aux = b->next_aux;
    b->next_aux = (b->next_aux + 1) % spin_batch::kAux;
    c.stream = b->aux[mb.aux];
    mb.big = spin_create_config(&c);
    if (!mb.big) return spin_last_status();  // status and message set by spin_create_config
    mb.active = true;
    return SPIN_OK;
  }
  mb.spins = (int8_t*)b->slab.get(mb.N);
  if (!mb.spins) return bfail(SPIN_ENOMEM, "spin allocation failed");
  BatchLattice& bl = b->h_lats[slot];
  bl.spins = mb.spins;
  bl.Jn = nullptr;
  bl.L = (uint32_t)s.L;
  bl.d = (uint32_t)s.d;
  bl.replica = s.replica;
  bl.t = 0;
  bl.keys = make_round_keys(s.seed);
  Lat lat;
  lat.spins = mb.spins;
  lat.J = nullptr;
  lat.L = bl.L;
  lat.d = bl.d;
  lat.N = mb.N;
  lat.replica = s.replica;
  lat.keys = bl.keys;
  hipError_t e = launch_init_spins(lat, b->stream);
  if (e != hipSuccess) return hfail(e, "hot start");
  if (s.model == SPIN_EA_PMJ) {
    const uint64_t nbytes = (uint64_t)s.d * mb.N;
    if (!s.couplings) {
      mb.key = std::make_tuple(s.coupling_seed, s.realisation, s.L, s.d);
      auto it = b->shared.find(mb.key);
      if (it == b->shared.end()) {
        uint32_t* jn = (uint32_t*)b->slab.get(nbytes / 2);
        if (!jn) return bfail(SPIN_ENOMEM, "coupling allocation failed");
        e = launch_couplings_nibble(jn, mb.N, (uint32_t)s.d, s.coupling_seed, s.realisation, b->stream);
        if (e != hipSuccess) {
          b->slab.put(jn, nbytes / 2);
          return hfail(e, "coupling generation");
        }
        it = b->shared.emplace(mb.key, Shared{jn, 0}).first;
      }
      ++it->second.refs;
      mb.jn = it->second.jn;
      mb.jn_shared = true;
    } else {
      mb.jn = (uint32_t*)b->slab.get(nbytes / 2);
      if (!mb.jn) return bfail(SPIN_ENOMEM, "coupling allocation failed");
      int8_t* tmp;
      if (!dmalloc(&tmp, nbytes)) return bfail(SPIN_ENOMEM, "coupling staging allocation failed");
      e = hipMemcpyAsync(tmp, s.couplings, nbytes, hipMemcpyHostToDevice, b->stream);
      if (e == hipSuccess) e = launch_pack_nibbles(tmp, mb.jn, nbytes, b->stream);
      if (e == hipSuccess) e = hipStreamSynchronize(b->stream);
      device_free(tmp);
      if (e != hipSuccess) return hfail(e, "coupling upload");
    }
    bl.Jn = mb.jn;
  }
  mb.active = true;
  if (upload) {
    e = hipMemcpyAsync(b->d_lats + slot, b->h_lats + slot, sizeof(BatchLattice), hipMemcpyHostToDevice, b->stream);
    if (e != hipSuccess) return hfail(e, "batch lattice upload");
  }
  return SPIN_OK;
}

// Take a slot (a free one first) and set the member up in it.  Slot index or
// a negative status.
static int add_member(spin_batch* b, const spin_desc& s, bool upload) {
  if (int rc = check_desc(s)) return rc;
  int slot;
  bool reused = false;
  if (!b->free_slots.empty()) {
    slot = b->free_slots.back();
    b->free_slots.pop_back();
    reused = true;
  } else {
    if (int rc = ensure_capacity(b, b->m.size() + 1)) return rc;
    slot = (int)b->m.size();
    b->m.push_back(Member());
  }
  const int rc = init_member(b, slot, s, upload);
  if (rc != SPIN_OK) {
    // init_member may have queued work on memory it took: let it drain
    (void)hipStreamSynchronize(b->stream);
    free_member(b, b->m[slot]);
    if (reused || slot + 1 != (int)b->m.size())
      b->free_slots.push_back(slot);
    else
      b->m.pop_back();
    return rc;
  }
  return slot;
}

// Make later work on the pool's stream wait for what the calls enqueued on
// the auxiliary streams marked in `used`.
static int join_aux(spin_batch* b, const bool* used) {
  for (int k = 0; k < spin_batch::kAux; ++k) {
    if (!used[k]) continue;
    hipError_t e = hipEventRecord(b->joined[k], b->aux[k]);
    if (e == hipSuccess) e = hipStreamWaitEvent(b->stream, b->joined[k], 0);
    if (e != hipSuccess) return hfail(e, "batch join");
  }
  return SPIN_OK;
}

static bool slot_ok(const spin_batch* b, int i) { return b && i >= 0 && i < (int)b->m.size() && b->m[i].active; }

// Advance slot i by n[i] sweeps at beta[i]; slot i's records go to device
// arrays dE, dM at the offset sum_{j<i} of the earlier slots' counts.
static int batch_run(spin_batch* b, const int* n, const double* beta, int every, int64_t* dE, int64_t* dM) {
  if (!b) return bfail(SPIN_EINVAL, "NULL batch");
  if (!n || !beta) return bfail(SPIN_EINVAL, "NULL n or beta array");
  if (every < 0) return bfail(SPIN_EINVAL, "every must be >= 0");
  const int S = (int)b->m.size();
  const bool cap = capturing(b);
  if (!cap)
    if (int rc = refresh_counters(b)) return rc;
  for (int i = 0; i < S; ++i) {
    const Member& mb = b->m[i];
    if (!mb.active) {
      if (n[i] != 0) return bfail(SPIN_EINVAL, "slot %d holds no lattice but n[%d] = %d", i, i, n[i]);
      continue;
    }
    if (cap && !mb.resident && (n[i] > 0 || rec_count(n[i], every)))
      return bfail(SPIN_ESTATE, "slot %d: a captured pool call can sweep only members held in LDS", i);
    if (n[i] < 0) return bfail(SPIN_EINVAL, "slot %d: n must be >= 0", i);
    if (std::isnan(beta[i]) || beta[i] < 0) return bfail(SPIN_EINVAL, "slot %d: bad beta %g", i, beta[i]);
    const uint64_t t = mb.big ? spin_sweeps_done(mb.big) : mb.t;
    if (t + (uint64_t)n[i] > ((uint64_t)1 << 32)) return bfail(SPIN_EINVAL, "slot %d: sweep index past 2^32", i);
    if (rec_count(n[i], every) && (!dE || !dM)) return bfail(SPIN_EINVAL, "NULL record arrays");
  }
  // the previous call's uploads must have been read before the host buffers change (a captured
  // call uploads nothing and changes nothing the previous upload reads)
  hipError_t e = cap ? hipSuccess : hipEventSynchronize(b->uploaded);
  if (e != hipSuccess) return hfail(e, "batch upload wait");
  std::vector<BatchCall> saved;
  if (cap) saved.assign(b->h_calls, b->h_calls + S);
  size_t rec = 0;
  std::map<std::tuple<int, int, uint32_t>, size_t> cls_index;
  std::vector<Class> classes;
  std::vector<std::pair<int, size_t>> bigs;  // slot, record offset
  for (int i = 0; i < S; ++i) {
    const Member& mb = b->m[i];
    if (!mb.active) continue;
    const size_t nr = rec_count(n[i], every);
    if (!mb.resident) {
      if (n[i] > 0 || nr) bigs.push_back({i, rec});
      rec += nr;
      continue;
    }
    BatchCall& c = b->h_calls[i];
    const Accept a = make_accept(beta[i], mb.d);
    c.n = (uint32_t)n[i];
    c.every = nr ? (uint32_t)every : 0u;
    c.never4 = 4u * a.never_level;
    for (int k = 0; k < 8; ++k) c.bound[k] = a.bound[k];
    c.E = nr ? dE + rec : nullptr;
    c.M = nr ? dM + rec : nullptr;
    rec += nr;
    if (c.n == 0 && c.every == 0) continue;
    Plan pl{0, 0};
    const bool planned = b->force_nt ? (pl = Plan{b->force_nt, b->force_per_cu}, true)
                                     : plan_for(mb.d, mb.model, mb.L, &pl);
    const uint32_t nt = planned ? pl.nt : batch_threads_for((uint32_t)mb.L, (uint32_t)mb.d);
    const auto key = std::make_tuple(mb.d, mb.model, nt);
    auto it = cls_index.find(key);
    if (it == cls_index.end()) {
      it = cls_index.emplace(key, classes.size()).first;
      classes.push_back(Class{(uint32_t)mb.d, mb.model == SPIN_EA_PMJ, nt, 0, {}, 0, false});
    }
    Class& cl = classes[it->second];
    cl.members.push_back((uint32_t)i);
    cl.lds = std::max(cl.lds, batch_lds_bytes((uint32_t)mb.L, (uint32_t)mb.d));
    if (planned)
      cl.per_cu = cl.per_cu ? std::min(cl.per_cu, pl.per_cu) : pl.per_cu;
    else
      cl.unplanned = true;
  }
  // members too large for one workgroup: the single-lattice kernels on their own streams, forked
  // before the persistent launches so that both run at once
  bool used[spin_batch::kAux] = {};
  if (!bigs.empty()) {
    e = hipEventRecord(b->fork, b->stream);
    if (e != hipSuccess) return hfail(e, "batch fork");
  }
  for (const auto& bg : bigs) {
    const int i = bg.first;
    const int k = b->m[i].aux;
    if (!used[k]) {
      e = hipStreamWaitEvent(b->aux[k], b->fork, 0);
      if (e != hipSuccess) return hfail(e, "batch fork wait");
      used[k] = true;
    }
    spin_lattice* h = b->m[i].big;
    int rc;
    if (n[i] > 0 && rec_count(n[i], every))
      rc = spin_sweep_record_device(h, n[i], beta[i], every, dE + bg.second, dM + bg.second);
    else if (n[i] > 0)
      rc = spin_sweep(h, n[i], beta[i]);
    else
      rc = record_device(h, dE + bg.second, dM + bg.second);
    if (rc != SPIN_OK) {
      join_aux(b, used);
      return rc;
    }
  }
  // task order: per class, largest work first (longest-processing-time order)
  uint32_t norder = 0;
  std::vector<std::pair<uint32_t, uint32_t>> ranges;
  for (Class& cl : classes) {
    const uint32_t start = norder;
    std::stable_sort(cl.members.begin(), cl.members.end(), [&](uint32_t x, uint32_t y) {
      return b->m[x].N * (uint64_t)b->h_calls[x].n > b->m[y].N * (uint64_t)b->h_calls[y].n;
    });
    for (uint32_t i : cl.members) b->h_order[norder++] = i;
    ranges.push_back({start, (uint32_t)cl.members.size()});
  }
  // upload the tables unless the device already holds them (same calls for the resident members,
  // same task order)
  bool same = norder && norder == b->last_order.size() && b->last_calls.size() == (size_t)S &&
              std::memcmp(b->last_order.data(), b->h_order, sizeof(uint32_t) * norder) == 0;
  for (int i = 0; same && i < S; ++i)
    if (b->m[i].active && b->m[i].resident)
      same = std::memcmp(&b->last_calls[i], &b->h_calls[i], sizeof(BatchCall)) == 0;
  if (norder && !same && cap) {
    std::copy(saved.begin(), saved.end(), b->h_calls);
    return bfail(SPIN_ESTATE,
                 "a captured pool call must repeat the arguments of the pool's previous call (make that call "
                 "once uncaptured first)");
  }
  if (norder && !same) {
    e = hipMemcpyAsync(b->d_calls, b->h_calls, sizeof(BatchCall) * S, hipMemcpyHostToDevice, b->stream);
    if (e == hipSuccess)
      e = hipMemcpyAsync(b->d_order, b->h_order, sizeof(uint32_t) * norder, hipMemcpyHostToDevice, b->stream);
    if (e == hipSuccess) e = hipEventRecord(b->uploaded, b->stream);
    if (e != hipSuccess) {
      b->last_calls.clear();
      b->last_order.clear();
      join_aux(b, used);
      return hfail(e, "batch upload");
    }
    b->last_calls.assign(b->h_calls, b->h_calls + S);
    b->last_order.assign(b->h_order, b->h_order + norder);
  }
  for (size_t k = 0; k < classes.size(); ++k) {
    const Class& cl = classes[k];
    const uint32_t ntasks = ranges[k].second;
    // workgroups per CU: the override, else the plan when every member has one (never more than
    // the class's LDS allows), else as many as threads and LDS allow
    uint32_t per_cu = max_per_cu(cl.nt, cl.lds);
    if (cl.per_cu && !cl.unplanned) per_cu = std::min(per_cu, cl.per_cu);
    if (b->wgs_override > 0) per_cu = (uint32_t)b->wgs_override;
    const uint32_t grid = std::min<uint32_t>(ntasks, per_cu * (uint32_t)b->num_cu);
    e = launch_batch(cl.d, cl.ea, cl.nt, b->d_lats, b->d_calls, b->d_order + ranges[k].first, ntasks,
                     b->d_counters + k, cl.lds, grid, b->stream);
    if (e != hipSuccess) {
      join_aux(b, used);
      return hfail(e, "batch launch");
    }
  }
  // join: later work on the pool's stream waits for the larger members
  if (int rc = join_aux(b, used)) return rc;
  if (cap) {
    b->t_stale = true;  // every replay advances the device counters
  } else {
    for (int i = 0; i < S; ++i)
      if (b->m[i].active && b->m[i].resident) b->m[i].t += (uint64_t)n[i];
  }
  return SPIN_OK;
}

static size_t record_total(const spin_batch* b, const int* n, int every) {
  size_t r = 0;
  for (size_t i = 0; i < b->m.size(); ++i)
    if (b->m[i].active) r += rec_count(n[i], every);
  return r;
}

extern "C" {

spin_batch* spin_batch_create(int count, const spin_desc* descs, void* stream) {
  if (count < 0 || (count > 0 && !descs)) {
    bfail(SPIN_EINVAL, "count must be >= 0 and descs non-NULL");
    return nullptr;
  }
  spin_batch* b = new spin_batch();
  b->stream = (hipStream_t)stream;
  int dev = 0;
  (void)hipGetDevice(&dev);
  (void)hipDeviceGetAttribute(&b->num_cu, hipDeviceAttributeMultiprocessorCount, dev);
  bool ok = hipEventCreateWithFlags(&b->uploaded, hipEventDisableTiming) == hipSuccess &&
            hipEventCreateWithFlags(&b->fork, hipEventDisableTiming) == hipSuccess;
  for (int k = 0; ok && k < spin_batch::kAux; ++k)
    ok = hipStreamCreateWithFlags(&b->aux[k], hipStreamNonBlocking) == hipSuccess &&
         hipEventCreateWithFlags(&b->joined[k], hipEventDisableTiming) == hipSuccess;
  if (!ok || !dmalloc(&b->d_counters, sizeof(uint32_t) * 64)) {
    (void)hipGetLastError();
    bfail(SPIN_ENOMEM, "batch allocation failed");
    batch_destroy(b);
    return nullptr;
  }
  if (ensure_capacity(b, (size_t)std::max(count, 1)) != SPIN_OK) {
    batch_destroy(b);
    return nullptr;
  }
  for (int i = 0; i < count; ++i) {
    const int rc = add_member(b, descs[i], false);
    if (rc < 0) {
      const std::string msg = "lattice " + std::to_string(i) + ": " + spin_last_error();
      batch_destroy(b);
      set_error(rc, msg.c_str());
      return nullptr;
    }
  }
  hipError_t e = hipSuccess;
  if (count)
    e = hipMemcpyAsync(b->d_lats, b->h_lats, sizeof(BatchLattice) * count, hipMemcpyHostToDevice, b->stream);
  for (int k = 0; k < spin_batch::kAux && e == hipSuccess; ++k) e = hipStreamSynchronize(b->aux[k]);
  if (e == hipSuccess) e = hipStreamSynchronize(b->stream);
  if (e != hipSuccess) {
    hfail(e, "batch setup");
    batch_destroy(b);
    return nullptr;
  }
  return b;
}

void spin_batch_free(spin_batch* b) { batch_destroy(b); }

int spin_batch_size(const spin_batch* b) { return b ? (int)b->m.size() : 0; }

int spin_batch_add(spin_batch* b, const spin_desc* desc) {
  if (!b || !desc) return bfail(SPIN_EINVAL, "NULL argument");
  return add_member(b, *desc, true);
}

int spin_batch_remove(spin_batch* b, int i) {
  if (!slot_ok(b, i)) return bfail(SPIN_EINVAL, "slot %d holds no lattice", i);
  // queued sweeps may still read the member's memory
  hipError_t e = hipStreamSynchronize(b->stream);
  if (e != hipSuccess) return hfail(e, "batch remove");
  free_member(b, b->m[i]);
  b->free_slots.push_back(i);
  return SPIN_OK;
}

int spin_batch_is_member(const spin_batch* b, int i) { return slot_ok(b, i) ? 1 : 0; }

uint64_t spin_batch_footprint(const spin_batch* b, int i) {
  if (!slot_ok(b, i)) return 0;
  const Member& mb = b->m[i];
  // spins, ping-pong copy, and for the glass the int8 couplings and their nibble-packed copy
  if (mb.big) return mb.N * 2 + (mb.model == SPIN_EA_PMJ ? (uint64_t)mb.d * mb.N + (uint64_t)mb.d * mb.N / 2 : 0);
  return mb.N + (mb.model == SPIN_EA_PMJ ? (uint64_t)mb.d * mb.N / 2 : 0);
}

int spin_batch_sweep_device(spin_batch* b, const int* n, const double* beta, int every, int64_t* E, int64_t* M) {
  return batch_run(b, n, beta, every, E, M);
}

int spin_batch_sweep(spin_batch* b, const int* n, const double* beta, int every, int64_t* E, int64_t* M) {
  if (!b) return bfail(SPIN_EINVAL, "NULL batch");
  if (!n) return bfail(SPIN_EINVAL, "NULL n array");
  if (every < 0) return bfail(SPIN_EINVAL, "every must be >= 0");
  const size_t nr = record_total(b, n, every);
  if (nr && (!E || !M)) return bfail(SPIN_EINVAL, "NULL record arrays");
  if (nr > b->rec_cap) {
    (void)hipStreamSynchronize(b->stream);
    device_free(b->d_rec);
    if (!dmalloc(&b->d_rec, 2 * nr * sizeof(int64_t))) {
      b->rec_cap = 0;
      return bfail(SPIN_ENOMEM, "record buffer allocation failed");
    }
    b->rec_cap = nr;
  }
  int rc = batch_run(b, n, beta, every, nr ? b->d_rec : nullptr, nr ? b->d_rec + nr : nullptr);
  if (rc != SPIN_OK) return rc;
  hipError_t e = hipSuccess;
  if (nr) {
    e = hipMemcpyAsync(E, b->d_rec, nr * sizeof(int64_t), hipMemcpyDeviceToHost, b->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(M, b->d_rec + nr, nr * sizeof(int64_t), hipMemcpyDeviceToHost, b->stream);
  }
  if (e == hipSuccess) e = hipStreamSynchronize(b->stream);
  if (e != hipSuccess) return hfail(e, "batch record copy");
  return SPIN_OK;
}

int spin_batch_measure(spin_batch* b, int64_t* E, int64_t* M) {
  if (!b || !E || !M) return bfail(SPIN_EINVAL, "NULL argument");
  const size_t S = b->m.size();
  std::vector<int> zero(S, 0);
  std::vector<double> beta(S, 0.0);
  std::vector<int64_t> e(S + 1), m(S + 1);
  int rc = spin_batch_sweep(b, zero.data(), beta.data(), 1, e.data(), m.data());
  if (rc != SPIN_OK) return rc;
  size_t k = 0;
  for (size_t i = 0; i < S; ++i) {
    if (b->m[i].active) {
      E[i] = e[k];
      M[i] = m[k];
      ++k;
    } else {
      E[i] = M[i] = 0;
    }
  }
  return SPIN_OK;
}

int spin_batch_get_spins(const spin_batch* b, int i, int8_t* out, size_t n) {
  if (!slot_ok(b, i) || !out) return bfail(SPIN_EINVAL, "slot %d holds no lattice, or NULL output", i);
  const Member& mb = b->m[i];
  if (n != mb.N) return bfail(SPIN_EINVAL, "n must equal L^d of slot %d", i);
  if (mb.big) return spin_get_spins(mb.big, out, n);
  hipError_t e = hipMemcpyAsync(out, mb.spins, n, hipMemcpyDeviceToHost, b->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(b->stream);
  if (e != hipSuccess) return hfail(e, "batch get spins");
  return SPIN_OK;
}

int spin_batch_set_spins(spin_batch* b, int i, const int8_t* in, size_t n) {
  if (!slot_ok(b, i) || !in) return bfail(SPIN_EINVAL, "slot %d holds no lattice, or NULL input", i);
  const Member& mb = b->m[i];
  if (n != mb.N) return bfail(SPIN_EINVAL, "n must equal L^d of slot %d", i);
  if (mb.big) return spin_set_spins(mb.big, in, n);
  for (size_t k = 0; k < n; ++k)
    if (in[k] != 1 && in[k] != -1) return bfail(SPIN_EINVAL, "spin %zu is not +-1", k);
  hipError_t e = hipMemcpyAsync(mb.spins, in, n, hipMemcpyHostToDevice, b->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(b->stream);
  if (e != hipSuccess) return hfail(e, "batch set spins");
  return SPIN_OK;
}

uint64_t spin_batch_sweeps_done(const spin_batch* b, int i) {
  if (!slot_ok(b, i)) return 0;
  if (b->t_stale && !capturing(b) && refresh_counters(const_cast<spin_batch*>(b)) != SPIN_OK) return 0;
  return b->m[i].big ? spin_sweeps_done(b->m[i].big) : b->m[i].t;
}

int spin_batch_set_workgroups_per_cu(spin_batch* b, int wgs) {
  if (!b) return bfail(SPIN_EINVAL, "NULL batch");
  if (wgs < 0 || wgs > 8) return bfail(SPIN_EINVAL, "workgroups per CU must be in 0..8");
  b->wgs_override = wgs;
  return SPIN_OK;
}

int spin_batch_autotune(spin_batch* b, double beta, int sweeps) {
  if (!b) return bfail(SPIN_EINVAL, "NULL batch");
  if (std::isnan(beta) || beta < 0) return bfail(SPIN_EINVAL, "bad beta %g", beta);
  if (sweeps < 1 || sweeps > 1000) return bfail(SPIN_EINVAL, "sweeps must be in 1..1000");
  if (int rc = refresh_counters(b)) return rc;
  std::map<std::tuple<int, int, int>, int> shapes;  // (d, model, L) -> members of the pool
  for (const Member& mb : b->m)
    if (mb.active && mb.resident) ++shapes[std::make_tuple(mb.d, mb.model, mb.L)];
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
    if (e0) (void)hipEventDestroy(e0);
    return hfail(hipGetLastError(), "autotune events");
  }
  int tuned = 0, rc = SPIN_OK;
  for (const auto& sh : shapes) {
    const int d = std::get<0>(sh.first), model = std::get<1>(sh.first), L = std::get<2>(sh.first);
    // scratch lattices of this shape, as many as the pool holds (at most four per CU): the launch
    // sees the same number of tasks per CU as the pool's own calls
    const int K = std::min(sh.second, 4 * b->num_cu);
    std::vector<spin_desc> descs(K);
    for (int r = 0; r < K; ++r) {
      descs[r].model = model;
      descs[r].L = L;
      descs[r].d = d;
      descs[r].couplings = nullptr;
      descs[r].coupling_seed = 0x5EED00000001ull;
      descs[r].realisation = (uint32_t)(r % 64);
      descs[r].seed = 0x5EED00000000ull;
      descs[r].replica = (uint32_t)r;
    }
    const size_t lds = batch_lds_bytes((uint32_t)L, (uint32_t)d);
    struct Cand {
      uint32_t nt, per_cu;
      float ms;
      uint64_t hash;
    };
    std::vector<Cand> cands;
    for (uint32_t nt : {256u, 512u, 576u, 1024u}) {
      if ((uint32_t)L / 8 > nt) continue;
      for (uint32_t pc = 1; pc <= max_per_cu(nt, lds); ++pc) cands.push_back(Cand{nt, pc, 3.4e38f, 0});
    }
    // every candidate is timed twice, the second round after all the first ones, and keeps its
    // faster time: a GPU that is still raising its clock, or a passing slow launch, favours no shape
    for (int round = 0; round < 2 && rc == SPIN_OK; ++round)
    for (Cand& c : cands) {
      spin_batch* t = spin_batch_create(K, descs.data(), b->stream);
      if (!t) {
        rc = spin_last_status();
        break;
      }
      t->force_nt = c.nt;
      t->force_per_cu = c.per_cu;
      std::vector<int> n(K, 1);
      std::vector<double> bt(K, beta);
      rc = batch_run(t, n.data(), bt.data(), 0, nullptr, nullptr);  // warm-up sweep
      std::fill(n.begin(), n.end(), sweeps);
      hipError_t e = rc == SPIN_OK ? hipEventRecord(e0, b->stream) : hipSuccess;
      if (rc == SPIN_OK && e == hipSuccess) rc = batch_run(t, n.data(), bt.data(), 0, nullptr, nullptr);
      if (rc == SPIN_OK && e == hipSuccess) e = hipEventRecord(e1, b->stream);
      if (rc == SPIN_OK && e == hipSuccess) e = hipEventSynchronize(e1);
      float ms = 0.f;
      if (rc == SPIN_OK && e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
      if (rc == SPIN_OK && e != hipSuccess) rc = hfail(e, "autotune timing");
      if (rc == SPIN_OK) c.ms = std::min(c.ms, ms);
      // FNV-1a over the final spins of three members: every candidate must give the same bits
      uint64_t h = 1469598103934665603ull;
      std::vector<int8_t> sp;
      for (int i : {0, K / 2, K - 1}) {
        if (rc != SPIN_OK) break;
        sp.resize(t->m[i].N);
        rc = spin_batch_get_spins(t, i, sp.data(), sp.size());
        for (int8_t v : sp) h = (h ^ (uint8_t)v) * 1099511628211ull;
      }
      c.hash = h;
      spin_batch_free(t);
      if (rc != SPIN_OK) break;
    }
    if (rc != SPIN_OK) break;
    const Cand* best = nullptr;
    const Cand* rule = nullptr;  // the static rule's shape
    const uint32_t rule_nt = batch_threads_for((uint32_t)L, (uint32_t)d);
    for (const Cand& c : cands) {
      if (c.hash != cands[0].hash) {
        rc = bfail(SPIN_EDEVICE, "autotune: launch shapes (%u, %u) and (%u, %u) gave different spins for L=%d d=%d",
                   c.nt, c.per_cu, cands[0].nt, cands[0].per_cu, L, d);
        break;
      }
      if (!best || c.ms < best->ms) best = &c;
      if (c.nt == rule_nt && c.per_cu == max_per_cu(rule_nt, lds)) rule = &c;
    }
    if (rc != SPIN_OK || !best) break;
    // a shape other than the static rule's must be at least 3 % faster to be taken: the scratch
    // pool holds one size class alone, the real pool runs its classes side by side
    if (rule && best->ms > 0.97f * rule->ms) best = rule;
    {
      std::lock_guard<std::mutex> lk(g_plan_mu);
      load_plans_locked();
      g_plan[sh.first] = Plan{best->nt, best->per_cu};
    }
    const double ns_per_sweep = 1e6 * best->ms / sweeps;
    tune_cache_append("batch", {d, model, L, (long long)best->nt, (long long)best->per_cu, (long long)ns_per_sweep});
    ++tuned;
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  return rc == SPIN_OK ? tuned : rc;
}

int spin_batch_plan(int d, int model, int L, int* threads, int* workgroups_per_cu) {
  if (!threads || !workgroups_per_cu) return bfail(SPIN_EINVAL, "NULL output");
  Plan pl{0, 0};
  if (!plan_for(d, model, L, &pl)) {
    *threads = *workgroups_per_cu = 0;
    return 0;
  }
  *threads = (int)pl.nt;
  *workgroups_per_cu = (int)pl.per_cu;
  return 1;
}

int spin_batch_synchronize(spin_batch* b) {
  if (!b) return bfail(SPIN_EINVAL, "NULL batch");
  hipError_t e = hipSuccess;
  for (int k = 0; k < spin_batch::kAux && e == hipSuccess; ++k) e = hipStreamSynchronize(b->aux[k]);
  if (e == hipSuccess) e = hipStreamSynchronize(b->stream);
  if (e != hipSuccess) return hfail(e, "batch synchronize");
  return SPIN_OK;
}

}  // extern "C"
