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
  *p = nullptr;
  if (hipMalloc((void**)p, bytes ? bytes : 16) != hipSuccess) {
    (void)hipGetLastError();
    *p = nullptr;
    return false;
  }
  return true;
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
      (void)hipFree(p);
      direct_.erase(it);
      return;
    }
    bytes = (bytes + 255) / 256 * 256;
    if (bytes == 0) bytes = 256;
    free_[bytes].push_back(p);
  }

  void release() {
    for (char* c : chunks_) (void)hipFree(c);
    for (void* p : direct_) (void)hipFree(p);
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
};

size_t rec_count(int n, int every) { return every > 0 ? (n > 0 ? (size_t)(n / every) : 1) : 0; }

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
};

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
  (void)hipFree(b->d_lats);
  (void)hipFree(b->d_calls);
  (void)hipFree(b->d_order);
  (void)hipFree(b->d_counters);
  (void)hipFree(b->d_rec);
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
    (void)hipFree(d_lats);
    (void)hipFree(d_calls);
    (void)hipFree(d_order);
    if (h_lats) (void)hipHostFree(h_lats);
    if (h_calls) (void)hipHostFree(h_calls);
    if (h_order) (void)hipHostFree(h_order);
    return bfail(SPIN_ENOMEM, "batch slot arrays (%zu slots)", cap);
  }
  (void)hipFree(b->d_lats);
  (void)hipFree(b->d_calls);
  (void)hipFree(b->d_order);
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
    if (!mb.big) return SPIN_EINVAL;  // message set by spin_create_config
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
      (void)hipFree(tmp);
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
  for (int i = 0; i < S; ++i) {
    const Member& mb = b->m[i];
    if (!mb.active) {
      if (n[i] != 0) return bfail(SPIN_EINVAL, "slot %d holds no lattice but n[%d] = %d", i, i, n[i]);
      continue;
    }
    if (n[i] < 0) return bfail(SPIN_EINVAL, "slot %d: n must be >= 0", i);
    if (std::isnan(beta[i]) || beta[i] < 0) return bfail(SPIN_EINVAL, "slot %d: bad beta %g", i, beta[i]);
    const uint64_t t = mb.big ? spin_sweeps_done(mb.big) : mb.t;
    if (t + (uint64_t)n[i] > ((uint64_t)1 << 32)) return bfail(SPIN_EINVAL, "slot %d: sweep index past 2^32", i);
    if (rec_count(n[i], every) && (!dE || !dM)) return bfail(SPIN_EINVAL, "NULL record arrays");
  }
  // the previous call's uploads must have been read before the host buffers change
  hipError_t e = hipEventSynchronize(b->uploaded);
  if (e != hipSuccess) return hfail(e, "batch upload wait");
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
    const uint32_t nt = batch_threads_for(mb.N / 8);
    const auto key = std::make_tuple(mb.d, mb.model, nt);
    auto it = cls_index.find(key);
    if (it == cls_index.end()) {
      it = cls_index.emplace(key, classes.size()).first;
      classes.push_back(Class{(uint32_t)mb.d, mb.model == SPIN_EA_PMJ, nt, 0, {}});
    }
    Class& cl = classes[it->second];
    cl.members.push_back((uint32_t)i);
    cl.lds = std::max(cl.lds, batch_lds_bytes((uint32_t)mb.L, (uint32_t)mb.d));
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
  if (norder) {
    e = hipMemcpyAsync(b->d_calls, b->h_calls, sizeof(BatchCall) * S, hipMemcpyHostToDevice, b->stream);
    if (e == hipSuccess)
      e = hipMemcpyAsync(b->d_order, b->h_order, sizeof(uint32_t) * norder, hipMemcpyHostToDevice, b->stream);
    if (e == hipSuccess) e = hipEventRecord(b->uploaded, b->stream);
    if (e != hipSuccess) {
      join_aux(b, used);
      return hfail(e, "batch upload");
    }
  }
  for (size_t k = 0; k < classes.size(); ++k) {
    const Class& cl = classes[k];
    const uint32_t ntasks = ranges[k].second;
    uint32_t per_cu = std::min<uint32_t>(2048u / cl.nt, (uint32_t)((160 * 1024 - 256) / cl.lds));
    if (b->wgs_override > 0) per_cu = (uint32_t)b->wgs_override;
    if (per_cu < 1) per_cu = 1;
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
  for (int i = 0; i < S; ++i)
    if (b->m[i].active && b->m[i].resident) b->m[i].t += (uint64_t)n[i];
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
  if (mb.big) return mb.N * (mb.model == SPIN_EA_PMJ ? 2 + mb.d : 2);  // spins, ping-pong copy, int8 couplings
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
    (void)hipFree(b->d_rec);
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
  return b->m[i].big ? spin_sweeps_done(b->m[i].big) : b->m[i].t;
}

int spin_batch_set_workgroups_per_cu(spin_batch* b, int wgs) {
  if (!b) return bfail(SPIN_EINVAL, "NULL batch");
  if (wgs < 0 || wgs > 8) return bfail(SPIN_EINVAL, "workgroups per CU must be in 0..8");
  b->wgs_override = wgs;
  return SPIN_OK;
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
