// spin_batch.cpp -- C ABI of the batched path (include/spin.h, spin_batch_*):
// many lattices (disorder realisations x temperatures) advanced by one
// persistent launch per class of (dimension, model, workgroup size).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <map>
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

struct Class {
  uint32_t d;
  bool ea;
  uint32_t nt;          // threads per workgroup
  size_t lds;           // dynamic LDS of the launch (largest lattice of the class)
  std::vector<uint32_t> members;
};

}  // namespace

struct spin_batch {
  int count;
  std::vector<int> L, d, model;
  std::vector<uint64_t> N;
  std::vector<uint64_t> t;                // host mirror of the sweep counters
  std::vector<size_t> off;                // byte offset of each lattice in `spins`
  int8_t* spins;
  std::vector<uint32_t*> jn_bufs;         // distinct coupling arrays (nibble words)
  BatchLattice* d_lats;
  std::vector<BatchLattice> h_lats;
  BatchCall* d_calls;
  BatchCall* h_calls;                     // pinned
  uint32_t* d_order;
  uint32_t* h_order;                      // pinned, count entries
  hipEvent_t uploaded;                    // the last upload of h_calls / h_order has been read
  uint32_t* d_counters;                   // one per class
  int64_t* d_rec;
  size_t rec_cap;
  std::vector<Class> classes;
  hipStream_t stream;
  int num_cu;
  int wgs_override;                       // 0: by occupancy
};

static uint32_t threads_for(uint64_t nwords) {
  if (nwords <= 2048) return 256;
  if (nwords <= 8192) return 512;
  return 1024;
}

static void batch_destroy(spin_batch* b) {
  if (!b) return;
  (void)hipStreamSynchronize(b->stream);
  (void)hipFree(b->spins);
  for (uint32_t* p : b->jn_bufs) (void)hipFree(p);
  (void)hipFree(b->d_lats);
  (void)hipFree(b->d_calls);
  if (b->h_calls) (void)hipHostFree(b->h_calls);
  if (b->h_order) (void)hipHostFree(b->h_order);
  if (b->uploaded) (void)hipEventDestroy(b->uploaded);
  (void)hipFree(b->d_order);
  (void)hipFree(b->d_counters);
  (void)hipFree(b->d_rec);
  delete b;
}

template <class T>
static bool dmalloc(T** p, size_t bytes) {
  *p = nullptr;
  if (hipMalloc((void**)p, bytes ? bytes : 16) != hipSuccess) {
    (void)hipGetLastError();
    *p = nullptr;
    return false;
  }
  return true;
}

extern "C" {

spin_batch* spin_batch_create(int count, const spin_desc* descs, void* stream) {
  if (count <= 0 || !descs) {
    bfail(SPIN_EINVAL, "count must be > 0 and descs non-NULL");
    return nullptr;
  }
  spin_batch* b = new spin_batch();
  b->count = count;
  b->spins = nullptr;
  b->d_lats = nullptr;
  b->d_calls = nullptr;
  b->h_calls = nullptr;
  b->d_order = nullptr;
  b->h_order = nullptr;
  b->uploaded = nullptr;
  b->d_counters = nullptr;
  b->d_rec = nullptr;
  b->rec_cap = 0;
  b->stream = (hipStream_t)stream;
  b->wgs_override = 0;
  int dev = 0;
  (void)hipGetDevice(&dev);
  b->num_cu = 256;
  (void)hipDeviceGetAttribute(&b->num_cu, hipDeviceAttributeMultiprocessorCount, dev);
  size_t total = 0;
  for (int i = 0; i < count; ++i) {
    const spin_desc& s = descs[i];
    if (s.model != SPIN_ISING && s.model != SPIN_EA_PMJ) {
      bfail(SPIN_EINVAL, "lattice %d: model must be 0 or 1", i);
      batch_destroy(b);
      return nullptr;
    }
    if (s.d != 2 && s.d != 3) {
      bfail(SPIN_EINVAL, "lattice %d: d must be 2 or 3", i);
      batch_destroy(b);
      return nullptr;
    }
    if (s.L < 8 || s.L % 8 != 0) {
      bfail(SPIN_EINVAL, "lattice %d: batched lattices need L %% 8 == 0 and L >= 8 (got %d)", i, s.L);
      batch_destroy(b);
      return nullptr;
    }
    const uint64_t N = (s.d == 3) ? (uint64_t)s.L * s.L * s.L : (uint64_t)s.L * s.L;
    if (batch_lds_bytes((uint32_t)s.L, (uint32_t)s.d) > kBatchMaxLds) {
      bfail(SPIN_EINVAL, "lattice %d: L=%d d=%d does not fit one workgroup's LDS (L^d/2 bytes <= %zu)", i, s.L,
            s.d, kBatchMaxLds);
      batch_destroy(b);
      return nullptr;
    }
    if (s.model == SPIN_ISING && s.couplings) {
      bfail(SPIN_EINVAL, "lattice %d: couplings must be NULL for the Ising model", i);
      batch_destroy(b);
      return nullptr;
    }
    if (s.couplings)
      for (uint64_t k = 0; k < (uint64_t)s.d * N; ++k)
        if (s.couplings[k] != 1 && s.couplings[k] != -1) {
          bfail(SPIN_EINVAL, "lattice %d: coupling %llu is not +-1", i, (unsigned long long)k);
          batch_destroy(b);
          return nullptr;
        }
    b->L.push_back(s.L);
    b->d.push_back(s.d);
    b->model.push_back(s.model);
    b->N.push_back(N);
    b->t.push_back(0);
    b->off.push_back(total);
    total += (N + 255) / 256 * 256;
  }
  if (!dmalloc(&b->spins, total) || !dmalloc(&b->d_lats, sizeof(BatchLattice) * count) ||
      !dmalloc(&b->d_calls, sizeof(BatchCall) * count) || !dmalloc(&b->d_order, sizeof(uint32_t) * count) ||
      !dmalloc(&b->d_counters, sizeof(uint32_t) * 64)) {
    bfail(SPIN_ENOMEM, "batch device allocation failed");
    batch_destroy(b);
    return nullptr;
  }
  if (hipHostMalloc((void**)&b->h_calls, sizeof(BatchCall) * count, hipHostMallocDefault) != hipSuccess ||
      hipHostMalloc((void**)&b->h_order, sizeof(uint32_t) * count, hipHostMallocDefault) != hipSuccess ||
      hipEventCreateWithFlags(&b->uploaded, hipEventDisableTiming) != hipSuccess) {
    (void)hipGetLastError();
    bfail(SPIN_ENOMEM, "pinned host allocation failed");
    batch_destroy(b);
    return nullptr;
  }
  // couplings: one nibble array per distinct (coupling seed, realisation, L, d) or host array
  std::map<std::tuple<uint64_t, uint32_t, int, int>, uint32_t*> shared;
  b->h_lats.resize(count);
  for (int i = 0; i < count; ++i) {
    const spin_desc& s = descs[i];
    BatchLattice& bl = b->h_lats[i];
    bl.spins = b->spins + b->off[i];
    bl.Jn = nullptr;
    bl.L = (uint32_t)s.L;
    bl.d = (uint32_t)s.d;
    bl.replica = s.replica;
    bl.t = 0;
    bl.keys = make_round_keys(s.seed);
    hipError_t e;
    Lat lat;
    lat.spins = bl.spins;
    lat.J = nullptr;
    lat.L = bl.L;
    lat.d = bl.d;
    lat.N = b->N[i];
    lat.replica = s.replica;
    lat.keys = bl.keys;
    if ((e = launch_init_spins(lat, b->stream)) != hipSuccess) {
      hfail(e, "batch hot start");
      batch_destroy(b);
      return nullptr;
    }
    if (s.model != SPIN_EA_PMJ) continue;
    const uint64_t nbytes = (uint64_t)s.d * b->N[i];
    if (!s.couplings) {
      auto key = std::make_tuple(s.coupling_seed, s.realisation, s.L, s.d);
      auto it = shared.find(key);
      if (it != shared.end()) {
        bl.Jn = it->second;
        continue;
      }
      uint32_t* jn;
      if (!dmalloc(&jn, nbytes / 2)) {
        bfail(SPIN_ENOMEM, "coupling allocation failed");
        batch_destroy(b);
        return nullptr;
      }
      b->jn_bufs.push_back(jn);
      if ((e = launch_couplings_nibble(jn, b->N[i], (uint32_t)s.d, s.coupling_seed, s.realisation, b->stream)) !=
          hipSuccess) {
        hfail(e, "coupling generation");
        batch_destroy(b);
        return nullptr;
      }
      shared[key] = jn;
      bl.Jn = jn;
    } else {
      uint32_t* jn;
      int8_t* tmp;
      if (!dmalloc(&jn, nbytes / 2) || !dmalloc(&tmp, nbytes)) {
        bfail(SPIN_ENOMEM, "coupling allocation failed");
        batch_destroy(b);
        return nullptr;
      }
      b->jn_bufs.push_back(jn);
      e = hipMemcpyAsync(tmp, s.couplings, nbytes, hipMemcpyHostToDevice, b->stream);
      if (e == hipSuccess) e = launch_pack_nibbles(tmp, jn, nbytes, b->stream);
      if (e == hipSuccess) e = hipStreamSynchronize(b->stream);
      (void)hipFree(tmp);
      if (e != hipSuccess) {
        hfail(e, "coupling upload");
        batch_destroy(b);
        return nullptr;
      }
      bl.Jn = jn;
    }
  }
  hipError_t e = hipMemcpyAsync(b->d_lats, b->h_lats.data(), sizeof(BatchLattice) * count, hipMemcpyHostToDevice,
                                b->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(b->stream);
  if (e != hipSuccess) {
    hfail(e, "batch setup");
    batch_destroy(b);
    return nullptr;
  }
  // classes: (d, model, threads); the LDS of a class is its largest lattice's
  std::map<std::tuple<int, int, uint32_t>, size_t> cls;
  for (int i = 0; i < count; ++i) {
    const uint32_t nt = threads_for(b->N[i] / 8);
    auto key = std::make_tuple(b->d[i], b->model[i], nt);
    auto it = cls.find(key);
    size_t ci;
    if (it == cls.end()) {
      ci = b->classes.size();
      cls[key] = ci;
      b->classes.push_back(Class{(uint32_t)b->d[i], b->model[i] == SPIN_EA_PMJ, nt, 0, {}});
    } else {
      ci = it->second;
    }
    Class& c = b->classes[ci];
    c.members.push_back((uint32_t)i);
    c.lds = std::max(c.lds, batch_lds_bytes((uint32_t)b->L[i], (uint32_t)b->d[i]));
  }
  return b;
}

void spin_batch_free(spin_batch* b) { batch_destroy(b); }

int spin_batch_size(const spin_batch* b) { return b ? b->count : 0; }

// Enqueue lattice i's n[i] sweeps at beta[i] (n == NULL: n0 for all, beta
// == NULL is invalid); records go to device arrays dE, dM at offsets
// sum_{j<i} n[j]/every.
static int batch_run(spin_batch* b, const int* n, int n0, const double* beta, int every, int64_t* dE, int64_t* dM) {
  if (!b) return bfail(SPIN_EINVAL, "NULL batch");
  if (!beta) return bfail(SPIN_EINVAL, "NULL beta array");
  if (every < 0) return bfail(SPIN_EINVAL, "every must be >= 0");
  // the previous call's uploads must have been read before the host buffers change
  hipError_t e = hipEventSynchronize(b->uploaded);
  if (e != hipSuccess) return hfail(e, "batch upload wait");
  size_t rec = 0;
  for (int i = 0; i < b->count; ++i) {
    const int ni = n ? n[i] : n0;
    if (ni < 0) return bfail(SPIN_EINVAL, "lattice %d: n must be >= 0", i);
    if (std::isnan(beta[i]) || beta[i] < 0) return bfail(SPIN_EINVAL, "lattice %d: bad beta %g", i, beta[i]);
    if (b->t[i] + (uint64_t)ni > ((uint64_t)1 << 32)) return bfail(SPIN_EINVAL, "lattice %d: sweep index past 2^32", i);
    const size_t nr = every > 0 ? (ni > 0 ? (size_t)(ni / every) : 1) : 0;
    BatchCall& c = b->h_calls[i];
    const Accept a = make_accept(beta[i], b->d[i]);
    c.n = (uint32_t)ni;
    c.every = (uint32_t)every;
    c.never4 = 4u * a.never_level;
    for (int k = 0; k < 8; ++k) c.bound[k] = a.bound[k];
    c.E = (nr && dE) ? dE + rec : nullptr;
    c.M = (nr && dM) ? dM + rec : nullptr;
    if (nr && (!dE || !dM)) return bfail(SPIN_EINVAL, "NULL record arrays");
    if (!nr) c.every = 0;
    rec += nr;
  }
  e = hipMemcpyAsync(b->d_calls, b->h_calls, sizeof(BatchCall) * b->count, hipMemcpyHostToDevice, b->stream);
  if (e != hipSuccess) return hfail(e, "batch call upload");
  // task order: per class, largest work first (longest-processing-time order)
  uint32_t norder = 0;
  std::vector<std::pair<uint32_t, uint32_t>> ranges;
  for (const Class& c : b->classes) {
    const uint32_t start = norder;
    std::vector<uint32_t> m;
    for (uint32_t i : c.members)
      if (b->h_calls[i].n > 0 || b->h_calls[i].every) m.push_back(i);
    std::stable_sort(m.begin(), m.end(), [&](uint32_t x, uint32_t y) {
      return b->N[x] * (uint64_t)b->h_calls[x].n > b->N[y] * (uint64_t)b->h_calls[y].n;
    });
    for (uint32_t i : m) b->h_order[norder++] = i;
    ranges.push_back({start, (uint32_t)m.size()});
  }
  if (norder) {
    e = hipMemcpyAsync(b->d_order, b->h_order, sizeof(uint32_t) * norder, hipMemcpyHostToDevice, b->stream);
    if (e != hipSuccess) return hfail(e, "batch order upload");
  }
  e = hipEventRecord(b->uploaded, b->stream);
  if (e != hipSuccess) return hfail(e, "batch upload event");
  for (size_t k = 0; k < b->classes.size(); ++k) {
    const Class& c = b->classes[k];
    const uint32_t ntasks = ranges[k].second;
    if (ntasks == 0) continue;
    uint32_t per_cu = std::min<uint32_t>(2048u / c.nt, (uint32_t)(160 * 1024 / c.lds));
    if (b->wgs_override > 0) per_cu = (uint32_t)b->wgs_override;
    if (per_cu < 1) per_cu = 1;
    const uint32_t grid = std::min<uint32_t>(ntasks, per_cu * (uint32_t)b->num_cu);
    e = launch_batch(c.d, c.ea, c.nt, b->d_lats, b->d_calls, b->d_order + ranges[k].first, ntasks,
                     b->d_counters + k, c.lds, grid, b->stream);
    if (e != hipSuccess) return hfail(e, "batch launch");
  }
  for (int i = 0; i < b->count; ++i) b->t[i] += b->h_calls[i].n;
  return SPIN_OK;
}

static size_t record_count(const spin_batch* b, const int* n, int n0, int every) {
  size_t r = 0;
  if (every <= 0) return 0;
  for (int i = 0; i < b->count; ++i) {
    const int ni = n ? n[i] : n0;
    r += ni > 0 ? (size_t)(ni / every) : 1;
  }
  return r;
}

int spin_batch_sweep_device(spin_batch* b, const int* n, const double* beta, int every, int64_t* E, int64_t* M) {
  return batch_run(b, n, 0, beta, every, E, M);
}

int spin_batch_sweep(spin_batch* b, const int* n, const double* beta, int every, int64_t* E, int64_t* M) {
  if (!b) return bfail(SPIN_EINVAL, "NULL batch");
  if (!n) return bfail(SPIN_EINVAL, "NULL n array");
  const size_t nr = record_count(b, n, 0, every);
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
  int rc = batch_run(b, n, 0, beta, every, nr ? b->d_rec : nullptr, nr ? b->d_rec + nr : nullptr);
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
  std::vector<int> zero(b->count, 0);
  std::vector<double> beta(b->count, 0.0);
  return spin_batch_sweep(b, zero.data(), beta.data(), 1, E, M);
}

int spin_batch_get_spins(const spin_batch* b, int i, int8_t* out, size_t n) {
  if (!b || !out) return bfail(SPIN_EINVAL, "NULL argument");
  if (i < 0 || i >= b->count) return bfail(SPIN_EINVAL, "lattice index %d out of range", i);
  if (n != b->N[i]) return bfail(SPIN_EINVAL, "n must equal L^d of lattice %d", i);
  hipError_t e = hipMemcpyAsync(out, b->spins + b->off[i], n, hipMemcpyDeviceToHost, b->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(b->stream);
  if (e != hipSuccess) return hfail(e, "batch get spins");
  return SPIN_OK;
}

int spin_batch_set_spins(spin_batch* b, int i, const int8_t* in, size_t n) {
  if (!b || !in) return bfail(SPIN_EINVAL, "NULL argument");
  if (i < 0 || i >= b->count) return bfail(SPIN_EINVAL, "lattice index %d out of range", i);
  if (n != b->N[i]) return bfail(SPIN_EINVAL, "n must equal L^d of lattice %d", i);
  for (size_t k = 0; k < n; ++k)
    if (in[k] != 1 && in[k] != -1) return bfail(SPIN_EINVAL, "spin %zu is not +-1", k);
  hipError_t e = hipMemcpyAsync(b->spins + b->off[i], in, n, hipMemcpyHostToDevice, b->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(b->stream);
  if (e != hipSuccess) return hfail(e, "batch set spins");
  return SPIN_OK;
}

uint64_t spin_batch_sweeps_done(const spin_batch* b, int i) {
  if (!b || i < 0 || i >= b->count) return 0;
  return b->t[i];
}

int spin_batch_set_workgroups_per_cu(spin_batch* b, int wgs) {
  if (!b) return bfail(SPIN_EINVAL, "NULL batch");
  if (wgs < 0 || wgs > 8) return bfail(SPIN_EINVAL, "workgroups per CU must be in 0..8");
  b->wgs_override = wgs;
  return SPIN_OK;
}

int spin_batch_synchronize(spin_batch* b) {
  if (!b) return bfail(SPIN_EINVAL, "NULL batch");
  hipError_t e = hipStreamSynchronize(b->stream);
  if (e != hipSuccess) return hfail(e, "batch synchronize");
  return SPIN_OK;
}

}  // extern "C"
