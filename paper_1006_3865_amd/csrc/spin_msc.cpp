// spin_msc.cpp -- C ABI of the multi-spin-coded +-J glass (include/spin.h,
// spin_msc_*): 32 systems in the bits of one word per site.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <utility>
#include <algorithm>
#include <vector>

#include "spin.h"
#include "spin_internal.h"
#include "spin_msc.h"

using namespace spin;

static int mfail(int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  std::vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  return set_error(code, buf);
}

struct spin_msc {
  int L, d;
  uint64_t N;
  uint64_t seed;
  uint32_t p0;
  uint64_t t;
  uint32_t* S;       // [N] current spins
  uint32_t* S2;      // [N] second buffer of the streaming kernel (allocated on first use)
  uint32_t TY, H, NT, XW;  // streaming shape; NT == 0: the per-colour phase kernel
  bool col;          // the register-column kernel (3D L = 512; shape TY, H)
  uint32_t* J;       // [d][N] (measurement)
  uint32_t* J6;      // [N/8][2][4][2d]: bonds of the active sites of each group and colour (phase kernel, on first use)
  int64_t* part;     // measurement partial counts
  int64_t* rec;      // records staging (2 * 32 * rec_cap)
  size_t rec_cap;
  hipStream_t stream;
};

static void msc_destroy(spin_msc* h) {
  if (!h) return;
  (void)hipStreamSynchronize(h->stream);
  device_free(h->S);
  device_free(h->S2);
  device_free(h->J);
  device_free(h->J6);
  device_free(h->part);
  device_free(h->rec);
  delete h;
}

template <class T>
static bool dalloc(T** p, size_t bytes) {
  *p = (T*)device_alloc(bytes);
  return *p != nullptr;
}

static MscArgs msc_args(const spin_msc* h, double beta) {
  const Accept acc = make_accept(beta, h->d);
  MscArgs a;
  std::memset(&a, 0, sizeof(a));
  a.keys = make_round_keys(h->seed);
  for (int u = 0; u < 3; ++u) a.thr[u] = (u < h->d) ? acc.T[2 * h->d - u] : ((uint64_t)1 << 32);
  a.N = h->N;
  a.L = (uint32_t)h->L;
  a.p0 = h->p0;
  return a;
}

// n sweeps; records (every > 0) of the 32 systems into device arrays dE, dM.
static int msc_run(spin_msc* h, int n, double beta, int every, int64_t* dE, int64_t* dM) {
  if (!h) return mfail(SPIN_EINVAL, "NULL handle");
  if (n < 0) return mfail(SPIN_EINVAL, "n must be >= 0");
  if (std::isnan(beta) || beta < 0) return mfail(SPIN_EINVAL, "beta must be >= 0 or +inf (got %g)", beta);
  if (h->t + (uint64_t)n > ((uint64_t)1 << 32)) return mfail(SPIN_EINVAL, "sweep index would exceed 2^32");
  MscArgs a = msc_args(h, beta);
  const bool streamed = h->NT || h->col;
  if (streamed && !h->S2 && n > 0 && !dalloc(&h->S2, h->N * 4)) return mfail(SPIN_ENOMEM, "second spin buffer");
  if (!streamed && !h->J6 && n > 0) {
    if (!dalloc(&h->J6, (size_t)2 * h->d * h->N * 4)) return mfail(SPIN_ENOMEM, "coupling copy");
    hipError_t e = launch_msc_bonds(h->J, h->J6, (uint32_t)h->L, (uint32_t)h->d, h->N, h->stream);
    if (e != hipSuccess) return mfail(SPIN_EDEVICE, "coupling copy: %s", hipGetErrorString(e));
  }
  uint32_t rec = 0;
  for (int i = 0; i < n; ++i) {
    a.t = (uint32_t)(h->t + (uint64_t)i);
    if (h->col) {
      hipError_t e = launch_msc_col(h->S, h->S2, h->J, a, (uint32_t)h->d, h->TY, h->H, h->stream);
      if (e != hipSuccess) return mfail(SPIN_EDEVICE, "multi-spin column launch: %s", hipGetErrorString(e));
      std::swap(h->S, h->S2);
    } else if (h->NT) {
      hipError_t e = launch_msc_stream(h->S, h->S2, h->J, a, (uint32_t)h->d, h->TY, h->H, h->NT, h->XW, h->stream);
      if (e != hipSuccess) return mfail(SPIN_EDEVICE, "multi-spin stream launch: %s", hipGetErrorString(e));
      std::swap(h->S, h->S2);
    } else {
      for (uint32_t c = 0; c < 2; ++c) {
        a.colour = c;
        hipError_t e = launch_msc_phase(h->S, h->J6, a, (uint32_t)h->d, h->stream);
        if (e != hipSuccess) return mfail(SPIN_EDEVICE, "multi-spin phase launch: %s", hipGetErrorString(e));
      }
    }
    if (every > 0 && (i + 1) % every == 0) {
      hipError_t e = launch_msc_measure(h->S, h->J, (uint32_t)h->L, (uint32_t)h->d, h->N, h->part, dE + 32 * rec,
                                        dM + 32 * rec, h->stream);
      if (e != hipSuccess) return mfail(SPIN_EDEVICE, "multi-spin measure launch: %s", hipGetErrorString(e));
      ++rec;
    }
  }
  h->t += (uint64_t)n;
  return SPIN_OK;
}

static int ensure_rec(spin_msc* h, size_t nrec) {
  if (nrec <= h->rec_cap) return SPIN_OK;
  (void)hipStreamSynchronize(h->stream);
  device_free(h->rec);
  h->rec_cap = 0;
  if (!dalloc(&h->rec, 2 * 32 * nrec * sizeof(int64_t))) return mfail(SPIN_ENOMEM, "record buffer allocation failed");
  h->rec_cap = nrec;
  return SPIN_OK;
}

extern "C" {

spin_msc* spin_msc_create(int L, int d, uint64_t coupling_seed, uint32_t realisation0, uint64_t seed,
                          uint32_t replica0, void* stream) {
  if (d != 2 && d != 3) {
    mfail(SPIN_EINVAL, "d must be 2 or 3 (got %d)", d);
    return nullptr;
  }
  if (L < 8 || L % 8 != 0) {
    mfail(SPIN_EINVAL, "L must be a multiple of 8 (got %d)", L);
    return nullptr;
  }
  uint64_t N = 1;
  for (int k = 0; k < d; ++k) N *= (uint64_t)L;
  if (N / 8 >= ((uint64_t)1 << 32)) {
    mfail(SPIN_EINVAL, "L^d/8 must be < 2^32");
    return nullptr;
  }
  spin_msc* h = new spin_msc();
  h->L = L;
  h->d = d;
  h->N = N;
  h->seed = seed;
  h->p0 = replica0;
  h->t = 0;
  h->S = nullptr;
  h->S2 = nullptr;
  h->J = nullptr;
  h->J6 = nullptr;
  // streaming shape, from measured rates: 3D whole rows in slabs of 16 rows (from L = 256 up, where
  // the ring fits LDS), else 8, else 4, and strips of planes sized so that the grid holds about one
  // workgroup per compute unit (at least 4 planes); 512 threads from L = 256 up, else 256.  2D rows
  // cut into segments of at most 2048 sites, strips of 16 rows, 256 threads.  Else the phase kernel.
  int cus = 256, dev = 0;
  if (hipGetDevice(&dev) == hipSuccess) {
    int v = 0;
    if (hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && v > 0) cus = v;
  }
  (void)hipGetLastError();
  h->NT = 0;
  h->col = false;
  h->TY = d == 3 ? 8u : 1u;
  h->H = 16;
  h->XW = (uint32_t)L;
  if (d == 3) {
    const uint32_t nt = L >= 256 ? 512u : 256u;
    const uint32_t first = L >= 256 ? 16u : 8u;
    for (uint32_t ty : {first, 8u, 4u}) {
      const uint32_t strips = std::max(1u, (uint32_t)cus / ((uint32_t)L / ty));
      const uint32_t H = std::min((uint32_t)L, std::max(4u, ((uint32_t)L + strips - 1) / strips));
      if (!h->NT && msc_stream_supported((uint32_t)L, 3, ty, H, nt, h->XW)) {
        h->TY = ty;
        h->H = H;
        h->NT = nt;
      }
    }
    // 3D L = 128, 256, 512: the register-column kernel with one workgroup per compute unit: slabs of
    // 4 rows at L = 512 and 8 below, strips of L^2 / (rows * CUs) planes (measured against the
    // plane-streaming kernel: L = 512 8430 vs 5370, 256 6610 vs 4550, 128 3050 vs 2020 attempts/ns)
    {
      const uint32_t ty = L == 512 ? 4u : 8u;
      uint32_t H = std::max(2u, (uint32_t)L * (uint32_t)L / (ty * (uint32_t)cus));
      while (H > 2 && ((uint32_t)L % H != 0 || H % 2 != 0)) --H;
      if (msc_col_supported((uint32_t)L, 3, ty, H)) {
        h->col = true;
        h->NT = 0;
        h->TY = ty;
        h->H = H;
      }
    }
  } else {
    while (h->XW > 2048 && (h->XW / 2) % 8 == 0) h->XW /= 2;
    h->TY = 1;
    h->H = 16;
    if (msc_stream_supported((uint32_t)L, 2, 1, h->H, 256, h->XW)) h->NT = 256;
  }
  h->part = nullptr;
  h->rec = nullptr;
  h->rec_cap = 0;
  h->stream = (hipStream_t)stream;
  if (!dalloc(&h->S, N * 4) || !dalloc(&h->J, (size_t)d * N * 4) ||
      !dalloc(&h->part, (size_t)msc_count_parts(N) * 64 * sizeof(int64_t))) {
    mfail(SPIN_ENOMEM, "device allocation failed (%llu sites)", (unsigned long long)N);
    msc_destroy(h);
    return nullptr;
  }
  hipError_t e = launch_msc_init(h->S, N, seed, replica0, h->stream);
  if (e == hipSuccess) e = launch_msc_couplings(h->J, N, (uint32_t)L, (uint32_t)d, coupling_seed, realisation0, h->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
  if (e != hipSuccess) {
    mfail(SPIN_EDEVICE, "multi-spin setup: %s", hipGetErrorString(e));
    msc_destroy(h);
    return nullptr;
  }
  return h;
}

void spin_msc_free(spin_msc* h) { msc_destroy(h); }

int spin_msc_sweep(spin_msc* h, int n, double beta) { return msc_run(h, n, beta, 0, nullptr, nullptr); }

int spin_msc_sweep_record(spin_msc* h, int n, double beta, int every, int64_t* E, int64_t* M) {
  if (!h || !E || !M) return mfail(SPIN_EINVAL, "NULL argument");
  if (every < 1) return mfail(SPIN_EINVAL, "every must be >= 1");
  const size_t nrec = (size_t)(n > 0 ? n / every : 0);
  if (int rc = ensure_rec(h, nrec ? nrec : 1)) return rc;
  int rc = msc_run(h, n, beta, every, h->rec, h->rec + 32 * h->rec_cap);
  if (rc != SPIN_OK) return rc;
  hipError_t e = hipSuccess;
  if (nrec) {
    e = hipMemcpyAsync(E, h->rec, 32 * nrec * sizeof(int64_t), hipMemcpyDeviceToHost, h->stream);
    if (e == hipSuccess)
      e = hipMemcpyAsync(M, h->rec + 32 * h->rec_cap, 32 * nrec * sizeof(int64_t), hipMemcpyDeviceToHost, h->stream);
  }
  if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
  if (e != hipSuccess) return mfail(SPIN_EDEVICE, "multi-spin records: %s", hipGetErrorString(e));
  return SPIN_OK;
}

int spin_msc_measure(spin_msc* h, int64_t* E, int64_t* M) {
  if (!h || !E || !M) return mfail(SPIN_EINVAL, "NULL argument");
  if (int rc = ensure_rec(h, 1)) return rc;
  hipError_t e = launch_msc_measure(h->S, h->J, (uint32_t)h->L, (uint32_t)h->d, h->N, h->part, h->rec,
                                    h->rec + 32 * h->rec_cap, h->stream);
  if (e == hipSuccess) e = hipMemcpyAsync(E, h->rec, 32 * sizeof(int64_t), hipMemcpyDeviceToHost, h->stream);
  if (e == hipSuccess)
    e = hipMemcpyAsync(M, h->rec + 32 * h->rec_cap, 32 * sizeof(int64_t), hipMemcpyDeviceToHost, h->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
  if (e != hipSuccess) return mfail(SPIN_EDEVICE, "multi-spin measure: %s", hipGetErrorString(e));
  return SPIN_OK;
}

int spin_msc_get_spins(const spin_msc* h, int system, int8_t* out, size_t n) {
  if (!h || !out) return mfail(SPIN_EINVAL, "NULL argument");
  if (system < 0 || system >= 32) return mfail(SPIN_EINVAL, "system must be in 0..31 (got %d)", system);
  if (n != h->N) return mfail(SPIN_EINVAL, "n must equal L^d");
  std::vector<uint32_t> w(h->N);
  hipError_t e = hipMemcpyAsync(w.data(), h->S, h->N * 4, hipMemcpyDeviceToHost, h->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
  if (e != hipSuccess) return mfail(SPIN_EDEVICE, "multi-spin get spins: %s", hipGetErrorString(e));
  for (size_t s = 0; s < n; ++s) out[s] = ((w[s] >> system) & 1u) ? (int8_t)-1 : (int8_t)1;
  return SPIN_OK;
}

uint64_t spin_msc_sweeps_done(const spin_msc* h) { return h ? h->t : 0; }

int spin_msc_set_kernel(spin_msc* h, int streaming, int rows, int planes, int threads, int width) {
  if (!h) return mfail(SPIN_EINVAL, "NULL handle");
  if (!streaming) {
    h->NT = 0;
    h->col = false;
    return SPIN_OK;
  }
  if (rows < 0 || planes < 0 || threads < 0 || width < 0) return mfail(SPIN_EINVAL, "negative streaming shape");
  if (streaming == 2) {
    const uint32_t TY = (uint32_t)(rows ? rows : 8), H = (uint32_t)(planes ? planes : 32);
    if (!msc_col_supported((uint32_t)h->L, (uint32_t)h->d, TY, H) || (threads && (uint32_t)threads != 64 * (TY + 2)) ||
        (width && width != h->L))
      return mfail(SPIN_EINVAL, "register-column shape rows=%d planes=%d threads=%d width=%d cannot run L=%d d=%d",
                   rows, planes, threads, width, h->L, h->d);
    h->col = true;
    h->NT = 0;
    h->TY = TY;
    h->H = H;
    h->XW = (uint32_t)h->L;
    return SPIN_OK;
  }
  if (streaming != 1) return mfail(SPIN_EINVAL, "streaming must be 0, 1 or 2 (got %d)", streaming);
  const uint32_t TY = h->d == 3 ? (uint32_t)(rows ? rows : 8) : 1u, H = (uint32_t)(planes ? planes : 16),
                 NT = (uint32_t)(threads ? threads : 512), XW = (uint32_t)(width ? width : h->L);
  if (!msc_stream_supported((uint32_t)h->L, (uint32_t)h->d, TY, H, NT, XW))
    return mfail(SPIN_EINVAL, "streaming shape rows=%d planes=%d threads=%d width=%d cannot run L=%d d=%d", rows,
                 planes, threads, width, h->L, h->d);
  h->TY = TY;
  h->H = H;
  h->NT = NT;
  h->XW = XW;
  h->col = false;
  return SPIN_OK;
}

int spin_msc_kernel(const spin_msc* h) {
  if (!h) return -1;
  return h->col ? 2 : (h->NT ? 1 : 0);
}

int spin_msc_synchronize(spin_msc* h) {
  if (!h) return mfail(SPIN_EINVAL, "NULL handle");
  hipError_t e = hipStreamSynchronize(h->stream);
  if (e != hipSuccess) return mfail(SPIN_EDEVICE, "multi-spin synchronize: %s", hipGetErrorString(e));
  return SPIN_OK;
}

}  // extern "C"
