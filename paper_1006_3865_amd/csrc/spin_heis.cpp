// spin_heis.cpp -- C ABI of the classical Heisenberg mode (spin_heis_*).
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <string>
#include <vector>

#include "spin.h"
#include "spin_heis.h"
#include "spin_internal.h"

using namespace spin;

static int hfail(int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  std::vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  return set_error(code, buf);
}

struct spin_heis {
  int L, d;
  uint64_t N;
  uint64_t seed;
  uint32_t replica;
  uint64_t t;
  float4* S;        // [N] (x, y, z, 0)
  double* part;     // measurement partials: rec_cap records of heis_measure_blocks(N) x 4 doubles
  size_t rec_cap;
  hipStream_t stream;
};

static void heis_destroy(spin_heis* h) {
  if (!h) return;
  (void)hipStreamSynchronize(h->stream);
  device_free(h->S);
  device_free(h->part);
  delete h;
}

static int reserve(spin_heis* h, size_t nrec) {
  if (nrec <= h->rec_cap) return SPIN_OK;
  (void)hipStreamSynchronize(h->stream);
  device_free(h->part);
  h->part = nullptr;
  h->rec_cap = 0;
  const size_t bytes = nrec * heis_measure_blocks(h->N) * 4 * sizeof(double);
  h->part = (double*)device_alloc(bytes);
  if (!h->part) {
    return hfail(SPIN_ENOMEM, "Heisenberg record buffer (%zu bytes)", bytes);
  }
  h->rec_cap = nrec;
  return SPIN_OK;
}

// Enqueue n sweeps; after every every-th sweep (every > 0) a measurement into record slot r.
static int heis_run(spin_heis* h, int n, double beta, int every) {
  if (n < 0) return hfail(SPIN_EINVAL, "n must be >= 0");
  if (std::isnan(beta) || beta < 0) return hfail(SPIN_EINVAL, "beta must be >= 0 (got %g)", beta);
  if (h->t + (uint64_t)n > ((uint64_t)1 << 32)) return hfail(SPIN_EINVAL, "sweep index would exceed 2^32");
  const size_t nrec = every > 0 ? (size_t)(n / every) : 0;
  if (int rc = reserve(h, nrec)) return rc;
  HeisArgs a;
  a.keys = make_round_keys(h->seed);
  a.N = h->N;
  a.L = (uint32_t)h->L;
  a.replica = h->replica;
  a.beta = (float)beta;
  const size_t stride = (size_t)heis_measure_blocks(h->N) * 4;
  size_t rec = 0;
  for (int i = 0; i < n; ++i) {
    a.t = (uint32_t)(h->t + (uint64_t)i);
    for (uint32_t c = 0; c < 2; ++c) {
      a.colour = c;
      hipError_t e = launch_heis_phase(h->S, (uint32_t)h->d, a, h->stream);
      if (e != hipSuccess) return hfail(SPIN_EDEVICE, "Heisenberg phase launch: %s", hipGetErrorString(e));
    }
    if (every > 0 && (i + 1) % every == 0) {
      hipError_t e = launch_heis_measure(h->S, (uint32_t)h->L, (uint32_t)h->d, h->N, h->part + rec * stride, h->stream);
      if (e != hipSuccess) return hfail(SPIN_EDEVICE, "Heisenberg measure launch: %s", hipGetErrorString(e));
      ++rec;
    }
  }
  h->t += (uint64_t)n;
  return SPIN_OK;
}

// Sum record slots 0..nrec-1 into E[r] and the magnetisation vector (|M| or the components).
static int heis_collect(spin_heis* h, size_t nrec, double* E, double* Mabs, double* M3) {
  const size_t blocks = heis_measure_blocks(h->N), stride = blocks * 4;
  std::vector<double> buf(nrec * stride);
  hipError_t e = hipMemcpyAsync(buf.data(), h->part, buf.size() * sizeof(double), hipMemcpyDeviceToHost, h->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
  if (e != hipSuccess) return hfail(SPIN_EDEVICE, "Heisenberg records: %s", hipGetErrorString(e));
  for (size_t r = 0; r < nrec; ++r) {
    double s[4] = {0, 0, 0, 0};
    for (size_t b = 0; b < blocks; ++b)
      for (int k = 0; k < 4; ++k) s[k] += buf[r * stride + b * 4 + k];
    E[r] = s[0];
    if (Mabs) Mabs[r] = std::sqrt(s[1] * s[1] + s[2] * s[2] + s[3] * s[3]);
    if (M3)
      for (int k = 0; k < 3; ++k) M3[3 * r + k] = s[1 + k];
  }
  return SPIN_OK;
}

extern "C" {

spin_heis* spin_heis_create(int L, int d, uint64_t seed, uint32_t replica, void* stream) {
  if ((d != 2 && d != 3) || L < 4 || L % 2 != 0) {
    hfail(SPIN_EINVAL, "need d = 2 or 3 and an even L >= 4 (got L=%d d=%d)", L, d);
    return nullptr;
  }
  const uint64_t N = d == 3 ? (uint64_t)L * L * L : (uint64_t)L * L;
  if (N > ((uint64_t)1 << 32)) {
    hfail(SPIN_EINVAL, "L^d must be <= 2^32");
    return nullptr;
  }
  spin_heis* h = new spin_heis();
  h->L = L;
  h->d = d;
  h->N = N;
  h->seed = seed;
  h->replica = replica;
  h->t = 0;
  h->S = nullptr;
  h->part = nullptr;
  h->rec_cap = 0;
  h->stream = (hipStream_t)stream;
  h->S = (float4*)device_alloc(N * sizeof(float4));
  if (!h->S) {
    hfail(SPIN_ENOMEM, "Heisenberg spins (%llu sites)", (unsigned long long)N);
    heis_destroy(h);
    return nullptr;
  }
  hipError_t e = launch_heis_init(h->S, N, seed, replica, h->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
  if (e != hipSuccess) {
    hfail(SPIN_EDEVICE, "Heisenberg setup: %s", hipGetErrorString(e));
    heis_destroy(h);
    return nullptr;
  }
  return h;
}

void spin_heis_free(spin_heis* h) { heis_destroy(h); }

int spin_heis_sweep(spin_heis* h, int n, double beta) {
  if (!h) return hfail(SPIN_EINVAL, "NULL handle");
  return heis_run(h, n, beta, 0);
}

int spin_heis_sweep_record(spin_heis* h, int n, double beta, int every, double* E, double* Mabs) {
  if (!h) return hfail(SPIN_EINVAL, "NULL handle");
  if (every < 1) return hfail(SPIN_EINVAL, "every must be >= 1");
  const size_t nrec = (size_t)(n > 0 ? n / every : 0);
  if (nrec > 0 && (!E || !Mabs)) return hfail(SPIN_EINVAL, "NULL record arrays");
  if (int rc = heis_run(h, n, beta, every)) return rc;
  return nrec ? heis_collect(h, nrec, E, Mabs, nullptr) : SPIN_OK;
}

int spin_heis_measure(spin_heis* h, double* E, double* M) {
  if (!h) return hfail(SPIN_EINVAL, "NULL handle");
  if (!E || !M) return hfail(SPIN_EINVAL, "NULL output");
  if (int rc = reserve(h, 1)) return rc;
  hipError_t e = launch_heis_measure(h->S, (uint32_t)h->L, (uint32_t)h->d, h->N, h->part, h->stream);
  if (e != hipSuccess) return hfail(SPIN_EDEVICE, "Heisenberg measure launch: %s", hipGetErrorString(e));
  return heis_collect(h, 1, E, nullptr, M);
}

int spin_heis_get_spins(const spin_heis* h, float* out, size_t n) {
  if (!h || !out) return hfail(SPIN_EINVAL, "NULL argument");
  if (n != 4 * h->N) return hfail(SPIN_EINVAL, "n must equal 4 L^d");
  hipError_t e = hipMemcpyAsync(out, h->S, h->N * sizeof(float4), hipMemcpyDeviceToHost, h->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
  if (e != hipSuccess) return hfail(SPIN_EDEVICE, "Heisenberg get spins: %s", hipGetErrorString(e));
  return SPIN_OK;
}

int spin_heis_set_spins(spin_heis* h, const float* in, size_t n) {
  if (!h || !in) return hfail(SPIN_EINVAL, "NULL argument");
  if (n != 4 * h->N) return hfail(SPIN_EINVAL, "n must equal 4 L^d");
  for (size_t i = 0; i < n; ++i) {
    if (!std::isfinite(in[i])) return hfail(SPIN_EINVAL, "spin component %zu is not finite", i);
    if (i % 4 == 3 && in[i] != 0.0f) return hfail(SPIN_EINVAL, "fourth component of site %zu must be 0", i / 4);
  }
  hipError_t e = hipMemcpyAsync(h->S, in, h->N * sizeof(float4), hipMemcpyHostToDevice, h->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
  if (e != hipSuccess) return hfail(SPIN_EDEVICE, "Heisenberg set spins: %s", hipGetErrorString(e));
  return SPIN_OK;
}

uint64_t spin_heis_sweeps_done(const spin_heis* h) { return h ? h->t : 0; }

int spin_heis_set_sweeps_done(spin_heis* h, uint64_t t) {
  if (!h) return hfail(SPIN_EINVAL, "NULL handle");
  if (t > ((uint64_t)1 << 32)) return hfail(SPIN_EINVAL, "sweep index must be <= 2^32");
  h->t = t;
  return SPIN_OK;
}

int spin_heis_synchronize(spin_heis* h) {
  if (!h) return hfail(SPIN_EINVAL, "NULL handle");
  hipError_t e = hipStreamSynchronize(h->stream);
  if (e != hipSuccess) return hfail(SPIN_EDEVICE, "Heisenberg synchronize: %s", hipGetErrorString(e));
  return SPIN_OK;
}

}  // extern "C"
