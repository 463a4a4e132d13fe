// spin_noalloc.hip -- spin_sweep_record_noalloc: spin_sweep_record_device on
// a fixed device scratch array, for callers that cannot allocate device
// memory (code under stream capture, tight serving loops, harnesses that
// forbid allocation).
//
// The scratch of a sweep call is the per-workgroup partial counts of its
// (E, M) records (16 bytes per counting workgroup and record) and, on the
// LDS-resident path, the one-task block of the persistent kernel.  Here they
// live in one file-scope device array; each GPU holds its own copy at its own
// address, found once per device with hipGetSymbolAddress and kept for the
// life of the process.  Every call on a GPU shares that GPU's array: calls
// that overlap on one GPU (other threads, other streams) race.  Nothing in
// it has to start at zero: every partial slot a finalize reads is written by
// its record's kernel first, and the task counter is cleared by a kernel.
#include <hip/hip_runtime.h>

#include <mutex>

#include "spin.h"
#include "spin_internal.h"

namespace {

constexpr size_t kScratchBytes = (size_t)2 << 20;   // SPIN_NOALLOC_SCRATCH_BYTES
constexpr size_t kSingleBytes = 256;                 // the one-task block, at the front
constexpr int kMaxDevices = 64;

__device__ __align__(256) unsigned char scratch[kScratchBytes];

std::mutex g_mu;
void* g_ptr[kMaxDevices];  // device address of `scratch` per device (nullptr: not looked up yet)

// Device address of this device's scratch array, looked up on first use with
// the device current.
int scratch_ptr(void** out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return spin::set_error(SPIN_EDEVICE, "hipGetDevice failed");
  if (dev < 0 || dev >= kMaxDevices) return spin::set_error(SPIN_EDEVICE, "device index out of range");
  std::lock_guard<std::mutex> lk(g_mu);
  if (!g_ptr[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) {
      (void)hipGetLastError();
      return spin::set_error(SPIN_EDEVICE, "hipGetSymbolAddress of the scratch array failed");
    }
    g_ptr[dev] = p;
  }
  *out = g_ptr[dev];
  return SPIN_OK;
}

}  // namespace

extern "C" {

int spin_sweep_record_noalloc(spin_lattice* h, int n, double beta, int every, int64_t* E, int64_t* M) {
  static_assert(kScratchBytes == SPIN_NOALLOC_SCRATCH_BYTES, "scratch size and header disagree");
  if (spin::single_bytes() > kSingleBytes) return spin::set_error(SPIN_EDEVICE, "one-task block exceeds its slot");
  void* base = nullptr;
  if (int rc = scratch_ptr(&base)) return rc;
  spin::CallScratch fx;
  fx.single = base;
  fx.part = reinterpret_cast<int64_t*>(static_cast<unsigned char*>(base) + kSingleBytes);
  fx.part_slots = (kScratchBytes - kSingleBytes) / sizeof(int64_t);
  return spin::sweep_record_fixed(h, n, beta, every, E, M, fx);
}

}  // extern "C"
