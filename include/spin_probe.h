/*
 * spin_probe.h -- ceiling probes exported by libspin.so.  Measurement only:
 * they establish what bounds the sweep (the generator's cost, the VALU issue
 * rates, the attainable HBM copy rate) and compute nothing of the chain.
 * Each call enqueues one kernel on the hipStream_t `stream` (NULL = null
 * stream), returns SPIN_OK or a negative spin_status (spin.h), and is timed by
 * the caller with events around it.  All pointers are device pointers owned
 * by the caller.
 */
#ifndef SPIN_PROBE_H
#define SPIN_PROBE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum spin_probe_kind {
  /* blocks*256 threads each evaluate `iters` Philox4x32-10 blocks (key = seed,
   * counter (i, 1, 0, 0)) with the sweep kernels' own code and fold the four
   * words with three XORs: 4*iters*blocks*256 words */
  SPIN_PROBE_PHILOX = 0,
  /* blocks*256 threads each run 8 independent chains of 4*iters links of one
   * 32x32 -> 64-bit product (v_mad_u64_u32) and one 32-bit add of its halves:
   * 32*iters links, 64*iters VALU instructions per thread */
  SPIN_PROBE_MAD64 = 1,
  /* 8 independent chains of 4*iters links of one 32-bit XOR-add (v_xad_u32):
   * 32*iters VALU instructions per thread */
  SPIN_PROBE_ALU32 = 2
};

/* One probe kernel of `kind`; out holds blocks*256 uint32 (one per thread,
 * written so the work is not optimised away).  SPIN_EINVAL for an unknown
 * kind, NULL out or zero sizes. */
int spin_probe_alu(int kind, uint32_t* out, uint32_t blocks, uint32_t iters, uint64_t seed, void* stream);

/* Copy `bytes` (a multiple of 16) from src to dst with `blocks` workgroups of
 * 256 threads, 16 bytes per thread per step, grid-stride. */
int spin_probe_copy(const void* src, void* dst, uint64_t bytes, uint32_t blocks, void* stream);

#ifdef __cplusplus
}
#endif

#endif /* SPIN_PROBE_H */
