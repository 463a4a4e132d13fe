/*
 * spin.h -- C ABI of the MI355X (gfx950) checkerboard Metropolis library.
 *
 * The library advances 2D (square) and 3D (simple cubic) lattices of +-1
 * spins, edge L, periodic boundaries, with single-spin-flip Metropolis
 * updates in red/black (checkerboard) order: the Ising ferromagnet of
 * Weigel, "Simulating spin models on GPU", Sec. 3, Eq. 1, and the +-J
 * Edwards-Anderson glass (same paper, Sec. 4, last paragraph).
 *
 * Definition of the chain computed (identical bits on every code path):
 *   - site s = x + L*(y + L*z), x fastest; colour(s) = (x+y+z) mod 2;
 *   - E = -sum_bonds J_b s_i s_j (each bond once; J_b = 1 for Ising),
 *     M = sum_i s_i, both exact 64-bit integers;
 *   - a sweep with absolute index t updates every colour-0 site, then every
 *     colour-1 site; site s flips iff r < T[(k+2d)/2], k = s_i*h_i, h_i the
 *     J-weighted neighbour sum (Sec. 3, Eq. 2: dE = 2k), where
 *     T = 2^32 for k <= 0 and floor(2^32*exp(-(beta*2k))) otherwise,
 *     computed on the host in IEEE double and compared as 64-bit integers;
 *   - r is word (s>>1)&3 of Philox4x32-10 (Salmon et al., SC'11) with key
 *     (seed_lo, seed_hi) and counter (s>>3, t, replica, colour);
 *   - hot start: spin s = +1 iff bit 31 of word s&3 of Philox with counter
 *     (s>>2, 0, replica, 2) is set;
 *   - generated couplings: J[dir][s] = -1 iff bit 31 of word s&3 of
 *     Philox(key = coupling seed, counter (s>>2, dir, realisation, 3)).
 *
 * Layouts: spins are int8 (+1/-1), N = L^d of them in site order.
 * Couplings are int8 (+1/-1), layout [dir][site]: J[dir*N + s] is the bond
 * between s and its +1 neighbour along dir (dir 0 = x, 1 = y, 2 = z).
 *
 * Errors: functions returning int give SPIN_OK (0) or a negative
 * spin_status; constructors return NULL.  spin_last_error() then holds a
 * message for the calling thread.  Work is enqueued on the handle's HIP
 * stream; a device fault surfaces at the next call that synchronises.
 *
 * Threading: a handle must not be used by two threads at once; different
 * handles are independent.  All host buffers belong to the caller and are
 * only read/written during the call.  Device memory belongs to the library.
 */
#ifndef SPIN_H
#define SPIN_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct spin_lattice spin_lattice;

enum spin_model { SPIN_ISING = 0, SPIN_EA_PMJ = 1 };

enum spin_status {
  SPIN_OK = 0,
  SPIN_EINVAL = -1,  /* bad argument (message says which) */
  SPIN_ENOMEM = -2,  /* device allocation failed */
  SPIN_EDEVICE = -3, /* HIP runtime or kernel error */
  SPIN_ESTATE = -4   /* call not valid in the handle's state */
};

/* Kernel families; the chain (and so every bit of output) is the same. */
enum spin_kernel {
  SPIN_KERNEL_AUTO = 0,     /* library picks */
  SPIN_KERNEL_GENERIC = 1,  /* per-site, global memory, any even L */
  SPIN_KERNEL_RESIDENT = 2, /* whole lattice in one workgroup's LDS, all sweeps in one launch */
  SPIN_KERNEL_TILED = 3,    /* LDS tile + halo per colour phase, needs L % 8 == 0 */
  SPIN_KERNEL_FUSED = 4,    /* Ising, both colours per launch on the shapes it is built for, ping-pong buffers */
  SPIN_KERNEL_STREAM = 5    /* both colours per launch streamed over planes, spins nibble-packed in LDS;
                               any L % 8 == 0 with L >= 16, both models, ping-pong buffers */
};

/* Source of the update draws (spin_set_rng).  SPIN_RNG_PHILOX is the
 * canonical chain above.  The others reproduce the generators of the
 * paper's RNG-quality experiment (Sec. 4, first paragraph) on the same
 * checkerboard chain: every 8-site group s>>3 owns one generator whose next
 * four numbers decide its four sites of a colour phase, in increasing x.
 *   SPIN_RNG_LCG32_ARRAY: x -> 1664525 x + 1013904223 (mod 2^32), draw x;
 *     each group seeded by word 0 of Philox (g, 0, replica, 6);
 *   SPIN_RNG_LCG32_DISJOINT: the same generator, one sequence from x0 =
 *     word 0 of Philox (0, 0, replica, 7), group g starting
 *     g * floor(2^32 / G) steps in (G = L^d/8 groups);
 *   SPIN_RNG_LCG64_DISJOINT: x -> 6364136223846793005 x +
 *     1442695040888963407 (mod 2^64), draw = high 32 bits; x0 = words 1:0
 *     of that Philox block; blocks of floor(2^64 / G). */
enum spin_rng {
  SPIN_RNG_PHILOX = 0,
  SPIN_RNG_LCG32_ARRAY = 1,
  SPIN_RNG_LCG32_DISJOINT = 2,
  SPIN_RNG_LCG64_DISJOINT = 3
};

/* Order of the updates within a sweep (spin_set_schedule). */
enum spin_schedule {
  SPIN_SCHEDULE_CHECKERBOARD = 0, /* the chain above (default) */
  SPIN_SCHEDULE_COARSE = 1        /* the paper's coarse-tile order with multi-hit: its own chain */
};

/* Full set of creation parameters. */
typedef struct {
  int model;                 /* spin_model */
  int L;                     /* edge, even, >= 4; L^d/8 < 2^32 */
  int d;                     /* 2 or 3 */
  const int8_t* couplings;   /* host, d*L^d values +-1 ([dir][site]); copied.
                                Ising: must be NULL.  EA: NULL means generate
                                from coupling_seed / realisation on the device. */
  uint64_t coupling_seed;    /* EA with couplings == NULL only */
  uint32_t realisation;      /* EA with couplings == NULL only */
  uint64_t seed;             /* Philox key of the hot start and of the updates */
  uint32_t replica;          /* third counter word of the hot start and updates */
  void* stream;              /* hipStream_t to enqueue on; NULL = null stream */
} spin_config;

/* Sec. 3 and Sec. 4: create a lattice in the seeded hot start (replica 0,
 * null stream).  couplings: NULL for SPIN_ISING; for SPIN_EA_PMJ a host
 * array of d*L^d values +-1, copied before return.  NULL on error. */
spin_lattice* spin_create(int model, int L, int d, const int8_t* couplings, uint64_t seed);

/* Same with every parameter (replica, stream, generated couplings). */
spin_lattice* spin_create_config(const spin_config* cfg);

/* Release a handle and its device memory; NULL is ignored.  Waits for the
 * handle's queued work first. */
void spin_free(spin_lattice* h);

/* Sec. 3, steps 1-7 (read as the plain red/black chain) with Eq. 2:
 * enqueue n >= 0 sweeps at inverse temperature beta (finite and >= 0, or
 * +inf for a zero-temperature quench; NaN or negative is SPIN_EINVAL).
 * Asynchronous.  The handle's sweep counter advances by n, so
 * spin_sweep(h,a,b); spin_sweep(h,c,b) equals spin_sweep(h,a+c,b). */
int spin_sweep(spin_lattice* h, int n, double beta);

/* As spin_sweep, and record (E, M) after every every-th sweep of this call
 * (n/every records; every >= 1).  E and M are HOST arrays of n/every int64;
 * the call synchronises before returning. */
int spin_sweep_record(spin_lattice* h, int n, double beta, int every, int64_t* E, int64_t* M);

/* As spin_sweep_record, but E and M are DEVICE arrays (n/every int64 each)
 * written asynchronously on the handle's stream. */
int spin_sweep_record_device(spin_lattice* h, int n, double beta, int every, int64_t* E, int64_t* M);

/* For callers that cannot allocate device memory (code under stream
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * call as spin_sweep_record_device -- same arguments, same bits, E and M
 * DEVICE arrays of n/every int64 owned by the caller -- that calls no
 * hipMalloc/hipFree (nor the allocator hook) and never synchronises.  Its
 * scratch (the per-workgroup partial counts of the records, and the task
 * block of the LDS-resident path) is one library-owned device array of
 * SPIN_NOALLOC_SCRATCH_BYTES per GPU, held until the process ends.  A call
 * whose records need more than that fails with SPIN_EINVAL before any work
 * (record fewer sweeps per call); a handle whose buffers for its kernel are
 * missing (possible only after another handle's spin_autotune changed the
 * automatic choice) fails with SPIN_ESTATE -- spin_create, spin_set_kernel,
 * spin_set_schedule and spin_autotune allocate them.  All calls on one GPU
 * share the array and keep the last call's contents: calls that overlap on
 * one GPU (two threads, or two streams running at once) race. */
#define SPIN_NOALLOC_SCRATCH_BYTES ((size_t)2 << 20)
int spin_sweep_record_noalloc(spin_lattice* h, int n, double beta, int every, int64_t* E, int64_t* M);

/* Sec. 4 (the energy and magnetisation measured between sweeps): current
 * E and M into host int64s.  Synchronises. */
int spin_measure(spin_lattice* h, int64_t* E, int64_t* M);

/* Copy the L^d spins to / from host memory (n must equal L^d; values put
 * must be +-1).  Synchronous. */
int spin_get_spins(const spin_lattice* h, int8_t* out, size_t n);
int spin_set_spins(spin_lattice* h, const int8_t* in, size_t n);

/* Couplings actually used (d*L^d int8, [dir][site]) into a host array.
 * SPIN_ESTATE for the Ising model. */
int spin_get_couplings(const spin_lattice* h, int8_t* out, size_t n);

/* Absolute index of the next sweep (number of sweeps done so far). */
uint64_t spin_sweeps_done(const spin_lattice* h);

/* Set the absolute sweep index of the next sweep (resume from a saved
 * state together with spin_set_spins).  index + later sweeps < 2^32. */
int spin_set_sweeps_done(spin_lattice* h, uint64_t t);

/* Sec. 4 (many independent runs of one system): the third Philox counter
 * word of later updates becomes `replica`; spins and sweep index stay, so the
 * chain continues as that replica's from the present state (the hot start of
 * a new handle also draws with the replica it was created with).
 * SPIN_ESTATE in the LCG draw modes, whose generators were seeded from the
 * replica when the mode was set. */
int spin_set_replica(spin_lattice* h, uint32_t replica);

/* Enqueue later work on this hipStream_t (NULL = null stream). */
int spin_set_stream(spin_lattice* h, void* stream);

/* Choose the kernel family and tile shape: tile_x (bytes, multiple of 8),
 * tile_y, tile_z (rows/planes) and threads per workgroup (multiple of 64).
 * 0 means the library default.  SPIN_EINVAL if the family cannot run this
 * lattice.  Results are bit-identical for every accepted choice.  2D Ising
 * in SPIN_KERNEL_FUSED with full rows (tile_x == L >= 4096): tile_y is the
 * strip height (even, >= 4) and tile_z 0 the row-streaming kernel, 1 its
 * register-column form; both count E/M inside the sweep when a record is due. */
int spin_set_kernel(spin_lattice* h, int kernel, int tile_x, int tile_y, int tile_z, int threads);

/* Sec. 3, steps 1-7, with the generalized multi-hit of the paragraph after
 * them: the paper's own update order, a chain of its own that depends on
 * tile and hits.  With SPIN_SCHEDULE_COARSE the lattice is cut into tiles
 * of edge `tile` (2D: 8, 16, 32 or 64; 3D: 8 or 16; L/tile even); a sweep
 * updates every tile whose tile coordinates sum to an even number, then
 * every odd one; inside a tile its colour-0 sites, then its colour-1
 * sites, `hits` times (>= 1), each from the current spins.  A sweep is
 * hits * L^d attempts; hit h of sweep t of site s with colour c draws word
 * (s>>1)&3 of Philox counter (s>>3, t*hits + h, replica, c), so
 * (sweep index + sweeps) * hits must stay <= 2^32.  The kernel family
 * setting does not apply.  SPIN_SCHEDULE_CHECKERBOARD (tile and hits
 * ignored) restores the canonical chain.  SPIN_EINVAL for other values. */
int spin_set_schedule(spin_lattice* h, int schedule, int tile, int hits);

/* Sec. 4 (tile sizes chosen by experiment): time every family and tile that
 * can run this handle's shape for `sweeps` (1..1000) sweeps at beta on a
 * scratch lattice of the same shape (the handle's spins, couplings and
 * sweep counter are untouched), select the fastest for the handle and
 * remember it for the process: handles of the same (model, L, d) in the
 * AUTO family use it from then on.  Synchronises.  Returns the chosen
 * spin_kernel value, or a negative status.  Bits never change. */
int spin_autotune(spin_lattice* h, double beta, int sweeps);

/* Select the draw source (enum spin_rng).  An LCG mode (Ising, L % 8 == 0,
 * checkerboard schedule only) (re)starts every group's generator from its
 * initial state; the sweeps then run one kernel per colour phase with the
 * spins in place.  SPIN_EINVAL for an unknown mode or a lattice it cannot
 * run; switching back to SPIN_RNG_PHILOX keeps the spins. */
int spin_set_rng(spin_lattice* h, int rng);

/* The LCG modes' generator states (uint64, one per 8-site group, n ==
 * L^d / 8) into a host array.  Synchronous.  SPIN_ESTATE under Philox. */
int spin_get_rng_state(const spin_lattice* h, uint64_t* out, size_t n);

/* Kernel family that spin_sweep will use next (spin_kernel value). */
int spin_get_kernel(const spin_lattice* h);

/* Tile shape that spin_sweep will use next (as spin_set_kernel takes it;
 * for the 2D row-streaming kernel tile_z == 1 selects its register-column
 * form).  Host ints; NULL pointers are skipped. */
int spin_get_tile(const spin_lattice* h, int* tile_x, int* tile_y, int* tile_z, int* threads);

/* Wait for the handle's queued work. */
int spin_synchronize(spin_lattice* h);

/* Device pointer to the current spins (valid until the next sweep call,
 * which may swap buffers).  NULL on error. */
const int8_t* spin_device_spins(const spin_lattice* h);

/* Sec. 3, Eq. 2: the acceptance table the library uses, T[(k+2d)/2] for
 * k = -2d..2d step 2 (2d+1 uint64 values written to T).  Host only. */
int spin_threshold_table(double beta, int d, uint64_t* T);

/* Install device allocation callbacks (NULL, NULL restores hipMalloc /
 * hipFree).  alloc(bytes, ctx) returns a device pointer or NULL;
 * release(ptr, ctx) frees it.  Affects handles created afterwards. */
void spin_set_allocator(void* (*alloc)(size_t, void*), void (*release)(void*, void*), void* ctx);

/* Test hooks for the out-of-memory paths (no passage of the paper; for
 * tests that force allocation failures).  spin_debug_fault_alloc(k) with
 * k >= 0: the library's next k device allocations succeed and the one after
 * them fails as if the device were out of memory (SPIN_ENOMEM from the call
 * that made it), after which injection is off again; k = -1 turns it off.
 * The environment variable SPIN_FAULT_ALLOC=k sets the same at the first
 * allocation of the process.  spin_debug_live_allocations: device blocks
 * the library holds now (lattices, pools and their buffers), for leak
 * checks. */
int spin_debug_fault_alloc(int64_t after);
int64_t spin_debug_live_allocations(void);

/* Message of the last failed call on this thread ("" if none). */
const char* spin_last_error(void);

/* Status code (spin_status) of that call: what a constructor that returned
 * NULL failed with. */
int spin_last_status(void);

/* Library version string. */
const char* spin_version(void);

/* ------------------------------------------------------------------ batches
 * Sec. 4, last paragraph (parallelism over many disorder realisations):
 * a pool of independent lattices advanced together.  A member whose spins
 * fit one workgroup's LDS (L % 8 == 0, L >= 8, L^d/2 bytes <= 150 KiB:
 * 2D L <= 552, 3D L <= 64) is swept by one persistent launch per class of
 * (d, model, size) that takes the members from a queue, largest work first;
 * any other valid lattice (even L >= 4) is advanced by the single-lattice
 * kernels within the same call, on internal streams that start after the
 * work already queued on the batch's stream and that the batch's stream
 * waits for before its later work, so they run alongside the persistent
 * launch and each other.  Every member follows
 * exactly the chain of a lone lattice with the same seed, replica and
 * couplings (same bits).
 *
 * Members live in numbered slots 0..spin_batch_size()-1.  spin_batch_add
 * reuses the most recently freed slot, if any, else appends one;
 * spin_batch_remove frees a slot.  Per-slot host arrays (n, beta, E, M of
 * spin_batch_measure) have spin_batch_size() entries; a free slot must get
 * n == 0 and its beta is ignored.
 */
typedef struct {
  int model;                 /* spin_model */
  int L, d;
  const int8_t* couplings;   /* host d*L^d +-1 ([dir][site]) copied before return, or NULL:
                                EA generates from coupling_seed/realisation (members of the
                                LDS-sized kind with the same four values (seed, realisation,
                                L, d) share one device copy), Ising: NULL */
  uint64_t coupling_seed;
  uint32_t realisation;
  uint64_t seed;
  uint32_t replica;
} spin_desc;

typedef struct spin_batch spin_batch;

/* Create a pool holding count >= 0 lattices (slots 0..count-1) in their hot
 * starts on hipStream_t stream (NULL = null stream).  NULL on error
 * (spin_last_error says which lattice). */
spin_batch* spin_batch_create(int count, const spin_desc* descs, void* stream);
void spin_batch_free(spin_batch* b);               /* NULL-safe; waits for queued work */

/* Number of slots (members and free slots). */
int  spin_batch_size(const spin_batch* b);

/* Add a lattice in its hot start; returns its slot (>= 0) or a negative
 * spin_status.  Work is enqueued on the batch's stream; may synchronise. */
int  spin_batch_add(spin_batch* b, const spin_desc* desc);

/* Remove the lattice in slot i and release its memory to the pool (device
 * memory returns to the system at spin_batch_free).  Synchronises. */
int  spin_batch_remove(spin_batch* b, int i);

/* 1 if slot i holds a lattice, else 0. */
int  spin_batch_is_member(const spin_batch* b, int i);

/* Device bytes that slot i's lattice may hold: spins (twice L^d for a
 * lattice beyond the LDS-sized kind: the streaming kernels' second buffer)
 * plus its couplings (d*L^d/2 packed for the LDS-sized kind, 3*d*L^d/2 --
 * int8 and packed -- otherwise), counted in full even when shared with
 * other members; 0 for a free slot.  An upper bound for admission control. */
uint64_t spin_batch_footprint(const spin_batch* b, int i);

/* Advance slot i by n[i] >= 0 sweeps at beta[i] (host arrays of
 * spin_batch_size() entries).  If every >= 1, record (E, M) after every
 * every-th sweep of each member; slot i's n[i]/every records (one record of
 * the current state when n[i] == 0) sit in E, M (HOST arrays) at offset
 * sum_{j<i} of the earlier slots' counts (free slots count 0).  Synchronises. */
int spin_batch_sweep(spin_batch* b, const int* n, const double* beta, int every, int64_t* E, int64_t* M);

/* Sec. 4 (tile sizes chosen by experiment), for the persistent launch: for
 * every lattice shape (d, model, L) among the pool's LDS-held members, time
 * each launch shape -- workgroups of 256, 512, 576 or 1024 threads, 1 .. as many
 * workgroups per CU as threads and LDS allow -- on scratch lattices of that
 * shape (as many as the pool holds, at most four per CU), `sweeps` sweeps at
 * beta each; check that every candidate leaves identical spins (else
 * SPIN_EDEVICE); keep the fastest as the shape's plan for every pool of the
 * process, and append it to the tuning cache file (SPIN_TUNE_CACHE, default
 * $HOME/.cache/spin-gfx950/tune.txt; records "batch <arch> d model L threads
 * workgroups_per_cu ns_per_sweep", read back at the first pool call of a
 * later process).  The pool's own lattices are not touched.  Returns the
 * number of shapes tuned or a negative status.  Synchronises. */
int spin_batch_autotune(spin_batch* b, double beta, int sweeps);

/* The plan of shape (d, model, L): 1 and its threads and workgroups per CU,
 * or 0 (outputs 0) when the shape has none and the static rule applies. */
int spin_batch_plan(int d, int model, int L, int* threads, int* workgroups_per_cu);

/* As spin_batch_sweep with DEVICE record arrays; asynchronous.
 * Graph capture: a call made while the pool's stream (a non-null stream
 * given at creation) is being captured enqueues only kernel launches -- the
 * queue counters are cleared by a kernel, and the per-slot tables must
 * already be on the device, so its arguments (n, beta, every, E, M) must
 * repeat those of the pool's previous, uncaptured call, and only members
 * held in LDS may sweep or record (else SPIN_ESTATE, nothing enqueued).
 * Every replay of the graph advances those members by n[i] sweeps from
 * where the previous replay left them and rewrites the same record slots;
 * spin_batch_sweeps_done and the next uncaptured call read the advanced
 * counters back from the device. */
int spin_batch_sweep_device(spin_batch* b, const int* n, const double* beta, int every, int64_t* E,
                            int64_t* M);

/* E, M of every slot (host arrays of spin_batch_size(); 0 for free slots).
 * Synchronises. */
int spin_batch_measure(spin_batch* b, int64_t* E, int64_t* M);

/* Spins of slot i to / from a host array of n == L^d values.  Synchronous. */
int spin_batch_get_spins(const spin_batch* b, int i, int8_t* out, size_t n);
int spin_batch_set_spins(spin_batch* b, int i, const int8_t* in, size_t n);

/* Absolute index of slot i's next sweep (0 for a free slot). */
uint64_t spin_batch_sweeps_done(const spin_batch* b, int i);

/* Workgroups resident per compute unit for the batch launches (0 = as many
 * as LDS and the workgroup size allow; 1..8 otherwise).  Bits never change. */
int spin_batch_set_workgroups_per_cu(spin_batch* b, int wgs);

/* Wait for the batch's queued work. */
int spin_batch_synchronize(spin_batch* b);

/* ---------------------------------------------------- continuous spins
 * Sec. 4, closing paragraph (the method generalises to continuous spins such
 * as the Heisenberg model, where single-precision floating point comes into
 * play): the classical Heisenberg ferromagnet, unit vectors S_s in R^3,
 * E = - sum_s sum_dir S_s . S_{s+e_dir}, periodic L^d (d = 2, 3, L even),
 * the red/black sweep of the canonical chain, arithmetic in float.
 * Site s draws Philox (s, 0, replica, 9) for its hot start and
 * (s, t, replica, 10 + c) in sweep t, colour c; with u_i = (w_i >> 8) 2^-24
 * a direction is z = 2 u0 - 1, phi = 2 pi u1, rho = sqrt(fma(-z, z, 1)),
 * (rho cos phi, rho sin phi, z); the trial S' replaces S iff dE <= 0 or
 * u2 < exp(-(beta dE)) (the Metropolis rule, Sec. 3, Eq. 2), dE = S.h - S'.h
 * with h the sum of the 2d neighbour vectors (order -x, +x, -y, +y, -z, +z)
 * and a.h = fma(a.x, h.x, fma(a.y, h.y, a.z h.z)).  cos, sin and exp are
 * evaluated by one stated method, each step a single IEEE float operation:
 * the angle reduced to its octant (o = floor(8 u1), exact) and Taylor
 * polynomials of cos and sin on [0, pi/4] to x^10 and x^9; exp(y) for
 * -87 < y < 0 as 2^k e^r with k = floor(y log2 e + 1/2), r = y - k ln 2
 * (ln 2 in two parts) and e^r by its Taylor polynomial to r^7; y <= -87
 * rejects.  Every result is therefore a definite float.  Spins live on the
 * device as float4 (x, y, z, 0).  A sweep is L^d attempts. */
typedef struct spin_heis spin_heis;

/* NULL on error (spin_last_error). */
spin_heis* spin_heis_create(int L, int d, uint64_t seed, uint32_t replica, void* stream);
void spin_heis_free(spin_heis* h);                 /* NULL-safe; waits for queued work */

/* n >= 0 sweeps at beta >= 0 (rounded to float); asynchronous. */
int spin_heis_sweep(spin_heis* h, int n, double beta);

/* As spin_heis_sweep, recording after every every-th sweep E[r] and |M|[r]
 * (n/every records, HOST arrays of double, sums accumulated in double).
 * Synchronises. */
int spin_heis_sweep_record(spin_heis* h, int n, double beta, int every, double* E, double* Mabs);

/* Current E and magnetisation vector M[3] (host, double).  Synchronises. */
int spin_heis_measure(spin_heis* h, double* E, double* M);

/* Spins into a host array of n == 4 L^d floats (x, y, z, 0 per site).
 * Synchronous. */
int spin_heis_get_spins(const spin_heis* h, float* out, size_t n);

/* Spins from a host array of n == 4 L^d floats (x, y, z, 0 per site):
 * components finite, the fourth 0 (SPIN_EINVAL otherwise); taken as given,
 * not normalised.  Synchronous. */
int spin_heis_set_spins(spin_heis* h, const float* in, size_t n);

/* Absolute index of the next sweep. */
uint64_t spin_heis_sweeps_done(const spin_heis* h);

/* Set the absolute index of the next sweep (resume from a saved state with
 * spin_heis_set_spins); index + later sweeps <= 2^32. */
int spin_heis_set_sweeps_done(spin_heis* h, uint64_t t);

/* Wait for the handle's queued work. */
int spin_heis_synchronize(spin_heis* h);

/* ---------------------------------------------------- multi-spin coding
 * Sec. 4, last paragraph (many disorder realisations at once, combined with
 * multi-spin coding): 32 +-J systems of edge L (L % 8 == 0, d = 2 or 3) in
 * the bits of one 32-bit word per site.  System b has the couplings of
 * realisation realisation0 + b and the hot start of replica replica0 + b,
 * by the rules at the top of this file (with the coupling seed and seed
 * given), so each system is the lattice spin_create_config would make.
 * A chain of its own: in sweep t, colour c, site s draws one word,
 * (s>>1)&3 of Philox(seed, counter (s>>3, t, replica0, 4 + c)), shared by
 * the 32 systems; system b flips s iff that word < T[(k_b+2d)/2] with its
 * own k_b (Eq. 2).  A sweep is 32 * L^d attempts. */
typedef struct spin_msc spin_msc;

/* NULL on error (spin_last_error). */
spin_msc* spin_msc_create(int L, int d, uint64_t coupling_seed, uint32_t realisation0, uint64_t seed,
                          uint32_t replica0, void* stream);
void spin_msc_free(spin_msc* h);                   /* NULL-safe; waits for queued work */

/* n >= 0 sweeps at beta (as spin_sweep); asynchronous. */
int spin_msc_sweep(spin_msc* h, int n, double beta);

/* As spin_msc_sweep, recording after every every-th sweep the 32 energies
 * and magnetisations: E[r*32 + b], M[r*32 + b] for record r (n/every
 * records; HOST arrays).  Synchronises. */
int spin_msc_sweep_record(spin_msc* h, int n, double beta, int every, int64_t* E, int64_t* M);

/* Current E[b], M[b] of the 32 systems (host arrays of 32).  Synchronises. */
int spin_msc_measure(spin_msc* h, int64_t* E, int64_t* M);

/* Spins of system b (0..31) into a host array of n == L^d int8.  Synchronous. */
int spin_msc_get_spins(const spin_msc* h, int system, int8_t* out, size_t n);

/* Absolute index of the next sweep. */
uint64_t spin_msc_sweeps_done(const spin_msc* h);

/* Kernel choice (bits never change): streaming == 1 sweeps both colours in
 * one launch streamed over planes, with rows (3D: rows per workgroup,
 * dividing L, <= 32), planes (per strip), threads (256 or 512) and width
 * (sites of a row per workgroup: a multiple of 8 dividing L), 0 meaning the
 * default (8, 16, 512, L); streaming == 2 (3D, L = 128, 256 or 512) is the
 * register-column kernel, which reads every coupling word once per sweep:
 * rows 4 or 8 (default 8), planes even and dividing L (default 32), threads
 * 0 or 64 * (rows + 2), width 0 or L; streaming == 0 launches one kernel per
 * colour.
 * At creation the library picks a streaming shape measured to be fast for
 * L and d where one fits, else the per-colour kernel.  SPIN_EINVAL if the
 * streaming shape does not fit L. */
int spin_msc_set_kernel(spin_msc* h, int streaming, int rows, int planes, int threads, int width);

/* The kernel the next sweep uses: 0 (one launch per colour), 1 (streamed
 * over planes) or 2 (register columns), as spin_msc_set_kernel's streaming;
 * -1 for a NULL handle. */
int spin_msc_kernel(const spin_msc* h);

/* Wait for the handle's queued work. */
int spin_msc_synchronize(spin_msc* h);

#ifdef __cplusplus
}
#endif

#endif /* SPIN_H */
