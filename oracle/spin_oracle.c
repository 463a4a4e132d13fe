/*
 * spin_oracle.c -- plain, single-threaded CPU oracle for checkerboard
 * Metropolis sweeps of the 2D/3D Ising ferromagnet and the +-J
 * Edwards-Anderson spin glass.
 *
 * THIS IS TEST INFRASTRUCTURE.  Only the test-suite, the smoke check and the
 * CPU-baseline leg of the benchmark load it.  It shares no code, header,
 * table or constant with the GPU library; it is written to be read against
 * the paper (Weigel, "Simulating spin models on GPU"), not to be fast.
 *
 * What it computes (the canonical chain):
 *
 *  Lattice (Sec. 3, Eq. 1 and the sentence after it): edge L (even), d = 2
 *  or 3, periodic boundaries, site index s = x + L*(y + L*z) with x
 *  fastest.  Colour of a site = (x + y + z) mod 2.
 *
 *  Energy (Sec. 3, Eq. 1, with J = 1 absorbed into beta; the +-J glass of
 *  Sec. 4, last paragraph, replaces J by a bond variable J_ij):
 *      E = - sum_s sum_dir J[dir][s] * s_s * s_{s + e_dir}
 *  every bond counted once.  For the ferromagnet J == 1.
 *
 *  Metropolis rule (Sec. 3, Eq. 2): flipping s_i changes the energy by
 *  dE = 2*k with k = s_i * h_i, h_i = sum of J-weighted neighbour spins.
 *  The move is accepted with probability min(1, exp(-beta*dE)).  With a
 *  uniform 32-bit integer r this is decided exactly as  r < T[k]  where
 *      T[k] = 2^32                                 for k <= 0,
 *      T[k] = floor(2^32 * exp(-(beta*(2k))))      for k  > 0,
 *  evaluated in IEEE double (one rounding of the product beta*dE, libm exp,
 *  exact scaling by 2^32, floor) and stored as a 64-bit integer, so the
 *  compare is between 64-bit integers.  The table is indexed by (k+z)/2,
 *  z = 2d.
 *
 *  Random numbers: Philox4x32-10 (Salmon, Moraes, Dror & Shaw, "Parallel
 *  random numbers: as easy as 1, 2, 3", SC'11) with key (seed_lo, seed_hi).
 *  The paper's per-thread LCG array (Sec. 4, first paragraph) is replaced
 *  by this counter-based generator; its period concerns are the reason.
 *  Counter layouts (c0, c1, c2, c3), word index in brackets:
 *      update of site s in sweep t, colour c : (s>>3, t, replica, c) [(s>>1)&3]
 *      hot-start spin of site s               : (s>>2, 0, replica, 2) [s&3]
 *      coupling J[dir][s] (key = coupling seed): (s>>2, dir, realisation, 3) [s&3]
 *  A hot-start spin is +1 when bit 31 of its word is set, else -1; a
 *  coupling is -1 when bit 31 of its word is set, else +1.
 *
 *  Sweep t (Sec. 3, steps 1-7, read as the plain red/black chain): first
 *  every colour-0 site, then every colour-1 site, each site updated from
 *  the current spins; the order inside a colour does not matter because no
 *  two sites of one colour are neighbours (Sec. 3, the sentence on the
 *  independence of sub-lattice sites).  The paper's coarse-tile ordering
 *  and its k-fold multi-hit repetition change the chain; they are a
 *  separate mode, oracle_coarse_sweeps below.
 *
 *  The paper's own schedule (Sec. 3, steps 1-7, with the generalized
 *  multi-hit of the paragraph after them), as an explicit mode with its own
 *  chain: the lattice is cut into tiles of edge T, B = L/T per edge (B
 *  even); a tile is even or odd by the parity of the sum of its tile
 *  coordinates.  Sweep t: for tile parity q = 0, then q = 1, in every tile
 *  of parity q, k times: update the tile's colour-0 sites, then its
 *  colour-1 sites (colour = (x+y+z) mod 2 as above), each from the current
 *  spins.  Tiles of one parity are never neighbours, so they are
 *  independent.  Hit h (0..k-1) of site s of colour c in sweep t draws
 *  word (s>>1)&3 of Philox counter (s>>3, t*k + h, replica, c).  With
 *  T = 1 and k = 1 this is the canonical chain.
 *
 *  Multi-spin coding of the +-J glass (Sec. 4, last paragraph: many
 *  disorder realisations at once, combined with asynchronous multi-spin
 *  coding), a mode with its own chain: 32 systems b = 0..31 of edge L
 *  share the lattice; system b has the couplings of realisation r0 + b and
 *  the hot start of replica p0 + b, both by the rules above.  In sweep t,
 *  colour c, site s draws ONE word, (s>>1)&3 of Philox counter
 *  (s>>3, t, p0, 4 + c), shared by the 32 systems; each system b flips its
 *  spin iff r < T[(k_b + z)/2] with its own k_b.  Each system alone is a
 *  Metropolis chain of its realisation; the systems are coupled only
 *  through the shared draws.
 *
 *  Linear congruential generators (Sec. 4, first paragraph: the RNG-quality
 *  experiment), a mode of the canonical chain with another source of draws:
 *  every 8-site group g = s>>3 (the "thread") owns one generator state; in
 *  each colour phase the group's four sites of that colour draw the next
 *  four numbers of its stream in increasing x.  Step x -> a x + c with
 *      32-bit: a = 1664525, c = 1013904223 (mod 2^32), draw = x,
 *      64-bit: a = 6364136223846793005, c = 1442695040888963407 (mod 2^64),
 *              draw = the high 32 bits of x,
 *  the new state being the draw's source.  Initial states, G = L^d/8 groups:
 *      mode 1 (array, one multiplier, random seeds): 32-bit, state of g =
 *              word 0 of Philox counter (g, 0, replica, 6);
 *      mode 2 (disjoint sub-sequences of one 32-bit LCG): x0 = word 0 of
 *              Philox counter (0, 0, replica, 7); group g starts g*len steps
 *              after x0, len = floor(2^32 / G);
 *      mode 3 (disjoint sub-sequences of one 64-bit LCG): x0 = word 1 of
 *              that block * 2^32 + word 0; len = floor(2^64 / G).
 *  Everything else (table, acceptance compare, colour order) is as above.
 *
 *  Continuous spins (Sec. 4, closing paragraph: the remark on generalising to models with
 *  continuous spins such as the Heisenberg model in single precision): the
 *  classical Heisenberg ferromagnet, unit vectors S_s in R^3, energy
 *  E = - sum_s sum_dir S_s . S_{s+e_dir}.  Same lattice, colours and sweep
 *  order as the canonical chain; arithmetic in IEEE single precision.
 *  Draw words of site s: hot start Philox (s, 0, replica, 9), update in
 *  sweep t, colour c Philox (s, t, replica, 10 + c); u_i = (w_i >> 8) 2^-24.
 *  A direction from (u0, u1): z = 2 u0 - 1, rho = sqrt(fma(-z, z, 1)),
 *  (rho cos phi, rho sin phi, z) with phi = 2 pi u1.  cos and sin are
 *  evaluated as follows (every step a single IEEE float operation, so the
 *  result is a definite float): the octant o = floor(8 u1) and r = 8 u1 - o
 *  (both exact); a = r for even o, 1 - r for odd o (exact); x = a * (pi/4
 *  rounded to float); C = 1 - x^2/2! + ... - x^10/10!, S = x - x^3/3! + ...
 *  + x^9/9! by Horner steps in x^2 with fma (coefficients 1/n! rounded to
 *  float); odd octants swap C and S; quadrant o>>1 rotates (C, S) by
 *  multiples of pi/2.  Update: h = sum of the 2d neighbour vectors (added
 *  in the order -x, +x, -y, +y, -z, +z, each component separately); trial
 *  S' from (u0, u1); dE = S.h - S'.h with a.h = fma(a.x, h.x, fma(a.y, h.y,
 *  a.z * h.z)); the Metropolis rule (Sec. 3, Eq. 2) accepts every dE <= 0
 *  (also at beta = inf, where beta * 0 would be undefined); otherwise
 *  y = -(beta * dE) (beta rounded to float) and accept iff y >= 0 (beta =
 *  0), or y > -87 and u2 < p with p = 2^k e^r: k = floor(y log2(e) +
 *  1/2) (fma), r = y - k ln2 in two fma steps with ln2 split into a high
 *  part exact in float and the rest, e^r = 1 + r + ... + r^7/7! by Horner
 *  with fma, and the scaling by 2^k exact (ldexp).
 */
#include <math.h>
#include <stddef.h>
#include <stdint.h>
#include <stdlib.h>

/* ---------------------------------------------------------------- Philox */

/* One Philox4x32-10 block: ten rounds of the S-box below, with the key
 * bumped by the Weyl constants between rounds (SC'11, Sec. 3.2). */
void oracle_philox4x32_10(const uint32_t ctr_in[4], const uint32_t key_in[2],
                          uint32_t out[4]) {
  const uint32_t M0 = 0xD2511F53u, M1 = 0xCD9E8D57u;
  const uint32_t W0 = 0x9E3779B9u, W1 = 0xBB67AE85u;
  uint32_t c0 = ctr_in[0], c1 = ctr_in[1], c2 = ctr_in[2], c3 = ctr_in[3];
  uint32_t k0 = key_in[0], k1 = key_in[1];
  for (int round = 0; round < 10; ++round) {
    uint64_t p0 = (uint64_t)M0 * (uint64_t)c0;
    uint64_t p1 = (uint64_t)M1 * (uint64_t)c2;
    uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
    uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
    uint32_t n0 = hi1 ^ c1 ^ k0;
    uint32_t n1 = lo1;
    uint32_t n2 = hi0 ^ c3 ^ k1;
    uint32_t n3 = lo0;
    c0 = n0; c1 = n1; c2 = n2; c3 = n3;
    if (round < 9) { k0 += W0; k1 += W1; }
  }
  out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

static uint32_t draw(uint64_t seed, uint32_t c0, uint32_t c1, uint32_t c2,
                     uint32_t c3, unsigned word) {
  uint32_t ctr[4] = {c0, c1, c2, c3};
  uint32_t key[2] = {(uint32_t)(seed & 0xffffffffu), (uint32_t)(seed >> 32)};
  uint32_t out[4];
  oracle_philox4x32_10(ctr, key, out);
  return out[word];
}

/* ------------------------------------------------------ threshold table */

/* T[(k+z)/2] for k = -z, -z+2, ..., z (Sec. 3, Eq. 2). */
void oracle_table(double beta, int d, uint64_t* T) {
  int z = 2 * d;
  for (int k = -z; k <= z; k += 2) {
    uint64_t v;
    if (k <= 0) {
      v = (uint64_t)1 << 32;
    } else {
      double dE = (double)(2 * k);
      double p = exp(-(beta * dE));
      v = (uint64_t)floor(ldexp(p, 32));
    }
    T[(k + z) / 2] = v;
  }
}

/* ------------------------------------------------------------- lattice */

static int64_t site_count(int L, int d) {
  int64_t n = 1;
  for (int i = 0; i < d; ++i) n *= L;
  return n;
}

/* Coordinates of site s. */
static void coords(int64_t s, int L, int d, int64_t x[3]) {
  x[0] = s % L;
  x[1] = (s / L) % L;
  x[2] = (d == 3) ? s / ((int64_t)L * L) : 0;
}

static int64_t index_of(const int64_t x[3], int L, int d) {
  int64_t s = x[0] + (int64_t)L * x[1];
  if (d == 3) s += (int64_t)L * L * x[2];
  return s;
}

/* Neighbour of s one step along +dir (sign=+1) or -dir (sign=-1). */
static int64_t neighbour(int64_t s, int dir, int sign, int L, int d) {
  int64_t x[3];
  coords(s, L, d, x);
  x[dir] = (x[dir] + sign + L) % L;
  return index_of(x, L, d);
}

static int colour_of(int64_t s, int L, int d) {
  int64_t x[3];
  coords(s, L, d, x);
  return (int)((x[0] + x[1] + x[2]) % 2);
}

static int valid_shape(int L, int d) {
  if (d != 2 && d != 3) return 0;
  if (L < 4 || (L % 2) != 0) return 0;
  if (site_count(L, d) / 8 >= ((int64_t)1 << 32)) return 0;
  return 1;
}

/* ---------------------------------------------------- inputs of the chain */

/* Seeded uniform hot start. */
int oracle_init_spins(int L, int d, uint64_t seed, uint32_t replica,
                      int8_t* spins) {
  if (!valid_shape(L, d)) return -1;
  int64_t N = site_count(L, d);
  for (int64_t s = 0; s < N; ++s) {
    uint32_t r = draw(seed, (uint32_t)(s >> 2), 0u, replica, 2u,
                      (unsigned)(s & 3));
    spins[s] = (r >> 31) ? (int8_t)1 : (int8_t)-1;
  }
  return 0;
}

/* +-J couplings, each sign with probability 1/2; layout [dir][site]. */
int oracle_couplings(int L, int d, uint64_t cseed, uint32_t realisation,
                     int8_t* J) {
  if (!valid_shape(L, d)) return -1;
  int64_t N = site_count(L, d);
  for (int dir = 0; dir < d; ++dir)
    for (int64_t s = 0; s < N; ++s) {
      uint32_t r = draw(cseed, (uint32_t)(s >> 2), (uint32_t)dir, realisation,
                        3u, (unsigned)(s & 3));
      J[(int64_t)dir * N + s] = (r >> 31) ? (int8_t)-1 : (int8_t)1;
    }
  return 0;
}

static int coupling(const int8_t* J, int dir, int64_t s, int64_t N) {
  return J ? (int)J[(int64_t)dir * N + s] : 1;
}

/* --------------------------------------------------------- observables */

/* E = -sum over bonds J s s (Eq. 1), M = sum of spins. */
void oracle_measure(int L, int d, const int8_t* J, const int8_t* spins,
                    int64_t* E, int64_t* M) {
  int64_t N = site_count(L, d);
  int64_t e = 0, m = 0;
  for (int64_t s = 0; s < N; ++s) {
    m += spins[s];
    for (int dir = 0; dir < d; ++dir) {
      int64_t t = neighbour(s, dir, +1, L, d);
      e -= (int64_t)coupling(J, dir, s, N) * spins[s] * spins[t];
    }
  }
  *E = e;
  *M = m;
}

/* Local field h_s = sum over the 2d neighbours of J_bond * s_neighbour. */
static int local_field(int64_t s, int L, int d, const int8_t* J,
                       const int8_t* spins, int64_t N) {
  int h = 0;
  for (int dir = 0; dir < d; ++dir) {
    int64_t up = neighbour(s, dir, +1, L, d);
    int64_t dn = neighbour(s, dir, -1, L, d);
    h += coupling(J, dir, s, N) * spins[up];   /* bond (s, s+e_dir)  */
    h += coupling(J, dir, dn, N) * spins[dn];  /* bond (s-e_dir, s)  */
  }
  return h;
}

/* ------------------------------------------------------------- sweeps */

/* Visiting order inside one colour: 0 forward, 1 reverse, 2 a seeded
 * shuffle.  All three give the same bits; the option exists so that the
 * tests can show it. */
static void visit_order(int64_t* list, int64_t n, int order, uint64_t salt) {
  if (order == 1) {
    for (int64_t i = 0; i < n / 2; ++i) {
      int64_t tmp = list[i];
      list[i] = list[n - 1 - i];
      list[n - 1 - i] = tmp;
    }
  } else if (order == 2) {
    uint64_t x = salt * 0x9E3779B97F4A7C15ull + 1;
    for (int64_t i = n - 1; i > 0; --i) {
      x ^= x << 13; x ^= x >> 7; x ^= x << 17;  /* xorshift64 */
      int64_t j = (int64_t)(x % (uint64_t)(i + 1));
      int64_t tmp = list[i];
      list[i] = list[j];
      list[j] = tmp;
    }
  }
}

/*
 * Run n sweeps, the first one with absolute index t0.  If every > 0,
 * (E, M) is written after each every-th sweep of this call (n/every
 * records).  stats, if not NULL, receives per class i = (k+z)/2 the number
 * of attempts stats[i] and acceptances stats[z+1+i].
 * Returns 0, or -1 on bad arguments.
 */
int oracle_sweeps(int L, int d, const int8_t* J, int8_t* spins, uint64_t seed,
                  uint32_t replica, uint64_t t0, int n, double beta, int every,
                  int64_t* E, int64_t* M, int order, uint64_t* stats) {
  if (!valid_shape(L, d) || n < 0) return -1;
  if (isnan(beta) || beta < 0) return -1;
  if (t0 + (uint64_t)n > ((uint64_t)1 << 32)) return -1;
  int z = 2 * d;
  uint64_t T[7];
  oracle_table(beta, d, T);
  int64_t N = site_count(L, d);
  int64_t* list = (int64_t*)malloc(sizeof(int64_t) * (size_t)(N / 2 + 1));
  if (!list) return -1;
  int rec = 0;
  for (int i = 0; i < n; ++i) {
    uint32_t t = (uint32_t)(t0 + (uint64_t)i);
    for (int c = 0; c < 2; ++c) {
      int64_t cnt = 0;
      for (int64_t s = 0; s < N; ++s)
        if (colour_of(s, L, d) == c) list[cnt++] = s;
      visit_order(list, cnt, order, (uint64_t)t * 2 + (uint64_t)c);
      for (int64_t q = 0; q < cnt; ++q) {
        int64_t s = list[q];
        int h = local_field(s, L, d, J, spins, N);
        int k = spins[s] * h;
        int cls = (k + z) / 2;
        uint32_t r = draw(seed, (uint32_t)(s >> 3), t, replica, (uint32_t)c,
                          (unsigned)((s >> 1) & 3));
        int accept = (uint64_t)r < T[cls];
        if (stats) {
          stats[cls] += 1;
          if (accept) stats[z + 1 + cls] += 1;
        }
        if (accept) spins[s] = (int8_t)(-spins[s]);
      }
    }
    if (every > 0 && (i + 1) % every == 0) {
      oracle_measure(L, d, J, spins, &E[rec], &M[rec]);
      ++rec;
    }
  }
  free(list);
  return 0;
}

/*
 * The coarse-tile schedule with k-fold multi-hit (see the header): n sweeps
 * from absolute sweep index t0, each updating every site k times.  Records
 * as in oracle_sweeps.  Requires T >= 1 dividing L with L/T even, k >= 1 and
 * (t0 + n) * k <= 2^32.  Returns 0, or -1 on bad arguments.
 */
int oracle_coarse_sweeps(int L, int d, const int8_t* J, int8_t* spins,
                         uint64_t seed, uint32_t replica, uint64_t t0, int n,
                         double beta, int T, int k, int every, int64_t* E,
                         int64_t* M) {
  if (!valid_shape(L, d) || n < 0 || T < 1 || k < 1) return -1;
  if (L % T != 0 || (L / T) % 2 != 0) return -1;
  if (isnan(beta) || beta < 0) return -1;
  if ((t0 + (uint64_t)n) * (uint64_t)k > ((uint64_t)1 << 32)) return -1;
  int z = 2 * d;
  uint64_t Tab[7];
  oracle_table(beta, d, Tab);
  int64_t N = site_count(L, d);
  int B = L / T;
  int nbz = (d == 3) ? B : 1, tz = (d == 3) ? T : 1;
  int rec = 0;
  for (int i = 0; i < n; ++i) {
    uint64_t t = t0 + (uint64_t)i;
    for (int q = 0; q < 2; ++q)
      for (int bz = 0; bz < nbz; ++bz)
        for (int by = 0; by < B; ++by)
          for (int bx = 0; bx < B; ++bx) {
            if ((bx + by + bz) % 2 != q) continue;
            for (int h = 0; h < k; ++h) {
              uint32_t hit = (uint32_t)(t * (uint64_t)k + (uint64_t)h);
              for (int c = 0; c < 2; ++c)
                for (int zz = 0; zz < tz; ++zz)
                  for (int yy = 0; yy < T; ++yy)
                    for (int xx = 0; xx < T; ++xx) {
                      int64_t x[3] = {(int64_t)bx * T + xx, (int64_t)by * T + yy,
                                      (int64_t)bz * tz + zz};
                      int64_t s = index_of(x, L, d);
                      if (colour_of(s, L, d) != c) continue;
                      int kk = spins[s] * local_field(s, L, d, J, spins, N);
                      uint32_t r = draw(seed, (uint32_t)(s >> 3), hit, replica,
                                        (uint32_t)c, (unsigned)((s >> 1) & 3));
                      if ((uint64_t)r < Tab[(kk + z) / 2])
                        spins[s] = (int8_t)(-spins[s]);
                    }
            }
          }
    if (every > 0 && (i + 1) % every == 0) {
      oracle_measure(L, d, J, spins, &E[rec], &M[rec]);
      ++rec;
    }
  }
  return 0;
}

/*
 * Multi-spin-coded +-J glass (see the header): spins[b*N + s] and
 * J[(b*d + dir)*N + s] hold the 32 systems' spins and couplings.  n sweeps
 * from absolute index t0; if every > 0, the 32 energies and magnetisations
 * after each every-th sweep go to E[rec*32 + b], M[rec*32 + b].
 */
int oracle_msc_sweeps(int L, int d, const int8_t* J, int8_t* spins,
                      uint64_t seed, uint32_t p0, uint64_t t0, int n,
                      double beta, int every, int64_t* E, int64_t* M) {
  if (!valid_shape(L, d) || n < 0 || !J) return -1;
  if (isnan(beta) || beta < 0) return -1;
  if (t0 + (uint64_t)n > ((uint64_t)1 << 32)) return -1;
  int z = 2 * d;
  uint64_t Tab[7];
  oracle_table(beta, d, Tab);
  int64_t N = site_count(L, d);
  int rec = 0;
  for (int i = 0; i < n; ++i) {
    uint32_t t = (uint32_t)(t0 + (uint64_t)i);
    for (int c = 0; c < 2; ++c)
      for (int64_t s = 0; s < N; ++s) {
        if (colour_of(s, L, d) != c) continue;
        uint32_t r = draw(seed, (uint32_t)(s >> 3), t, p0, 4u + (uint32_t)c,
                          (unsigned)((s >> 1) & 3));
        for (int b = 0; b < 32; ++b) {
          int8_t* sb = spins + (int64_t)b * N;
          const int8_t* Jb = J + (int64_t)b * d * N;
          int kk = sb[s] * local_field(s, L, d, Jb, sb, N);
          if ((uint64_t)r < Tab[(kk + z) / 2]) sb[s] = (int8_t)(-sb[s]);
        }
      }
    if (every > 0 && (i + 1) % every == 0) {
      for (int b = 0; b < 32; ++b)
        oracle_measure(L, d, J + (int64_t)b * d * N, spins + (int64_t)b * N,
                       &E[rec * 32 + b], &M[rec * 32 + b]);
      ++rec;
    }
  }
  return 0;
}

/* ------------------------------------------------- LCG experiment mode */

#define LCG32_A 1664525u
#define LCG32_C 1013904223u
#define LCG64_A 6364136223846793005ull
#define LCG64_C 1442695040888963407ull

static uint64_t lcg_step(int mode, uint64_t x) {
  if (mode == 3) return x * LCG64_A + LCG64_C;
  return (uint64_t)(uint32_t)((uint32_t)x * LCG32_A + LCG32_C);
}

static uint32_t lcg_draw(int mode, uint64_t x) {
  return mode == 3 ? (uint32_t)(x >> 32) : (uint32_t)x;
}

/* x advanced by k steps.  f(x) = a x + c composed with itself is
 * x -> a^2 x + (a + 1) c; binary powers of f are combined for the set bits
 * of k (all arithmetic mod 2^64, then reduced mod 2^32 for the 32-bit
 * generator). */
uint64_t oracle_lcg_skip(int mode, uint64_t x, uint64_t k) {
  uint64_t A = mode == 3 ? LCG64_A : LCG32_A, C = mode == 3 ? LCG64_C : LCG32_C;
  uint64_t ga = 1, gc = 0; /* accumulated map g(x) = ga x + gc */
  while (k) {
    if (k & 1) {
      ga = A * ga;
      gc = A * gc + C;
    }
    C = (A + 1) * C;
    A = A * A;
    k >>= 1;
  }
  uint64_t r = ga * x + gc;
  return mode == 3 ? r : (uint64_t)(uint32_t)r;
}

/* floor(2^32 / G) and floor(2^64 / G) for G >= 1. */
static uint64_t block_len(int mode, uint64_t G) {
  if (mode != 3) return (((uint64_t)1) << 32) / G;
  uint64_t q = UINT64_MAX / G;
  return (UINT64_MAX % G == G - 1) ? q + 1 : q; /* G divides 2^64 */
}

/* Initial generator states of the G = L^d/8 groups (see the header).
 * Returns 0, or -1 on bad arguments (mode not 1..3, L % 8 != 0). */
int oracle_lcg_init(int L, int d, int mode, uint64_t seed, uint32_t replica, uint64_t* state) {
  if (!valid_shape(L, d) || L % 8 != 0 || mode < 1 || mode > 3) return -1;
  uint64_t G = (uint64_t)site_count(L, d) / 8;
  if (mode == 1) {
    for (uint64_t g = 0; g < G; ++g) state[g] = draw(seed, (uint32_t)g, 0, replica, 6, 0);
    return 0;
  }
  uint64_t x0 = draw(seed, 0, 0, replica, 7, 0);
  if (mode == 3) x0 |= (uint64_t)draw(seed, 0, 0, replica, 7, 1) << 32;
  uint64_t len = block_len(mode, G);
  for (uint64_t g = 0; g < G; ++g) state[g] = oracle_lcg_skip(mode, x0, g * len);
  return 0;
}

/* n sweeps of the canonical chain with LCG draws (modes 1..3); state[G] is
 * advanced in place.  Records as in oracle_sweeps.  Returns 0, or -1 on bad
 * arguments. */
int oracle_lcg_sweeps(int L, int d, const int8_t* J, int8_t* spins, uint64_t* state, int mode, int n,
                      double beta, int every, int64_t* E, int64_t* M) {
  if (!valid_shape(L, d) || L % 8 != 0 || mode < 1 || mode > 3 || n < 0) return -1;
  if (isnan(beta) || beta < 0) return -1;
  int z = 2 * d;
  uint64_t T[7];
  oracle_table(beta, d, T);
  int64_t N = site_count(L, d);
  int rec = 0;
  for (int i = 0; i < n; ++i) {
    for (int colour = 0; colour < 2; ++colour) {
      for (int64_t s = 0; s < N; ++s) {
        if (colour_of(s, L, d) != colour) continue;
        const int field = local_field(s, L, d, J, spins, N);
        const int k = spins[s] * field;
        uint64_t* st = &state[s >> 3];
        *st = lcg_step(mode, *st);
        uint32_t r = lcg_draw(mode, *st);
        if ((uint64_t)r < T[(k + z) / 2]) spins[s] = (int8_t)(-spins[s]);
      }
    }
    if (every > 0 && (i + 1) % every == 0) {
      oracle_measure(L, d, J, spins, &E[rec], &M[rec]);
      ++rec;
    }
  }
  return 0;
}

/* ------------------------------------------------- Heisenberg (float) */

static float unit_uniform(uint32_t w) { return (float)(w >> 8) * 0x1p-24f; }

/* cos and sin of x in [0, pi/4] (Taylor polynomials, Horner steps in x^2). */
static void cos_sin_octant(float x, float* c, float* sn) {
  const float x2 = x * x;
  float pc = -1.0f / 3628800.0f;
  pc = fmaf(pc, x2, 1.0f / 40320.0f);
  pc = fmaf(pc, x2, -1.0f / 720.0f);
  pc = fmaf(pc, x2, 1.0f / 24.0f);
  pc = fmaf(pc, x2, -0.5f);
  *c = fmaf(pc, x2, 1.0f);
  float ps = 1.0f / 362880.0f;
  ps = fmaf(ps, x2, -1.0f / 5040.0f);
  ps = fmaf(ps, x2, 1.0f / 120.0f);
  ps = fmaf(ps, x2, -1.0f / 6.0f);
  *sn = fmaf(ps * x2, x, x);
}

static void direction(uint32_t w0, uint32_t w1, float v[3]) {
  const float z = 2.0f * unit_uniform(w0) - 1.0f;
  const float rho = sqrtf(fmaf(-z, z, 1.0f));
  const float t = 8.0f * unit_uniform(w1);
  const int o = (int)t;
  const float r = t - (float)o;
  const float a = (o & 1) ? 1.0f - r : r;
  float c, sn;
  cos_sin_octant(a * 0.785398163397448309616f, &c, &sn);
  if (o & 1) {
    const float tmp = c;
    c = sn;
    sn = tmp;
  }
  float cx, sy;
  switch (o >> 1) {
    case 0: cx = c; sy = sn; break;
    case 1: cx = -sn; sy = c; break;
    case 2: cx = -c; sy = -sn; break;
    default: cx = sn; sy = -c; break;
  }
  v[0] = rho * cx;
  v[1] = rho * sy;
  v[2] = z;
}

/* Metropolis acceptance u < exp(y) for the float y = -(beta dE). */
static int accept_exp(float u, float y) {
  if (y >= 0.0f) return 1;
  if (!(y > -87.0f)) return 0;    /* exp(y) < 2^-125: p stays a normal float above this */
  const float k = floorf(fmaf(y, 1.44269504088896340736f, 0.5f));
  float r = fmaf(-k, 0.693145751953125f, y);       /* ln2 high part, exact in float */
  r = fmaf(-k, 1.428606765330187045e-06f, r);      /* the rest of ln2 */
  float p = 1.0f / 5040.0f;
  p = fmaf(p, r, 1.0f / 720.0f);
  p = fmaf(p, r, 1.0f / 120.0f);
  p = fmaf(p, r, 1.0f / 24.0f);
  p = fmaf(p, r, 1.0f / 6.0f);
  p = fmaf(p, r, 0.5f);
  p = fmaf(p, r, 1.0f);
  p = fmaf(p, r, 1.0f);
  return u < ldexpf(p, (int)k);
}

/* The two float steps above, exported so that tests can pin them against cos, sin and exp in
 * double precision. */
void oracle_heis_direction(uint32_t w0, uint32_t w1, float v[3]) { direction(w0, w1, v); }

int oracle_heis_accept(float u, float y) { return accept_exp(u, y); }

static float dot_h(const float a[3], const float h[3]) {
  return fmaf(a[0], h[0], fmaf(a[1], h[1], a[2] * h[2]));
}

/* Hot start: spins[4 s + 0..2] the direction of site s, [4 s + 3] = 0. */
int oracle_heis_init(int L, int d, uint64_t seed, uint32_t replica, float* spins) {
  if (!valid_shape(L, d)) return -1;
  int64_t N = site_count(L, d);
  for (int64_t s = 0; s < N; ++s) {
    uint32_t ctr[4] = {(uint32_t)s, 0u, replica, 9u}, key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)}, w[4];
    oracle_philox4x32_10(ctr, key, w);
    direction(w[0], w[1], &spins[4 * s]);
    spins[4 * s + 3] = 0.0f;
  }
  return 0;
}

/* E = -sum of bond dot products and M = (sum S), accumulated in double. */
void oracle_heis_measure(int L, int d, const float* spins, double* E, double M[3]) {
  int64_t N = site_count(L, d);
  double e = 0, m[3] = {0, 0, 0};
  for (int64_t s = 0; s < N; ++s) {
    for (int k = 0; k < 3; ++k) m[k] += spins[4 * s + k];
    for (int dir = 0; dir < d; ++dir) {
      int64_t u = neighbour(s, dir, +1, L, d);
      double b = 0;
      for (int k = 0; k < 3; ++k) b += (double)spins[4 * s + k] * (double)spins[4 * u + k];
      e -= b;
    }
  }
  *E = e;
  for (int k = 0; k < 3; ++k) M[k] = m[k];
}

/* n sweeps from absolute sweep t0 (records of E and |M| after every every-th
 * sweep).  Returns 0, or -1 on bad arguments. */
int oracle_heis_sweeps(int L, int d, float* spins, uint64_t seed, uint32_t replica, uint64_t t0, int n, double beta,
                       int every, double* E, double* Mabs) {
  if (!valid_shape(L, d) || n < 0 || isnan(beta) || beta < 0) return -1;
  if (t0 + (uint64_t)n > ((uint64_t)1 << 32)) return -1;
  const float bf = (float)beta;
  int64_t N = site_count(L, d);
  int rec = 0;
  for (int i = 0; i < n; ++i) {
    uint32_t t = (uint32_t)(t0 + (uint64_t)i);
    for (int colour = 0; colour < 2; ++colour) {
      for (int64_t s = 0; s < N; ++s) {
        if (colour_of(s, L, d) != colour) continue;
        float h[3] = {0.0f, 0.0f, 0.0f};
        for (int dir = 0; dir < d; ++dir) {
          int64_t dn = neighbour(s, dir, -1, L, d), up = neighbour(s, dir, +1, L, d);
          for (int k = 0; k < 3; ++k) h[k] = h[k] + spins[4 * dn + k];
          for (int k = 0; k < 3; ++k) h[k] = h[k] + spins[4 * up + k];
        }
        uint32_t ctr[4] = {(uint32_t)s, t, replica, 10u + (uint32_t)colour};
        uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)}, w[4];
        oracle_philox4x32_10(ctr, key, w);
        float trial[3];
        direction(w[0], w[1], trial);
        const float dE = dot_h(&spins[4 * s], h) - dot_h(trial, h);
        if (dE <= 0.0f || accept_exp(unit_uniform(w[2]), -(bf * dE)))
          for (int k = 0; k < 3; ++k) spins[4 * s + k] = trial[k];
      }
    }
    if (every > 0 && (i + 1) % every == 0) {
      double m[3];
      oracle_heis_measure(L, d, spins, &E[rec], m);
      Mabs[rec] = sqrt(m[0] * m[0] + m[1] * m[1] + m[2] * m[2]);
      ++rec;
    }
  }
  return 0;
}
