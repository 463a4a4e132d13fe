"""Plant plausible mistakes in copies of the oracle and show the pins catch each.

Every mutant is a text edit of ``oracle/spin_oracle.c`` (a dropped term, a
wrong sign, a swapped operand or index, a wrong counter word, a wrong
colour order...).  Each is compiled on the CPU and run through a quick
subset of the pins of ``test_oracle_pins.py``; at least one pin must fail.
The unmodified source must pass the same subset.
"""
import math
import os

import numpy as np
import pytest

import bruteforce as bf
import oracle

MUTANTS = {
    "heis_dE_sign": ("const float dE = dot_h(&spins[4 * s], h) - dot_h(trial, h);",
                     "const float dE = dot_h(trial, h) - dot_h(&spins[4 * s], h);"),
    "heis_phi_from_first_word": ("const float t = 8.0f * unit_uniform(w1);", "const float t = 8.0f * unit_uniform(w0);"),
    "heis_odd_octant_not_reflected": ("const float a = (o & 1) ? 1.0f - r : r;", "const float a = r;"),
    "heis_third_quadrant_sign": ("case 2: cx = -c; sy = -sn; break;", "case 2: cx = c; sy = -sn; break;"),
    "heis_cos_series_short": ("pc = fmaf(pc, x2, 1.0f / 40320.0f);", "pc = fmaf(pc, x2, 0.0f);"),
    "heis_exp_ln2_tail_dropped": ("r = fmaf(-k, 1.428606765330187045e-06f, r);", "r = fmaf(-k, 0.0f, r);"),
    "heis_exp_series_short": ("p = fmaf(p, r, 1.0f / 720.0f);", "p = fmaf(p, r, 0.0f);"),
    "heis_exp_cutoff_early": ("if (!(y > -87.0f)) return 0;", "if (!(y > -60.0f)) return 0;"),
    "heis_zero_dE_rejected": ("if (dE <= 0.0f || accept_exp(", "if (dE < 0.0f || accept_exp("),
    "heis_drop_upper_neighbour": ("for (int k = 0; k < 3; ++k) h[k] = h[k] + spins[4 * up + k];", "(void)up;"),
    "heis_update_counter_colour": ("uint32_t ctr[4] = {(uint32_t)s, t, replica, 10u + (uint32_t)colour};",
                                   "uint32_t ctr[4] = {(uint32_t)s, t, replica, 10u};"),
    "lcg64_low_word": ("return mode == 3 ? (uint32_t)(x >> 32) : (uint32_t)x;", "return (uint32_t)x;"),
    "lcg_draw_before_step": ("*st = lcg_step(mode, *st);\n        uint32_t r = lcg_draw(mode, *st);",
                             "uint32_t r = lcg_draw(mode, *st);\n        *st = lcg_step(mode, *st);"),
    "lcg_block_len_wrong_count": ("uint64_t len = block_len(mode, G);", "uint64_t len = block_len(mode, G + 1);"),
    "lcg_stream_per_four_sites": ("uint64_t* st = &state[s >> 3];",
                                  "uint64_t* st = &state[(uint64_t)(s >> 2) % ((uint64_t)N / 8)];"),
    "lcg_skip_square_wrong": ("    C = (A + 1) * C;", "    C = A * C;"),
    "lcg32_multiplier": ("#define LCG32_A 1664525u", "#define LCG32_A 1664521u"),
    "drop_backward_neighbour": ("h += coupling(J, dir, dn, N) * spins[dn];", "(void)dn;"),
    "wrong_sign_of_k": ("int k = spins[s] * h;", "int k = -spins[s] * h;"),
    "dE_is_k_not_2k": ("double dE = (double)(2 * k);", "double dE = (double)k;"),
    "colour_order_swapped": ("for (int c = 0; c < 2; ++c) {", "for (int c = 1; c >= 0; --c) {"),
    "update_counter_word_s_over_4": ("draw(seed, (uint32_t)(s >> 3), t, replica", "draw(seed, (uint32_t)(s >> 2), t, replica"),
    "update_word_index": ("t, replica, (uint32_t)c,\n                          (unsigned)((s >> 1) & 3));",
                          "t, replica, (uint32_t)c,\n                          (unsigned)(s & 3));"),
    "coarse_update_word_index": ("(uint32_t)c, (unsigned)((s >> 1) & 3));", "(uint32_t)c, (unsigned)(s & 3));"),
    "philox_swapped_high_words": ("uint32_t n0 = hi1 ^ c1 ^ k0;", "uint32_t n0 = hi0 ^ c1 ^ k0;"),
    "philox_key_not_bumped": ("if (round < 9) { k0 += W0; k1 += W1; }", "if (round < 9) { k0 += W0; }"),
    "energy_sign": ("e -= (int64_t)coupling(J, dir, s, N) * spins[s] * spins[t];",
                    "e += (int64_t)coupling(J, dir, s, N) * spins[s] * spins[t];"),
    "hot_start_inverted": ("spins[s] = (r >> 31) ? (int8_t)1 : (int8_t)-1;",
                           "spins[s] = (r >> 31) ? (int8_t)-1 : (int8_t)1;"),
    "coupling_of_wrong_bond": ("h += coupling(J, dir, s, N) * spins[up];", "h += coupling(J, dir, up, N) * spins[up];"),
    "y_coordinate_wraps_wrong": ("x[1] = (s / L) % L;", "x[1] = (s / L) % (L - 1);"),
    "table_index_off_by_one": ("int accept = (uint64_t)r < T[cls];", "int accept = (uint64_t)r < T[cls > 0 ? cls - 1 : 0];"),
    "table_ceil": ("v = (uint64_t)floor(ldexp(p, 32));", "v = (uint64_t)ceil(ldexp(p, 32));"),
    # the coarse-tile multi-hit schedule
    "coarse_odd_tiles_first": ("if ((bx + by + bz) % 2 != q) continue;", "if ((bx + by + bz) % 2 == q) continue;"),
    "coarse_hit_counter_ignores_k": ("uint32_t hit = (uint32_t)(t * (uint64_t)k + (uint64_t)h);",
                                     "uint32_t hit = (uint32_t)(t + (uint64_t)h);"),
    "coarse_fine_colours_swapped": ("              for (int c = 0; c < 2; ++c)\n                for (int zz",
                                    "              for (int c = 1; c >= 0; --c)\n                for (int zz"),
    "coarse_single_hit": ("for (int h = 0; h < k; ++h) {", "for (int h = 0; h < 1; ++h) {"),
    "coarse_last_tiles_skipped": ("int B = L / T;", "int B = L / T - 1;"),
    # the multi-spin-coded glass
    "msc_counter_space": ("t, p0, 4u + (uint32_t)c,", "t, p0, (uint32_t)c,"),
    "msc_all_systems_share_couplings": ("const int8_t* Jb = J + (int64_t)b * d * N;", "const int8_t* Jb = J;"),
    "msc_draw_from_wrong_replica": ("(uint32_t)(s >> 3), t, p0, 4u", "(uint32_t)(s >> 3), t, p0 + 1u, 4u"),
}


def _quick_pins(lib, rocrand_philox):
    """Raise AssertionError on the first pin that fails."""
    # Philox against rocRAND
    ctrs = np.array([[0, 0, 0, 0], [7, 3, 2, 1], [0xFFFFFFFF] * 4], dtype=np.uint64)
    key = (0x00000001, 0x10063865)
    np.testing.assert_array_equal(np.array([lib.philox4x32_10(c, key) for c in ctrs]), rocrand_philox(ctrs, key))
    # table closed form at a few betas
    for beta in (0.3, 0.5, 2.0):
        T = lib.table(beta, 3)
        for i, k in enumerate(range(-6, 7, 2)):
            want = 1 << 32 if k <= 0 else math.floor(math.ldexp(math.exp(-beta * 2 * k), 32))
            assert int(T[i]) == want
    # inputs of the chain against rocRAND bit rules
    L, d, seed = 4, 2, 0x1006386500000003
    words = rocrand_philox([(s >> 2, 0, 0, 2) for s in range(L * L)], (seed & 0xFFFFFFFF, seed >> 32))
    expect = np.array([1 if words[s, s & 3] >> 31 else -1 for s in range(L * L)], dtype=np.int8)
    np.testing.assert_array_equal(lib.init_spins(L, d, seed, 0), expect)
    # measurement against brute force
    rng = np.random.default_rng(0)
    for (L, d) in ((6, 2), (4, 3)):
        s = rng.choice(np.array([-1, 1], dtype=np.int8), size=L ** d)
        J = rng.choice(np.array([-1, 1], dtype=np.int8), size=d * L ** d)
        assert lib.measure(L, d, J, s) == (bf.energy(s, L, d, J), bf.magnetisation(s))
    # sweeps against the brute-force restatement with rocRAND draws
    for (L, d, ea, beta) in ((4, 2, False, 0.44), (6, 2, True, 0.8), (4, 3, True, 0.5)):
        seed, rep, t0, n = 0x1006386500000009, 1, 2, 2
        J = rng.choice(np.array([-1, 1], dtype=np.int8), size=d * L ** d) if ea else None
        s0 = rng.choice(np.array([-1, 1], dtype=np.int8), size=L ** d)
        got = s0.copy()
        lib.sweeps(L, d, J, got, seed, rep, t0, n, beta)
        N = L ** d
        ctrs, keys = [], []
        for t in range(t0, t0 + n):
            for c in (0, 1):
                for g in range((N + 7) // 8):
                    ctrs.append((g, t, rep, c))
                    keys.append((g, t, c))
        w = dict(zip(keys, rocrand_philox(ctrs, (seed & 0xFFFFFFFF, seed >> 32))))
        ref = s0.copy()
        for t in range(t0, t0 + n):
            bf.sweep(ref, L, d, J, beta, t, lambda s, tt, c: int(w[(s >> 3, tt, c)][(s >> 1) & 3]))
        np.testing.assert_array_equal(got, ref)
    # coarse-tile multi-hit sweeps against their brute-force restatement
    for (L, d, ea, T, k, beta) in ((8, 2, False, 2, 2, 0.44), (4, 3, True, 2, 2, 0.5)):
        seed, rep, t0, n = 0x1006386500000009, 1, 3, 1
        J = rng.choice(np.array([-1, 1], dtype=np.int8), size=d * L ** d) if ea else None
        s0 = rng.choice(np.array([-1, 1], dtype=np.int8), size=L ** d)
        got = s0.copy()
        lib.coarse_sweeps(L, d, J, got, seed, rep, t0, n, beta, T, k)
        N = L ** d
        ctrs, keys = [], []
        for t in range(t0, t0 + n):
            for h in range(k):
                for c in (0, 1):
                    for g in range((N + 7) // 8):
                        ctrs.append((g, t * k + h, rep, c))
                        keys.append((g, t * k + h, c))
        w = dict(zip(keys, rocrand_philox(ctrs, (seed & 0xFFFFFFFF, seed >> 32))))
        ref = s0.copy()
        for t in range(t0, t0 + n):
            bf.coarse_sweep(ref, L, d, J, beta, t, T, k, lambda s, hit, c: int(w[(s >> 3, hit, c)][(s >> 1) & 3]))
        np.testing.assert_array_equal(got, ref)

    # multi-spin-coded systems against single-system brute force with the shared draws
    L, d, beta, r0, p0, t0, n = 6, 2, 0.3, 3, 40, 1, 2
    J = np.stack([lib.couplings(L, d, 0x51, r0 + b) for b in range(32)])
    spins = np.stack([lib.init_spins(L, d, 0x52, p0 + b) for b in range(32)])
    start = spins.copy()
    lib.msc_sweeps(L, d, J, spins, 0x52, p0, t0, n, beta)
    keys = [(g, t, c) for t in range(t0, t0 + n) for c in (0, 1) for g in range(5)]
    w = dict(zip(keys, rocrand_philox([(g, t, p0, 4 + c) for (g, t, c) in keys], (0x52, 0))))
    for b in (0, 7, 31):
        ref = start[b].copy()
        for t in range(t0, t0 + n):
            bf.sweep(ref, L, d, J[b], beta, t, lambda s, tt, c: int(w[(s >> 3, tt, c)][(s >> 1) & 3]))
        np.testing.assert_array_equal(spins[b], ref)

    # LCG mode: published sequence, skip-ahead, contiguous blocks, brute force with per-group streams
    x, seq = 0, []
    for _ in range(3):
        x = lib.lcg_skip(1, x, 1)
        seq.append(x)
    assert seq == [1013904223, 1196435762, 3519870697]
    for mode, mod in ((1, 1 << 32), (3, 1 << 64)):
        a, c = (1664525, 1013904223) if mode == 1 else (6364136223846793005, 1442695040888963407)
        y = 987654321
        for _ in range(7):
            y = (a * y + c) % mod
        assert lib.lcg_skip(mode, 987654321, 7) == y
    for mode in (2, 3):
        st = lib.lcg_init(16, 2, mode, 0x77, 1)
        ln = (1 << (64 if mode == 3 else 32)) // 32
        assert all(lib.lcg_skip(mode, int(st[g]), ln) == int(st[g + 1]) for g in range(31))
    for mode in (2, 3):
        L, d, beta = 8, 2, 0.44
        spins = lib.init_spins(L, d, 0x77, 1)
        state = lib.lcg_init(L, d, mode, 0x77, 1)
        ref, py = spins.copy(), [int(v) for v in state]
        lib.lcg_sweeps(L, d, None, spins, state, mode, 1, beta)

        def lcg_draw(s, t, c, mode=mode, py=py):
            g = s >> 3
            if mode == 3:
                py[g] = (6364136223846793005 * py[g] + 1442695040888963407) % (1 << 64)
                return py[g] >> 32
            py[g] = (1664525 * py[g] + 1013904223) % (1 << 32)
            return py[g]
        bf.sweep(ref, L, d, None, beta, 0, lcg_draw)
        np.testing.assert_array_equal(spins, ref)


    # Heisenberg mode: beta = 0 takes every trial; one sweep against brute force in double precision
    L, d, rep, hs = 4, 2, 1, 0x5A
    sp = lib.heis_init(L, d, hs, rep)
    lib.heis_sweeps(L, d, sp, hs, rep, 0, 1, 0.0)
    N = L * L
    col = [((s % L) + (s // L)) & 1 for s in range(N)]
    w = rocrand_philox([(s, 0, rep, 10 + col[s]) for s in range(N)], (hs, 0))
    u = (np.asarray(w, dtype=np.uint64) >> 8).astype(np.float64) * 2.0 ** -24
    zz = 2 * u[:, 0] - 1
    ph = 2 * math.pi * u[:, 1]
    rr = np.sqrt(1 - zz * zz)
    np.testing.assert_allclose(sp[:, :3], np.stack([rr * np.cos(ph), rr * np.sin(ph), zz], axis=1), atol=2e-6)
    beta = 0.7
    sp = lib.heis_init(L, d, hs, rep)
    S = sp[:, :3].astype(np.float64).copy()

    def e_of(S):
        g = S.reshape(L, L, 3)
        return -float((g * np.roll(g, -1, axis=1)).sum() + (g * np.roll(g, -1, axis=0)).sum())
    for c in (0, 1):
        for s in range(N):
            if col[s] != c:
                continue
            ww = rocrand_philox([(s, 0, rep, 10 + c)], (hs, 0))[0]
            uu = (np.asarray(ww, dtype=np.uint64) >> 8).astype(np.float64) * 2.0 ** -24
            z1, p1 = 2 * uu[0] - 1, 2 * math.pi * uu[1]
            trial = np.array([math.sqrt(1 - z1 * z1) * math.cos(p1), math.sqrt(1 - z1 * z1) * math.sin(p1), z1])
            e0, old = e_of(S), S[s].copy()
            S[s] = trial
            if not uu[2] < math.exp(-beta * (e_of(S) - e0)):
                S[s] = old
    lib.heis_sweeps(L, d, sp, hs, rep, 0, 1, beta)
    np.testing.assert_allclose(sp[:, :3], S, atol=2e-5)
    # the float direction and acceptance steps against cos, sin and exp in double precision
    hw = np.random.default_rng(9).integers(0, 1 << 32, size=(600, 2), dtype=np.uint64).tolist()
    for a, b in hw + [[0, 0], [0xFFFFFFFF, 0xFFFFFFFF], [1 << 31, 1 << 29], [1 << 31, 3 << 29]]:
        z1, p1 = 2 * ((a >> 8) * 2.0 ** -24) - 1, 2 * math.pi * ((b >> 8) * 2.0 ** -24)
        r1 = math.sqrt(1 - z1 * z1)
        np.testing.assert_allclose(lib.heis_direction(a, b), [r1 * math.cos(p1), r1 * math.sin(p1), z1], atol=3e-7)
    for y in np.linspace(-86.9, -1e-4, 300).astype(np.float32).tolist():
        e = math.exp(y)
        assert lib.heis_accept(e * (1 - 1e-6), y) and not lib.heis_accept(e * (1 + 1e-6), y), y
    # dE = 0 at beta = inf is accepted: colour-1 spins (0, 0, s(x) s(y)), s = (+, +, -, -), cancel
    # around every colour-0 site of the L = 4 square lattice
    sp = lib.heis_init(4, 2, hs, 0)
    for s in range(16):
        if (s % 4 + s // 4) & 1:
            sp[s] = [0.0, 0.0, (1.0 if s % 4 < 2 else -1.0) * (1.0 if s // 4 < 2 else -1.0), 0.0]
    lib.heis_sweeps(4, 2, sp, hs, 0, 0, 1, math.inf)
    for s in range(16):
        if (s % 4 + s // 4) & 1 == 0:
            ww = rocrand_philox([(s, 0, 0, 10)], (hs, 0))[0]
            np.testing.assert_array_equal(sp[s, :3], lib.heis_direction(int(ww[0]), int(ww[1])))


def test_unmodified_oracle_passes_quick_pins(oracle_mod, rocrand_philox):
    _quick_pins(oracle_mod.default(), rocrand_philox)


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_planted_mistake_is_caught(name, tmp_path, rocrand_philox):
    src = open(oracle.SOURCE).read()
    old, new = MUTANTS[name]
    assert src.count(old) == 1, "mutation anchor must match exactly once: " + old
    path = os.path.join(str(tmp_path), "mutant.c")
    with open(path, "w") as f:
        f.write(src.replace(old, new))
    so = oracle.compile_oracle(path, os.path.join(str(tmp_path), "libmutant.so"))
    lib = oracle.OracleLib(so)
    with pytest.raises(AssertionError):
        _quick_pins(lib, rocrand_philox)
