#!/usr/bin/env python3
"""Benchmark of the checkerboard Metropolis path on one MI355X.

Default workload ``ising2d_L8192``: three 2D Ising lattices, L = 8192
(67,108,864 int8 spins each), one per inverse temperature 0.30, 0.4406868 and
0.60, all from the same seeded hot start.  One *step* advances each lattice
by 10 sweeps and records E and M once (the recording cadence of the
workload), so the default 200 steps are the whole 2000-sweep job.  Lattices
are created and initialised before the timed region (inputs resident in HBM).

Printed: one JSON line with the whole-job throughput (spin-flip attempts per
ns, measurement included), the sweep-only rate (measurement excluded, the
paper's timing convention), the roofline of the dominant kernel (its launch
duration timed with HIP events on the stream it runs on) and the CPU oracle
timed on a bounded sample of the same workload.

``--gpus N`` with N > 1 exits: this build runs on one GPU.
"""
import argparse
import hashlib
import json
import os
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E
# vector ALU: 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz, one 32-bit lane op per lane per clock
VALU_PEAK_TOPS = 256 * 4 * 16 * 2.4e9 / 1e12
# Algorithmic 32-bit lane operations per spin-flip attempt: Philox4x32-10 gives 4 words per
# 10 rounds of (2 32x32->64 multiplies + 2 three-input XORs) = 10 per attempt.  The update of an
# 8-site group (4 attempts of one colour) with the active sites packed into one dword: gathers
# (active bytes, other-colour bytes, the shifted side, 2d - 2 row/plane neighbours), 2d mask-XORs,
# the sums of 2d terms (2 in 2D, 3 in 3D), 4 x (extract, compare, select), 2 flip XORs and 1
# counter: 2D 5 + 4 + 2 + 12 + 2 + 1 = 26 -> 6.5; 3D 7 + 6 + 3 + 12 + 2 + 1 = 31 -> 7.75.
ALG_OPS_PER_ATTEMPT = {2: 10.0 + 26 / 4.0, 3: 10.0 + 31 / 4.0}
BYTES_PER_ATTEMPT = 2.0  # int8 spin read once and written once per sweep (Ising)
# LDS: 256 CUs x 128 bytes per clock x 2.4 GHz.  Algorithmic LDS bytes of the streaming kernels per
# 8-site group and sweep: the row (2D) or plane-slice row (3D) stored once (8 B); per colour unit the
# group and its in-LDS neighbours (2D: 3 x 8 B + 2 x 4 B = 32 B; 3D: 5 x 8 B + 2 x 4 B = 48 B) and four
# 4-byte bound lookups (16 B); colour 0 stores the group back (8 B).  2D: 8 + 56 + 48 = 112 B, 3D:
# 8 + 72 + 64 = 144 B, per 8 attempts.
LDS_PEAK_GBS = 256 * 128 * 2.4
LDS_BYTES_PER_ATTEMPT = {2: 112 / 8.0, 3: 144 / 8.0}
# The 3D register-column kernel (L = 512) keeps z columns and the wave's own rows in registers: per
# 8-site group and sweep it stores the loaded row and the colour-0 result (16 B), reads per colour
# unit the active-parity half of one y neighbour (4 B; groups are held parity-split) and the bounds
# of its four sites (two 8-byte pair-table entries, 16 B): 56 B per 8 attempts.
LDS_BYTES_PER_ATTEMPT_3R = 56 / 8.0
# The 2D register-column form keeps every row of its column in registers: per 8-site group and sweep
# the bounds of four sites per colour unit (32 B) and one 4-byte segment-end word for colour 1 (4 B).
LDS_BYTES_PER_ATTEMPT_2C = 36 / 8.0


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default="ising2d_L8192", choices=["ising2d_L8192", "ising3d_L512", "ising2d_L64"])
    ap.add_argument("--kernel", default="auto", choices=["auto", "fused", "tiled", "generic", "resident"])
    ap.add_argument("--tile", default="", help="x,y,z,threads")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-c3", action="store_true", help="skip the 3D Ising L=512 leg")
    ap.add_argument("--c3-steps", type=int, default=100, help="steps of 10 sweeps of the 3D leg (100: whole job)")
    ap.add_argument("--no-large", action="store_true", help="skip the 2D L=16384 sensitivity row")
    ap.add_argument("--no-c1", action="store_true", help="skip the 2D Ising L=64 leg")
    ap.add_argument("--no-ceilings", action="store_true", help="skip the probe kernels")
    ap.add_argument("--copy-probe-mib", type=int, default=0,
                    help="also run a plain device copy of this many MiB (counter calibration)")
    ap.add_argument("--no-batched", action="store_true", help="skip the batched 3D EA workload")
    ap.add_argument("--batched-static-only", action="store_true",
                    help="batched workload: one call with the static launch rule only (no autotuner, no graph)")
    ap.add_argument("--no-serving", action="store_true", help="skip the serving workload")
    ap.add_argument("--serve-jobs", type=int, default=100)
    ap.add_argument("--no-coarse", action="store_true", help="skip the coarse-tile multi-hit schedule")
    ap.add_argument("--no-autocorr", action="store_true",
                    help="skip the multi-hit autocorrelation measurement near the critical point")
    ap.add_argument("--no-msc", action="store_true", help="skip the multi-spin-coded +-J glass")
    ap.add_argument("--no-rng-quality", action="store_true", help="skip the RNG-quality experiment")
    ap.add_argument("--no-heisenberg", action="store_true", help="skip the continuous-spin (Heisenberg) model")
    ap.add_argument("--coarse-only", default="", help="L,T,k: time only this coarse-tile configuration")
    ap.add_argument("--heis-shapes", default="4096x2,256x3", help="Heisenberg lattices as LxD, comma separated")
    ap.add_argument("--batched-sweeps", type=int, default=5000)
    ap.add_argument("--msc-shapes", default="512x3,256x3,128x3,4096x2",
                    help="multi-spin-coded lattices as LxD, comma separated")
    return ap.parse_args()


# Source files that define each profiled kernel (its counters are valid while they are unchanged).
KERNEL_SOURCES = {
    "k_stream2d": ("spin_stream2d.hip", "spin_phase.h", "spin_device.h", "spin_packed.h"),
    "k_stream2c": ("spin_stream2d.hip", "spin_phase.h", "spin_device.h", "spin_packed.h"),
    "k_stream3d": ("spin_stream3d.hip", "spin_phase.h", "spin_device.h", "spin_packed.h"),
    "k_stream3r": ("spin_stream3d.hip", "spin_phase.h", "spin_device.h", "spin_packed.h"),
    "k_streamg": ("spin_stream_kernels.hip", "spin_nibble.h", "spin_device.h"),
    "k_batch": ("spin_batch_kernels.hip", "spin_nibble.h", "spin_device.h"),
    "k_msc_stream": ("spin_msc_kernels.hip", "spin_msc.h", "spin_device.h"),
    "k_msc_col": ("spin_msc_kernels.hip", "spin_msc.h", "spin_device.h"),
    "k_coarse": ("spin_coarse_kernels.hip", "spin_nibble.h", "spin_device.h"),
    "k_heis_phase": ("spin_heis_kernels.hip", "spin_heis.h", "spin_device.h"),
}


def kernel_sources_sha(kernel_tag):
    files = KERNEL_SOURCES.get(kernel_tag)
    if files is None:
        return None
    h = hashlib.sha256()
    for f in files:
        h.update(open(os.path.join(ROOT, "paper_1006_3865_amd", "csrc", f), "rb").read())
    return h.hexdigest()


def profiled_traffic(kernel_tag, L):
    """HBM bytes per launch from the committed rocprofv3 summary, if the kernel is unchanged."""
    pdir = os.path.join(ROOT, "profiles")
    if not os.path.isdir(pdir):
        return None
    sha = kernel_sources_sha(kernel_tag)
    if sha is None:
        return None
    for f in sorted(os.listdir(pdir)):
        if not f.endswith(".md"):
            continue
        for line in open(os.path.join(pdir, f)):
            m = re.match(r"traffic-record: kernel=(\S+) L=(\d+) bytes_per_launch=(\d+) source_sha256=(\w+)", line)
            if m and m.group(1) == kernel_tag and int(m.group(2)) == L and m.group(4) == sha:
                return int(m.group(3))
    return None


def host_cpu():
    """CPU model, logical CPUs of the host and CPUs this process may run on."""
    model = "unknown"
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    try:
        usable = len(os.sched_getaffinity(0))
    except AttributeError:
        usable = os.cpu_count() or 1
    return {"model": model, "nproc": os.cpu_count() or 1, "usable": usable}


def cpu_baseline(cfg, seconds_hint):
    """The C oracle, single-threaded, on a bounded sample of the workload: each lattice is built (hot
    start) before its timed window, which covers the sweeps (with their E/M records) only."""
    import oracle
    L, d = cfg["L"], cfg["d"]
    n_sweeps = 2 if L ** d >= 1 << 26 else (20 if L ** d >= 1 << 20 else 200)
    attempts = 0
    used = 0
    busy = 0.0
    for b in cfg["betas"]:
        ch = oracle.Chain(L, d, cfg["seed"])
        t0 = time.perf_counter()
        ch.sweep(n_sweeps, b, every=max(1, min(cfg["every"], n_sweeps)))
        busy += time.perf_counter() - t0
        attempts += n_sweeps * L ** d
        used += 1
        if busy > seconds_hint:
            break
    cpu = host_cpu()
    return {"value": round(attempts / (busy * 1e9), 5), "unit": "spin-flip attempts/ns", "cores": 1,
            "kind": "oracle", "cpu_model": cpu["model"], "nproc": cpu["nproc"], "usable_cpus": cpu["usable"],
            "sample": "%d sweeps (E/M recorded) of the L=%d d=%d lattice at each of %d beta(s) from the hot "
                      "start (built outside the timed window); %.1f s of sweeps on one host core"
                      % (n_sweeps, L, d, used, busy)}


def _oracle_worker(args):
    """One oracle process: build its lattice untimed, then time `sweeps` sweeps."""
    import oracle
    L, d, seed, replica, cseed, realisation, beta, sweeps = args
    J = oracle.couplings(L, d, cseed, realisation) if cseed is not None else None
    ch = oracle.Chain(L, d, seed, replica, J=J)
    t0 = time.perf_counter()
    ch.sweep(sweeps, beta)
    return sweeps * L ** d, time.perf_counter() - t0


def cpu_aggregate(workloads, kind, procs, seconds=5.0, oracle_rate=0.015):
    """Labelled aggregate of P independent single-threaded oracle processes, one lattice each, run at
    the same time (P = the CPUs this process may use, at most 16): the ±J batch's lattices (kind
    "ea3d_batch") or the served trace's jobs ("serve_trace"), each for about `seconds` of sweeps
    (sweep counts from an assumed `oracle_rate` attempts/ns).  Aggregate = summed attempts / the
    longest process's sweep time."""
    import multiprocessing as mp
    work = []
    if kind == "ea3d_batch":
        descs = workloads.ea_batch()
        step = max(1, len(descs) // procs)
        for d in descs[::step][:procs]:
            n = max(1, int(seconds * oracle_rate * 1e9 / d["L"] ** 3))
            work.append((d["L"], 3, d["seed"], d["replica"], d["coupling_seed"], d["realisation"], d["beta"], n))
    else:
        for j in workloads.serve_trace(jobs=procs):
            n = max(1, min(j["sweeps"], int(seconds * oracle_rate * 1e9 / j["L"] ** j["d"])))
            work.append((j["L"], j["d"], j["seed"], 0, j["coupling_seed"] if j["model"] == 1 else None, 0,
                         j["beta"], n))
    ctx = mp.get_context("fork")
    with ctx.Pool(len(work)) as pool:
        res = pool.map(_oracle_worker, work)
    att = sum(a for a, _ in res)
    span = max(t for _, t in res)
    return {"value": round(att / (span * 1e9), 4), "unit": "spin-flip attempts/ns", "cores": len(work),
            "kind": "oracle aggregate", "workload": kind,
            "sample": "%d independent single-threaded oracle processes at once, one lattice each (%s), "
                      "%.1f s longest" % (len(work), "first lattices of the batch, evenly spaced" if
                                          kind == "ea3d_batch" else "the trace's first jobs, sweeps capped", span)}


def bench_batched(torch, spin, workloads, sweeps, every=100, plain_sweeps=100, static_only=False):
    """Batched 3D +-J EA workload: 512 realisations (L in 16..64) x 16 betas = 8192 lattices, all
    advanced `sweeps` sweeps by one pool call, (E, M) every `every` sweeps.  Plain: the same
    lattices on lone handles one after another; its time is the sum over lattices of L^3 * sweeps
    at the rate measured on two lattices of each size over `plain_sweeps` sweeps (steady state)."""
    import numpy as np
    descs = workloads.ea_batch()
    betas = np.array([d["beta"] for d in descs])
    N = np.array([d["L"] ** 3 for d in descs], dtype=np.float64)
    stream = torch.cuda.Stream()
    attempts = float(N.sum()) * sweeps

    def one_call(tag):
        """The whole workload as one pool call on a fresh pool: (wall s, GPU ms)."""
        b = spin.Batch(descs, stream=stream)
        nrec = int(b.record_counts(sweeps, every).sum())
        E = torch.zeros(max(nrec, 1), dtype=torch.int64, device="cuda")
        M = torch.zeros(max(nrec, 1), dtype=torch.int64, device="cuda")
        b.sweep(2, betas, 0)          # warm-up: module load, LDS attributes
        b.synchronize()
        torch.cuda.synchronize()
        ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        t0 = time.perf_counter()
        ev0.record(stream)
        b.sweep_device(sweeps, betas, every, E, M)
        ev1.record(stream)
        b.synchronize()
        wall = time.perf_counter() - t0
        print("bench: batched %s %.1f ms" % (tag, wall * 1e3), file=sys.stderr, flush=True)
        h = [int(E[-1]), int(M[-1])]
        b.close()
        return wall, ev0.elapsed_time(ev1), h

    wall_static, ms_static, h_static = one_call("static plan")
    if static_only:
        return {"workload": "ea3d_batch", "lattices": len(descs), "sweeps": sweeps, "record_every": every,
                "attempts": attempts, "static_plan_attempts_per_ns": round(attempts / (wall_static * 1e9), 2),
                "static_plan_gpu_ms": round(ms_static, 2)}
    # the project's autotuner picks each lattice shape's launch plan by timing (outside the timed region)
    b = spin.Batch(descs, stream=stream)
    t0 = time.perf_counter()
    ntuned = b.autotune(float(np.median(betas)), 20)
    tune_s = time.perf_counter() - t0
    b.close()
    plans = {"L%d" % L: spin.batch_plan(3, 1, L) for L in sorted({d["L"] for d in descs})}
    wall, gpu_ms, h_tuned = one_call("tuned plan")
    # the same workload as replays of one captured 100-sweep call (hipGraph)
    g_sweeps = 100
    reps = sweeps // g_sweeps
    b = spin.Batch(descs, stream=stream)
    nrec = int(b.record_counts(g_sweeps, every).sum())
    E = torch.zeros(max(nrec, 1), dtype=torch.int64, device="cuda")
    M = torch.zeros(max(nrec, 1), dtype=torch.int64, device="cuda")
    b.sweep(2, betas, 0)                           # the same 2 warm-up sweeps as one_call
    b.sweep_device(g_sweeps, betas, every, E, M)   # uploads the call's tables (uncaptured)
    b.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=stream):
        b.sweep_device(g_sweeps, betas, every, E, M)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps - 1):
        g.replay()
    torch.cuda.synchronize()
    graph_wall = time.perf_counter() - t0
    h_graph = [int(E[-1]), int(M[-1])]
    del g
    b.close()
    graph_att = float(N.sum()) * g_sweeps * (reps - 1)
    rates = {}
    for L in sorted({d["L"] for d in descs}):
        sel = [d for d in descs if d["L"] == L][:2]
        att = 0.0
        ms = 0.0
        for d in sel:
            lat = spin.Lattice(1, L, 3, d["seed"], coupling_seed=d["coupling_seed"], realisation=d["realisation"],
                               replica=d["replica"], stream=stream)
            lat.sweep(5, d["beta"])
            a, bb = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record(stream)
            lat.sweep(plain_sweeps, d["beta"])
            bb.record(stream)
            lat.synchronize()
            ms += a.elapsed_time(bb)
            att += plain_sweeps * L ** 3
            kname = spin.KERNEL_NAMES[lat.kernel]
            lat.close()
        rates[L] = (att / (ms * 1e6), kname)
    plain_s = sum(L ** 3 * sweeps / (rates[L][0] * 1e9) for L in (d["L"] for d in descs))
    batched = attempts / (wall * 1e9)
    plain = attempts / (plain_s * 1e9)
    return {"workload": "ea3d_batch", "lattices": len(descs), "realisations": len(descs) // 16,
            "sizes": sorted(rates), "sweeps": sweeps, "record_every": every, "attempts": attempts,
            "batched_attempts_per_ns": round(batched, 2), "batched_gpu_ms": round(gpu_ms, 2),
            "plan": "autotuned (%d shapes in %.1f s): %s" % (ntuned, tune_s, plans),
            "static_plan_attempts_per_ns": round(attempts / (wall_static * 1e9), 2),
            "static_plan_gpu_ms": round(ms_static, 2),
            "graph": {"captured_sweeps": g_sweeps, "replays_timed": reps - 1,
                      "attempts_per_ns": round(graph_att / (graph_wall * 1e9), 2)},
            "final_record_identical": {"tuned_vs_static": h_static == h_tuned, "graph_vs_static": h_static == h_graph},
            "plain_attempts_per_ns": round(plain, 3), "ratio": round(batched / plain, 2),
            "plain_rate_by_L": {str(L): {"attempts_per_ns": round(r, 3), "kernel": k} for L, (r, k) in rates.items()},
            "plain_method": "lone handles, %d sweeps on 2 lattices per L, summed over the workload" % plain_sweeps}


def bench_coarse(torch, spin, workloads, sizes=(1024, 8192), tiles=(16, 32, 64), hits=(1, 2, 4, 8)):
    """The paper's own schedule (coarse tiles, k-fold multi-hit): 2D Ising at beta 0.4406868, attempts/ns
    (k * L^2 attempts per sweep) for each tile edge and hit count, HIP events on the lattice's stream."""
    stream = torch.cuda.Stream()
    out = {}
    for L in sizes:
        lat = spin.Lattice(0, L, 2, workloads.seed(2), stream=stream)
        for T in tiles:
            for k in hits:
                lat.set_schedule(spin.SPIN_SCHEDULE_COARSE, T, k)
                # about 3e10 attempts per point (tens of milliseconds): shorter windows catch the
                # GPU's clock still rising and scatter by several per cent
                n = max(2, int(3e10 / (k * L * L)))
                n = min(n, 2000)
                lat.sweep(1, workloads.BETA_2D_CRIT)
                a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                a.record(stream)
                lat.sweep(n, workloads.BETA_2D_CRIT)
                b.record(stream)
                lat.synchronize()
                out["L%d_T%d_k%d" % (L, T, k)] = round(n * k * L * L / (a.elapsed_time(b) * 1e6), 2)
        lat.close()
    res = {"workload": "ising2d coarse-tile multi-hit", "beta": workloads.BETA_2D_CRIT,
           "unit": "spin-flip attempts/ns", "attempts_per_ns": out}
    traffic = profiled_traffic("k_coarse", 8192)
    if traffic is not None:  # counted HBM bytes per launch (one tile parity) of the L=8192, T=32, k=8 case
        res["traffic_L8192_T32_k8_bytes_per_launch"] = traffic
    return res


def bench_multihit_autocorr(torch, spin, workloads, L=64, T=16, hits=(1, 2, 4, 8), sweeps=200_000, therm=5_000,
                            chunk=20_000):
    """The autocorrelation cost of the multi-hit schedule near the critical point (Sec. 3, multi-hit
    paragraph): 2D Ising L=64 at beta 0.4406868, the canonical checkerboard and coarse tiles of edge T
    with k hits; E and M recorded after every sweep (device records), integrated autocorrelation times
    of E and |M| in sweeps (self-consistent window, c = 6), and the GPU time per independent sample
    (tau_int x time per sweep, records included)."""
    import numpy as np
    from paper_1006_3865_amd import analysis
    beta = workloads.BETA_2D_CRIT
    stream = torch.cuda.Stream()
    N = L * L
    out = {}
    for k in (0,) + tuple(hits):
        lat = spin.Lattice(0, L, 2, workloads.seed(0x30), stream=stream)
        if k:
            lat.set_schedule(spin.SPIN_SCHEDULE_COARSE, T, k)
        lat.sweep(therm, beta)
        E = torch.zeros(sweeps, dtype=torch.int64, device="cuda")
        M = torch.zeros(sweeps, dtype=torch.int64, device="cuda")
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(stream)
        for c0 in range(0, sweeps, chunk):
            lat.sweep_record_device(chunk, beta, 1, E[c0:], M[c0:])
        b.record(stream)
        lat.synchronize()
        ms = a.elapsed_time(b)
        lat.close()
        e, m = E.cpu().numpy(), np.abs(M.cpu().numpy())
        tE, wE, dE = analysis.tau_int(e)
        tM, wM, dM = analysis.tau_int(m)
        us = ms * 1e3 / sweeps
        name = "checkerboard" if k == 0 else "coarse_T%d_k%d" % (T, k)
        out[name] = {"hits": max(k, 1), "us_per_sweep": round(us, 3),
                     "attempts_per_ns": round(max(k, 1) * N * sweeps / (ms * 1e6), 2),
                     "tau_int_E": round(tE, 2), "tau_int_E_err": round(dE, 2),
                     "tau_int_absM": round(tM, 1), "tau_int_absM_err": round(dM, 1),
                     "us_per_independent_E": round(tE * us, 2), "us_per_independent_absM": round(tM * us, 1),
                     "mean_e_per_site": round(float(e.mean()) / N, 6)}
    # attempts per independent sample in units of N attempts (hits x tau), relative to the checkerboard
    ref = out["checkerboard"]
    for v in out.values():
        v["attempt_sweeps_per_independent_E"] = round(v["hits"] * v["tau_int_E"], 1)
        v["attempt_sweeps_per_independent_absM"] = round(v["hits"] * v["tau_int_absM"], 1)
        v["penalty_E"] = round(v["hits"] * v["tau_int_E"] / ref["tau_int_E"], 3)
        v["penalty_absM"] = round(v["hits"] * v["tau_int_absM"] / ref["tau_int_absM"], 3)
    return {"workload": "2D Ising L=%d at beta 0.4406868, %d sweeps recorded after %d" % (L, sweeps, therm),
            "tile": T, "window_c": 6, "modes": out}


def bench_rng_quality(torch, spin, workloads, L=64, sweeps=200_000, therm=10_000, chunk=20_000):
    """The RNG-quality experiment (Sec. 4, first paragraph): the canonical 2D Ising chain at L=64 and
    beta 0.4406868 with Philox and with the three LCG set-ups (an array of 32-bit LCGs with one
    multiplier and random seeds; disjoint sub-sequences of one 32-bit LCG; of one 64-bit LCG); E after
    every sweep; u and the specific heat c per site with jackknife errors (50 blocks) against the exact
    finite-lattice values (Kaufman's partition function), as z-scores."""
    from paper_1006_3865_amd import analysis
    beta = workloads.BETA_2D_CRIT
    N = L * L
    u_ex, c_ex = analysis.exact_u_c(L, beta)
    stream = torch.cuda.Stream()
    names = {spin.SPIN_RNG_PHILOX: "philox4x32_10", spin.SPIN_RNG_LCG32_ARRAY: "lcg32_array_random_seeds",
             spin.SPIN_RNG_LCG32_DISJOINT: "lcg32_disjoint_subsequences",
             spin.SPIN_RNG_LCG64_DISJOINT: "lcg64_disjoint_subsequences"}
    out = {}
    for mode, name in names.items():
        lat = spin.Lattice(0, L, 2, workloads.seed(0x31), stream=stream)
        if mode != spin.SPIN_RNG_PHILOX:
            lat.set_rng(mode)
        lat.sweep(therm, beta)
        E = torch.zeros(sweeps, dtype=torch.int64, device="cuda")
        M = torch.zeros(sweeps, dtype=torch.int64, device="cuda")
        t0 = time.perf_counter()
        for c0 in range(0, sweeps, chunk):
            lat.sweep_record_device(chunk, beta, 1, E[c0:], M[c0:])
        lat.synchronize()
        wall = time.perf_counter() - t0
        lat.close()
        u, du, c, dc = analysis.energy_stats(E.cpu().numpy(), N, beta)
        out[name] = {"u": round(u, 6), "u_err": round(du, 6), "z_u": round((u - u_ex) / du, 2),
                     "c": round(c, 4), "c_err": round(dc, 4), "z_c": round((c - c_ex) / dc, 2),
                     "wall_s": round(wall, 2)}
    return {"workload": "2D Ising L=%d at beta 0.4406868, %d sweeps after %d, E every sweep" % (L, sweeps, therm),
            "exact_u": round(u_ex, 8), "exact_c": round(c_ex, 6), "modes": out}


def bench_heisenberg(torch, spin, workloads, shapes=((4096, 2), (256, 3)), beta=0.7):
    """Continuous spins (classical Heisenberg, float): attempts/ns over back-to-back sweeps (one launch
    per colour), HIP events on the handle's stream, with the HBM rate of the algorithmic traffic (each
    site's float4 read and written once and read once more as a neighbour per sweep: 48 B per attempt)."""
    stream = torch.cuda.Stream()
    out = {}
    for (L, d) in shapes:
        h = spin.Heis(L, d, workloads.seed(0x12), stream=stream)
        N = L ** d
        n = max(4, min(200, int(2e9 / N)))
        h.sweep(2, beta)
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(stream)
        h.sweep(n, beta)
        b.record(stream)
        h.synchronize()
        ms = a.elapsed_time(b)
        h.close()
        rate = N * n / (ms * 1e6)
        rec = {"attempts_per_ns": round(rate, 1), "ms_per_sweep": round(ms / n, 4), "sweeps": n,
               "alg_hbm_GBps": round(48 * rate, 1), "alg_hbm_frac": round(48 * rate / HBM_PEAK_GBS, 4)}
        traffic = profiled_traffic("k_heis_phase", L) if d == 2 else None
        if traffic is not None:  # counted HBM bytes per colour launch
            rec["traffic_bytes_per_sweep"] = 2 * traffic
            rec["traffic_GBps"] = round(2 * traffic / (ms / n * 1e6), 1)
        out["d%d_L%d" % (d, L)] = rec
    return {"workload": "classical Heisenberg, float, beta %g" % beta, "rates": out}


def bench_msc(torch, spin, workloads, shapes=((512, 3), (256, 3), (128, 3), (4096, 2))):
    """Multi-spin-coded +-J glass: 32 realisations per word, attempts/ns (32 * L^d per sweep) at the
    middle of the batch's temperature ladder, HIP events on the handle's stream."""
    stream = torch.cuda.Stream()
    beta = workloads.ea_betas()[7]
    out = {}
    for (L, d) in shapes:
        m = spin.Msc(L, d, workloads.seed(0x11), 0, workloads.seed(0x10), 0, stream=stream)
        N = L ** d
        n = max(4, min(400, int(2e11 / (32 * N))))
        m.sweep(2, beta)
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(stream)
        m.sweep(n, beta)
        b.record(stream)
        m.synchronize()
        ms = a.elapsed_time(b)
        # fewest HBM bytes a sweep can move: read and write each site word, read the d coupling words
        hbm_min = N * (8 + 4 * d)
        kname = {0: "k_msc_phase", 1: "k_msc_stream", 2: "k_msc_col"}.get(m.kernel, "?")
        rec = {"kernel": kname, "attempts_per_ns": round(32 * N * n / (ms * 1e6), 1),
               "ps_per_attempt": round(ms * 1e9 / (32 * N * n), 4), "sweeps": n,
               "ms_per_sweep": round(ms / n, 4),
               "min_hbm_GBps": round(hbm_min * n / (ms * 1e6), 1),
               "min_hbm_frac": round(hbm_min * n / (ms * 1e-3) / 8e12, 4)}
        traffic = profiled_traffic(kname, L) if d == 3 else None
        if traffic is not None:   # HBM bytes per sweep counted by rocprofv3 for this kernel and L
            rec["traffic_bytes_per_sweep"] = traffic
            rec["traffic_GBps"] = round(traffic * n / (ms * 1e6), 1)
        out["d%d_L%d" % (d, L)] = rec
        m.close()
    return {"workload": "ea multi-spin-coded (32 realisations per word)", "beta": beta, "rates": out}


def serve_class(job, lds_resident):
    """Size class of a served job: 'lds' (swept by the pool's persistent kernel), 'mid' (below 4 M
    sites, on the single-lattice kernels), 'big' (4 M sites and more: fills the GPU on its own)."""
    N = job["L"] ** job["d"]
    if lds_resident(job["L"], job["d"]):
        return "lds"
    return "mid" if N < (1 << 22) else "big"


def bench_serving(torch, serve, workloads, jobs):
    """Serving workload (a9).  Capacity: the served loop with every job submitted at t = 0 against the
    plain path's capacity (the same jobs one at a time on lone handles: total work / summed service
    times), overall and per size class (each class served alone at t = 0).  Latency: a Poisson stream at
    0.8 x the served capacity, 1 GiB pool budget, 512 slots; p50/p99 served vs plain FIFO (latencies by
    the FIFO recurrence over the measured service times)."""
    unit = workloads.serve_trace(jobs=jobs, rate_per_s=1.0)
    work = sum(j["L"] ** j["d"] * j["sweeps"] for j in unit)
    stream = torch.cuda.Stream()

    def run(trace):
        ex = serve.PoolExecutor(stream=stream)
        srv = serve.Server(ex, budget_bytes=1 << 30, max_slots=512)
        res = srv.serve(trace)
        ex.close()
        return res, srv.ticks

    sat, _ = run([dict(j, arrival=0.0) for j in unit])
    cap = work / max(r["finished"] for r in sat.values())          # attempts/s, saturated
    lam = 0.8 * cap / (work / len(unit))                            # jobs/s
    trace = [dict(j, arrival=j["arrival"] / lam) for j in unit]
    served, ticks = run(trace)
    plain = serve.plain_fifo(trace, serve.lone_service)
    plain_busy = sum(r["service"] for r in plain.values())
    plain_cap = work / plain_busy
    s_sum = serve.summarize(served, trace)
    p_sum = serve.summarize(plain, trace)
    same = all((served[k]["E"], served[k]["M"]) == (plain[k]["E"], plain[k]["M"]) for k in served)
    classes = {}
    for c in ("lds", "mid", "big"):
        sub = [j for j in unit if serve_class(j, serve.lds_resident) == c]
        if not sub:
            continue
        w = sum(j["L"] ** j["d"] * j["sweeps"] for j in sub)
        res_c, _ = run([dict(j, arrival=0.0) for j in sub])
        served_s = max(r["finished"] for r in res_c.values())
        plain_s = sum(plain[j["job"]]["service"] for j in sub)
        classes[c] = {"jobs": len(sub), "work_share": round(w / work, 4),
                      "served_attempts_per_ns": round(w / served_s / 1e9, 2),
                      "plain_attempts_per_ns": round(w / plain_s / 1e9, 2),
                      "ratio": round(plain_s / served_s, 2), "served_s": round(served_s, 4),
                      "plain_s": round(plain_s, 4)}
    # classes served one after another: the ratio a served run can reach on this trace without running
    # classes concurrently, from the per-class capacities
    seq_served = sum(v["served_s"] for v in classes.values())
    return {"workload": "serve_trace", "jobs": jobs, "mean_attempts_per_job": work / len(unit),
            "saturated_attempts_per_ns": round(cap / 1e9, 2),
            "plain_saturated_attempts_per_ns": round(plain_cap / 1e9, 2),
            "saturated_ratio": round(cap / plain_cap, 2),
            "classes": classes,
            "class_sequential_ratio": round(plain_busy / seq_served, 2) if seq_served > 0 else None,
            "arrival_rate_per_s": round(lam, 2),
            "budget_bytes": 1 << 30, "max_slots": 512, "ticks": ticks,
            "served": {k: round(v, 5) for k, v in s_sum.items()},
            "plain_fifo": {k: round(v, 5) for k, v in p_sum.items()},
            "p50_ratio": round(p_sum["p50_s"] / s_sum["p50_s"], 2),
            "p99_ratio": round(p_sum["p99_s"] / s_sum["p99_s"], 2),
            "results_identical": bool(same)}


SETTLE_S = 0.3  # seconds of untimed sweeps before a single-lattice job's warm-up steps


def lattice_job(torch, spin, workloads, name, steps, warmup, kern=0, tile=(0, 0, 0, 0), so_sweeps=200):
    """One single-lattice workload: `steps` steps of 10 sweeps with the workload's E/M records, on
    lattices created and initialised before the timed region; then `so_sweeps` back-to-back sweeps
    without records (the sweep-only rate, HIP events on the lattice's stream) and the roofline of the
    dominant kernel from them."""
    cfg = workloads.CONFIGS[name]
    L, d, every = cfg["L"], cfg["d"], cfg["every"]
    N = L ** d
    sweeps_per_step = 10  # one record interval of the L=8192 / L=512 workloads
    # one stream per lattice: the lattices are independent chains, so one lattice's sweep can start on
    # CUs that another's sweep has already left
    streams = [torch.cuda.Stream() for _ in cfg["betas"]]
    stream = streams[0]
    torch.cuda.synchronize()
    lats = []
    for b, st in zip(cfg["betas"], streams):
        lat = spin.Lattice(cfg["model"], L, d, cfg["seed"], stream=st)
        if kern:
            lat.set_kernel(kern, *tile)
        lats.append((lat, b))
    kname = spin.KERNEL_NAMES[lats[0][0].kernel]
    ktile = lats[0][0].tile
    recs_per_step = sweeps_per_step // every
    nrec = steps * recs_per_step
    Erec = [torch.zeros(max(1, nrec), dtype=torch.int64, device="cuda") for _ in lats]
    Mrec = [torch.zeros(max(1, nrec), dtype=torch.int64, device="cuda") for _ in lats]
    for st in streams:
        st.wait_stream(torch.cuda.current_stream())
    for lat, _ in lats:
        lat.synchronize()

    # clock settle: a cold GPU needs tens of milliseconds under load before it reaches its steady
    # clock (back-to-back repeats of 600 sweeps at 2D L=8192: 1644, then 1851 and 1864 attempts/ns),
    # so the same sweeps run for SETTLE_S seconds before the warm-up steps; like them they only
    # advance the chains
    t_settle = time.perf_counter()
    while time.perf_counter() - t_settle < SETTLE_S:
        for lat, b in lats:
            lat.sweep(sweeps_per_step, b)
        torch.cuda.synchronize()
    # warmup (advances the same chains; the kernels' cost does not depend on the state)
    for i in range(warmup):
        for lat, b in lats:
            lat.sweep(sweeps_per_step, b)
    torch.cuda.synchronize()

    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(steps):
        for j, (lat, b) in enumerate(lats):
            lat.sweep_record_device(sweeps_per_step, b, every, Erec[j][i * recs_per_step:],
                                    Mrec[j][i * recs_per_step:])
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0

    # sweep-only segment (measurement excluded): the same kernel, HIP events on its stream
    ev_a = torch.cuda.Event(enable_timing=True)
    ev_b = torch.cuda.Event(enable_timing=True)
    k0 = 1 if len(lats) > 1 else 0
    lat0, b0 = lats[k0]
    ev_a.record(streams[k0])
    lat0.sweep(so_sweeps, b0)
    ev_b.record(streams[k0])
    torch.cuda.synchronize()
    so_ms = ev_a.elapsed_time(ev_b)
    for lat, _ in lats:
        lat.close()
    res = {"workload": name, "kernel": kname, "lattices": len(lats), "steps": steps, "warmup": warmup,
           "settle_s": SETTLE_S,
           "sweeps_per_step": sweeps_per_step, "record_every": every,
           "value": round(steps * sweeps_per_step * N * len(lats) / (wall * 1e9), 2),
           "ms_per_step": round(wall * 1e3 / max(1, steps), 4)}
    res.update(roofline_of(kname, L, d, N, so_sweeps, so_ms, ktile))
    return res


def roofline_of(kname, L, d, N, so_sweeps, so_ms, tile=(0, 0, 0, 0)):
    """Sweep-only rate and the roofline of the dominant kernel from so_sweeps back-to-back sweeps that
    took so_ms (HIP events on the lattice's stream)."""
    launches_per_sweep = {"fused": 1, "tiled": 2, "generic": 2}.get(kname, 0)
    launches = so_sweeps * launches_per_sweep if launches_per_sweep else 1
    kernel_avg_us = so_ms * 1e3 / launches
    attempts_per_launch = so_sweeps * N / launches
    sweep_only_rate = so_sweeps * N / (so_ms * 1e6)  # attempts per ns
    alg_ops = ALG_OPS_PER_ATTEMPT[d]
    alu_tops = alg_ops * attempts_per_launch / (kernel_avg_us * 1e-6) / 1e12
    hbm_gbs = BYTES_PER_ATTEMPT * attempts_per_launch / (kernel_avg_us * 1e-6) / 1e9
    col2 = d == 2 and tile[0] == L and tile[2] == 1   # the register-column form of the 2D row streaming
    kernel_tag = {("fused", 2): "k_stream2c" if col2 else "k_stream2d",
                  ("fused", 3): "k_stream3r" if L == 512 else "k_stream3d",
                  ("tiled", 3): "k_tiled3d"}.get((kname, d), kname)
    traffic = profiled_traffic(kernel_tag, L)
    roof = {"bound": "alu", "achieved": round(alu_tops, 2), "peak": round(VALU_PEAK_TOPS, 2),
            "unit": "Tops/s", "frac": round(alu_tops / VALU_PEAK_TOPS, 4), "traffic": traffic,
            "kernel": kernel_tag, "kernel_avg_us": round(kernel_avg_us, 2),
            "alg_ops_per_attempt": alg_ops, "attempts_per_launch": int(attempts_per_launch),
            "hbm": {"achieved": round(hbm_gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                    "frac": round(hbm_gbs / HBM_PEAK_GBS, 4),
                    "alg_bytes_per_launch": int(BYTES_PER_ATTEMPT * attempts_per_launch)}}
    if kname == "fused":  # the streaming kernels
        lb = {"k_stream3r": LDS_BYTES_PER_ATTEMPT_3R, "k_stream2c": LDS_BYTES_PER_ATTEMPT_2C}.get(
            kernel_tag, LDS_BYTES_PER_ATTEMPT[d])
        lds_gbs = lb * attempts_per_launch / (kernel_avg_us * 1e-6) / 1e9
        roof["lds"] = {"achieved": round(lds_gbs, 1), "peak": round(LDS_PEAK_GBS, 1), "unit": "GB/s",
                       "frac": round(lds_gbs / LDS_PEAK_GBS, 4),
                       "alg_bytes_per_launch": int(lb * attempts_per_launch)}
    return {"sweep_only_attempts_per_ns": round(sweep_only_rate, 2),
            "hbm_frac_sweep_only": round(hbm_gbs / HBM_PEAK_GBS, 4), "roofline": roof}


def bench_c1(torch, spin, workloads):
    """The 2D Ising L = 64 job (1000 sweeps at beta 0.4406868, E and M after every sweep): one call of
    1000 sweeps with the 1000 records, and the same as 100 calls of 10 sweeps.  The lattice (4 KiB)
    sits in one workgroup's LDS for a whole call, so the rate is one CU's, bound by latency: no
    chip-wide roofline applies."""
    cfg = workloads.CONFIGS["ising2d_L64"]
    L, beta, n = cfg["L"], cfg["betas"][0], cfg["sweeps"]
    stream = torch.cuda.Stream()
    E = torch.zeros(n, dtype=torch.int64, device="cuda")
    M = torch.zeros(n, dtype=torch.int64, device="cuda")
    res = {"workload": "ising2d_L64", "sweeps": n, "record_every": 1, "beta": beta}
    warm = spin.Lattice(0, L, 2, cfg["seed"], stream=stream)
    warm.sweep_record_device(10, beta, 1, E, M)   # module load and first launch outside the timing
    warm.synchronize()
    warm.close()
    for tag, calls in (("one_call", 1), ("calls_of_10", n // 10)):
        lat = spin.Lattice(0, L, 2, cfg["seed"], stream=stream)
        lat.synchronize()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        per = n // calls
        a.record(stream)
        for c in range(calls):
            lat.sweep_record_device(per, beta, 1, E[c * per:], M[c * per:])
        b.record(stream)
        lat.synchronize()
        ms = a.elapsed_time(b)
        res[tag] = {"kernel": spin.KERNEL_NAMES[lat.kernel], "us_per_sweep": round(ms * 1e3 / n, 3),
                    "attempts_per_ns": round(n * L * L / (ms * 1e6), 3)}
        lat.close()
    res["note"] = "latency-bound: the lattice lives in one CU's LDS for the whole call"
    return res


def bench_large2d(torch, spin, workloads, L=16384, sweeps=100):
    """Sensitivity row above the 256 MB Infinity Cache: 2D Ising L = 16384 (256 MiB of spins, 512 MiB
    with the second buffer), sweep-only rate on the row-streaming kernel (not one of the workloads)."""
    stream = torch.cuda.Stream()
    lat = spin.Lattice(0, L, 2, workloads.seed(2), stream=stream)
    lat.sweep(2, workloads.BETA_2D_CRIT)
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record(stream)
    lat.sweep(sweeps, workloads.BETA_2D_CRIT)
    b.record(stream)
    lat.synchronize()
    kname = spin.KERNEL_NAMES[lat.kernel]
    ktile = lat.tile
    lat.close()
    out = {"workload": "ising2d_L%d (sensitivity, not a workload)" % L, "beta": workloads.BETA_2D_CRIT,
           "kernel": kname, "sweeps": sweeps, "ping_pong_bytes": 2 * L * L}
    out.update(roofline_of(kname, L, 2, L * L, sweeps, a.elapsed_time(b), ktile))
    return out


def bench_ceilings(torch, spin):
    """What bounds the sweep on this GPU, from the probe kernels in the library (include/spin_probe.h):
    Philox4x32-10 blocks evaluated by the sweep kernels' own code (words/ns), the issue rate of the
    32x32 -> 64-bit multiply-add the generator is built from and of a plain 32-bit operation (VALU
    lane-instructions per second against 256 CUs x 64 lanes x 2.4 GHz), and a device copy (GB/s of
    bytes read + written) of a buffer above the 256 MB Infinity Cache and of one inside it."""
    lib = spin.load()
    stream = torch.cuda.Stream()
    sp = stream.cuda_stream
    blocks = 256 * 16
    out = torch.empty(blocks * 256, dtype=torch.int32, device="cuda")
    threads = blocks * 256

    def timed(fn, reps=3):
        fn()
        best = None
        for _ in range(reps):
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record(stream)
            fn()
            b.record(stream)
            stream.synchronize()
            ms = a.elapsed_time(b)
            best = ms if best is None else min(best, ms)
        return best

    res = {}
    it = 1024
    ms = timed(lambda: spin._check(lib.spin_probe_alu(spin.SPIN_PROBE_PHILOX, out.data_ptr(), blocks, it, 7, sp)))
    words = 4.0 * it * threads
    res["philox_words_per_ns"] = round(words / (ms * 1e6), 1)
    res["philox_blocks_per_ns"] = round(words / 4 / (ms * 1e6), 1)
    it = 512
    ms = timed(lambda: spin._check(lib.spin_probe_alu(spin.SPIN_PROBE_MAD64, out.data_ptr(), blocks, it, 7, sp)))
    mad_ops = 64.0 * it * threads
    res["mad64_probe_lane_instr_per_s"] = round(mad_ops / (ms * 1e-3), -9)
    res["mad64_probe_frac_of_valu_peak"] = round(mad_ops / (ms * 1e-3) / (VALU_PEAK_TOPS * 1e12), 4)
    ms = timed(lambda: spin._check(lib.spin_probe_alu(spin.SPIN_PROBE_ALU32, out.data_ptr(), blocks, it, 7, sp)))
    alu_ops = 32.0 * it * threads
    res["alu32_probe_lane_instr_per_s"] = round(alu_ops / (ms * 1e-3), -9)
    res["alu32_probe_frac_of_valu_peak"] = round(alu_ops / (ms * 1e-3) / (VALU_PEAK_TOPS * 1e12), 4)
    res["valu_peak_lane_instr_per_s"] = VALU_PEAK_TOPS * 1e12
    for mib in (1024, 64):
        nb = mib << 20
        src = torch.empty(nb, dtype=torch.uint8, device="cuda")
        dst = torch.empty_like(src)
        ms = timed(lambda: spin._check(lib.spin_probe_copy(src.data_ptr(), dst.data_ptr(), nb, 256 * 64, sp)))
        res["copy_%dMiB_GBps" % mib] = round(2.0 * nb / (ms * 1e6), 1)
        del src, dst
    # the canonical chain's ceiling if the generator ran alone at the measured rate and the update
    # cost nothing: one word per attempt
    res["note"] = ("philox words/ns bounds attempts/ns from the generator alone; the sweep adds the "
                   "update's VALU work on top")
    return res


def main():
    args = parse()
    # tuning records are neither read nor written unless the caller names a cache file: the
    # benchmark runs its own autotuner where it uses one
    os.environ.setdefault("SPIN_TUNE_CACHE", "")
    if args.gpus != 1:
        print("bench.py runs on one GPU only: this build has no multi-GPU path (asked for --gpus %d)" % args.gpus,
              file=sys.stderr)
        sys.exit(2)
    import torch
    from paper_1006_3865_amd import spin, workloads

    assert torch.cuda.is_available(), "no GPU"
    torch.cuda.set_device(0)
    spin.load()
    kern = {"auto": 0, "generic": 1, "resident": 2, "tiled": 3, "fused": 4}[args.kernel]
    tile = [int(v) for v in args.tile.split(",")] if args.tile else [0, 0, 0, 0]
    head = lattice_job(torch, spin, workloads, args.workload, args.steps, args.warmup, kern, tile)
    cfg = workloads.CONFIGS[args.workload]

    if args.copy_probe_mib:
        nb = args.copy_probe_mib << 20
        a = torch.empty(nb, dtype=torch.uint8, device="cuda")
        bb = torch.empty_like(a)
        bb.copy_(a)
        torch.cuda.synchronize()
        del a, bb

    out = {
        "metric": "spin-flip attempts/ns + % HBM roofline; batched vs plain flips/ns; p50/p99 job latency",
        "value": head["value"],
        "unit": "spin-flip attempts/ns",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": head["ms_per_step"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "int8", "data": "synthetic",
        "config": {"workload": args.workload, "model": "ising", "L": cfg["L"], "d": cfg["d"],
                   "betas": [float(b) for b in cfg["betas"]], "sweeps_per_step": head["sweeps_per_step"],
                   "record_every": cfg["every"], "lattices": head["lattices"], "kernel": head["kernel"],
                   "untimed_settle_s": head["settle_s"], "parallelism": "single GPU"},
        "sweep_only_attempts_per_ns": head["sweep_only_attempts_per_ns"],
        "hbm_frac_sweep_only": head["hbm_frac_sweep_only"],
        "roofline": head["roofline"],
    }
    if not args.no_c3 and args.workload != "ising3d_L512":
        # the 3D workload as its own leg: the whole 1000-sweep job (100 steps of 10 sweeps, E/M every 10)
        out["ising3d_L512"] = lattice_job(torch, spin, workloads, "ising3d_L512", args.c3_steps, 2)
        print("ising3d_L512:", json.dumps(out["ising3d_L512"]), file=sys.stderr, flush=True)
    if not args.no_c1 and args.workload != "ising2d_L64":
        out["ising2d_L64"] = bench_c1(torch, spin, workloads)
        print("ising2d_L64:", json.dumps(out["ising2d_L64"]), file=sys.stderr, flush=True)
    if not args.no_large:
        out["large2d_L16384"] = bench_large2d(torch, spin, workloads)
    if not args.no_ceilings:
        out["ceilings"] = bench_ceilings(torch, spin)
        print("ceilings:", json.dumps(out["ceilings"]), file=sys.stderr, flush=True)
    if not args.no_batched:
        out["batched"] = bench_batched(torch, spin, workloads, args.batched_sweeps,
                                       static_only=args.batched_static_only)
        print("batched:", json.dumps(out["batched"]), file=sys.stderr, flush=True)
    if not args.no_coarse:
        if args.coarse_only:
            cL, cT, ck = (int(v) for v in args.coarse_only.split(","))
            out["coarse_schedule"] = bench_coarse(torch, spin, workloads, (cL,), (cT,), (ck,))
        else:
            out["coarse_schedule"] = bench_coarse(torch, spin, workloads)
    if not args.no_coarse and not args.no_autocorr and not args.coarse_only:
        out["multihit_autocorr"] = bench_multihit_autocorr(torch, spin, workloads)
        print("coarse:", json.dumps(out["coarse_schedule"]), file=sys.stderr, flush=True)
    if not args.no_heisenberg:
        hshapes = tuple(tuple(int(v) for v in t.split("x")) for t in args.heis_shapes.split(",") if t)
        out["heisenberg"] = bench_heisenberg(torch, spin, workloads, hshapes)
    if not args.no_rng_quality:
        out["rng_quality"] = bench_rng_quality(torch, spin, workloads)
    if not args.no_msc:
        shapes = tuple(tuple(int(v) for v in t.split("x")) for t in args.msc_shapes.split(",") if t)
        out["multispin"] = bench_msc(torch, spin, workloads, shapes)
        print("multispin:", json.dumps(out["multispin"]), file=sys.stderr, flush=True)
    if not args.no_serving:
        from paper_1006_3865_amd import serve
        out["serving"] = bench_serving(torch, serve, workloads, args.serve_jobs)
        print("serving:", json.dumps(out["serving"]), file=sys.stderr, flush=True)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(cfg, 25.0)
        procs = min(16, host_cpu()["usable"])
        out["cpu_baseline_aggregates"] = {
            "ea3d_batch": cpu_aggregate(workloads, "ea3d_batch", procs),
            "serve_trace": cpu_aggregate(workloads, "serve_trace", procs)}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
