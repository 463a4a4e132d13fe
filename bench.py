#!/usr/bin/env python3
"""Benchmark of the checkerboard Metropolis path on one MI355X.

Workload (default ``ising2d_L8192``): three 2D Ising lattices, L = 8192
(67,108,864 int8 spins each), one per inverse temperature 0.30, 0.4406868 and
0.60, all from the same seeded hot start; one *step* advances each lattice
by 10 sweeps and records E and M once (the recording cadence of the
workload).  200 steps are the whole 2000-sweep job.  Lattices are created
and initialised before the timed region (inputs resident in HBM).

Printed: one JSON line with the whole-job throughput (spin-flip attempts
per ns, measurement included), the sweep-only rate, the roofline of the
dominant kernel (timed with HIP events on the stream it runs on) and the CPU
oracle timed on a bounded sample.

``--gpus N`` with N > 1 exits: this build runs on one GPU.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0            # MI355X HBM3E, GB/s
VALU_PEAK_TOPS = 256 * 4 * 16 * 2.4e9 / 1e12   # 256 CUs x 4 SIMD x 16 lanes x 2.4 GHz (32-bit lane ops)
PHILOX_OPS_PER_ATTEMPT = 10.0    # 10 rounds x (2 mul-hi/lo + 2 three-way xor) per 4 words


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default="ising2d_L8192", choices=["ising2d_L8192", "ising3d_L512", "ising2d_L64"])
    ap.add_argument("--kernel", default="auto", choices=["auto", "fused", "tiled", "generic", "resident"])
    ap.add_argument("--tile", default="", help="x,y,z,threads")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--copy-probe-mib", type=int, default=0,
                    help="also run a plain device copy of this many MiB (counter calibration)")
    return ap.parse_args()


def cpu_baseline(cfg, seconds_hint):
    """The C oracle, single-threaded, on a bounded sample of the workload."""
    import numpy as np
    import oracle
    L, d = cfg["L"], cfg["d"]
    n_sweeps = 2 if L ** d >= 1 << 26 else (20 if L ** d >= 1 << 20 else 200)
    attempts = 0
    t0 = time.perf_counter()
    for b in cfg["betas"]:
        ch = oracle.Chain(L, d, cfg["seed"])
        tb = time.perf_counter()
        ch.sweep(n_sweeps, b, every=max(1, min(cfg["every"], n_sweeps)))
        attempts += n_sweeps * L ** d
        if time.perf_counter() - t0 > seconds_hint:
            break
    dt = time.perf_counter() - t0
    return {"value": attempts / (dt * 1e9), "unit": "spin-flip attempts/ns", "cores": 1, "kind": "oracle",
            "sample": "%d sweeps (E/M recorded) of the L=%d d=%d lattice at each of %d betas, from the hot start; "
                      "%.1f s" % (n_sweeps, L, d, len(cfg["betas"]), dt)}


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: this build has no multi-GPU path (asked for --gpus %d)" % args.gpus,
              file=sys.stderr)
        sys.exit(2)
    import torch
    from paper_1006_3865_amd import spin, workloads

    assert torch.cuda.is_available(), "no GPU"
    torch.cuda.set_device(0)
    spin.load()
    cfg = workloads.CONFIGS[args.workload]
    L, d, every = cfg["L"], cfg["d"], cfg["every"]
    N = L ** d
    sweeps_per_step = 10  # one record interval of the L=8192 / L=512 workloads
    kern = {"auto": 0, "generic": 1, "resident": 2, "tiled": 3, "fused": 4}[args.kernel]
    tile = [int(v) for v in args.tile.split(",")] if args.tile else [0, 0, 0, 0]

    stream = torch.cuda.Stream()
    torch.cuda.synchronize()
    lats = []
    for b in cfg["betas"]:
        lat = spin.Lattice(cfg["model"], L, d, cfg["seed"], stream=stream)
        if kern:
            lat.set_kernel(kern, *tile)
        lats.append((lat, b))
    kname = spin.KERNEL_NAMES[lats[0][0].kernel]
    nrec = args.steps * sweeps_per_step // every
    Erec = [torch.zeros(max(1, nrec), dtype=torch.int64, device="cuda") for _ in lats]
    Mrec = [torch.zeros(max(1, nrec), dtype=torch.int64, device="cuda") for _ in lats]
    stream.wait_stream(torch.cuda.current_stream())
    for lat, _ in lats:
        lat.synchronize()

    # warmup (advances the same chains; costs are state-independent)
    for i in range(args.warmup):
        for lat, b in lats:
            lat.sweep(sweeps_per_step, b)
    torch.cuda.synchronize()

    events = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        for j, (lat, b) in enumerate(lats):
            ev0 = torch.cuda.Event(enable_timing=True)
            ev0.record(stream)
            lat.sweep_record_device(sweeps_per_step, b, every, Erec[j][i * (sweeps_per_step // every):],
                                    Mrec[j][i * (sweeps_per_step // every):])
            ev1 = torch.cuda.Event(enable_timing=True)
            ev1.record(stream)
            events.append((ev0, ev1))
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    step_gpu_ms = sum(a.elapsed_time(b) for a, b in events)

    # sweep-only segment: the same kernel without measurement, timed with events on its stream
    so_sweeps = min(200, max(20, args.steps))
    ev_a = torch.cuda.Event(enable_timing=True)
    ev_b = torch.cuda.Event(enable_timing=True)
    lat0, b0 = lats[1] if len(lats) > 1 else lats[0]
    ev_a.record(stream)
    lat0.sweep(so_sweeps, b0)
    ev_b.record(stream)
    torch.cuda.synchronize()
    so_ms = ev_a.elapsed_time(ev_b)
    launches_per_sweep = 1 if kname in ("fused",) else (0 if kname == "resident" else 2)
    if launches_per_sweep:
        kernel_avg_ms = so_ms / (so_sweeps * launches_per_sweep)
    else:
        kernel_avg_ms = so_ms
    attempts_per_launch = N if launches_per_sweep == 1 else (N // 2 if launches_per_sweep == 2 else N * so_sweeps)
    bytes_per_attempt = 2.0
    # algorithmic bytes per launch: each site read once and written once per sweep
    alg_bytes = bytes_per_attempt * (N if launches_per_sweep else N * so_sweeps) / max(1, launches_per_sweep)
    hbm_gbs = alg_bytes / (kernel_avg_ms * 1e-3) / 1e9
    sweep_only_rate = so_sweeps * N / (so_ms * 1e6)
    alu_tops = PHILOX_OPS_PER_ATTEMPT * sweep_only_rate * 1e9 / 1e12

    total_attempts = args.steps * sweeps_per_step * N * len(lats)
    value = total_attempts / (wall * 1e9)
    hbm_frac = hbm_gbs / HBM_PEAK_GBS
    alu_frac = alu_tops / VALU_PEAK_TOPS
    roof = {"bound": "hbm", "achieved": round(hbm_gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(hbm_frac, 4), "traffic": None, "kernel": kname,
            "kernel_avg_us": round(kernel_avg_ms * 1e3, 2),
            "alg_bytes_per_launch": int(alg_bytes)}
    if alu_frac > hbm_frac:
        roof = {"bound": "alu", "achieved": round(alu_tops, 2), "peak": round(VALU_PEAK_TOPS, 2),
                "unit": "Tops/s", "frac": round(alu_frac, 4), "traffic": None, "kernel": kname,
                "kernel_avg_us": round(kernel_avg_ms * 1e3, 2),
                "alg_ops_per_attempt": PHILOX_OPS_PER_ATTEMPT, "hbm_frac": round(hbm_frac, 4)}

    if args.copy_probe_mib:
        nb = args.copy_probe_mib << 20
        a = torch.empty(nb, dtype=torch.uint8, device="cuda")
        bb = torch.empty_like(a)
        bb.copy_(a)
        torch.cuda.synchronize()

    out = {
        "metric": "spin-flip attempts/ns + % HBM roofline; batched vs plain flips/ns; p50/p99 job latency",
        "value": round(value, 2),
        "unit": "spin-flip attempts/ns",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(wall * 1e3 / max(1, args.steps), 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "int8", "data": "synthetic",
        "config": {"workload": args.workload, "model": "ising", "L": L, "d": d,
                   "betas": [float(b) for b in cfg["betas"]], "sweeps_per_step": sweeps_per_step,
                   "record_every": every, "lattices": len(lats), "kernel": kname,
                   "parallelism": "single GPU"},
        "sweep_only_attempts_per_ns": round(sweep_only_rate, 2),
        "hbm_frac_sweep_only": round(hbm_frac, 4),
        "gpu_busy_ms_per_step": round(step_gpu_ms / max(1, args.steps), 4),
        "roofline": roof,
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(cfg, 25.0)
    for lat, _ in lats:
        lat.close()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
