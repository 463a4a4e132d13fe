"""Write the full-length oracle records of the benchmark configurations.

Runs the CPU oracle only (oracle/), over the whole schedule of each
configuration, and stores what a GPU run must reproduce bit for bit:

  ising2d_L8192_b{0,1,2}.json  2D Ising L=8192 at beta 0.30, 0.4406868, 0.60:
                                2000 sweeps, (E, M) after every 10th, SHA-256
                                of the int8 spins after sweeps 10, 100, 2000.
  ising3d_L512.json             3D Ising L=512 at beta 0.2216544: 1000 sweeps,
                                (E, M) every 10th, spins after 10 and 1000.
  ea3d_subset_{0..3}.json       3D +-J EA, the stratified subset of the batched
                                workload (2 realisations of each L x 16 betas =
                                160 lattices, split in 4 files): 5000 sweeps,
                                (E, M) every 100th, spins after 5000.

Sweeps run in calls of `every` sweeps, so records fall on absolute sweeps
every, 2 every, ...  Hours of single-core work per file; run the files in
parallel processes:  python tests/golden/make_full_runs.py [name ...]
"""
import hashlib
import json
import multiprocessing as mp
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

from oracle import oracle as O  # noqa: E402
from paper_1006_3865_amd import workloads as W  # noqa: E402  (seeds and sizes only)


def sha(spins):
    return hashlib.sha256(spins.tobytes()).hexdigest()


def ea_subset():
    """2 realisations of each size (the first two in realisation order) x 16 betas."""
    descs = W.ea_batch()
    picked = []
    for L in (16, 24, 32, 48, 64):
        rs = sorted({d["realisation"] for d in descs if d["L"] == L})[:2]
        picked += [d for d in descs if d["realisation"] in rs]
    return picked


def run_single(model, L, d, seed, beta, sweeps, every, checkpoints, log):
    ch = O.Chain(L, d, seed, 0)
    E, M, hashes = [], [], {}
    t0 = time.time()
    while ch.t < sweeps:
        e, m = ch.sweep(every, beta, every=every)
        E += [int(x) for x in e]
        M += [int(x) for x in m]
        if ch.t in checkpoints:
            hashes[str(ch.t)] = sha(ch.spins)
        if ch.t % (10 * every) == 0:
            print("%s t=%d %.0fs" % (log, ch.t, time.time() - t0), flush=True)
    return dict(model=model, L=L, d=d, seed=seed, replica=0, beta_hex=float.hex(beta), sweeps=sweeps,
                every=every, E=E, M=M, spins_sha256=hashes)


def job(name):
    if name.startswith("ising2d_L8192_b"):
        i = int(name[-1])
        c = W.CONFIGS["ising2d_L8192"]
        out = run_single(0, 8192, 2, c["seed"], c["betas"][i], c["sweeps"], c["every"], {10, 100, 2000}, name)
    elif name == "ising3d_L512":
        c = W.CONFIGS["ising3d_L512"]
        out = run_single(0, 512, 3, c["seed"], c["betas"][0], c["sweeps"], c["every"], {10, 1000}, name)
    elif name.startswith("ea3d_subset_"):
        part = int(name[-1])
        descs = ea_subset()[part::4]
        lats = []
        t0 = time.time()
        for k, d in enumerate(descs):
            J = O.couplings(d["L"], 3, d["coupling_seed"], d["realisation"])
            ch = O.Chain(d["L"], 3, d["seed"], d["replica"], J=J)
            E, M = [], []
            while ch.t < 5000:
                e, m = ch.sweep(100, d["beta"], every=100)
                E += [int(x) for x in e]
                M += [int(x) for x in m]
            lats.append(dict(realisation=d["realisation"], L=d["L"], replica=d["replica"],
                             beta_hex=float.hex(d["beta"]), E=E, M=M, spins_sha256={"5000": sha(ch.spins)}))
            print("%s lattice %d/%d %.0fs" % (name, k + 1, len(descs), time.time() - t0), flush=True)
        out = dict(model=1, d=3, coupling_seed=W.seed(0x11), seed=W.seed(0x10), sweeps=5000, every=100,
                   lattices=lats)
    else:
        raise SystemExit("unknown record " + name)
    out["generator"] = "tests/golden/make_full_runs.py (CPU oracle)"
    path = os.path.join(HERE, "full_" + name + ".json")
    with open(path + ".tmp", "w") as f:
        json.dump(out, f)
    os.replace(path + ".tmp", path)
    return name


ALL = ["ising2d_L8192_b0", "ising2d_L8192_b1", "ising2d_L8192_b2", "ising3d_L512"] + \
      ["ea3d_subset_%d" % i for i in range(4)]

if __name__ == "__main__":
    names = sys.argv[1:] or ALL
    O.build()
    with mp.Pool(len(names)) as pool:
        for n in pool.imap_unordered(job, names):
            print("done", n, flush=True)
