"""Serving loop on the GPU: every job's result is the same bits alone and in the mix.

A short trace of the serving workload's kinds (2D Ising, 3D Ising, 3D +-J),
with LDS-sized lattices and larger ones (single-lattice kernels in the same
ticks), sweeps capped so the test runs in seconds.  Each job's final spins
and (E, M) from the pool are compared with the job run alone on a lone
lattice, and with the oracle where the oracle is quick.
"""
import sys

import numpy as np
import pytest

from paper_1006_3865_amd import serve, spin, workloads

pytestmark = pytest.mark.gpu


def note(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module", autouse=True)
def gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("no GPU visible")
    spin.load()
    return torch


def trace(jobs=40):
    tr = workloads.serve_trace(jobs=jobs, rate_per_s=400.0)
    for j in tr:
        if j["d"] == 2:
            j["L"] = min(j["L"], 1024)
        else:
            j["L"] = min(j["L"], 80)
        j["sweeps"] = min(j["sweeps"], 300)
    return tr


def test_served_equals_alone_and_oracle(oracle_mod):
    tr = trace()
    kinds = {(j["model"], j["d"], serve.lds_resident(j["L"], j["d"])) for j in tr}
    note("kinds", sorted(kinds))
    assert any(not k[2] for k in kinds) and any(k[2] for k in kinds)
    ex = serve.PoolExecutor()
    srv = serve.Server(ex, budget_bytes=256 << 20, max_slots=16, tick_s=0.002, keep_spins=True)
    res = srv.serve(tr)
    note("ticks", srv.ticks, serve.summarize(res, tr))
    assert srv.ticks > len(tr) // 4
    alone = {}
    for j in tr:
        E, M, _ = serve.lone_service(j, spins_out=alone)
        r = res[j["job"]]
        np.testing.assert_array_equal(r["spins"], alone[j["job"]], err_msg="job %d spins" % j["job"])
        assert (r["E"], r["M"]) == (E, M), "job %d" % j["job"]
        if j["L"] ** j["d"] * j["sweeps"] <= 3 * 10 ** 7:
            d = serve.job_desc(j)
            J = oracle_mod.couplings(d["L"], d["d"], d["coupling_seed"], 0) if j["model"] == 1 else None
            ch = oracle_mod.Chain(d["L"], d["d"], d["seed"], 0, J=J)
            ch.sweep(j["sweeps"], j["beta"])
            np.testing.assert_array_equal(r["spins"], ch.spins, err_msg="job %d vs oracle" % j["job"])
            assert (r["E"], r["M"]) == ch.measure()
    ex.close()


def test_pool_footprint_matches_host_rule():
    b = spin.Batch([])
    for desc in (dict(model=1, L=16, d=3, seed=1, coupling_seed=5), dict(model=0, L=1024, d=2, seed=2),
                 dict(model=1, L=72, d=3, seed=3, coupling_seed=5), dict(model=0, L=12, d=2, seed=4)):
        s = b.add(desc)
        assert b.footprint(s) == serve.footprint(desc), desc
    b.close()
