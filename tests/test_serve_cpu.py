"""Host logic of the serving loop (no GPU): admission, quanta, retirement, latency bookkeeping.

A fake executor stands in for the pool: it counts sweeps per slot, checks the
budget and slot limits, and advances a virtual clock by a cost model.  An
oracle-backed executor checks that splitting a job's sweeps into ticks gives
the same final state as running it in one call.
"""
import numpy as np
import pytest

from paper_1006_3865_amd import serve, workloads


class Clock:
    def __init__(self):
        self.t = 0.0

    def __call__(self):
        return self.t


class FakeExecutor:
    def __init__(self, clock, budget, max_slots, cost_per_attempt=1e-12, overhead=1e-4):
        self.clock = clock
        self.budget = budget
        self.max_slots = max_slots
        self.cost = cost_per_attempt
        self.overhead = overhead
        self.slot_job = []
        self.free = []
        self.done_sweeps = {}
        self.admit_order = []
        self.peak_used = 0
        self.peak_slots = 0

    def used(self):
        return sum(serve.footprint(j) for j in self.slot_job if j is not None)

    def add(self, job):
        if self.free:
            s = self.free.pop()
            self.slot_job[s] = job
        else:
            s = len(self.slot_job)
            self.slot_job.append(job)
        self.done_sweeps[job["job"]] = 0
        self.admit_order.append(job["job"])
        self.peak_used = max(self.peak_used, self.used())
        self.peak_slots = max(self.peak_slots, sum(j is not None for j in self.slot_job))
        assert self.used() <= self.budget
        return s

    def remove(self, s):
        assert self.slot_job[s] is not None
        self.slot_job[s] = None
        self.free.append(s)

    def slots(self):
        return len(self.slot_job)

    def run(self, n, beta):
        assert len(n) == len(self.slot_job)
        work = 0
        longest = 0.0
        for s, j in enumerate(self.slot_job):
            if j is None:
                assert n[s] == 0
                continue
            assert n[s] >= 1, "a resident job got no sweeps"
            assert beta[s] == j["beta"]
            self.done_sweeps[j["job"]] += int(n[s])
            a = int(n[s]) * j["L"] ** j["d"]
            work += a
            longest = max(longest, a / 2e9)
        self.clock.t += self.overhead + max(longest, work * self.cost)

    def measure(self):
        S = len(self.slot_job)
        E = np.zeros(S, dtype=np.int64)
        M = np.zeros(S, dtype=np.int64)
        for s, j in enumerate(self.slot_job):
            if j is not None:
                E[s] = -j["job"]
                M[s] = self.done_sweeps[j["job"]]
        return E, M

    def spins(self, s):
        return np.zeros(1, dtype=np.int8)


def small_trace(jobs=60, rate=200.0):
    tr = workloads.serve_trace(jobs=jobs, rate_per_s=rate)
    for j in tr:
        j["sweeps"] = min(j["sweeps"], 400)
    return tr


def test_every_job_gets_exactly_its_sweeps():
    clock = Clock()
    tr = small_trace()
    ex = FakeExecutor(clock, 1 << 30, 512)
    srv = serve.Server(ex, budget_bytes=1 << 30, max_slots=512, clock=clock)
    res = srv.serve(tr)
    assert sorted(res) == sorted(j["job"] for j in tr)
    for j in tr:
        r = res[j["job"]]
        assert r["E"] == -j["job"]
        assert r["M"] == j["sweeps"]
        assert ex.done_sweeps[j["job"]] == j["sweeps"]
        assert r["finished"] >= j["arrival"]
        assert r["latency"] == pytest.approx(r["finished"] - j["arrival"])
        assert r["admitted"] >= j["arrival"]


def test_budget_and_slots_respected_and_fifo():
    clock = Clock()
    tr = small_trace(80, rate=5000.0)
    budget = 64 << 20
    tr = [j for j in tr if serve.footprint(j) <= budget]
    ex = FakeExecutor(clock, budget, 7)
    srv = serve.Server(ex, budget_bytes=budget, max_slots=7, clock=clock)
    res = srv.serve(tr)
    assert len(res) == len(tr)
    assert ex.peak_used <= budget
    assert ex.peak_slots <= 7
    arrival = {j["job"]: (j["arrival"], j["job"]) for j in tr}
    order = [arrival[k] for k in ex.admit_order]
    assert order == sorted(order), "admission is not first come first served"


def test_job_over_budget_is_rejected():
    clock = Clock()
    job = dict(job=0, arrival=0.0, model=0, d=2, L=4096, beta=0.4, sweeps=10, seed=1)
    srv = serve.Server(FakeExecutor(clock, 1 << 20, 4), budget_bytes=1 << 20, clock=clock)
    with pytest.raises(ValueError):
        srv.serve([job])


def test_quantum_bounds():
    srv = serve.Server(None, tick_s=0.01, rate_wg=1e9, rate_big=1e12, sweep_floor_s=1e-5, streams=4)
    small = dict(L=16, d=3, left=10 ** 6)
    assert srv.quantum(small, 0) == int(0.01 * 1e9 / 16 ** 3)
    assert srv.quantum(dict(L=16, d=3, left=5), 0) == 5
    big = dict(L=4096, d=2, left=10 ** 6)                   # chip-rate bound, 8 jobs share 4 streams
    assert srv.quantum(big, 8) == int(0.01 * 1e12 / (4096 ** 2 * 2))
    assert srv.quantum(big, 3) == int(0.01 * 1e12 / 4096 ** 2)
    mid = dict(L=72, d=3, left=10 ** 6)                     # latency-floor bound: tick / floor sweeps
    assert abs(srv.quantum(mid, 1) - 1000) <= 1
    huge = dict(L=1 << 15, d=2, left=7)
    assert srv.quantum(huge, 100) == 1  # at least one sweep per tick


def test_idle_gaps_jump_to_next_arrival():
    clock = Clock()
    tr = [dict(job=0, arrival=0.0, model=0, d=2, L=16, beta=0.4, sweeps=10, seed=1),
          dict(job=1, arrival=100.0, model=0, d=2, L=16, beta=0.4, sweeps=10, seed=2)]
    ex = FakeExecutor(clock, 1 << 30, 4)
    res = serve.Server(ex, clock=clock).serve(tr)
    assert res[1]["admitted"] == 100.0
    assert res[1]["latency"] < 1.0


def test_percentile_nearest_rank():
    v = [5, 1, 4, 2, 3]
    assert serve.percentile(v, 50) == 3
    assert serve.percentile(v, 99) == 5
    assert serve.percentile(v, 100) == 5
    assert serve.percentile(list(range(1, 101)), 99) == 99
    assert serve.percentile(list(range(1, 101)), 50) == 50


def test_plain_fifo_recurrence():
    tr = [dict(job=0, arrival=0.0), dict(job=1, arrival=0.5), dict(job=2, arrival=10.0)]
    svc = {0: 2.0, 1: 1.0, 2: 0.5}
    res = serve.plain_fifo(tr, lambda j: (0, 0, svc[j["job"]]))
    assert res[0]["finished"] == 2.0 and res[0]["latency"] == 2.0
    assert res[1]["finished"] == 3.0 and res[1]["latency"] == 2.5
    assert res[2]["finished"] == 10.5 and res[2]["latency"] == 0.5


def test_footprint_rule():
    assert serve.lds_resident(552, 2) and not serve.lds_resident(560, 2)
    assert serve.lds_resident(64, 3) and not serve.lds_resident(72, 3)
    assert not serve.lds_resident(12, 2)
    assert serve.footprint(dict(model=1, L=16, d=3)) == 4096 + 3 * 4096 // 2
    assert serve.footprint(dict(model=0, L=1024, d=2)) == 2 * 1024 ** 2
    assert serve.footprint(dict(model=1, L=72, d=3)) == 2 * 72 ** 3 + 3 * 72 ** 3 + 3 * 72 ** 3 // 2


class OracleExecutor:
    """Pool stand-in on the CPU oracle: per-slot chains."""

    def __init__(self, oracle_mod):
        self.o = oracle_mod
        self.chains = []

    def add(self, job):
        d = serve.job_desc(job)
        J = None
        if d["model"] == 1:
            J = self.o.couplings(d["L"], d["d"], d["coupling_seed"], d["realisation"])
        ch = self.o.Chain(d["L"], d["d"], d["seed"], d["replica"], J=J)
        if None in self.chains:
            s = self.chains.index(None)
            self.chains[s] = ch
        else:
            s = len(self.chains)
            self.chains.append(ch)
        return s

    def remove(self, s):
        self.chains[s] = None

    def slots(self):
        return len(self.chains)

    def run(self, n, beta):
        for s, ch in enumerate(self.chains):
            if ch is not None and n[s]:
                ch.sweep(int(n[s]), float(beta[s]))

    def measure(self):
        S = len(self.chains)
        E = np.zeros(S, dtype=np.int64)
        M = np.zeros(S, dtype=np.int64)
        for s, ch in enumerate(self.chains):
            if ch is not None:
                E[s], M[s] = ch.measure()
        return E, M

    def spins(self, s):
        return self.chains[s].spins.copy()


def test_ticked_jobs_equal_one_shot_runs(oracle_mod):
    """Splitting a job's sweeps into ticks, with other jobs in the pool, leaves its chain unchanged."""
    tr = []
    rng = np.random.default_rng(3)
    for k in range(12):
        model = k % 3 == 2
        d = 2 if k % 3 == 0 else 3
        L = int(rng.choice([8, 12, 16])) if d == 3 else int(rng.choice([16, 24, 32]))
        tr.append(dict(job=k, arrival=0.001 * k, model=int(model), d=d, L=L, beta=float(rng.uniform(0.1, 1.0)),
                       sweeps=int(rng.integers(5, 60)), seed=workloads.seed(0x3000 + k),
                       coupling_seed=workloads.seed(0x4000 + k)))
    clock = Clock()
    ex = OracleExecutor(oracle_mod)

    def tick_clock():
        clock.t += 1e-4
        return clock.t

    # tiny quanta force many ticks per job
    srv = serve.Server(ex, tick_s=1e-4, rate_wg=2e6, rate_big=2e6, clock=tick_clock, keep_spins=True)
    res = srv.serve(tr)
    assert srv.ticks > 10
    for j in tr:
        d = serve.job_desc(j)
        J = oracle_mod.couplings(d["L"], d["d"], d["coupling_seed"], 0) if j["model"] == 1 else None
        ch = oracle_mod.Chain(d["L"], d["d"], d["seed"], 0, J=J)
        ch.sweep(j["sweeps"], j["beta"])
        np.testing.assert_array_equal(res[j["job"]]["spins"], ch.spins)
        assert (res[j["job"]]["E"], res[j["job"]]["M"]) == ch.measure()


def test_cancel_waiting_job_never_admitted():
    """A job cancelled while it waits for budget is dropped without being admitted."""
    clock = Clock()
    budget = 3 << 20
    tr = [dict(job=k, arrival=0.0, model=0, d=2, L=1024, beta=0.4, sweeps=2000, seed=k) for k in range(3)]
    ex = FakeExecutor(clock, budget, 8)
    srv = serve.Server(ex, budget_bytes=budget, max_slots=8, clock=clock)
    res = srv.serve(tr, cancel={2: 0.0})
    assert res[2]["cancelled"] and res[2]["reason"] == "cancelled" and res[2]["sweeps_done"] == 0
    assert 2 not in ex.admit_order
    for k in (0, 1):
        assert not res[k].get("cancelled") and ex.done_sweeps[k] == 2000 and res[k]["M"] == 2000


def test_cancel_resident_job_frees_slot_and_budget():
    """Cancelling a running job frees its slot and budget for the job queued behind it."""
    clock = Clock()
    budget = 2 << 20                                 # one L = 1024 job (2 MiB) at a time
    tr = [dict(job=0, arrival=0.0, model=0, d=2, L=1024, beta=0.4, sweeps=10 ** 6, seed=1),
          dict(job=1, arrival=0.0, model=0, d=2, L=1024, beta=0.4, sweeps=300, seed=2)]
    ex = FakeExecutor(clock, budget, 1)
    srv = serve.Server(ex, budget_bytes=budget, max_slots=1, clock=clock)
    res = srv.serve(tr, cancel={0: 0.05})
    r0 = res[0]
    assert r0["cancelled"] and 0 < r0["sweeps_done"] < 10 ** 6
    assert r0["sweeps_done"] == ex.done_sweeps[0]
    assert r0["finished"] >= 0.05
    assert ex.admit_order == [0, 1]
    assert not res[1].get("cancelled") and ex.done_sweeps[1] == 300
    assert res[1]["admitted"] >= r0["finished"]
    assert ex.peak_used <= budget


def test_deadline_watchdog_cancels_overdue_jobs():
    clock = Clock()
    tr = [dict(job=0, arrival=0.0, model=0, d=2, L=2048, beta=0.4, sweeps=10 ** 6, seed=1, deadline_s=0.2),
          dict(job=1, arrival=0.0, model=0, d=2, L=32, beta=0.4, sweeps=100, seed=2, deadline_s=100.0)]
    ex = FakeExecutor(clock, 1 << 30, 8)
    res = serve.Server(ex, clock=clock).serve(tr)
    assert res[0]["cancelled"] and res[0]["reason"] == "deadline"
    assert res[0]["latency"] > 0.2 and res[0]["sweeps_done"] < 10 ** 6   # stopped at the first tick past it
    assert not res[1].get("cancelled") and ex.done_sweeps[1] == 100
    s = serve.summarize(res, tr)
    assert s["jobs"] == 2


def test_cancellation_leaves_other_results_unchanged(oracle_mod):
    """Jobs that share the pool with a cancelled one end in the same state as run alone."""
    tr = [dict(job=k, arrival=0.0, model=k % 2, d=3 if k % 2 else 2, L=16 if k % 2 else 32,
               beta=0.3 + 0.1 * k, sweeps=40, seed=workloads.seed(0x5000 + k),
               coupling_seed=workloads.seed(0x6000 + k)) for k in range(5)]
    clock = Clock()

    def tick_clock():
        clock.t += 1e-4
        return clock.t

    ex = OracleExecutor(oracle_mod)
    srv = serve.Server(ex, tick_s=1e-4, rate_wg=4e6, rate_big=4e6, clock=tick_clock, keep_spins=True)
    res = srv.serve(tr, cancel={2: 5e-4})
    assert res[2]["cancelled"] and 0 < res[2]["sweeps_done"] < 40
    for j in tr:
        if j["job"] == 2:
            continue
        d = serve.job_desc(j)
        J = oracle_mod.couplings(d["L"], d["d"], d["coupling_seed"], 0) if j["model"] == 1 else None
        ch = oracle_mod.Chain(d["L"], d["d"], d["seed"], 0, J=J)
        ch.sweep(j["sweeps"], j["beta"])
        np.testing.assert_array_equal(res[j["job"]]["spins"], ch.spins)
        assert (res[j["job"]]["E"], res[j["job"]]["M"]) == ch.measure()
