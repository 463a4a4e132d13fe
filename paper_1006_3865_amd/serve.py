"""Serving loop over the lattice pool: continuous batching of simulation jobs.

A job is one lattice (model, L, d, beta, seed[, coupling seed]) to be swept
`sweeps` times, returning its final (E, M).  Jobs arrive over time; the
server keeps every admitted job's state on the device (a slot of a
spin_batch pool) and advances all of them together in ticks:

  1. admit arrived jobs in arrival order while the pool's HBM budget and
     slot count allow (first come, first served: a job that does not fit
     holds back the ones behind it);
  2. give every resident job a sweep quantum sized so that its share of the
     tick takes about `tick_s` seconds, at most its remaining sweeps, and
     run one pool call (one persistent launch per kernel class for the
     LDS-sized lattices, the single-lattice kernels for larger ones);
  3. measure (E, M) of the jobs that finished and retire them.

Each job's chain depends only on its own seed, replica and couplings, so its
result is the same bits whatever else shares the pool and however its sweeps
are split into ticks.

Time: the trace's arrival times are seconds from the start.  The loop runs
on a trace clock that advances by the measured wall time of each tick and
jumps to the next arrival when the pool is empty, so latencies are those of
a server that is never idle while work is queued, without sleeping through
the gaps.  The plain baseline runs the same jobs one at a time in arrival
order through lone lattices; its latencies follow from the measured service
times by the single-server FIFO recurrence.
"""
import math
import time

import numpy as np

LDS_BYTES = 150 * 1024  # packed (2 sites per byte) lattice limit of the persistent kernel


def lds_resident(L, d):
    """Whether the pool's persistent kernel holds this lattice (else the single-lattice kernels)."""
    return L >= 8 and L % 8 == 0 and (L ** d) // 2 <= LDS_BYTES


def footprint(job):
    """Device bytes of a job in the pool: spins (a second buffer for the streaming kernels of
    larger lattices) plus its couplings (nibble-packed in the persistent kernel's layout; int8 and
    nibble-packed for the larger lattices)."""
    N = job["L"] ** job["d"]
    if lds_resident(job["L"], job["d"]):
        return N + (job["d"] * N // 2 if job["model"] == 1 else 0)
    return 2 * N + (job["d"] * N + job["d"] * N // 2 if job["model"] == 1 else 0)


def percentile(values, q):
    """Nearest-rank percentile (q in (0, 100])."""
    v = sorted(values)
    if not v:
        return float("nan")
    k = max(1, int(math.ceil(q / 100.0 * len(v))))
    return v[k - 1]


def job_desc(job):
    d = dict(model=job["model"], L=job["L"], d=job["d"], seed=job["seed"], replica=job.get("replica", 0))
    if job["model"] == 1:
        d["coupling_seed"] = job["coupling_seed"]
        d["realisation"] = job.get("realisation", 0)
    return d


class PoolExecutor:
    """Executor over a spin_batch pool on the GPU."""

    def __init__(self, stream=None):
        from . import spin
        self.spin = spin
        self.pool = spin.Batch([], stream=stream)

    def add(self, job):
        return self.pool.add(job_desc(job))

    def remove(self, slot):
        self.pool.remove(slot)

    def slots(self):
        return self.pool.count

    def run(self, n, beta):
        """Advance slot i by n[i] sweeps at beta[i]; returns when done."""
        self.pool.sweep(n, beta, 0)

    def measure(self):
        return self.pool.measure()

    def spins(self, slot):
        return self.pool.spins(slot)

    def close(self):
        self.pool.close()


class Server:
    """Admission, tick scheduling and retirement; the executor does the sweeping."""

    def __init__(self, executor, budget_bytes=1 << 30, max_slots=512, tick_s=0.02,
                 rate_wg=2.0e9, rate_big=8.0e11, sweep_floor_s=15e-6, streams=4, clock=time.perf_counter,
                 keep_spins=False):
        self.ex = executor
        self.budget = budget_bytes
        self.max_slots = max_slots
        self.tick_s = tick_s
        self.rate_wg = rate_wg              # attempts/s of one workgroup on an LDS-resident lattice
        self.rate_big = rate_big            # attempts/s of the whole chip on a larger lattice
        self.sweep_floor_s = sweep_floor_s  # shortest sweep of a larger lattice (launch and pipeline latency)
        self.streams = streams              # larger lattices the pool runs at once
        self.clock = clock
        self.keep_spins = keep_spins
        self.ticks = 0

    def quantum(self, job, nbig):
        """Sweeps for this tick: what the job's own rate estimate does in tick_s, sharing the
        pool's streams with the other larger jobs; at least 1, at most what is left."""
        N = job["L"] ** job["d"]
        if lds_resident(job["L"], job["d"]):
            q = self.tick_s * self.rate_wg / N
        else:
            rate = min(self.rate_big, N / self.sweep_floor_s)
            share = max(1.0, nbig / float(self.streams))
            q = self.tick_s * rate / (N * share)
        return int(min(job["left"], max(1, math.floor(q))))

    def _cancelled(self, j, now, cancel):
        """Why job j is to be cancelled at trace time now, or None."""
        at = cancel.get(j["job"]) if cancel else None
        if at is not None and at <= now:
            return "cancelled"
        dl = j.get("deadline_s")
        if dl is not None and now - j["arrival"] > dl:
            return "deadline"
        return None

    def serve(self, trace, cancel=None):
        """Run every job of the trace; returns dict job -> result (E, M, latency, ...).

        cancel: optional dict job -> trace time of a cancellation request.  A job with a
        "deadline_s" field is cancelled by the watchdog once its age (now - arrival) exceeds it.
        Both take effect at the next tick boundary: a waiting job is dropped, a resident one leaves
        the pool and frees its slot and budget; its result is {cancelled: True, reason, sweeps_done,
        arrival, finished, latency}.  The other jobs' results do not change."""
        jobs = sorted((dict(j) for j in trace), key=lambda j: (j["arrival"], j["job"]))
        for j in jobs:
            if footprint(j) > self.budget:
                raise ValueError("job %d needs %d bytes, more than the budget" % (j["job"], footprint(j)))
        results = {}
        waiting = list(jobs)          # arrival order
        resident = {}                 # slot -> job
        used = 0
        now = 0.0
        while waiting or resident:
            t0 = self.clock()
            # cancellations and the watchdog
            for j in [j for j in waiting if j["arrival"] <= now and self._cancelled(j, now, cancel)]:
                waiting.remove(j)
                results[j["job"]] = dict(cancelled=True, reason=self._cancelled(j, now, cancel), sweeps_done=0,
                                         arrival=j["arrival"], finished=now, latency=now - j["arrival"])
            for s in [s for s, j in resident.items() if self._cancelled(j, now, cancel)]:
                j = resident.pop(s)
                self.ex.remove(s)
                used -= footprint(j)
                results[j["job"]] = dict(cancelled=True, reason=self._cancelled(j, now, cancel),
                                         sweeps_done=j["sweeps"] - j["left"], arrival=j["arrival"],
                                         admitted=j["admitted"], finished=now, latency=now - j["arrival"])
            if not waiting and not resident:
                break
            # admission, first come first served
            while waiting and waiting[0]["arrival"] <= now:
                j = waiting[0]
                fp = footprint(j)
                if used + fp > self.budget or len(resident) >= self.max_slots:
                    break
                waiting.pop(0)
                j["slot"] = self.ex.add(j)
                j["left"] = j["sweeps"]
                j["admitted"] = now
                used += fp
                resident[j["slot"]] = j
            if not resident:
                now = max(now + (self.clock() - t0), waiting[0]["arrival"])
                continue
            S = self.ex.slots()
            n = np.zeros(S, dtype=np.int32)
            beta = np.zeros(S)
            nbig = sum(1 for j in resident.values() if not lds_resident(j["L"], j["d"]))
            for s, j in resident.items():
                n[s] = self.quantum(j, nbig)
                beta[s] = j["beta"]
            self.ex.run(n, beta)
            for s, j in resident.items():
                j["left"] -= int(n[s])
            done = [s for s, j in resident.items() if j["left"] == 0]
            finished = []
            if done:
                E, M = self.ex.measure()
                for s in done:
                    j = resident.pop(s)
                    r = dict(E=int(E[s]), M=int(M[s]), arrival=j["arrival"], admitted=j["admitted"])
                    if self.keep_spins:
                        r["spins"] = self.ex.spins(s)
                    self.ex.remove(s)
                    used -= footprint(j)
                    results[j["job"]] = r
                    finished.append(r)
            now += self.clock() - t0
            for r in finished:
                r["finished"] = now
                r["latency"] = now - r["arrival"]
            self.ticks += 1
        return results


def plain_fifo(trace, service):
    """Single-server FIFO in arrival order: service(job) runs one job alone and returns
    (E, M, seconds).  Returns dict job -> result with latency from the recurrence
    start = max(arrival, previous finish)."""
    jobs = sorted(trace, key=lambda j: (j["arrival"], j["job"]))
    results = {}
    free_at = 0.0
    for j in jobs:
        E, M, secs = service(j)
        start = max(j["arrival"], free_at)
        free_at = start + secs
        results[j["job"]] = dict(E=E, M=M, arrival=j["arrival"], finished=free_at,
                                 latency=free_at - j["arrival"], service=secs)
    return results


def lone_service(job, spins_out=None):
    """Run one job alone on a single-lattice handle (the library's own kernel choice)."""
    from . import spin
    d = job_desc(job)
    lat = spin.Lattice(d["model"], d["L"], d["d"], d["seed"], coupling_seed=d.get("coupling_seed"),
                       realisation=d.get("realisation", 0), replica=d["replica"])
    lat.synchronize()
    t0 = time.perf_counter()
    lat.sweep(job["sweeps"], job["beta"])
    E, M = lat.measure()
    secs = time.perf_counter() - t0
    if spins_out is not None:
        spins_out[job["job"]] = lat.spins()
    lat.close()
    return E, M, secs


def summarize(results, trace):
    lat = [r["latency"] for r in results.values() if not r.get("cancelled")]
    work = sum(j["L"] ** j["d"] * j["sweeps"] for j in trace)
    span = max(r["finished"] for r in results.values()) - min(j["arrival"] for j in trace)
    return dict(jobs=len(results), p50_s=percentile(lat, 50), p99_s=percentile(lat, 99),
                attempts_per_ns=work / span / 1e9 if span > 0 else float("nan"), makespan_s=span)
