"""Continuous-batching solve server for one GPU.

Solve requests (a lattice case and a step budget) arrive over time.  The
server keeps every admitted lattice resident in device memory until its last
step and advances all resident lattices together: each round is one batched
step sequence of the library (one launch per kernel for all lattices, each
lattice taking its own number of steps, at most one chunk).  Between rounds it
retires finished requests (their fields are read back, which completes the
request) and admits queued requests in arrival order while their device bytes
fit the memory budget and a slot is free.  A round is sized to about
`round_s` seconds at the measured update rate and shared equally in work among
the resident requests: each takes as many steps as its share of lattice
updates buys (at least one), so small requests finish in few rounds instead of
advancing in lock-step with the largest ones, and an arriving request waits at
most about one round for admission.

Failures are isolated per request.  After every round the backend reports
each resident lattice's failure flag (the library sets it when a temperature
iteration does not converge, which is how a non-physical or non-finite state
shows itself); a flagged request is retired at once with an error and its
memory released, while the others continue untouched (their lattices share
launches but no data).  A request whose lattice cannot be created, or whose
result cannot be read back, is failed the same way.

Scheduling is host logic over a small backend interface, so it is tested on
the CPU with a simulated backend; `GpuBackend` is the one that runs the step.
"""
from __future__ import annotations

import time
from dataclasses import dataclass


@dataclass
class Request:
    rid: int
    arrival: float          # seconds after the server starts
    case: dict
    steps: int
    nodes: int = 0
    nbytes: int = 0
    admitted: float | None = None
    done: float | None = None
    result: dict | None = None
    error: str | None = None

    @property
    def failed(self):
        return self.error is not None

    @property
    def latency(self):
        return None if self.done is None else self.done - self.arrival


class GpuBackend:
    """Lattices in device memory, stepped through the library's batches."""

    def __init__(self, mech, storage="f32dev", keep="fields"):
        from . import rlbm
        self.rlbm = rlbm
        self.mech = rlbm.Mechanism(mech) if isinstance(mech, dict) else mech
        self.storage = storage
        self.keep = keep            # "fields", "populations" or "none"
        self._batches = []
        self._batch_key = None

    def nbytes(self, case):
        return self.rlbm.lattice_bytes(case, self.mech, self.storage) + 256

    def create(self, case):
        return self.rlbm.Lattice(case, storage=self.storage, mech=self.mech).set_state()

    def step(self, lattices, steps):
        """Enqueue one round (asynchronous), then gather every lattice's
        failure flag (one small read per batch, which waits for the round);
        returns the flags in the order of `lattices`."""
        # one batch per storage layout: lattices with a slaved species and
        # weakly coupled ones (one lattice more) cannot share launches
        groups = {}
        for k, lat in enumerate(lattices):
            groups.setdefault(lat.L, []).append(k)
        key = tuple((L, tuple(id(lattices[k]) for k in ks)) for L, ks in sorted(groups.items()))
        if key != self._batch_key:
            self._batches = [(self.rlbm.Batch([lattices[k] for k in ks]), ks)
                             for _, ks in sorted(groups.items())]
            self._batch_key = key
        for batch, ks in self._batches:
            batch.step([steps[k] for k in ks])
        status = [0] * len(lattices)
        for batch, ks in self._batches:
            for k, st in zip(ks, batch.status()):
                status[k] = st
        return status

    def finish(self, lat):
        if self.keep == "fields":
            return lat.fields()
        if self.keep == "populations":
            return {"populations": lat.populations()}
        lat.invariants()            # synchronises and checks for non-finite state
        return {}

    def release(self, lat):
        # batches that hold the lattice go first; the next round builds new ones
        self._batches = []
        self._batch_key = None
        lat.close()


class Server:
    """First-come-first-served admission under a byte budget and a slot cap;
    continuous batching of everything resident."""

    def __init__(self, backend, budget_bytes=200e9, max_slots=256, round_s=0.05,
                 rate_guess=3e8, min_chunk=1, max_chunk=2000, clock=time.perf_counter,
                 sleep=time.sleep):
        self.backend = backend
        self.budget = float(budget_bytes)
        self.max_slots = int(max_slots)
        self.round_s = float(round_s)
        self.rate = float(rate_guess)          # lattice updates per second, measured
        self.min_chunk, self.max_chunk = int(min_chunk), int(max_chunk)
        self.clock, self.sleep = clock, sleep
        self.rounds = 0
        self.updates = 0

    def _steps(self, active):
        """Steps of each resident request in the next round: an equal share
        of the round's updates, within [min_chunk, max_chunk] and the steps
        it has left."""
        share = self.round_s * self.rate / len(active)
        return [min(a[2], max(self.min_chunk, min(self.max_chunk, int(share / a[0].nodes))))
                for a in active]

    def run(self, requests, on_done=None):
        """Serve `requests` (arrival times relative to the start); returns them
        with admitted/done times and results filled in.  on_done(request), if
        given, is called as each request completes or fails."""
        queue = sorted(requests, key=lambda r: (r.arrival, r.rid))
        for r in queue:
            r.nodes = int(r.case["nx"]) * int(r.case["ny"]) * int(r.case["nz"])
            r.nbytes = self.backend.nbytes(r.case)
            if r.nbytes > self.budget:
                raise ValueError(f"request {r.rid} needs {r.nbytes} B, more than the budget")
        active = []                  # [request, lattice, steps left]
        used = 0
        head = 0
        t0 = self.clock()
        while head < len(queue) or active:
            now = self.clock() - t0
            # admission, in arrival order, while the head fits
            while head < len(queue) and queue[head].arrival <= now and len(active) < self.max_slots \
                    and used + queue[head].nbytes <= self.budget:
                r = queue[head]
                head += 1
                try:
                    lat = self.backend.create(r.case)
                except Exception as e:          # the request fails, the server goes on
                    r.error = f"create: {e}"
                    r.done = self.clock() - t0
                    if on_done:
                        on_done(r)
                    continue
                r.admitted = self.clock() - t0
                used += r.nbytes
                active.append([r, lat, r.steps])
            if not active:
                if head < len(queue):
                    self.sleep(max(0.0, queue[head].arrival - (self.clock() - t0)))
                continue
            steps = self._steps(active)
            ts = self.clock()
            status = self.backend.step([a[1] for a in active], steps)
            if status is None:
                status = [0] * len(active)
            work = sum(a[0].nodes * s for a, s, st in zip(active, steps, status) if not st)
            dt = self.clock() - ts
            if dt > 0 and work > 0:
                self.rate = 0.5 * self.rate + 0.5 * work / dt
            self.updates += work
            self.rounds += 1
            keep = []
            for a, s, st in zip(active, steps, status):
                a[2] -= s
                r, lat = a[0], a[1]
                if st:
                    # quarantine: retire the failed request alone
                    r.error = f"failure flag {st}: a temperature iteration did not converge " \
                              f"(non-physical or non-finite state)"
                elif a[2] == 0:
                    try:
                        r.result = self.backend.finish(lat)
                    except Exception as e:
                        r.error = f"read-back: {e}"
                else:
                    keep.append(a)
                    continue
                r.done = self.clock() - t0
                self.backend.release(lat)
                used -= r.nbytes
                if on_done:
                    on_done(r)
            active = keep
        return queue


def percentile(values, p):
    """Nearest-rank percentile (p in [0, 100])."""
    v = sorted(values)
    if not v:
        return None
    k = max(0, min(len(v) - 1, int(-(-p * len(v) // 100)) - 1))
    return v[k]


def summarize(requests, wall_s):
    """Throughput over the completed requests' lattice updates; latency
    percentiles over the completed requests (failed ones are counted apart)."""
    ok = [r for r in requests if not r.failed]
    lat = [r.latency for r in ok]
    work = sum(r.nodes * r.steps for r in ok)
    return {"requests": len(requests), "failed": len(requests) - len(ok), "wall_s": wall_s,
            "updates": work, "mlups": work / wall_s / 1e6 if wall_s > 0 else None,
            "p50_s": percentile(lat, 50), "p99_s": percentile(lat, 99),
            "max_s": max(lat) if lat else None}
