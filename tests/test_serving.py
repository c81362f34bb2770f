"""Continuous-batching server: scheduling on a simulated backend (CPU), and on
the GPU the identity of every result served in a mix with the same request
solved alone."""
import numpy as np
import pytest

from paper_2108_07605_amd.serving import Request, Server, percentile, summarize


class SimClock:
    def __init__(self):
        self.t = 0.0

    def __call__(self):
        return self.t

    def sleep(self, dt):
        self.t += max(dt, 1e-6)


class SimBackend:
    """Lattices are dicts counting the steps they were given; a step round
    costs updates / rate seconds of simulated time."""

    def __init__(self, clock, rate=1e6):
        self.clock, self.rate = clock, rate
        self.resident = 0
        self.peak_bytes = 0
        self.peak_slots = 0
        self.live = set()
        self.used = 0
        self.rounds = []

    def nbytes(self, case):
        return case["bytes"]

    def create(self, case):
        lat = {"case": case, "steps": 0, "id": len(self.rounds) * 1000 + len(self.live)}
        self.live.add(id(lat))
        self.used += case["bytes"]
        self.peak_bytes = max(self.peak_bytes, self.used)
        self.peak_slots = max(self.peak_slots, len(self.live))
        return lat

    def step(self, lats, steps):
        assert len(lats) == len(steps) and all(s >= 1 for s in steps)
        work = 0
        for lat, s in zip(lats, steps):
            lat["steps"] += s
            work += lat["case"]["nx"] * s
        self.rounds.append(len(lats))
        self.clock.t += work / self.rate

    def finish(self, lat):
        return {"steps": lat["steps"]}

    def release(self, lat):
        self.live.discard(id(lat))
        self.used -= lat["case"]["bytes"]


def _req(rid, arrival, nx, steps, nbytes):
    return Request(rid, arrival, {"nx": nx, "ny": 1, "nz": 1, "bytes": nbytes}, steps)


def test_budget_fifo_and_exact_step_counts():
    clock = SimClock()
    be = SimBackend(clock)
    rng = np.random.default_rng(3)
    reqs = [_req(k, float(0.01 * k), int(rng.integers(10, 500)), int(rng.integers(1, 300)),
                 int(rng.integers(1, 5)) * 100) for k in range(60)]
    srv = Server(be, budget_bytes=1000, max_slots=5, round_s=0.01, rate_guess=1e6,
                 clock=clock, sleep=clock.sleep)
    out = srv.run(reqs)
    assert be.peak_bytes <= 1000 and be.peak_slots <= 5
    assert be.used == 0 and not be.live
    for r in out:
        assert r.result["steps"] == r.steps                  # every request got exactly its budget
        assert r.arrival <= r.admitted <= r.done
    # first come first served: admission times follow arrival order
    adm = [r.admitted for r in sorted(out, key=lambda r: (r.arrival, r.rid))]
    assert all(a <= b for a, b in zip(adm, adm[1:]))
    assert srv.updates == sum(r.nodes * r.steps for r in out)


def test_batching_mixes_requests():
    clock = SimClock()
    be = SimBackend(clock)
    reqs = [_req(k, 0.0, 100, 50 + 10 * k, 10) for k in range(8)]
    srv = Server(be, budget_bytes=1e9, max_slots=64, round_s=0.001, rate_guess=1e6,
                 clock=clock, sleep=clock.sleep)
    srv.run(reqs)
    assert max(be.rounds) == 8            # all eight resident together
    assert len(be.rounds) > 8             # advanced in several rounds (chunks)


def test_idle_server_waits_for_arrivals():
    clock = SimClock()
    be = SimBackend(clock, rate=1e9)
    reqs = [_req(0, 5.0, 10, 3, 1), _req(1, 9.0, 10, 3, 1)]
    out = Server(be, clock=clock, sleep=clock.sleep).run(reqs)
    assert out[0].admitted >= 5.0 and out[1].admitted >= 9.0


def test_oversized_request_is_rejected():
    clock = SimClock()
    with pytest.raises(ValueError):
        Server(SimBackend(clock), budget_bytes=100, clock=clock, sleep=clock.sleep).run(
            [_req(0, 0.0, 10, 1, 101)])


def test_percentile_nearest_rank():
    v = list(range(1, 101))
    assert percentile(v, 50) == 50 and percentile(v, 99) == 99 and percentile(v, 100) == 100
    assert percentile([7.0], 99) == 7.0 and percentile([], 50) is None
    s = summarize([Request(0, 0.0, {}, 10, nodes=5, done=2.0)], 4.0)
    assert s["updates"] == 50 and s["p50_s"] == 2.0


@pytest.mark.gpu
def test_served_results_identical_to_alone(mech9):
    """Requests of different kinds and sizes served together (admitted at
    different times, stepped in chunks of varying length, weakly coupled ones
    in a batch of their own, one with the linearly implicit update) end
    bit-identical to the same requests stepped alone."""
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2108_07605_amd import rlbm, workloads as wl
    from paper_2108_07605_amd.serving import GpuBackend
    print("case serving mix of 8 requests, f32dev", flush=True)
    cases = [
        wl.make_case("reactor", seed=1, nx=6, ny=6, nz=6, mech=mech9, T0=1300.0),
        wl.make_case("tube", seed=2, nx=150, mech=mech9),
        wl.make_case("channel2d", seed=3, nx=40, ny=10, nz=1, mech=mech9),
        wl.make_case("tube", seed=4, nx=77, mech=mech9),
        wl.make_case("channel3d", seed=5, nx=16, ny=8, nz=6, mech=mech9),
        wl.make_case("reactor", seed=6, nx=4, ny=5, nz=3, mech=mech9, T0=1200.0),
        wl.make_case("tube", seed=7, nx=90, mech=mech9, coupling="weak"),
        wl.make_case("channel2d", seed=8, nx=24, ny=8, nz=1, mech=mech9, coupling="weak",
                     reaction="implicit"),
    ]
    steps = [23, 41, 17, 60, 9, 33, 29, 14]
    reqs = [Request(k, 0.002 * k, c, s) for k, (c, s) in enumerate(zip(cases, steps))]
    be = GpuBackend(mech9, storage="f32dev", keep="populations")
    srv = Server(be, budget_bytes=1e10, max_slots=4, round_s=1e-4, rate_guess=1e8, min_chunk=3,
                 max_chunk=7)
    out = srv.run(reqs)
    mech = rlbm.Mechanism(mech9)
    for r in out:
        alone = rlbm.Lattice(r.case, storage="f32dev", mech=mech).set_state()
        alone.step(r.steps)
        assert np.array_equal(alone.populations(), r.result["populations"]), r.rid


class FailingBackend(SimBackend):
    """A lattice whose case names `fail_after` reports a failure flag in the
    first round that takes it past that many steps; a case with `bad` cannot
    be created."""

    def create(self, case):
        if case.get("bad"):
            raise RuntimeError("invalid request")
        return super().create(case)

    def step(self, lats, steps):
        super().step(lats, steps)
        return [1 if lat["case"].get("fail_after") is not None and lat["steps"] > lat["case"]["fail_after"]
                else 0 for lat in lats]


def test_failed_request_is_quarantined():
    """A request whose lattice is flagged is retired at once with an error and
    its memory released; one that cannot be created fails at admission; every
    other request is served its full budget."""
    clock = SimClock()
    be = FailingBackend(clock)
    reqs = [_req(k, 0.001 * k, 100 + 10 * k, 40, 10) for k in range(6)]
    reqs[2].case["fail_after"] = 5
    reqs[4].case["bad"] = True
    srv = Server(be, budget_bytes=1e9, max_slots=8, round_s=1e-4, rate_guess=1e6, min_chunk=2,
                 max_chunk=4, clock=clock, sleep=clock.sleep)
    out = {r.rid: r for r in srv.run(reqs)}
    assert out[2].failed and "failure flag" in out[2].error and out[2].result is None
    assert out[4].failed and out[4].error.startswith("create") and out[4].admitted is None
    for k in (0, 1, 3, 5):
        assert not out[k].failed and out[k].result["steps"] == 40
    # retired early, after the round that flagged it, and nothing left behind
    assert out[2].done < min(out[k].done for k in (0, 1, 3, 5))
    assert be.used == 0 and not be.live
    summ = summarize(list(out.values()), 1.0)
    assert summ["failed"] == 2 and summ["updates"] == sum(out[k].nodes * 40 for k in (0, 1, 3, 5))


def test_equal_work_share_lets_small_requests_finish_first():
    """A small request arriving with a large one finishes after a few rounds,
    not after as many rounds as the large one needs."""
    clock = SimClock()
    be = SimBackend(clock)
    reqs = [_req(0, 0.0, 100000, 200, 10), _req(1, 0.0, 100, 200, 10)]
    srv = Server(be, round_s=0.01, rate_guess=1e6, clock=clock, sleep=clock.sleep)
    out = {r.rid: r for r in srv.run(reqs)}
    assert out[1].done < 0.05 * out[0].done
    assert out[0].result["steps"] == 200 and out[1].result["steps"] == 200


def _poison(lat):
    """An impossible state: every energy population NaN.  The kernels'
    bounded temperature iteration gives up and flags the lattice; every
    kernel still finishes."""
    pops = lat.populations()
    pops[-1] = np.nan
    lat.write_populations(pops)
    return lat


@pytest.mark.gpu
def test_flagged_lattice_is_isolated_in_a_batch(mech9):
    """One lattice of a batch holds a non-physical state: the batch reports
    its flag and no other, and the other lattices end bit-identical to
    stepping them alone."""
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2108_07605_amd import rlbm, workloads as wl
    print("case batch with one poisoned lattice, f32dev", flush=True)
    cases = [wl.make_case("tube", seed=11, nx=100, mech=mech9),
             wl.make_case("channel2d", seed=12, nx=32, ny=8, nz=1, mech=mech9),
             wl.make_case("reactor", seed=13, nx=4, ny=4, nz=4, mech=mech9, T0=1300.0)]
    m = rlbm.Mechanism(mech9)
    lats = [rlbm.Lattice(c, storage="f32dev", mech=m).set_state() for c in cases]
    _poison(lats[1])
    b = rlbm.Batch(lats)
    b.step([20, 20, 20])
    assert b.status() == [0, 1, 0]
    assert b.status() == [0, 0, 0]           # read and cleared
    for k in (0, 2):
        alone = rlbm.Lattice(cases[k], storage="f32dev", mech=m).set_state()
        alone.step(20)
        assert alone.status() == 0
        assert np.array_equal(alone.populations(), lats[k].populations()), k
    with pytest.raises(rlbm.RlbmError):
        lats[1].fields()                     # read-out reports the state too


@pytest.mark.gpu
def test_server_quarantines_a_failed_request(mech9):
    """A served request whose state turns non-physical is retired with an
    error while the requests served beside it finish bit-identical to
    running alone."""
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2108_07605_amd import rlbm, workloads as wl
    from paper_2108_07605_amd.serving import GpuBackend

    class PoisonBackend(GpuBackend):
        def create(self, case):
            lat = super().create(case)
            return _poison(lat) if case.get("poison") else lat

    print("case serving mix with one poisoned request, f32dev", flush=True)
    cases = [wl.make_case("tube", seed=21, nx=120, mech=mech9),
             wl.make_case("channel2d", seed=22, nx=32, ny=8, nz=1, mech=mech9),
             wl.make_case("reactor", seed=23, nx=4, ny=4, nz=4, mech=mech9, T0=1250.0),
             wl.make_case("tube", seed=24, nx=80, mech=mech9)]
    cases[1]["poison"] = True
    steps = [30, 40, 25, 35]
    reqs = [Request(k, 0.0, c, s) for k, (c, s) in enumerate(zip(cases, steps))]
    be = PoisonBackend(mech9, storage="f32dev", keep="populations")
    srv = Server(be, budget_bytes=1e10, max_slots=8, round_s=1e-4, rate_guess=1e8, min_chunk=4,
                 max_chunk=9)
    out = {r.rid: r for r in srv.run(reqs)}
    assert out[1].failed and "failure flag" in out[1].error
    mech = rlbm.Mechanism(mech9)
    for k in (0, 2, 3):
        r = out[k]
        assert not r.failed, r.error
        alone = rlbm.Lattice(r.case, storage="f32dev", mech=mech).set_state()
        alone.step(r.steps)
        assert np.array_equal(alone.populations(), r.result["populations"]), k


@pytest.mark.gpu
def test_served_requests_match_the_oracle(mech9):
    """One small request of each served kind (reactor, flame tube, 2D and 3D
    channels) through the server in FP32 deviation storage: the fields read
    back match the FP64 oracle to 1e-5 in mass fractions and temperature."""
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from oracle import Oracle
    from paper_2108_07605_amd import workloads as wl
    from paper_2108_07605_amd.serving import GpuBackend
    print("case served reactor/tube/channel2d/channel3d vs oracle, f32dev", flush=True)
    cases = [wl.make_case("reactor", seed=51, nx=4, ny=4, nz=4, mech=mech9, T0=1350.0),
             wl.make_case("tube", seed=52, nx=96, mech=mech9),
             wl.make_case("channel2d", seed=53, nx=48, ny=12, nz=1, mech=mech9),
             wl.make_case("channel3d", seed=54, nx=20, ny=8, nz=6, mech=mech9)]
    steps = [40, 45, 30, 20]
    reqs = [Request(k, 0.001 * k, c, s) for k, (c, s) in enumerate(zip(cases, steps))]
    be = GpuBackend(mech9, storage="f32dev", keep="fields")
    srv = Server(be, budget_bytes=1e10, max_slots=8, round_s=1e-4, rate_guess=1e8, min_chunk=5,
                 max_chunk=12)
    out = {r.rid: r for r in srv.run(reqs)}
    for k, (c, n) in enumerate(zip(cases, steps)):
        r = out[k]
        assert not r.failed, r.error
        o = Oracle(c)
        o.step(n)
        of, gf = o.fields(), r.result
        eT = float(np.abs(gf["T"] - of["T"]).max() / np.abs(of["T"]).max())
        eY = max(float(np.abs(gf["Y"][a] - of["Y"][a]).max() / max(np.abs(of["Y"][a]).max(), 1e-6))
                 for a in range(of["Y"].shape[0]))
        print(f"served {c['name']} vs oracle after {n} steps: Y {eY:.2e} T {eT:.2e}", flush=True)
        assert eY <= 1e-5 and eT <= 1e-5, (k, eY, eT)
