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
