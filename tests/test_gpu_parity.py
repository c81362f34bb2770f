"""HIP path versus the FP64 CPU oracle, element by element, through the C ABI.

Tolerances: FP64 storage agrees with the oracle to 1e-10 in the field-normalised
max norm (the two sides differ only in rounding order: LU with pivoting vs
Gaussian elimination, collapsed vs per-species polynomials, exp/log ulps);
FP32 deviation storage agrees to 1e-5 in mass fractions and temperature.
"""
import math

import numpy as np
import pytest

from oracle import Oracle
from paper_2108_07605_amd import workloads as wl

pytestmark = pytest.mark.gpu

TOL64 = 1e-10
TOL32 = 1e-5


def _gpu():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2108_07605_amd import rlbm
    return rlbm


def _nerr(a, b, floor=0.0):
    return float(np.abs(a - b).max() / max(np.abs(b).max(), floor, 1e-300))


def _compare_pops(gpu_pops, ora_pops, tol):
    worst = 0.0
    for l in range(ora_pops.shape[0]):
        e = _nerr(gpu_pops[l], ora_pops[l])
        worst = max(worst, e)
        assert e <= tol, (l, e)
    return worst


def _compare_fields(gf, of, tol, u_floor):
    assert _nerr(gf["rho"], of["rho"]) <= tol
    assert _nerr(gf["T"], of["T"]) <= tol
    for a in range(of["Y"].shape[0]):
        assert _nerr(gf["Y"][a], of["Y"][a], 1e-12) <= tol, a
    assert _nerr(gf["u"], of["u"], u_floor) <= tol


def _u_floor(case):
    fl = case["init"]
    th = float(np.median(fl["T"])) * case["mech"]["R_univ"] / 20.0
    return 1e-3 * math.sqrt(th)


def _run_pair(case, steps_list, storage="f64"):
    rlbm = _gpu()
    lat = rlbm.Lattice(case, storage=storage)
    lat.set_state()
    ora = Oracle(case)
    done = 0
    out = []
    for n in steps_list:
        lat.step(n - done)
        ora.step(n - done)
        done = n
        out.append((lat.populations(), ora.populations(), lat.fields(), ora.fields()))
    return lat, ora, out


@pytest.mark.parametrize("storage", ["f64"])
def test_abc_box_parity(storage):
    print("case abc_box 32x8x8 M=3 f64", flush=True)
    case = wl.make_case("abc_box")
    lat, ora, out = _run_pair(case, [1, 10, 200])
    for gp, op, gf, of in out:
        _compare_pops(gp, op, TOL64)
        _compare_fields(gf, of, TOL64, _u_floor(case))


@pytest.mark.parametrize("storage", ["f64", "f32dev"])
@pytest.mark.parametrize("wall_type", ["wall", "bounceback"])
@pytest.mark.parametrize("coupling", ["strong", "weak"])
def test_closed_box_corners_parity(coupling, wall_type, storage):
    """A box closed by walls on all six faces (edges on two walls, corners
    on three, with 15 and 19 incoming links), TMS or bounce-back, with a
    slaved species or the weakly coupled storage, against the oracle."""
    print(f"case closed box 10x8x6 M=3 {coupling} {wall_type} {storage}", flush=True)
    case = wl.make_case("abc_box", nx=10, ny=8, nz=6, mech=wl.mechanism_abc(), coupling=coupling)
    if wall_type == "wall":
        face = {"type": "wall", "T_lo": 1000.0, "T_hi": 1000.0, "x0": 0.0, "width": 1.0}
    else:
        face = {"type": "bounceback"}
    case["faces"] = [dict(face) for _ in range(6)]
    lat, ora, out = _run_pair(case, [1, 20], storage=storage)
    for gp, op, gf, of in out:
        if storage == "f64":
            _compare_pops(gp, op, TOL64)
            _compare_fields(gf, of, TOL64, _u_floor(case))
        else:
            assert _nerr(gf["T"], of["T"]) <= TOL32
            assert max(_nerr(gf["Y"][a], of["Y"][a], 1e-6) for a in range(3)) <= TOL32


@pytest.mark.parametrize("storage", ["f64", "f32dev"])
@pytest.mark.parametrize("wall_type", ["wall", "bounceback"])
@pytest.mark.parametrize("species", [2, 4])
def test_closed_box_other_species_counts(species, wall_type, storage):
    """The boundary kernels compiled for two and four species (their LDS
    holds every lattice in both storages) in boxes closed on all six faces,
    against the oracle."""
    print(f"case closed box 10x8x6 M={species} {wall_type} {storage}", flush=True)
    if species == 2:
        case = wl.make_case("binary", nx=10, ny=8, nz=6, amp=1e-2)
        T_w = 300.0
    else:
        case = wl.make_case("abc_box", nx=10, ny=8, nz=6, mech=wl.mechanism_abcd())
        T_w = 1000.0
    if wall_type == "wall":
        face = {"type": "wall", "T_lo": T_w, "T_hi": T_w, "x0": 0.0, "width": 1.0}
    else:
        face = {"type": "bounceback"}
    case["faces"] = [dict(face) for _ in range(6)]
    lat, ora, out = _run_pair(case, [1, 20], storage=storage)
    for gp, op, gf, of in out:
        if storage == "f64":
            _compare_pops(gp, op, TOL64)
            _compare_fields(gf, of, TOL64, _u_floor(case))
        else:
            assert _nerr(gf["T"], of["T"]) <= TOL32
            assert max(_nerr(gf["Y"][a], of["Y"][a], 1e-6) for a in range(species)) <= TOL32


@pytest.mark.parametrize("storage", ["f64", "f32dev"])
def test_bounce_back_channel_with_inlet_and_outlet_parity(mech9, storage):
    """A 2D channel whose y walls are bounce-back walls, with the flux inlet
    and the LODI outlet: the bounce-back kernel path beside inlet and outlet
    tiles, and the edge nodes where a bounce-back face meets the inlet and
    outlet faces (the wall is taken there)."""
    print(f"case channel2d 40x10 bounce-back walls {storage}", flush=True)
    case = wl.make_case("channel2d", nx=40, ny=10, nz=1, mech=mech9)
    for f in (2, 3):
        case["faces"][f] = {"type": "bounceback"}
    lat, ora, out = _run_pair(case, [1, 40], storage=storage)
    for gp, op, gf, of in out:
        if storage == "f64":
            _compare_pops(gp, op, TOL64)
            _compare_fields(gf, of, TOL64, _u_floor(case))
        else:
            assert _nerr(gf["T"], of["T"]) <= TOL32
            assert max(_nerr(gf["Y"][a], of["Y"][a], 1e-6) for a in range(of["Y"].shape[0])) <= TOL32


def test_abc_box_initial_state_exact():
    rlbm = _gpu()
    case = wl.make_case("abc_box")
    lat = rlbm.Lattice(case).set_state()
    ora = Oracle(case)
    _compare_pops(lat.populations(), ora.populations(), 1e-14)
    gf = lat.fields()
    np.testing.assert_allclose(gf["T"], case["init"]["T"], rtol=1e-13)


@pytest.mark.parametrize("name,kw,steps", [
    ("channel2d", dict(nx=48, ny=12, nz=1), [1, 30]),
    ("channel3d", dict(nx=20, ny=8, nz=6, perturb=0.5), [1, 12]),
    ("tube", dict(nx=96), [1, 60]),
    ("reactor", dict(nx=4, ny=4, nz=4, T0=1500.0), [1, 40]),
    ("bbbox", dict(nx=12, ny=8, nz=6), [1, 30]),
    ("channel2d", dict(nx=48, ny=12, nz=1, inlet="inlet_local"), [1, 30]),
    ("channel2d", dict(nx=40, ny=10, nz=1, substeps=4), [1, 20]),
    ("channel2d", dict(nx=48, ny=12, nz=1, reaction="implicit"), [1, 30]),
    ("reactor", dict(nx=4, ny=4, nz=4, T0=1500.0, X_radical=0.01, reaction="implicit", substeps=1), [1, 40]),
    ("channel2d", dict(nx=48, ny=12, nz=1, coupling="weak"), [1, 30]),
    ("channel3d", dict(nx=20, ny=8, nz=6, perturb=0.5, coupling="weak"), [1, 12]),
    ("bbbox", dict(nx=12, ny=8, nz=6, coupling="weak"), [1, 30]),
    ("tube", dict(nx=96, coupling="weak"), [1, 60]),
    ("reactor", dict(nx=3, ny=3, nz=2, T0=1500.0, X_radical=0.01, reaction="implicit", coupling="weak"), [1, 30]),
    ("channel2d", dict(nx=40, ny=10, nz=1, inlet="inlet_local", coupling="weak", substeps=3), [1, 20]),
    ("channel3d", dict(nx=256, ny=4, nz=3, perturb=0.5), [1, 6]),    # full 256-node blocks
    # rows of 80 nodes: some 64-node tiles lie in one row, others span two
    ("channel3d", dict(nx=80, ny=5, nz=4, perturb=0.5), [1, 10]),
    ("channel3d", dict(nx=80, ny=5, nz=4, perturb=0.5, coupling="weak"), [1, 10]),
])
def test_nine_species_parity(mech9, name, kw, steps):
    print(f"case {name} {kw} M=9 f64", flush=True)
    case = wl.make_case(name, mech=mech9, **kw)
    lat, ora, out = _run_pair(case, steps)
    for gp, op, gf, of in out:
        _compare_pops(gp, op, TOL64)
        _compare_fields(gf, of, TOL64, _u_floor(case))


@pytest.mark.parametrize("l", [1, 3])
def test_stiff_reactor_linearly_implicit(mech9, l):
    """Rates x1e4 (one forward-Euler sub-step overshoots to negative mass
    fractions here): the linearly implicit update with partial pivoting
    matches the oracle in a perturbed radical-seeded box, so every node
    differs, while the mixture burns."""
    mech = wl.scaled_rates(mech9, 1e4)
    case = wl.make_case("reactor", nx=6, ny=4, nz=3, mech=mech, T0=1500.0, X_radical=0.01,
                        reaction="implicit", substeps=l)
    rng = np.random.default_rng(70 + l)
    case["init"]["T"] = case["init"]["T"] * (1.0 + 0.02 * rng.standard_normal(case["N"]))
    case["init"]["u"] = 0.01 * rng.standard_normal((3, case["N"]))
    print(f"case stiff reactor 6x4x3 x1e4 implicit l={l} f64", flush=True)
    lat, ora, out = _run_pair(case, [1, 5, 20])
    for gp, op, gf, of in out:
        _compare_pops(gp, op, TOL64)
        _compare_fields(gf, of, TOL64, _u_floor(case))
    assert out[-1][3]["T"].min() > 1800.0


def test_weak_coupling_three_species_parity():
    """Weakly coupled storage (all M species lattices, L = M + 2) with three
    species in a perturbed periodic box, against the oracle, and its
    separately conserved densities."""
    rlbm = _gpu()
    print("case abc_box 32x8x8 M=3 weak f64", flush=True)
    case = wl.make_case("abc_box", coupling="weak")
    lat, ora, out = _run_pair(case, [1, 10, 100])
    assert lat.L == 5 and lat.slaved == rlbm.SLAVED_NONE
    for gp, op, gf, of in out:
        _compare_pops(gp, op, TOL64)
        _compare_fields(gf, of, TOL64, _u_floor(case))
    gi, oi = lat.invariants(), ora.invariants()
    np.testing.assert_allclose(gi[[0, 4, 5, 6]], oi[[0, 4, 5, 6]], rtol=1e-13)
    pops = lat.populations()
    rho_sp = pops[:3].sum(axis=1)
    rho = pops[3].sum(axis=0)
    assert np.abs(rho_sp.sum(axis=0) - rho).max() > 1e-8 * rho.max()      # the densities drift apart
    assert abs(rho_sp.sum() - ora.fa.sum()) <= 1e-13 * ora.fa.sum()


def test_bounce_back_box_conservation():
    """A duct closed by bounce-back walls (eq. bb) keeps its mass, energy and
    element totals on the GPU in both storage formats while it reacts."""
    rlbm = _gpu()
    case = wl.make_case("bbbox", nx=24, ny=10, nz=8)
    E = len(case["mech"]["elements"])
    for storage, tol in (("f64", 1e-12), ("f32dev", 1e-7)):
        print(f"case bbbox 24x10x8 {storage} 200 steps", flush=True)
        lat = rlbm.Lattice(case, storage=storage).set_state()
        inv0 = lat.invariants()
        lat.step(200)
        inv1 = lat.invariants()
        assert inv1[-1] == 0.0
        for k in [0, 4] + list(range(5, 5 + E)):
            assert abs(inv1[k] - inv0[k]) <= tol * abs(inv0[k]), (storage, k)


@pytest.mark.parametrize("coupling", ["strong", "weak"])
def test_three_species_linearly_implicit(coupling):
    """The linearly implicit update with three species (a 2x2 reduced system)
    and rates x10 (the box burns from 1000 to 2060 K in 30 steps), with a
    slaved species and in the weakly coupled storage."""
    mech = wl.scaled_rates(wl.mechanism_abc(), 10.0)
    case = wl.make_case("abc_box", nx=12, ny=4, nz=4, mech=mech, reaction="implicit", substeps=1,
                        coupling=coupling)
    print(f"case abc_box 12x4x4 M=3 implicit x10 {coupling}", flush=True)
    lat, ora, out = _run_pair(case, [1, 30])
    for gp, op, gf, of in out:
        _compare_pops(gp, op, TOL64)
        _compare_fields(gf, of, TOL64, _u_floor(case))


def test_long_periodic_box_parity():
    """A periodic box 256 nodes long in x (every block one x row, the
    stencils wrapping at both ends of the row)."""
    print("case abc_box 256x2x2 M=3 f64", flush=True)
    case = wl.make_case("abc_box", nx=256, ny=2, nz=2)
    lat, ora, out = _run_pair(case, [1, 20])
    for gp, op, gf, of in out:
        _compare_pops(gp, op, TOL64)
        _compare_fields(gf, of, TOL64, _u_floor(case))


@pytest.mark.parametrize("coupling", ["strong", "weak"])
def test_binary_parity(coupling):
    print(f"case binary 64 M=2 f64 {coupling}", flush=True)
    case = wl.make_case("binary", nx=64, amp=1e-2, coupling=coupling)
    lat, ora, out = _run_pair(case, [1, 100])
    for gp, op, gf, of in out:
        _compare_pops(gp, op, TOL64)
        _compare_fields(gf, of, TOL64, _u_floor(case))


def test_tiny_and_degenerate_boxes():
    """2x2x2 and 1x1x1 periodic boxes (every neighbour is the node itself or
    its image) and a 3x1x1 line."""
    for nx, ny, nz, coupling in ((2, 2, 2, "strong"), (1, 1, 1, "strong"), (3, 1, 1, "strong"),
                                 (1, 1, 1, "weak"), (3, 1, 1, "weak")):
        print(f"case abc_box {nx}x{ny}x{nz} {coupling}", flush=True)
        case = wl.make_case("abc_box", nx=nx, ny=ny, nz=nz, coupling=coupling)
        lat, ora, out = _run_pair(case, [5])
        for gp, op, gf, of in out:
            _compare_pops(gp, op, TOL64)


def test_f32_deviation_storage_vs_oracle():
    print("case abc_box f32dev", flush=True)
    case = wl.make_case("abc_box")
    lat, ora, out = _run_pair(case, [200], storage="f32dev")
    gp, op, gf, of = out[-1]
    ey = [_nerr(gf["Y"][a], of["Y"][a]) for a in range(of["Y"].shape[0])]
    et = _nerr(gf["T"], of["T"])
    print(f"f32dev vs oracle, abc_box 200 steps: Y {max(ey):.3e} T {et:.3e}", flush=True)
    assert max(ey) <= TOL32 and et <= TOL32


@pytest.mark.parametrize("name,kw,steps", [
    ("channel2d", dict(nx=48, ny=12, nz=1), 30),
    # rows of 80 nodes: 64-node tiles inside one row and tiles across two
    ("channel3d", dict(nx=80, ny=5, nz=4, perturb=0.5), 10),
])
def test_f32_deviation_channel_vs_oracle(mech9, name, kw, steps):
    print(f"case {name} {kw} f32dev", flush=True)
    case = wl.make_case(name, mech=mech9, **kw)
    lat, ora, out = _run_pair(case, [steps], storage="f32dev")
    gp, op, gf, of = out[-1]
    ey = [_nerr(gf["Y"][a], of["Y"][a], 1e-6) for a in range(of["Y"].shape[0])]
    et = _nerr(gf["T"], of["T"])
    print(f"f32dev vs oracle, {name} {steps} steps: Y {max(ey):.3e} T {et:.3e}", flush=True)
    assert max(ey) <= TOL32 and et <= TOL32


def test_f32_deviation_weak_coupling_vs_oracle(mech9):
    print("case channel2d 48x12 f32dev weak", flush=True)
    case = wl.make_case("channel2d", nx=48, ny=12, nz=1, mech=mech9, coupling="weak")
    lat, ora, out = _run_pair(case, [30], storage="f32dev")
    gp, op, gf, of = out[-1]
    ey = [_nerr(gf["Y"][a], of["Y"][a], 1e-6) for a in range(of["Y"].shape[0])]
    et = _nerr(gf["T"], of["T"])
    print(f"f32dev weak vs oracle, channel2d 48x12 30 steps: Y {max(ey):.3e} T {et:.3e}", flush=True)
    assert max(ey) <= TOL32 and et <= TOL32


def test_f32_deviation_long_run_vs_f64(mech9):
    """FP32 deviation storage against FP64 storage on the GPU over 1000 steps
    of a walled channel with inlet and outlet: mass fractions (each species
    normalised by its own maximum) and temperature within 1e-5."""
    rlbm = _gpu()
    print("case channel2d 256x32 1000 steps f32dev vs f64", flush=True)
    case = wl.make_case("channel2d", nx=256, ny=32, nz=1, mech=mech9)
    a = rlbm.Lattice(case, storage="f64").set_state()
    b = rlbm.Lattice(case, storage="f32dev").set_state()
    a.step(1000)
    b.step(1000)
    fa, fb = a.fields(), b.fields()
    ey = [_nerr(fb["Y"][k], fa["Y"][k]) for k in range(fa["Y"].shape[0])]
    et = _nerr(fb["T"], fa["T"])
    print(f"f32dev vs f64, 1000 steps: Y {max(ey):.3e} T {et:.3e}", flush=True)
    assert max(ey) <= TOL32 and et <= TOL32


def test_invariants_match_oracle():
    rlbm = _gpu()
    case = wl.make_case("abc_box")
    lat = rlbm.Lattice(case).set_state()
    ora = Oracle(case)
    lat.step(20)
    ora.step(20)
    gi, oi = lat.invariants(), ora.invariants()
    np.testing.assert_allclose(gi[[0, 4, 5, 6]], oi[[0, 4, 5, 6]], rtol=1e-13)
    assert np.abs(gi[1:4]).max() < 1e-11
    assert gi[-1] == 0.0


@pytest.mark.parametrize("storage,coupling", [("f64", "strong"), ("f32dev", "strong"), ("f32dev", "weak")])
def test_populations_round_trip(storage, coupling, mech9):
    """FP64 populations read out and written straight back are unchanged
    (the FP32 encoding against the same references is idempotent)."""
    rlbm = _gpu()
    case = wl.make_case("channel2d", nx=32, ny=8, nz=1, mech=mech9, coupling=coupling)
    lat = rlbm.Lattice(case, storage=storage).set_state()
    lat.step(5)
    saved = lat.populations()
    lat.write_populations(saved)
    assert np.array_equal(lat.populations(), saved)
    lat.step(3)
    p3 = lat.populations()
    lat.write_populations(p3)
    assert np.array_equal(lat.populations(), p3)


@pytest.mark.parametrize("storage,coupling", [("f64", "strong"), ("f32dev", "strong"), ("f32dev", "weak")])
def test_state_snapshot_resume(storage, coupling, mech9):
    """Checkpoint/resume: a raw snapshot taken after 5 steps, loaded back into
    the same lattice after 7 more steps or into a fresh lattice, continues
    bit-identically."""
    rlbm = _gpu()
    case = wl.make_case("channel2d", nx=32, ny=8, nz=1, mech=mech9, coupling=coupling)
    lat = rlbm.Lattice(case, storage=storage).set_state()
    lat.step(5)
    snap = lat.save_state()
    lat.step(7)
    a = lat.populations()
    fa = lat.fields()
    lat.load_state(snap)
    lat.step(7)
    assert np.array_equal(lat.populations(), a)
    lat2 = rlbm.Lattice(case, storage=storage).load_state(snap)
    lat2.step(7)
    assert np.array_equal(lat2.populations(), a)
    f2 = lat2.fields()
    for key in ("rho", "T", "Y", "u"):
        assert np.array_equal(f2[key], fa[key]), key
    other = rlbm.Lattice(wl.make_case("channel2d", nx=16, ny=8, nz=1, mech=mech9), storage=storage)
    with pytest.raises(rlbm.RlbmError):
        other.load_state(snap)
    flip = "strong" if coupling == "weak" else "weak"
    other = rlbm.Lattice(wl.make_case("channel2d", nx=32, ny=8, nz=1, mech=mech9, coupling=flip), storage=storage)
    with pytest.raises(rlbm.RlbmError):
        other.load_state(snap)


def test_determinism(mech9):
    rlbm = _gpu()
    case = wl.make_case("channel3d", nx=24, ny=8, nz=8, mech=mech9)
    p = []
    for _ in range(2):
        lat = rlbm.Lattice(case).set_state()
        lat.step(10)
        p.append(lat.populations())
    assert np.array_equal(p[0], p[1])


def test_batch_equals_alone(mech9):
    """Uneven lattices in one batched launch give bit-identical results to
    stepping each alone, including different step counts and a lattice with
    the linearly implicit reaction update among explicit ones."""
    rlbm = _gpu()
    cases = [wl.make_case("tube", seed=s, nx=n, mech=mech9, reaction=r)
             for s, n, r in ((1, 64, "explicit"), (2, 300, "implicit"), (3, 129, "explicit"))]
    steps = [20, 7, 13]
    alone = []
    for c, n in zip(cases, steps):
        lat = rlbm.Lattice(c).set_state()
        lat.step(n)
        alone.append(lat.populations())
    lats = [rlbm.Lattice(c).set_state() for c in cases]
    b = rlbm.Batch(lats)
    b.step([s - 3 for s in steps])
    b.step([3, 3, 3])
    for lat, ref in zip(lats, alone):
        assert np.array_equal(lat.populations(), ref)


def test_batch_matches_oracle(mech9):
    """Three uneven lattices in one batch (a flame tube with inlet and outlet,
    a walled 2D channel on the linearly implicit update, a periodic reactor),
    stepped by two batch calls with different counts per lattice (whole
    16-step chunks replay the captured graph, the rest are direct launches):
    each against its own oracle, FP64 storage."""
    rlbm = _gpu()
    cases = [wl.make_case("tube", seed=31, nx=96, mech=mech9),
             wl.make_case("channel2d", seed=32, nx=40, ny=10, nz=1, mech=mech9, reaction="implicit"),
             wl.make_case("reactor", seed=33, nx=4, ny=4, nz=4, mech=mech9, T0=1400.0)]
    print("case batch tube 96 + channel2d 40x10 implicit + reactor 4^3 vs oracle, f64", flush=True)
    m = rlbm.Mechanism(mech9)
    lats = [rlbm.Lattice(c, storage="f64", mech=m).set_state() for c in cases]
    oras = [Oracle(c) for c in cases]
    b = rlbm.Batch(lats)
    for call in ([30, 17, 20], [7, 21, 3]):
        b.step(call)
        for o, n in zip(oras, call):
            o.step(n)
        assert b.status() == [0, 0, 0]
        for lat, o, c in zip(lats, oras, cases):
            _compare_pops(lat.populations(), o.populations(), TOL64)
            _compare_fields(lat.fields(), o.fields(), TOL64, _u_floor(c))


def test_batch_graph_replays_match_direct_launches(mech9):
    """Four calls of 16 steps each (one replay of the captured chunk per
    call), with reads and synchronisations between them: after every call
    the batch equals the same lattices stepped by direct launches, bit for
    bit."""
    rlbm = _gpu()
    print("case batch graph replays vs direct launches, f32dev", flush=True)
    cases = [wl.make_case("tube", seed=41, nx=70, mech=mech9),
             wl.make_case("channel2d", seed=42, nx=24, ny=8, nz=1, mech=mech9)]
    m = rlbm.Mechanism(mech9)
    lats = [rlbm.Lattice(c, storage="f32dev", mech=m).set_state() for c in cases]
    alone = [rlbm.Lattice(c, storage="f32dev", mech=m).set_state() for c in cases]
    b = rlbm.Batch(lats)
    for _ in range(4):
        b.step([16, 16])
        for a in alone:
            a.step(16)
        for lat, a in zip(lats, alone):
            assert np.array_equal(lat.populations(), a.populations())


def test_long_walled_channel_vs_oracle(mech9):
    """A 64x16x1 channel with TMS walls, flux inlet and LODI outlet over 300
    steps (the outlet state and the wall temperature ramp act all the
    while), FP64 storage, every node against the oracle."""
    rlbm = _gpu()
    print("case channel2d 64x16 300 steps f64", flush=True)
    case = wl.make_case("channel2d", nx=64, ny=16, nz=1, mech=mech9)
    lat, ora, out = _run_pair(case, [100, 300])
    for gp, op, gf, of in out:
        _compare_pops(gp, op, TOL64)
        _compare_fields(gf, of, TOL64, _u_floor(case))


@pytest.mark.parametrize("storage", ["f64", "f32dev"])
def test_unit_prandtl_number_parity(mech9, storage):
    """Pr = 1 (omega_1 = omega): the energy update's singularity-free form
    on the GPU against the oracle on a walled channel."""
    print(f"case channel2d 48x12 Pr=1 {storage}", flush=True)
    case = wl.make_case("channel2d", nx=48, ny=12, nz=1, mech=wl.with_prandtl(mech9, 1.0))
    lat, ora, out = _run_pair(case, [1, 30], storage=storage)
    for gp, op, gf, of in out:
        if storage == "f64":
            _compare_pops(gp, op, TOL64)
            _compare_fields(gf, of, TOL64, _u_floor(case))
    gf, of = out[-1][2], out[-1][3]
    assert _nerr(gf["T"], of["T"]) <= (TOL64 if storage == "f64" else TOL32)
    assert max(_nerr(gf["Y"][a], of["Y"][a], 1e-6) for a in range(of["Y"].shape[0])) <= TOL32


@pytest.mark.parametrize("storage", ["f64", "f32dev"])
def test_four_species_parity(storage):
    """The four-species kernels (three reacting species and an inert one) in
    the perturbed periodic box against the oracle."""
    print(f"case abc_box 32x8x8 M=4 {storage}", flush=True)
    case = wl.make_case("abc_box", mech=wl.mechanism_abcd())
    lat, ora, out = _run_pair(case, [1, 10, 100], storage=storage)
    for gp, op, gf, of in out:
        if storage == "f64":
            _compare_pops(gp, op, TOL64)
            _compare_fields(gf, of, TOL64, _u_floor(case))
        else:
            assert _nerr(gf["T"], of["T"]) <= TOL32
            assert max(_nerr(gf["Y"][a], of["Y"][a], 1e-6) for a in range(4)) <= TOL32


def _window(pops, case, cx, cy, cz, h=2):
    nx, ny, nz = case["nx"], case["ny"], case["nz"]
    xs = [(cx + d) % nx for d in range(-h, h + 1)]
    ys = [(cy + d) % ny for d in range(-h, h + 1)]
    zs = [(cz + d) % nz for d in range(-h, h + 1)]
    idx = np.array([(z * ny + y) * nx + x for z in zs for y in ys for x in xs])
    return idx


def test_full_size_channel2d_vs_oracle(mech9):
    """The 1024x64x1 channel at its full size, every node (TMS walls, flux
    inlet and LODI outlet included): FP64 storage against the oracle element
    by element after 1 and 3 steps, and FP32 deviation storage within its
    tolerance after 3."""
    rlbm = _gpu()
    print("case channel2d 1024x64x1 f64 + f32dev, all nodes", flush=True)
    case = wl.make_case("channel2d", mech=mech9)
    assert (case["nx"], case["ny"], case["nz"]) == (1024, 64, 1)
    lat64 = rlbm.Lattice(case, storage="f64").set_state()
    lat32 = rlbm.Lattice(case, storage="f32dev").set_state()
    ora = Oracle(case)
    done = 0
    for n in (1, 3):
        lat64.step(n - done)
        lat32.step(n - done)
        ora.step(n - done)
        done = n
        of = ora.fields()
        _compare_pops(lat64.populations(), ora.populations(), TOL64)
        _compare_fields(lat64.fields(), of, TOL64, _u_floor(case))
    gf = lat32.fields()
    ey = [_nerr(gf["Y"][a], of["Y"][a], 1e-6) for a in range(of["Y"].shape[0])]
    et = _nerr(gf["T"], of["T"])
    print(f"f32dev vs oracle, channel2d 1024x64 3 steps: Y {max(ey):.3e} T {et:.3e}", flush=True)
    assert max(ey) <= TOL32 and et <= TOL32


def test_full_size_channel3d_sampled(mech9):
    """512x64x64 channel in the benchmark's launch configuration: the
    post-step populations at sampled interior nodes equal the oracle's update
    of a 5x5x5 neighbourhood (which fixes that node's update exactly)."""
    rlbm = _gpu()
    import torch
    print("case channel3d 512x64x64 f64 sampled", flush=True)
    case = wl.make_case("channel3d", mech=mech9)
    lat = rlbm.Lattice(case).set_state()
    lat.step(3)
    L, N = lat.L, lat.N
    buf = torch.empty(L * 27 * N, dtype=torch.float64, device="cuda")
    rlbm._check(rlbm.lib().rlbm_read_populations(lat.handle, rlbm.c_void_p(buf.data_ptr()), 1))
    rng = np.random.default_rng(7)
    samples = [(int(rng.integers(3, 509)), int(rng.integers(3, 61)), int(rng.integers(3, 61)))
               for _ in range(6)]
    before = {}
    for s in samples:
        idx = torch.as_tensor(_window(None, case, *s), device="cuda")
        before[s] = buf.view(L, 27, N)[:, :, idx].cpu().numpy()
    lat.step(1)
    rlbm._check(rlbm.lib().rlbm_read_populations(lat.handle, rlbm.c_void_p(buf.data_ptr()), 1))
    after = buf.view(L, 27, N)
    for s in samples:
        node = (s[2] * 64 + s[1]) * 512 + s[0]
        got = after[:, :, node].cpu().numpy()
        win = wl.make_case("reactor", nx=5, ny=5, nz=5, mech=mech9, T0=300.0)
        win["slaved"] = case["slaved"]
        ora = Oracle(win)
        ora.set_populations(before[s])
        ora.T[:] = 300.0
        ora.step(1)
        exp = ora.populations()[:, :, 62]
        for l in range(L):
            err = np.abs(got[l] - exp[l]).max() / np.abs(exp[l]).max()
            assert err <= TOL64, (s, l, err)
