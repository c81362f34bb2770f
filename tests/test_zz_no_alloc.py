"""The allocation-free group step (rlbm_step_group) against the batch step
(rlbm_batch_step) on the same lattices, through the C ABI."""
import ctypes

import numpy as np
import pytest

from paper_2108_07605_amd import workloads as wl

pytestmark = pytest.mark.gpu


def _gpu():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2108_07605_amd import rlbm
    return rlbm


def _cases(mech9, specs):
    return [wl.make_case(kind, seed=seed, mech=mech9, **kw) for kind, seed, kw in specs]


def test_group_step_equals_batch_step(mech9):
    """Two group calls in a row, the second over fewer and smaller lattices,
    each against a batch step of the same lattices from the same state: bit
    for bit (same kernels, tables in the library's own device array)."""
    rlbm = _gpu()
    m = rlbm.Mechanism(mech9)
    calls = [
        (_cases(mech9, [("tube", 61, dict(nx=130)),
                        ("channel2d", 62, dict(nx=40, ny=10, nz=1, reaction="implicit")),
                        ("reactor", 63, dict(nx=4, ny=4, nz=4, T0=1300.0)),
                        ("channel3d", 64, dict(nx=16, ny=8, nz=6))]), [23, 17, 9, 20]),
        (_cases(mech9, [("tube", 65, dict(nx=70)),
                        ("reactor", 66, dict(nx=3, ny=3, nz=2, T0=1250.0))]), [11, 5]),
    ]
    for storage in ("f32dev", "f64"):
        for cases, steps in calls:
            print(f"case group step vs batch step: {len(cases)} lattices, {storage}", flush=True)
            grp = [rlbm.Lattice(c, storage=storage, mech=m).set_state() for c in cases]
            ref = [rlbm.Lattice(c, storage=storage, mech=m).set_state() for c in cases]
            rlbm.step_group(grp, steps)
            b = rlbm.Batch(ref)
            b.step(steps)
            for g, r in zip(grp, ref):
                assert g.status() == 0 and r.status() == 0
                assert np.array_equal(g.populations(), r.populations())
            # and a second round on the same lattices
            rlbm.step_group(grp, [s // 2 + 1 for s in steps])
            b.step([s // 2 + 1 for s in steps])
            for g, r in zip(grp, ref):
                assert np.array_equal(g.populations(), r.populations())
                np.testing.assert_array_equal(g.fields()["T"], r.fields()["T"])


def test_group_step_rejects_too_many_and_mixed_streams(mech9):
    rlbm = _gpu()
    import torch
    m = rlbm.Mechanism(mech9)
    c = wl.make_case("reactor", seed=67, nx=2, ny=2, nz=2, mech=mech9, T0=1200.0)
    lat = rlbm.Lattice(c, mech=m).set_state()
    k = rlbm.GROUP_MAX_LATTICES + 1
    arr = (ctypes.c_void_p * k)(*([lat.handle.value] * k))
    st = (ctypes.c_int64 * k)(*([1] * k))
    rc = rlbm.lib().rlbm_step_group(arr, k, st)
    assert rc == -1 and b"RLBM_GROUP_MAX_LATTICES" in rlbm.lib().rlbm_last_error()
    other = rlbm.Lattice(c, mech=m, stream=torch.cuda.Stream()).set_state()
    with pytest.raises(rlbm.RlbmError):
        rlbm.step_group([lat, other], [1, 1])
    with pytest.raises(rlbm.RlbmError):
        rlbm.step_group([lat, lat], [1, 1])
