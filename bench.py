"""Benchmark: MLUPS of the fused reactive-mixture LBM step on one MI355X.

A "step" is one time step of the whole hot path (advection, boundaries,
moments, gradients, Stefan-Maxwell, reaction sub-steps, collision of all M+1
stored lattices) over the whole lattice.  Default workload: the 3D channel
512x64x64 with the 9-species / 21-reaction synthetic mechanism, TMS walls on
the four side faces, flux inlet and LODI outlet, FP32 deviation storage with
FP64 arithmetic; the same workload in FP64 storage is measured beside it.

Prints one JSON line.  Inputs are resident in HBM before the timed region.
"""
import argparse
import hashlib
import json
import os
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "k_update_channel3d_512x64x64_traffic.json")


def _kernel_hash():
    """Hash of the kernel sources' code (the kernels, the physics and the
    launch shapes): // comments and blank lines are dropped, so commentary
    edits keep the recorded counters valid."""
    h = hashlib.sha256()
    for f in ("physics.hpp", "launch.hpp", "kernels.hip"):
        with open(os.path.join(ROOT, "paper_2108_07605_amd", "csrc", f)) as fh:
            lines = (re.sub(r"//.*$", "", ln).rstrip() for ln in fh.read().splitlines())
            h.update("\n".join(ln for ln in lines if ln).encode())
    return h.hexdigest()[:16]


def _traffic_all(storage, dims):
    """HBM bytes per launch of every step kernel from committed rocprofv3
    counter runs (FETCH_SIZE + WRITE_SIZE, scaled by the same counters on a
    copy kernel of known size): {kernel: bytes}, or {} when absent, taken on
    another workload, or taken on different kernel sources."""
    try:
        with open(TRAFFIC_FILE) as fh:
            t = json.load(fh)
    except (OSError, ValueError):
        return {}
    if t.get("kernel_hash") != _kernel_hash() or t.get("dims") != list(dims):
        return {}
    return {k: v["bytes_per_launch"] for k, v in t.get(storage, {}).items() if "bytes_per_launch" in v}


def _traffic(storage, kernel, dims):
    """Counted HBM bytes per launch of one kernel, or None (see _traffic_all)."""
    return _traffic_all(storage, dims).get(kernel)


def _host():
    """The host the CPU baseline ran on: logical CPUs and model name."""
    model = None
    try:
        with open("/proc/cpuinfo") as fh:
            for ln in fh:
                if ln.startswith("model name"):
                    model = ln.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"nproc": os.cpu_count(), "cpu_model": model}


def _time_storage(case, storage, steps, warmup):
    import torch
    from paper_2108_07605_amd import rlbm
    lat = rlbm.Lattice(case, storage=storage)
    lat.set_state()
    stream = lat.stream
    lat.step(warmup)
    lat.kernel_times()                  # drop anything recorded so far
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    # the dominant kernel's duration: the library records HIP events around
    # every k_update launch on the lattice stream during the timed steps
    # themselves (only that kernel, so the other launches run back to back)
    lat.set_timing(True, kernels=("update",))
    e0.record(stream)
    t0 = time.perf_counter()
    lat.step(steps)
    e1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms = e0.elapsed_time(e1)
    lat.set_timing(False)
    kt_timed = lat.kernel_times()
    # the breakdown of the step by kernel, from a few more steps with events
    # around every launch (after the timed region)
    lat.set_timing(True)
    lat.step(min(steps, 10))
    lat.set_timing(False)
    kt = lat.kernel_times()
    inv = lat.invariants()
    ok = inv[-1] == 0.0
    del lat
    torch.cuda.empty_cache()
    return {"ms_total": ms, "wall_s": wall, "kernels": kt, "update_timed": kt_timed["update"],
            "finite": bool(ok)}


def _step_roofline(storage, case, N, bytes_node, ms_step):
    """The whole step against the HBM roofline: algorithmic bytes (every
    stored population read and written once) per step over the step time,
    and the counted bytes of all of its kernels (rocprofv3, when recorded
    for these sources) over the algorithmic ones."""
    alg = bytes_node * N
    counted = _traffic_all(storage, (case["nx"], case["ny"], case["nz"]))
    tot = sum(counted.values()) if counted else None
    achieved = alg / (ms_step * 1e-3) / 1e9
    return {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS, "alg_bytes_per_step": alg,
            "counted_bytes_per_step": tot, "counted_over_algorithmic": None if tot is None else tot / alg}


def _cpu_baseline(budget_s=20.0):
    """The oracle, as it stands, on a bounded sample of the same workload: a
    64x16x16 channel with the same mechanism and boundaries, stepped until
    about budget_s of CPU time."""
    from threadpoolctl import threadpool_limits
    from oracle import Oracle
    from paper_2108_07605_amd import workloads as wl
    case = wl.make_case("channel3d", nx=64, ny=16, nz=16)
    with threadpool_limits(limits=1):      # BLAS/OpenMP pools of NumPy: one thread
        o = Oracle(case)
        o.step(1)
        t0 = time.perf_counter()
        n = 0
        while time.perf_counter() - t0 < budget_s:
            o.step(1)
            n += 1
        dt = time.perf_counter() - t0
    N = case["nx"] * case["ny"] * case["nz"]
    return {"value": N * n / dt / 1e6, "unit": "MLUPS", "cores": 1, "kind": "oracle",
            "sample": f"channel3d 64x16x16 (16384 nodes), same mechanism and boundaries, "
                      f"{n} steps in {dt:.1f} s, FP64 NumPy, 1 thread",
            "host": _host()}


def _bench_tubes(args):
    """The uneven flame-tube batch: tubes of U{64..2048} nodes (inlet,
    outlet, FP32 deviation storage) advanced by one launch per kernel for all
    tubes, against stepping one lattice at a time."""
    import torch
    from paper_2108_07605_amd import rlbm, workloads as wl
    mech = wl.mechanism_h2air9()
    cases = wl.tube_batch(args.tubes, mech=mech)
    m = rlbm.Mechanism(mech)
    lats = [rlbm.Lattice(c, storage="f32dev", mech=m).set_state() for c in cases]
    k = len(lats)
    nodes = sum(c["N"] for c in cases)
    batch = rlbm.Batch(lats)
    batch.step([args.warmup] * k)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    batch.step([args.steps] * k)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    finite = all(l.invariants()[-1] == 0.0 for l in lats)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    for l in lats:
        l.step(args.seq_steps)
    torch.cuda.synchronize()
    dt_seq = time.perf_counter() - t1
    v = nodes * args.steps / dt / 1e6
    v_seq = nodes * args.seq_steps / dt_seq / 1e6
    return {"metric": "MLUPS, batched uneven instances", "value": v, "unit": "MLUPS", "n_gpus": 1,
            "steps": args.steps, "warmup": args.warmup, "ms_per_step": dt / args.steps * 1e3,
            "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
            "data": "synthetic",
            "config": {"workload": f"{k} flame tubes, lengths U{{64..2048}} (total {nodes} nodes), "
                                   "9 species / 21 reactions, flux inlet + LODI outlet, f32dev storage",
                       "instances": k, "nodes": nodes},
            "one_at_a_time": {"value": v_seq, "unit": "MLUPS", "steps": args.seq_steps},
            "batched_over_one_at_a_time": v / v_seq, "finite": finite}


def _bench_serve(args):
    """The continuous-batching server on a seeded Poisson trace (mean 20
    requests/s) over reactor 16^3, flame tube 1024, channel 512x64x1 and
    channel 256x64x64 requests; step budgets U{1000..5000} scaled by
    --step-scale; admission budget 200 GB of device memory.  Latency is
    arrival to fields read back."""
    import torch
    from paper_2108_07605_amd import workloads as wl
    from paper_2108_07605_amd.serving import GpuBackend, Request, Server, summarize
    mech = wl.mechanism_h2air9()
    trace = wl.serving_trace(args.requests)
    reqs = [Request(k, q["arrival_s"], wl.request_case(q, mech=mech, scale_steps=args.step_scale),
                    max(1, int(q["steps"] * args.step_scale))) for k, q in enumerate(trace)]
    backend = GpuBackend(mech, storage="f32dev", keep="fields")
    # warm up the kernels once on a small request
    warm = Server(backend, budget_bytes=200e9)
    warm.run([Request(-1, 0.0, wl.request_case(trace[0], mech=mech, scale_steps=0.01), 3)])
    torch.cuda.synchronize()
    srv = Server(backend, budget_bytes=200e9, max_slots=256, round_s=0.05)
    t0 = time.perf_counter()
    done = [0]

    def progress(r):
        done[0] += 1
        print(f"request {r.rid} done ({done[0]}/{len(reqs)}) at {time.perf_counter() - t0:.1f} s, "
              f"latency {r.latency:.2f} s{' FAILED' if r.failed else ''}", file=sys.stderr, flush=True)

    out = srv.run(reqs, on_done=progress)
    wall = time.perf_counter() - t0
    summ = summarize(out, wall)
    kinds = {}
    for q, r in zip(trace, out):
        kinds.setdefault(q["kind"], []).append(r.latency)
    offered = sum(r.nodes * r.steps for r in out) / max(q["arrival_s"] for q in trace)
    return {"metric": "p50/p99 solve latency + MLUPS, continuous batching", "value": summ["mlups"],
            "unit": "MLUPS", "n_gpus": 1, "steps": None, "warmup": 1, "ms_per_step": None,
            "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
            "data": "synthetic",
            "config": {"workload": f"{len(out)} requests, Poisson 20/s over reactor 16^3 / tube 1024 / "
                                   f"channel 512x64x1 / channel 256x64x64, steps U{{1000..5000}} x "
                                   f"{args.step_scale}, 200 GB admission budget, f32dev storage",
                       "requests": len(out), "step_scale": args.step_scale},
            "latency_s": {"p50": summ["p50_s"], "p99": summ["p99_s"], "max": summ["max_s"]},
            "failed": summ["failed"],
            "offered_load_mlups": offered / 1e6,
            "latency_p50_by_kind_s": {k: sorted(v)[len(v) // 2] for k, v in kinds.items()},
            "rounds": srv.rounds, "wall_s": wall}


def _field_errors(a, b, u_floor, dims):
    """Field-normalised max errors of a against b: max|a-b| / max|b| per
    mass fraction, for T, and for |u| (normalised by max(max|u|, u_floor));
    with the node (x, y, z) of the largest mass-fraction error."""
    import numpy as np
    nx, ny, _ = dims
    Y = [float(np.abs(a["Y"][k] - b["Y"][k]).max() / max(np.abs(b["Y"][k]).max(), 1e-300))
         for k in range(b["Y"].shape[0])]
    kw = int(np.argmax(Y))
    n = int(np.argmax(np.abs(a["Y"][kw] - b["Y"][kw])))
    T = float(np.abs(a["T"] - b["T"]).max() / np.abs(b["T"]).max())
    nT = int(np.argmax(np.abs(a["T"] - b["T"])))
    du = np.sqrt(((a["u"] - b["u"]) ** 2).sum(axis=0)).max()
    um = np.sqrt((b["u"] ** 2).sum(axis=0)).max()
    xyz = lambda m: [m % nx, (m // nx) % ny, m // (nx * ny)]
    return {"Y_max": max(Y), "Y": Y, "T": T, "u": float(du / max(um, u_floor)),
            "Y_abs_max": float(np.abs(a["Y"] - b["Y"]).max()),
            "T_abs_max_K": float(np.abs(a["T"] - b["T"]).max()),
            "Y_worst_species": kw, "Y_worst_node": xyz(n), "T_worst_node": xyz(nT)}


def _bench_substeps(args):
    """Cost of the reaction sub-steps (eq. R3): the 512x64x64 channel in
    FP32-deviation storage with l = 1, 2, 4 forward-Euler sub-steps and one
    mechanism (screened for l = 1), step time relative to l = 1.  The paper
    reports about +6 % (l = 2) and +15 % (l = 4) for its CPU solver.  Rows
    "implicit l" time the linearly implicit sub-steps on the same channel."""
    from paper_2108_07605_amd import workloads as wl
    mech = wl.mechanism_h2air9(substeps=1)
    rows = {}
    for key, l, scheme in ((1, 1, "explicit"), (2, 2, "explicit"), (4, 4, "explicit"),
                           ("implicit 1", 1, "implicit"), ("implicit 2", 2, "implicit")):
        case = wl.make_case("channel3d", nx=args.nx, ny=args.ny, nz=args.nz, mech=mech, substeps=l,
                            reaction=scheme)
        r = _time_storage(case, "f32dev", args.steps, args.warmup)
        ms = r["ms_total"] / args.steps
        rows[key] = {"ms_per_step": ms,
                     "local_ms": r["kernels"]["local"][0] / max(r["kernels"]["local"][1], 1),
                     "gradients_ms": r["kernels"]["gradients"][0] / max(r["kernels"]["gradients"][1], 1),
                     "finite": r["finite"]}
    N = args.nx * args.ny * args.nz
    for key in rows:
        rows[key]["increase_vs_l1"] = rows[key]["ms_per_step"] / rows[1]["ms_per_step"] - 1.0
        rows[key]["mlups"] = N / (rows[key]["ms_per_step"] * 1e-3) / 1e6
    return {"metric": "step time vs reaction sub-steps l", "value": rows[4]["increase_vs_l1"],
            "unit": "fraction (l=4 over l=1)", "n_gpus": 1, "steps": args.steps,
            "warmup": args.warmup, "higher_is_better": False, "dtype": "f64",
            "data": "synthetic",
            "config": {"workload": f"channel3d {args.nx}x{args.ny}x{args.nz}, 9 species, f32dev storage"},
            "substeps": rows,
            "paper_cpu_increase": {"2": 0.06, "4": 0.15}}


def _bench_coupling(args):
    """Cost of the weakly coupled storage (all M species lattices, L = M + 2)
    against the slaved one (L = M + 1) on the 512x64x64 channel in both
    storages: MLUPS, per-kernel times and k_update's algorithmic HBM rate
    (2 L 27 s bytes per node)."""
    from paper_2108_07605_amd import workloads as wl
    mech = wl.mechanism_h2air9()
    N = args.nx * args.ny * args.nz
    rows = {}
    for coupling in ("strong", "weak"):
        case = wl.make_case("channel3d", nx=args.nx, ny=args.ny, nz=args.nz, mech=mech, coupling=coupling)
        L = mech["M"] + (2 if coupling == "weak" else 1)
        for st in ("f32dev", "f64"):
            r = _time_storage(case, st, args.steps, args.warmup)
            ms = r["ms_total"] / args.steps
            upd_ms, upd_n = r["update_timed"]
            upd = upd_ms / max(upd_n, 1)
            s_b = 4 if st == "f32dev" else 8
            rows[f"{coupling} {st}"] = {
                "L": L, "ms_per_step": ms, "mlups": N / (ms * 1e-3) / 1e6,
                "kernels_ms_avg": {k: v[0] / max(v[1], 1) for k, v in r["kernels"].items()},
                "update_GBps": 2 * L * 27 * s_b * N / (upd * 1e-3) / 1e9, "finite": r["finite"]}
    return {"metric": "MLUPS, weakly coupled vs slaved storage", "value": rows["weak f32dev"]["mlups"],
            "unit": "MLUPS", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
            "higher_is_better": True, "dtype": "f64", "data": "synthetic",
            "config": {"workload": f"channel3d {args.nx}x{args.ny}x{args.nz}, 9 species"},
            "rows": rows}


def _bench_precision(args):
    """FP32-deviation storage against FP64 storage from the same initial
    state: the 512x64x64 channel after --steps steps (2000 in the recipe) and
    the 1024x64x1 channel after 2.5x as many, with the errors at 1/8, 1/4,
    1/2 and all of the steps."""
    import math
    import torch
    from paper_2108_07605_amd import rlbm, workloads as wl
    mech = wl.mechanism_h2air9()
    m = rlbm.Mechanism(mech)
    out = {"metric": "FP32-deviation vs FP64 storage: field-normalised max error", "unit": "relative",
           "n_gpus": 1, "dtype": "f64", "data": "synthetic", "higher_is_better": False, "cases": {}}
    for name, kw, steps in (("channel3d", dict(nx=args.nx, ny=args.ny, nz=args.nz), args.steps),
                            ("channel2d", dict(nx=1024, ny=64, nz=1), int(2.5 * args.steps))):
        case = wl.make_case(name, mech=mech, **kw)
        dims = (case["nx"], case["ny"], case["nz"])
        th = float(case["init"]["T"].mean()) * mech["R_univ"] / 20.0
        lats = {st: rlbm.Lattice(case, storage=st, mech=m).set_state() for st in ("f64", "f32dev")}
        done, rows = 0, []
        for n in (steps // 8, steps // 4, steps // 2, steps):
            for lat in lats.values():
                lat.step(n - done)
            done = n
            f = {st: lat.fields() for st, lat in lats.items()}
            err = _field_errors(f["f32dev"], f["f64"], 1e-3 * math.sqrt(th), dims)
            rows.append({"steps": n, **err})
        finite = all(lat.invariants()[-1] == 0.0 for lat in lats.values())
        for lat in lats.values():
            lat.close()
        # sensitivity of the FP64 run itself: the same case with the initial
        # temperature perturbed by 1e-10 (relative, seeded noise)
        import numpy as np
        init = dict(case["init"])
        rng = np.random.default_rng(11)
        init["T"] = init["T"] * (1.0 + 1e-10 * rng.uniform(-1.0, 1.0, init["T"].shape))
        a = rlbm.Lattice(case, storage="f64", mech=m).set_state()
        bl = rlbm.Lattice(case, storage="f64", mech=m).set_state(init)
        done, sens = 0, []
        for n in (steps // 8, steps // 4, steps // 2, steps):
            a.step(n - done)
            bl.step(n - done)
            done = n
            e = _field_errors(bl.fields(), a.fields(), 1e-3 * math.sqrt(th), dims)
            sens.append({k: e[k] for k in ("Y_max", "T", "u", "Y_abs_max")} | {"steps": n})
        a.close()
        bl.close()
        err = rows[-1]
        out["cases"][name] = {"dims": list(dims), "steps": steps, "errors": err,
                              "history": [{k: r[k] for k in ("steps", "Y_max", "T", "u", "Y_abs_max")}
                                          for r in rows],
                              "f64_perturbed_1e-10": sens,
                              "pass_1e-5_Y_T": err["Y_max"] <= 1e-5 and err["T"] <= 1e-5, "finite": finite}
    out["value"] = max(c["errors"]["Y_max"] for c in out["cases"].values())
    return out


def _bench_configs(args):
    """The two smaller configurations at their full sizes and step counts:
    the 32x8x8 three-species box (200 steps) and the 1024x64x1 nine-species
    channel (5000 steps).  For each: GPU MLUPS in FP64 and FP32-deviation
    storage with the step's fraction of the HBM roofline (algorithmic bytes
    2 L 27 s per node), the FP32 against FP64 field errors at the end, and
    the oracle's MLUPS on the host (the box in full; the channel on a prefix
    bounded by --cpu-budget seconds)."""
    import numpy as np
    import torch
    from threadpoolctl import threadpool_limits
    from oracle import Oracle
    from paper_2108_07605_amd import rlbm, workloads as wl
    rows = {}
    for name, case, steps in (("cfg1 abc_box 32x8x8 M=3", wl.make_case("abc_box"), 200),
                              ("cfg2 channel2d 1024x64x1 M=9", wl.make_case("channel2d"), 5000)):
        N = case["nx"] * case["ny"] * case["nz"]
        M = case["mech"]["M"]
        L = M + 1
        row = {"nodes": N, "steps": steps, "species": M}
        fields = {}
        for st, sb in (("f64", 8), ("f32dev", 4)):
            lat = rlbm.Lattice(case, storage=st).set_state()
            lat.step(min(steps, 20))                  # warm-up, then the full run from a fresh state
            lat.set_state()
            torch.cuda.synchronize()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(lat.stream)
            lat.step(steps)
            e1.record(lat.stream)
            torch.cuda.synchronize()
            ms = e0.elapsed_time(e1) / steps
            mlups = N / (ms * 1e-3) / 1e6
            row[st] = {"mlups": mlups, "ms_per_step": ms,
                       "frac_of_hbm_roofline": mlups * 1e6 * 2 * L * 27 * sb / (HBM_PEAK_GBS * 1e9),
                       "status": lat.status()}
            fields[st] = lat.fields()
            lat.close()
        th = float(np.mean(case["init"]["T"])) * case["mech"]["R_univ"] / 20.0
        err = _field_errors(fields["f32dev"], fields["f64"], 1e-3 * th ** 0.5, (case["nx"], case["ny"], case["nz"]))
        row["f32dev_vs_f64"] = {"Y_max": err["Y_max"], "T": err["T"], "u": err["u"]}
        with threadpool_limits(limits=1):
            o = Oracle(case)
            t0 = time.perf_counter()
            n = 0
            while n < steps and (n == 0 or time.perf_counter() - t0 < args.cpu_budget):
                o.step(1)
                n += 1
            dt = time.perf_counter() - t0
        row["oracle"] = {"mlups": N * n / dt / 1e6, "steps": n, "cores": 1}
        if n == steps:
            of = o.fields()
            e64 = _field_errors(fields["f64"], of, 1e-3 * th ** 0.5, (case["nx"], case["ny"], case["nz"]))
            row["f64_vs_oracle"] = {"Y_max": e64["Y_max"], "T": e64["T"], "u": e64["u"]}
        rows[name] = row
    return {"metric": "MLUPS (all M+2 LBEs) + % HBM roofline, FP32-store vs FP64", "unit": "MLUPS",
            "value": rows["cfg2 channel2d 1024x64x1 M=9"]["f32dev"]["mlups"], "n_gpus": 1,
            "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
            "data": "synthetic", "config": {"workload": "configurations 1 and 2 at full size"},
            "rows": rows, "host": _host()}


def _copy_probe(mib):
    """A copy kernel of known size: 5 launches of an out-of-place elementwise
    copy reading and writing mib MiB each."""
    import torch
    n = mib * (1 << 20) // 4
    a = torch.rand(n, device="cuda")
    b = torch.empty_like(a)
    for _ in range(5):
        torch.mul(a, 1.0, out=b)
    torch.cuda.synchronize()
    print(json.dumps({"copy_probe_bytes_read": n * 4, "copy_probe_bytes_written": n * 4, "launches": 5}))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--nx", type=int, default=512)
    ap.add_argument("--ny", type=int, default=64)
    ap.add_argument("--nz", type=int, default=64)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-budget", type=float, default=20.0)
    ap.add_argument("--storage", default="both", choices=["both", "f32dev", "f64"])
    ap.add_argument("--workload", default="channel3d",
                    choices=["channel3d", "tubes", "serve", "precision", "substeps", "coupling", "configs"],
                    help="channel3d: the 512x64x64 channel (default); tubes: 256 uneven flame "
                         "tubes in batched launches vs one lattice at a time; serve: the "
                         "continuous-batching server on a Poisson request trace; precision: "
                         "FP32-deviation vs FP64 storage field errors after --steps steps; "
                         "substeps: step time with l = 1, 2, 4 reaction sub-steps; coupling: the "
                         "weakly coupled storage (all M species lattices) vs the slaved one; "
                         "configs: the 32x8x8 box and the 1024x64x1 channel at full size in both "
                         "storages, with the oracle's rate")
    ap.add_argument("--tubes", type=int, default=256)
    ap.add_argument("--seq-steps", type=int, default=20,
                    help="steps of the one-lattice-at-a-time comparison (tubes)")
    ap.add_argument("--requests", type=int, default=200)
    ap.add_argument("--step-scale", type=float, default=1.0,
                    help="scale of the trace's step budgets (serve)")
    ap.add_argument("--copy-probe", type=int, default=0, metavar="MIB",
                    help="only run a plain device copy of MIB MiB five times (calibrates the "
                         "FETCH_SIZE / WRITE_SIZE counters) and exit")
    args = ap.parse_args()
    if args.copy_probe:
        _copy_probe(args.copy_probe)
        return
    if args.gpus != 1:
        print("bench.py runs on one GPU only: the library has no multi-GPU path",
              file=sys.stderr)
        sys.exit(2)
    import torch
    from paper_2108_07605_amd import workloads as wl
    torch.cuda.set_device(0)
    if args.workload == "tubes":
        print(json.dumps(_bench_tubes(args)))
        return
    if args.workload == "serve":
        print(json.dumps(_bench_serve(args)))
        return
    if args.workload == "precision":
        print(json.dumps(_bench_precision(args)))
        return
    if args.workload == "substeps":
        print(json.dumps(_bench_substeps(args)))
        return
    if args.workload == "coupling":
        print(json.dumps(_bench_coupling(args)))
        return
    if args.workload == "configs":
        print(json.dumps(_bench_configs(args)))
        return
    case = wl.make_case("channel3d", nx=args.nx, ny=args.ny, nz=args.nz)
    N = case["nx"] * case["ny"] * case["nz"]
    M = case["mech"]["M"]
    L = M + 1
    res = {}
    storages = ["f32dev", "f64"] if args.storage == "both" else [args.storage]
    for st in storages:
        r = _time_storage(case, st, args.steps, args.warmup)
        s = 4 if st == "f32dev" else 8
        bytes_node = 2 * L * 27 * s                      # populations read + written once
        ms_step = r["ms_total"] / args.steps
        mlups = N / (ms_step * 1e-3) / 1e6
        # dominant kernel: the collision (k_update), the largest share of the
        # step, whose algorithmic traffic is the population read + write; its
        # duration is the average over the timed steps
        coll_name = "update"
        coll_ms, coll_n = r["update_timed"]
        coll_avg = coll_ms / max(coll_n, 1)
        achieved = bytes_node * N / (coll_avg * 1e-3) / 1e9
        traffic = _traffic(st, "k_" + coll_name, (case["nx"], case["ny"], case["nz"]))
        res[st] = {
            "mlups": mlups, "ms_per_step": ms_step, "finite": r["finite"],
            "kernels_ms_avg": {k: v[0] / max(v[1], 1) for k, v in r["kernels"].items()},
            "update_ms_avg_timed": coll_avg,
            "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS,
                         "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
                         "traffic": traffic,
                         "kernel": "k_" + coll_name, "alg_bytes_per_node": bytes_node},
            "step_frac_of_hbm_roofline": mlups * 1e6 * bytes_node / (HBM_PEAK_GBS * 1e9),
            "step_roofline": _step_roofline(st, case, N, bytes_node, ms_step),
        }
    main_st = storages[0]
    m = res[main_st]
    out = {
        "metric": "MLUPS (all M+2 LBEs) + % HBM roofline, FP32-store vs FP64; p50/p99 solve latency",
        "value": m["mlups"],
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": m["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"channel3d {case['nx']}x{case['ny']}x{case['nz']}, 9 species / "
                               f"{len(case['mech']['lnA'])} reversible reactions, TMS walls on y/z, "
                               f"flux inlet, LODI outlet, {main_st} storage",
                   "nodes": N, "storage": main_st, "species": M, "substeps": case["substeps"]},
        "roofline": m["roofline"],
        "step_roofline": m["step_roofline"],
        "storages": res,
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = _cpu_baseline(args.cpu_budget)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
