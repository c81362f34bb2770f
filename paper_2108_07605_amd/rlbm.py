"""Thin Python binding of librlbm.so (the C ABI in include/rlbm.h).

Argument marshalling only: every step of the method runs in the HIP kernels of
the library.  PyTorch provides device memory and the stream.  If the shared
library is missing the import of this module fails loudly; there is no CPU
fallback.
"""
from __future__ import annotations

import ctypes
import os
from ctypes import POINTER, c_double, c_int, c_int32, c_int64, c_size_t, c_void_p

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "librlbm.so")

FACE_PERIODIC, FACE_WALL, FACE_INLET, FACE_OUTLET, FACE_BOUNCEBACK, FACE_INLET_LOCAL = 0, 1, 2, 3, 4, 5
STORAGE_F64, STORAGE_F32_DEV = 0, 1
REACTION_EXPLICIT, REACTION_LINEARLY_IMPLICIT = 0, 1
SLAVED_NONE = -2   # weakly coupled storage: all M species lattices stored
_FACE_CODES = {"periodic": FACE_PERIODIC, "wall": FACE_WALL, "inlet": FACE_INLET,
               "outlet": FACE_OUTLET, "bounceback": FACE_BOUNCEBACK, "inlet_local": FACE_INLET_LOCAL}
_STORAGE = {"f64": STORAGE_F64, "f32dev": STORAGE_F32_DEV}
_REACTION = {"explicit": REACTION_EXPLICIT, "implicit": REACTION_LINEARLY_IMPLICIT}
# kernels of one step, in launch order (rlbm_kernel_times)
KERNELS = ("boundary", "local", "gradients", "update")

EXPORTS = (
    "rlbm_mech_create", "rlbm_mech_destroy", "rlbm_lattice_bytes", "rlbm_lattice_create",
    "rlbm_lattice_destroy", "rlbm_set_state", "rlbm_step", "rlbm_read_fields",
    "rlbm_read_populations", "rlbm_write_populations", "rlbm_invariants",
    "rlbm_lattice_shape", "rlbm_set_timing", "rlbm_kernel_times", "rlbm_batch_bytes",
    "rlbm_state_bytes", "rlbm_save_state", "rlbm_load_state",
    "rlbm_batch_create", "rlbm_batch_step", "rlbm_batch_destroy", "rlbm_last_error",
    "rlbm_lattice_status", "rlbm_batch_status", "rlbm_step_group",
)


class RlbmError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"rlbm error {code}: {msg}")
        self.code = code


class MechDesc(ctypes.Structure):
    _fields_ = [
        ("M", c_int32), ("R", c_int32), ("E", c_int32),
        ("molar_mass", POINTER(c_double)), ("nasa", POINTER(c_double)),
        ("composition", POINTER(c_int32)),
        ("R_univ", c_double), ("ln_cstd", c_double),
        ("nu_f", POINTER(c_int32)), ("nu_r", POINTER(c_int32)),
        ("lnA", POINTER(c_double)), ("beta", POINTER(c_double)), ("Ta", POINTER(c_double)),
        ("reversible", POINTER(c_int32)),
        ("T_ref", c_double), ("P_ref", c_double), ("mu_ref", c_double), ("mu_exp", c_double),
        ("Pr", c_double), ("D_exp", c_double), ("D_ref", POINTER(c_double)),
    ]


class Face(ctypes.Structure):
    _fields_ = [
        ("type", c_int32),
        ("T_lo", c_double), ("T_hi", c_double), ("x0", c_double), ("width", c_double),
        ("rho_in", c_double), ("u_in", c_double), ("T_in", c_double),
        ("Y_in", POINTER(c_double)),
        ("P_inf", c_double), ("sigma", c_double),
    ]


class LatticeDesc(ctypes.Structure):
    _fields_ = [
        ("nx", c_int32), ("ny", c_int32), ("nz", c_int32),
        ("faces", Face * 6),
        ("storage", c_int32), ("substeps", c_int32), ("slaved", c_int32),
        ("reaction", c_int32),
    ]


_lib_handle = None


def lib():
    """Load librlbm.so once; raise if it has not been built."""
    global _lib_handle
    if _lib_handle is not None:
        return _lib_handle
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with "
                          "`python -m paper_2108_07605_amd.build` (no CPU fallback exists)")
    L = ctypes.CDLL(LIB_PATH)
    vp = c_void_p
    sig = {
        "rlbm_mech_create": (c_int, [POINTER(MechDesc), POINTER(vp)]),
        "rlbm_mech_destroy": (None, [vp]),
        "rlbm_lattice_bytes": (c_int, [POINTER(LatticeDesc), vp, POINTER(c_size_t)]),
        "rlbm_lattice_create": (c_int, [POINTER(LatticeDesc), vp, vp, c_size_t, vp, POINTER(vp)]),
        "rlbm_lattice_destroy": (None, [vp]),
        "rlbm_set_state": (c_int, [vp, vp, vp, vp, vp, c_int]),
        "rlbm_step": (c_int, [vp, c_int64]),
        "rlbm_read_fields": (c_int, [vp, vp, vp, vp, vp, vp, c_int]),
        "rlbm_read_populations": (c_int, [vp, vp, c_int]),
        "rlbm_write_populations": (c_int, [vp, vp, c_int]),
        "rlbm_invariants": (c_int, [vp, POINTER(c_double), c_int]),
        "rlbm_lattice_shape": (c_int, [vp, POINTER(c_int32), POINTER(c_int64), POINTER(c_int64),
                                       POINTER(c_int32)]),
        "rlbm_set_timing": (c_int, [vp, c_int]),
        "rlbm_kernel_times": (c_int, [vp, POINTER(c_double), POINTER(c_int64), c_int]),
        "rlbm_batch_bytes": (c_int, [c_int32, POINTER(c_size_t)]),
        "rlbm_state_bytes": (c_int, [vp, POINTER(c_size_t)]),
        "rlbm_save_state": (c_int, [vp, vp, c_int]),
        "rlbm_load_state": (c_int, [vp, vp, c_int]),
        "rlbm_batch_create": (c_int, [POINTER(vp), c_int32, vp, c_size_t, POINTER(vp)]),
        "rlbm_batch_step": (c_int, [vp, POINTER(c_int64)]),
        "rlbm_batch_destroy": (None, [vp]),
        "rlbm_lattice_status": (c_int, [vp, POINTER(c_int32)]),
        "rlbm_batch_status": (c_int, [vp, POINTER(c_int32)]),
        "rlbm_step_group": (c_int, [POINTER(vp), c_int32, POINTER(c_int64)]),
        "rlbm_last_error": (ctypes.c_char_p, []),
    }
    for name, (res, args) in sig.items():
        fn = getattr(L, name)
        fn.restype = res
        fn.argtypes = args
    _lib_handle = L
    return L


def _check(rc):
    if rc != 0:
        raise RlbmError(rc, lib().rlbm_last_error().decode())


def _dptr(a, dtype):
    return a.ctypes.data_as(POINTER(dtype))


class Mechanism:
    """Mechanism descriptor (lattice units) copied into the library."""

    def __init__(self, mech):
        M = int(mech["M"])
        R = len(mech["lnA"])
        comp = np.ascontiguousarray(mech.get("composition", []), dtype=np.int32).reshape(M, -1) \
            if mech.get("composition") else np.zeros((M, 0), dtype=np.int32)
        E = comp.shape[1]
        self._keep = keep = {
            "m": np.ascontiguousarray(mech["molar_mass"], dtype=np.float64),
            "nasa": np.ascontiguousarray(mech["nasa"], dtype=np.float64).reshape(M, 7),
            "comp": comp,
            "nu_f": np.ascontiguousarray(mech["nu_f"], dtype=np.int32).reshape(R, M) if R else np.zeros((1, M), np.int32),
            "nu_r": np.ascontiguousarray(mech["nu_r"], dtype=np.int32).reshape(R, M) if R else np.zeros((1, M), np.int32),
            "lnA": np.ascontiguousarray(mech["lnA"] or [0.0], dtype=np.float64),
            "beta": np.ascontiguousarray(mech["beta"] or [0.0], dtype=np.float64),
            "Ta": np.ascontiguousarray(mech["Ta"] or [0.0], dtype=np.float64),
            "rev": np.ascontiguousarray(mech["reversible"] or [0], dtype=np.int32),
            "D": np.ascontiguousarray(mech["transport"]["D_ref"], dtype=np.float64).reshape(M, M),
        }
        tr = mech["transport"]
        d = MechDesc()
        d.M, d.R, d.E = M, R, E
        d.molar_mass = _dptr(keep["m"], c_double)
        d.nasa = _dptr(keep["nasa"], c_double)
        d.composition = _dptr(keep["comp"], c_int32) if E else None
        d.R_univ = float(mech["R_univ"])
        d.ln_cstd = float(mech["ln_cstd"])
        d.nu_f = _dptr(keep["nu_f"], c_int32)
        d.nu_r = _dptr(keep["nu_r"], c_int32)
        d.lnA = _dptr(keep["lnA"], c_double)
        d.beta = _dptr(keep["beta"], c_double)
        d.Ta = _dptr(keep["Ta"], c_double)
        d.reversible = _dptr(keep["rev"], c_int32)
        d.T_ref, d.P_ref = float(tr["T_ref"]), float(tr["P_ref"])
        d.mu_ref, d.mu_exp, d.Pr = float(tr["mu_ref"]), float(tr["mu_exp"]), float(tr["Pr"])
        d.D_exp = float(tr["D_exp"])
        d.D_ref = _dptr(keep["D"], c_double)
        self.M, self.R, self.E = M, R, E
        h = c_void_p()
        _check(lib().rlbm_mech_create(ctypes.byref(d), ctypes.byref(h)))
        self.handle = h

    def __del__(self):
        if getattr(self, "handle", None) and _lib_handle is not None:
            _lib_handle.rlbm_mech_destroy(self.handle)
            self.handle = None


def lattice_desc(case, storage="f64"):
    """Build an rlbm_lattice_desc from a workload case; returns (desc, keep)."""
    d = LatticeDesc()
    d.nx, d.ny, d.nz = int(case["nx"]), int(case["ny"]), int(case["nz"])
    keep = []
    for k, f in enumerate(case["faces"]):
        fc = d.faces[k]
        fc.type = _FACE_CODES[f["type"]]
        if f["type"] == "wall":
            fc.T_lo, fc.T_hi, fc.x0, fc.width = f["T_lo"], f["T_hi"], f["x0"], f["width"]
        elif f["type"] in ("inlet", "inlet_local"):
            y = np.ascontiguousarray(f["Y"], dtype=np.float64)
            keep.append(y)
            fc.rho_in, fc.u_in, fc.T_in = f["rho"], f["u"], f["T"]
            fc.Y_in = _dptr(y, c_double)
        elif f["type"] == "outlet":
            fc.P_inf, fc.sigma = f["P_inf"], f["sigma"]
    d.storage = _STORAGE[storage]
    d.substeps = int(case.get("substeps", 2))
    coupling = case.get("coupling", "strong")
    if coupling not in ("strong", "weak"):
        raise KeyError("unknown coupling %r" % (coupling,))
    d.slaved = SLAVED_NONE if coupling == "weak" else int(case.get("slaved", -1))
    d.reaction = _REACTION[case.get("reaction", "explicit")]
    return d, keep


def lattice_bytes(case, mech: Mechanism, storage="f64"):
    d, _keep = lattice_desc(case, storage)
    n = c_size_t()
    _check(lib().rlbm_lattice_bytes(ctypes.byref(d), mech.handle, ctypes.byref(n)))
    return n.value


class Lattice:
    """One lattice in torch-owned device memory on the current CUDA (HIP) device."""

    def __init__(self, case, storage="f64", mech: Mechanism | None = None, stream=None):
        import torch
        self.torch = torch
        self.case = case
        self.mech = mech or Mechanism(case["mech"])
        self.M = self.mech.M
        self.N = int(case["nx"]) * int(case["ny"]) * int(case["nz"])
        self.storage = storage
        d, keep = lattice_desc(case, storage)
        nbytes = c_size_t()
        _check(lib().rlbm_lattice_bytes(ctypes.byref(d), self.mech.handle, ctypes.byref(nbytes)))
        self.nbytes = nbytes.value
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        self._mem = torch.empty(self.nbytes + 256, dtype=torch.uint8, device="cuda")
        base = self._mem.data_ptr()
        aligned = (base + 255) & ~255
        h = c_void_p()
        _check(lib().rlbm_lattice_create(ctypes.byref(d), self.mech.handle, c_void_p(aligned),
                                         self.nbytes, c_void_p(self.stream.cuda_stream),
                                         ctypes.byref(h)))
        self.handle = h
        Lc, Nc, nif, sl = c_int32(), c_int64(), c_int64(), c_int32()
        _check(lib().rlbm_lattice_shape(h, ctypes.byref(Lc), ctypes.byref(Nc), ctypes.byref(nif),
                                        ctypes.byref(sl)))
        self.L, self.n_interface = Lc.value, nif.value
        del keep

    @property
    def slaved(self):
        sl = c_int32()
        _check(lib().rlbm_lattice_shape(self.handle, None, None, None, ctypes.byref(sl)))
        return sl.value

    def __del__(self):
        self.close()

    def close(self):
        """Destroy the lattice and release its device memory (after the
        work queued on its stream)."""
        if getattr(self, "handle", None) and _lib_handle is not None:
            _lib_handle.rlbm_lattice_destroy(self.handle)
            self.handle = None
            self.stream.synchronize()
            self._mem = None

    def set_state(self, init=None):
        init = init or self.case["init"]
        arrs = [np.ascontiguousarray(init[k], dtype=np.float64) for k in ("rho", "u", "T", "Y")]
        _check(lib().rlbm_set_state(self.handle, *[a.ctypes.data_as(c_void_p) for a in arrs], 0))
        return self

    def step(self, n=1):
        _check(lib().rlbm_step(self.handle, int(n)))

    def fields(self):
        torch = self.torch
        N, M = self.N, self.M
        out = {k: torch.empty(s, dtype=torch.float64, device="cuda")
               for k, s in (("rho", N), ("u", 3 * N), ("T", N), ("Y", M * N), ("P", N))}
        _check(lib().rlbm_read_fields(self.handle, *[c_void_p(out[k].data_ptr())
                                                     for k in ("rho", "u", "T", "Y", "P")], 1))
        res = {k: v.cpu().numpy() for k, v in out.items()}
        res["u"] = res["u"].reshape(3, N)
        res["Y"] = res["Y"].reshape(M, N)
        return res

    def populations(self):
        torch = self.torch
        buf = torch.empty(self.L * 27 * self.N, dtype=torch.float64, device="cuda")
        _check(lib().rlbm_read_populations(self.handle, c_void_p(buf.data_ptr()), 1))
        return buf.cpu().numpy().reshape(self.L, 27, self.N)

    def write_populations(self, pops):
        torch = self.torch
        buf = torch.as_tensor(np.ascontiguousarray(pops, dtype=np.float64).ravel(), device="cuda")
        _check(lib().rlbm_write_populations(self.handle, c_void_p(buf.data_ptr()), 1))

    def save_state(self):
        """Raw snapshot (host bytes) for bit-exact resume."""
        n = c_size_t()
        _check(lib().rlbm_state_bytes(self.handle, ctypes.byref(n)))
        buf = np.empty(n.value, dtype=np.uint8)
        _check(lib().rlbm_save_state(self.handle, buf.ctypes.data_as(c_void_p), 0))
        return buf

    def load_state(self, buf):
        buf = np.ascontiguousarray(buf, dtype=np.uint8)
        _check(lib().rlbm_load_state(self.handle, buf.ctypes.data_as(c_void_p), 0))
        return self

    def invariants(self):
        n = 6 + self.mech.E
        out = (c_double * n)()
        _check(lib().rlbm_invariants(self.handle, out, n))
        return np.array(out[:])

    def status(self):
        """Failure bits set since the last call (0: healthy); clears them."""
        st = c_int32()
        _check(lib().rlbm_lattice_status(self.handle, ctypes.byref(st)))
        return st.value

    def set_timing(self, on=True, kernels=None):
        """HIP events around the launches of the named kernels (all when
        `kernels` is None) while `on`."""
        names = KERNELS if kernels is None else kernels
        mask = sum(1 << KERNELS.index(k) for k in names) if on else 0
        _check(lib().rlbm_set_timing(self.handle, mask))

    def kernel_times(self):
        ms = (c_double * len(KERNELS))()
        cnt = (c_int64 * len(KERNELS))()
        _check(lib().rlbm_kernel_times(self.handle, ms, cnt, len(KERNELS)))
        return {name: (ms[k], cnt[k])
                for k, name in enumerate(KERNELS)}


GROUP_MAX_LATTICES = 256


def step_group(lattices, steps):
    """Advance lattices together without any allocation (rlbm_step_group):
    all on one stream, at most GROUP_MAX_LATTICES of them."""
    k = len(lattices)
    arr = (c_void_p * k)(*[lat.handle.value for lat in lattices])
    st = (c_int64 * k)(*[int(s) for s in steps])
    _check(lib().rlbm_step_group(arr, k, st))


class Batch:
    """Independent lattices advanced by shared launches (rlbm_batch_*)."""

    def __init__(self, lattices):
        import torch
        self.lattices = list(lattices)
        k = len(self.lattices)
        nb = c_size_t()
        _check(lib().rlbm_batch_bytes(k, ctypes.byref(nb)))
        self._mem = torch.empty(nb.value + 256, dtype=torch.uint8, device="cuda")
        aligned = (self._mem.data_ptr() + 255) & ~255
        arr = (c_void_p * k)(*[lat.handle.value for lat in self.lattices])
        h = c_void_p()
        _check(lib().rlbm_batch_create(arr, k, c_void_p(aligned), nb.value, ctypes.byref(h)))
        self.handle = h

    def step(self, steps):
        k = len(self.lattices)
        arr = (c_int64 * k)(*[int(s) for s in steps])
        _check(lib().rlbm_batch_step(self.handle, arr))

    def status(self):
        """Failure bits of every lattice since the last call (0: healthy);
        clears them."""
        k = len(self.lattices)
        arr = (c_int32 * k)()
        _check(lib().rlbm_batch_status(self.handle, arr))
        return list(arr)

    def __del__(self):
        if getattr(self, "handle", None) and _lib_handle is not None:
            _lib_handle.rlbm_batch_destroy(self.handle)
            self.handle = None
