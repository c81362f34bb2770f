"""Seeded synthetic inputs: mechanisms, lattices and initial fields.

This module only *produces inputs*.  It is shared by the HIP path (through
the Python binding) and by the CPU oracle, and it holds none of the lattice
Boltzmann arithmetic: no equilibria, moments, collision, transport or
temperature solve.  What it does compute is parameter selection:

* unit conversion of physical Arrhenius constants into lattice units
  (acoustic scaling, paper section 3.6, with the reference state of section 3.6:
  T0 = 298.15 K, P0 = 1 atm);
* initial densities from the ideal-gas law (paper section 2.1) so that the
  initial pressure is uniform, as the workloads prescribe;
* a stiffness screen that lowers pre-exponential factors which would make the
  explicit reaction sub-steps of section 2.3 unstable.  It evaluates the
  seeded Arrhenius law and an equilibrium-constant bound on a temperature grid
  and only ever *changes inputs*; neither side of a parity test uses its
  numbers.

The paper's own runs need a detailed hydrogen/air mechanism with tabulated
thermochemistry and transport, a DNS reference and a kinetics library, none of
which are available; every mechanism here is synthetic and seeded.
Species are labelled by their H/O/N composition only; thermochemical
coefficients are drawn from broad seeded ranges, never from tables.

Thermo model (one NASA-7 range per species, T in kelvin):
    cp/R      = a0 + a1 T + a2 T^2 + a3 T^3 + a4 T^4
    h/(R T)   = a0 + a1 T/2 + a2 T^2/3 + a3 T^3/4 + a4 T^4/5 + a5/T
    s/R       = a0 ln T + a1 T + a2 T^2/2 + a3 T^3/3 + a4 T^4/4 + a6
with R the species gas constant R_U/m_a.

Transport model (synthetic power laws standing in for mixture-averaged
transport of section 3.5):
    mu(T)      = mu_ref (T/T_ref)^mu_exp,   lambda = mu cp / Pr
    D_ab(T, P) = D_ref[a][b] (T/T_ref)^D_exp (P_ref/P)
"""
from __future__ import annotations

import copy
import itertools
import math
from dataclasses import dataclass

import numpy as np

ROOT_SEED = 2108_07605

# Physical constants (SI)
R_U_SI = 8.314462618          # J/(mol K)
P_ATM = 101325.0              # Pa
T0_STD = 298.15               # K, standard-state temperature of section 3.6

# Lattice unit map (acoustic scaling).  The lightest species at the hottest
# admissible temperature has theta = R_a T = THETA_CAP, which keeps every
# product-form factor of the species equilibria non-negative.
THETA_CAP = 0.5
T_CAP = 3000.0

FACE_NAMES = ("x-", "x+", "y-", "y+", "z-", "z+")


def _rng(*key):
    ss = np.random.SeedSequence([ROOT_SEED, *[int(k) for k in key]])
    return np.random.default_rng(ss)


# ---------------------------------------------------------------------------
# species sets
# ---------------------------------------------------------------------------
ELEMENT_MASS = {"H": 1.0, "O": 16.0, "N": 14.0}

# Nine species with H/O/N-like compositions; molar masses follow from the
# composition: {2, 32, 18, 1, 16, 17, 33, 34, 28}.
SPECIES9 = [
    ("H2", {"H": 2}),
    ("O2", {"O": 2}),
    ("H2O", {"H": 2, "O": 1}),
    ("H", {"H": 1}),
    ("O", {"O": 1}),
    ("OH", {"H": 1, "O": 1}),
    ("HO2", {"H": 1, "O": 2}),
    ("H2O2", {"H": 2, "O": 2}),
    ("N2", {"N": 2}),
]
INERT9 = 8
FUEL9 = 0
OXID9 = 1

# Seeded ranges for the synthetic thermochemistry: formation enthalpy h_f/R
# (kelvin) and standard entropy s0/R at T0.
_HF_RANGE = {
    "H2": (0.0, 0.0), "O2": (0.0, 0.0), "N2": (0.0, 0.0),
    "H2O": (-30000.0, -27000.0), "H": (24000.0, 27000.0),
    "O": (27000.0, 31000.0), "OH": (3000.0, 5000.0),
    "HO2": (0.0, 2000.0), "H2O2": (-17000.0, -15000.0),
}


def _atoms(comp):
    return sum(comp.values())


def _cp0(comp):
    n = _atoms(comp)
    return 2.5 if n == 1 else (3.5 if n == 2 else 4.0)


def _s0_range(comp):
    n = _atoms(comp)
    return (13.0, 20.0) if n == 1 else ((15.0, 25.0) if n == 2 else (22.0, 29.0))


def _molar_mass(comp):
    return sum(ELEMENT_MASS[e] * k for e, k in comp.items())


def _nasa_coeffs(rng, comp, hf_over_R):
    """Seeded NASA-7 coefficients.  a5/a6 are offsets chosen so that h/R at T0
    is close to the seeded formation enthalpy and s/R close to the seeded
    standard entropy; only a0 T0 and a0 ln T0 are removed (the small a1/a2
    terms are left in, which merely shifts the synthetic values)."""
    a0 = _cp0(comp)
    a1 = rng.uniform(0.0, 3.0e-4)
    a2 = rng.uniform(-3.0e-8, 0.0)
    s0 = rng.uniform(*_s0_range(comp))
    a5 = hf_over_R - a0 * T0_STD
    a6 = s0 - a0 * math.log(T0_STD)
    return [a0, a1, a2, 0.0, 0.0, a5, a6]


# ---------------------------------------------------------------------------
# unit map
# ---------------------------------------------------------------------------
@dataclass
class UnitMap:
    m_min: float            # g/mol of the lightest species
    rho_scale: float        # kg/m^3 per lattice density unit
    dt_phys: float          # s per lattice time step
    dx_phys: float          # m per lattice spacing

    @property
    def R_univ(self):       # universal gas constant in lattice units
        return THETA_CAP * self.m_min / T_CAP

    @property
    def c_unit(self):       # m/s per lattice velocity unit
        return math.sqrt(R_U_SI * 1e3 / self.R_univ)

    @property
    def conc_scale(self):   # mol/m^3 per lattice concentration unit
        return self.rho_scale * 1e3

    def P_lat(self, P_pa):  # pressure to lattice units
        # lattice pressure unit = rho_scale * c_unit^2
        return P_pa / (self.rho_scale * self.c_unit ** 2)

    def speed_lat(self, v_ms):
        return v_ms / self.c_unit


def _mix_mass_from_X(masses, X):
    return float(np.dot(masses, X))


def _Y_from_X(masses, X):
    w = np.asarray(masses) * np.asarray(X)
    return w / w.sum()


# ---------------------------------------------------------------------------
# reactions
# ---------------------------------------------------------------------------
def _enumerate_reactions(species, active):
    """All element-balanced reactions with one or two reactant molecules and
    one or two product molecules among the `active` species (repeats allowed),
    each unordered pair of sides listed once."""
    comps = [c for _, c in species]
    sides = []
    for n in (1, 2):
        for combo in itertools.combinations_with_replacement(active, n):
            sides.append(combo)

    def elems(side):
        tot = {}
        for s in side:
            for e, k in comps[s].items():
                tot[e] = tot.get(e, 0) + k
        return tot

    out = []
    seen = set()
    for a in sides:
        for b in sides:
            if a == b or len(a) + len(b) < 3:   # 1<->1 is not mass-changing here
                continue
            if set(a) & set(b):                  # no spectator species
                continue
            if elems(a) != elems(b):
                continue
            key = tuple(sorted([a, b]))
            if key in seen:
                continue
            seen.add(key)
            out.append((a, b))
    return out


def _side_vector(side, M):
    v = np.zeros(M, dtype=np.int64)
    for s in side:
        v[s] += 1
    return v


def _nasa_h_RT(a, T):
    return (a[0] + a[1] * T / 2 + a[2] * T ** 2 / 3 + a[3] * T ** 3 / 4
            + a[4] * T ** 4 / 5 + a[5] / T)


def _nasa_s_R(a, T):
    return (a[0] * np.log(T) + a[1] * T + a[2] * T ** 2 / 2 + a[3] * T ** 3 / 3
            + a[4] * T ** 4 / 4 + a[6])


def _screen_rates(mech, substeps, T_lo=250.0, T_hi=T_CAP, margin=0.5):
    """Stiffness screen (input selection only).  Lowers ln A of a reaction so
    that, for T in [T_lo, T_hi] and concentrations up to the total
    concentration at (P0, T_lo), no single reaction consumes more than
    `margin` of a partner per reaction sub-step, in either direction."""
    T = np.linspace(T_lo, T_hi, 400)
    R_U = mech["R_univ"]
    c_max = mech["P0"] / (R_U * T_lo)
    nasa = np.asarray(mech["nasa"])
    gRT = np.array([_nasa_h_RT(a, T) - _nasa_s_R(a, T) for a in nasa])  # [M, nT]
    capped = []
    for r in range(len(mech["lnA"])):
        nu_f = np.asarray(mech["nu_f"][r])
        nu_r = np.asarray(mech["nu_r"][r])
        dnu = nu_r - nu_f
        ln_kf = mech["lnA"][r] + mech["beta"][r] * np.log(T) - mech["Ta"][r] / T
        worst = np.max(ln_kf + (nu_f.sum() - 1) * math.log(c_max))
        if mech["reversible"][r]:
            ln_Kc = -(dnu @ gRT) + dnu.sum() * (mech["ln_cstd"] - np.log(T))
            worst = max(worst, np.max(ln_kf - ln_Kc + (nu_r.sum() - 1) * math.log(c_max)))
        limit = math.log(margin * substeps)
        if worst > limit:
            cut = worst - limit
            mech["lnA"][r] -= cut
            capped.append((r, cut / math.log(10.0)))
    mech["capped"] = capped
    return mech


# ---------------------------------------------------------------------------
# mechanisms
# ---------------------------------------------------------------------------
def _transport(mech, T_ref, rho_ref, P_ref, nu_P=0.125, Pr=0.7, Sc=0.7,
               pair_ref=(0, 1)):
    """Synthetic transport constants in lattice units.  mu_ref = nu_P * P_ref;
    the binary diffusivity of the reference pair equals the reference
    kinematic viscosity over Sc, other pairs scale with sqrt(1/m_a + 1/m_b)."""
    m = np.asarray(mech["molar_mass"])
    mu_ref = nu_P * P_ref
    nu_ref = mu_ref / rho_ref
    i, j = pair_ref
    base = math.sqrt(1.0 / m[i] + 1.0 / m[j])
    D = nu_ref / Sc * np.sqrt(1.0 / m[:, None] + 1.0 / m[None, :]) / base
    mech["transport"] = {
        "T_ref": T_ref, "P_ref": P_ref, "mu_ref": mu_ref, "mu_exp": 0.7,
        "Pr": Pr, "D_ref": D.tolist(), "D_exp": 1.75,
    }
    return mech


def mechanism_abc(seed: int = 1, substeps: int = 2):
    """Three species A(2), B(32), C(17) and one irreversible step A+B->2C.

    Arrhenius constants: A log-uniform in [1e3, 1e5] m^3/(mol s), beta = 0,
    Ea/R uniform in [2000, 8000] K.  The physical time step is chosen so that
    the seeded rate at the mean initial state (T = 1000 K, Y_A = 0.1,
    Y_B = 0.9) consumes about 20% of A over 200 steps."""
    rng = _rng(1, seed)
    species = [("A", {"H": 2}), ("B", {"O": 2}), ("C", {"H": 1, "O": 1})]
    masses = [2.0, 32.0, 17.0]
    hf = {"A": 0.0, "B": 0.0, "C": rng.uniform(-6000.0, -4000.0)}
    nasa = [_nasa_coeffs(rng, c, hf[n]) for n, c in species]
    A_si = 10.0 ** rng.uniform(3.0, 5.0)
    Ta = rng.uniform(2000.0, 8000.0)

    T_ref, YA, YB = 1000.0, 0.1, 0.9
    m_ref = 1.0 / (YA / 2.0 + YB / 32.0)
    rho_phys = P_ATM * m_ref * 1e-3 / (R_U_SI * T_ref)
    # rate of A per unit time at the mean state: k c_B
    cB_phys = rho_phys * YB / 32e-3
    k_phys = A_si * math.exp(-Ta / T_ref)
    dt_phys = (0.2 / 200.0) / (k_phys * cB_phys)
    units = UnitMap(m_min=2.0, rho_scale=rho_phys, dt_phys=dt_phys, dx_phys=0.0)
    units.dx_phys = units.c_unit * dt_phys

    R_U = units.R_univ
    P0 = units.P_lat(P_ATM)
    mech = {
        "name": "synthetic A+B->2C",
        "species": [n for n, _ in species],
        "M": 3,
        "molar_mass": masses,
        "elements": ["H", "O"],
        "composition": [[c.get("H", 0), c.get("O", 0)] for _, c in species],
        "nasa": nasa,
        "R_univ": R_U,
        "P0": P0,
        "ln_cstd": math.log(P0 / R_U),
        "nu_f": [[1, 1, 0]],
        "nu_r": [[0, 0, 2]],
        "lnA": [math.log(A_si * units.conc_scale * dt_phys)],
        "beta": [0.0],
        "Ta": [Ta],
        "reversible": [0],
        "units": units.__dict__ | {"R_univ": R_U, "c_unit": units.c_unit},
    }
    _transport(mech, T_ref=T_ref, rho_ref=1.0, P_ref=P0, pair_ref=(0, 1))
    _screen_rates(mech, substeps)
    return mech


def mechanism_abcd(seed: int = 1, substeps: int = 2):
    """Four species: the three of mechanism_abc and an inert D(28) that takes
    part in transport and thermo only (one reaction A+B->2C)."""
    mech = mechanism_abc(seed=seed, substeps=substeps)
    rng = _rng(3, seed)
    out = copy.deepcopy(mech)
    out["name"] = "synthetic A+B->2C with inert D"
    out["species"] = mech["species"] + ["D"]
    out["M"] = 4
    out["molar_mass"] = mech["molar_mass"] + [28.0]
    out["elements"] = ["H", "O", "N"]
    out["composition"] = [row + [0] for row in mech["composition"]] + [[0, 0, 2]]
    out["nasa"] = mech["nasa"] + [_nasa_coeffs(rng, {"N": 2}, 0.0)]
    out["nu_f"] = [row + [0] for row in mech["nu_f"]]
    out["nu_r"] = [row + [0] for row in mech["nu_r"]]
    _transport(out, T_ref=out["transport"]["T_ref"], rho_ref=1.0, P_ref=out["P0"], pair_ref=(0, 1))
    _screen_rates(out, substeps)
    return out


def with_prandtl(mech, Pr: float):
    """Copy of a mechanism with another Prandtl number (Pr = 1 makes the
    energy lattice's two relaxation rates equal, omega_1 = omega)."""
    out = copy.deepcopy(mech)
    out["transport"]["Pr"] = float(Pr)
    out["name"] = "%s, Pr %g" % (mech["name"], Pr)
    return out


def mechanism_h2air9(seed: int = 2, substeps: int = 2, n_reactions: int = 21,
                     dx_phys: float = 1e-3 / 64):
    """Nine species, `n_reactions` reversible element-balanced reactions drawn
    from all 1<->2 and 2<->2 candidates among the eight non-inert species.
    Each reaction is oriented so that its forward direction releases heat at
    T0.  log10 A ~ U[8, 14] in cm^3/mol/s units, beta ~ U[-1, 1],
    Ea/R ~ U[0, 20000] K; then the stiffness screen."""
    rng = _rng(2, seed)
    M = len(SPECIES9)
    masses = [_molar_mass(c) for _, c in SPECIES9]
    hf = {n: rng.uniform(*_HF_RANGE[n]) if _HF_RANGE[n][0] != _HF_RANGE[n][1]
          else _HF_RANGE[n][0] for n, _ in SPECIES9}
    nasa = [_nasa_coeffs(rng, c, hf[n]) for n, c in SPECIES9]

    # reference state: lean premix at 300 K, 1 atm
    X = np.zeros(M)
    X[FUEL9], X[INERT9], X[OXID9] = 0.1, 0.7, 0.2
    m_ref = _mix_mass_from_X(masses, X)
    T_ref = 300.0
    rho_phys = P_ATM * m_ref * 1e-3 / (R_U_SI * T_ref)
    units = UnitMap(m_min=min(masses), rho_scale=rho_phys, dt_phys=0.0,
                    dx_phys=dx_phys)
    units.dt_phys = dx_phys / units.c_unit
    R_U = units.R_univ
    P0 = units.P_lat(P_ATM)

    cand = _enumerate_reactions(SPECIES9, active=list(range(8)))
    pick = rng.choice(len(cand), size=min(n_reactions, len(cand)), replace=False)
    nu_f, nu_r, lnA, beta, Ta = [], [], [], [], []
    hf_vec = np.array([hf[n] for n, _ in SPECIES9])
    for k in sorted(pick):
        a, b = cand[k]
        va, vb = _side_vector(a, M), _side_vector(b, M)
        if (vb - va) @ hf_vec > 0:         # orient exothermic forward
            va, vb = vb, va
        order = int(va.sum())
        log10A = rng.uniform(8.0, 14.0)
        A_si = 10.0 ** log10A * (1e-6) ** (order - 1)
        A_lat = A_si * units.conc_scale ** (order - 1) * units.dt_phys
        nu_f.append(va.tolist())
        nu_r.append(vb.tolist())
        lnA.append(math.log(A_lat))
        beta.append(rng.uniform(-1.0, 1.0))
        Ta.append(rng.uniform(0.0, 20000.0))
    mech = {
        "name": "synthetic 9-species H/O/N",
        "species": [n for n, _ in SPECIES9],
        "M": M,
        "molar_mass": masses,
        "elements": ["H", "O", "N"],
        "composition": [[c.get("H", 0), c.get("O", 0), c.get("N", 0)]
                        for _, c in SPECIES9],
        "nasa": nasa,
        "R_univ": R_U,
        "P0": P0,
        "ln_cstd": math.log(P0 / R_U),
        "nu_f": nu_f,
        "nu_r": nu_r,
        "lnA": lnA,
        "beta": beta,
        "Ta": Ta,
        "reversible": [1] * len(nu_f),
        "units": units.__dict__ | {"R_univ": R_U, "c_unit": units.c_unit},
    }
    _transport(mech, T_ref=T_ref, rho_ref=1.0, P_ref=P0,
               pair_ref=(OXID9, INERT9))
    _screen_rates(mech, substeps)
    return mech


# ---------------------------------------------------------------------------
# lattices and initial fields
# ---------------------------------------------------------------------------
def _coords(nx, ny, nz):
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    return x.ravel().astype(float), y.ravel().astype(float), z.ravel().astype(float)


def _rho_from_state(mech, P, T, Y):
    """Ideal-gas density for the requested initial pressure (input recipe)."""
    m = np.asarray(mech["molar_mass"])
    inv_m = (Y / m[:, None]).sum(axis=0)
    return P / (mech["R_univ"] * T * inv_m)


def periodic_faces():
    return [{"type": "periodic"} for _ in FACE_NAMES]


def wall_ramp(T_lo, T_hi, nx):
    """Isothermal wall with a tanh temperature ramp along x centred at nx/20,
    of width nx/100."""
    return {"type": "wall", "T_lo": T_lo, "T_hi": T_hi, "x0": nx / 20.0,
            "width": max(nx / 100.0, 1e-12)}


def wall_profile(face, x):
    """Wall temperature at node coordinate x (input recipe, evaluated by the
    generator only to initialise the bulk temperature)."""
    return face["T_lo"] + (face["T_hi"] - face["T_lo"]) * 0.5 * (
        1.0 + np.tanh((x - face["x0"]) / face["width"]))


def make_case(name: str, seed: int = 0, **kw):
    """Build a named case.

    Names: 'abc_box' (32x8x8 periodic, 3 species), 'reactor' (homogeneous
    periodic box), 'channel2d' (1024x64x1), 'channel3d' (512x64x64), 'tube'
    (Lx1x1 flame tube), 'binary' (two-species periodic box), 'bbbox' (duct
    with bounce-back walls), plus keyword
    overrides nx, ny, nz, storage ('f64' | 'f32dev'), substeps, reaction
    ('explicit' | 'implicit'), coupling ('strong': one slaved species;
    'weak': all M species lattices stored), steps."""
    builders = {
        "abc_box": _case_abc_box,
        "reactor": _case_reactor,
        "channel2d": _case_channel2d,
        "channel3d": _case_channel3d,
        "tube": _case_tube,
        "binary": _case_binary,
        "bbbox": _case_bbbox,
    }
    case = builders[name](seed=seed, **kw)
    case.setdefault("storage", kw.get("storage", "f64"))
    case.setdefault("substeps", kw.get("substeps", 2))
    case.setdefault("reaction", kw.get("reaction", "explicit"))
    case.setdefault("coupling", kw.get("coupling", "strong"))
    case["name"] = name
    case["N"] = case["nx"] * case["ny"] * case["nz"]
    return case


def _slaved_auto(Y):
    """Largest domain-mean mass fraction; ties go to the lowest index."""
    return int(np.argmax(Y.mean(axis=1)))


def _case_abc_box(seed=0, nx=32, ny=8, nz=8, steps=200, substeps=2, perturb=True, **kw):
    mech = kw.get("mech") or mechanism_abc(substeps=substeps)
    rng = _rng(10, seed)
    x, _, _ = _coords(nx, ny, nz)
    ph1, ph2 = rng.uniform(0, 2 * np.pi, 2)
    amp_y, amp_t = (0.05, 0.02) if perturb else (0.0, 0.0)
    YA = 0.1 * (1 + amp_y * np.sin(2 * np.pi * x / nx + ph1))
    if mech["M"] == 4:          # with the inert D at a uniform 30% by mass
        Y = np.stack([0.7 * YA, 0.7 * (1 - YA), np.zeros_like(YA), np.full_like(YA, 0.3)])
    else:
        Y = np.stack([YA, 1 - YA, np.zeros_like(YA)])
    T = 1000.0 * (1 + amp_t * np.sin(2 * np.pi * x / nx + ph2))
    rho = _rho_from_state(mech, mech["P0"], T, Y)
    u = np.zeros((3, x.size))
    return {"mech": mech, "nx": nx, "ny": ny, "nz": nz, "faces": periodic_faces(),
            "substeps": substeps, "slaved": _slaved_auto(Y), "steps": steps,
            "init": {"rho": rho, "u": u, "T": T, "Y": Y}}


def _case_reactor(seed=0, nx=16, ny=16, nz=16, steps=1000, substeps=2, mech=None,
                  T0=1200.0, X_fuel=0.1, X_radical=0.0, **kw):
    """Homogeneous periodic box of fuel, oxidiser and inert; X_radical > 0
    adds that mole fraction of every other species (a radical pool, so the
    fast reactions run from the first step)."""
    mech = mech or mechanism_h2air9(substeps=substeps)
    M = mech["M"]
    N = nx * ny * nz
    X = np.zeros(M)
    if M == 9:
        X[:] = X_radical
        X[FUEL9], X[INERT9], X[OXID9] = X_fuel, 0.7 - 6 * X_radical, 0.0
        X[OXID9] = 1.0 - X.sum()
    else:
        X[:] = 1.0 / M
    Y = np.repeat(_Y_from_X(mech["molar_mass"], X)[:, None], N, axis=1)
    T = np.full(N, T0)
    rho = _rho_from_state(mech, mech["P0"], T, Y)
    return {"mech": mech, "nx": nx, "ny": ny, "nz": nz, "faces": periodic_faces(),
            "substeps": substeps, "slaved": _slaved_auto(Y), "steps": steps,
            "init": {"rho": rho, "u": np.zeros((3, N)), "T": T, "Y": Y}}


def _premix_Y(mech, X_fuel=0.1, X_inert=0.7):
    M = mech["M"]
    X = np.zeros(M)
    X[FUEL9], X[INERT9] = X_fuel, X_inert
    X[OXID9] = 1.0 - X_fuel - X_inert
    return _Y_from_X(mech["molar_mass"], X)


def _channel(mech, nx, ny, nz, u_ms, T_in, T_wall_hi, walls_y, walls_z,
             perturb, rng, X_fuel=0.1, inlet="inlet"):
    N = nx * ny * nz
    units = mech["units"]
    u_in = u_ms / units["c_unit"]
    Yin = _premix_Y(mech, X_fuel)
    wall = wall_ramp(T_in, T_wall_hi, nx)
    x, _, _ = _coords(nx, ny, nz)
    T = wall_profile(wall, x)
    Y = np.repeat(Yin[:, None], N, axis=1)
    rho = _rho_from_state(mech, mech["P0"], T, Y)
    u = np.zeros((3, N))
    u[0] = u_in
    if perturb > 0:
        u += perturb * u_in * rng.uniform(-1.0, 1.0, size=(3, N))
    rho_in = float(_rho_from_state(mech, mech["P0"], np.array([T_in]), Yin[:, None])[0])
    faces = [
        {"type": inlet, "rho": rho_in, "u": u_in, "T": T_in, "Y": Yin.tolist()},
        {"type": "outlet", "P_inf": mech["P0"], "sigma": 0.25},
        dict(wall) if walls_y else {"type": "periodic"},
        dict(wall) if walls_y else {"type": "periodic"},
        dict(wall) if walls_z else {"type": "periodic"},
        dict(wall) if walls_z else {"type": "periodic"},
    ]
    return faces, {"rho": rho, "u": u, "T": T, "Y": Y}


def _case_channel2d(seed=0, nx=1024, ny=64, nz=1, steps=5000, substeps=2, mech=None,
                    u_ms=0.5, inlet="inlet", **kw):
    """inlet: 'inlet' (velocity and temperature imposed) or 'inlet_local'
    (the simplified flux inlet that keeps the local values)."""
    mech = mech or mechanism_h2air9(substeps=substeps)
    faces, init = _channel(mech, nx, ny, nz, u_ms, 300.0, 1300.0, True, False, 0.0,
                           _rng(20, seed), inlet=inlet)
    return {"mech": mech, "nx": nx, "ny": ny, "nz": nz, "faces": faces,
            "substeps": substeps, "slaved": _slaved_auto(init["Y"]), "steps": steps,
            "init": init}


def _case_channel3d(seed=0, nx=512, ny=64, nz=64, steps=2000, substeps=2, mech=None,
                    u_ms=0.5, perturb=0.01, **kw):
    mech = mech or mechanism_h2air9(substeps=substeps)
    faces, init = _channel(mech, nx, ny, nz, u_ms, 300.0, 1300.0, True, True, perturb,
                           _rng(30, seed))
    return {"mech": mech, "nx": nx, "ny": ny, "nz": nz, "faces": faces,
            "substeps": substeps, "slaved": _slaved_auto(init["Y"]), "steps": steps,
            "init": init}


def _case_bbbox(seed=0, nx=16, ny=8, nz=6, steps=200, substeps=2, mech=None,
                perturb=True, **kw):
    """Closed duct: periodic along x, adiabatic bounce-back walls on the four
    y and z faces; the lean premix with seeded sinusoidal composition and
    temperature modes along x and seeded velocity noise (perturb=False: a
    uniform mixture at rest at 1200 K)."""
    mech = mech or mechanism_h2air9(substeps=substeps)
    rng = _rng(60, seed)
    N = nx * ny * nz
    x, _, _ = _coords(nx, ny, nz)
    Y = np.repeat(_premix_Y(mech)[:, None], N, axis=1)
    T = np.full(N, 1200.0)
    u = np.zeros((3, N))
    if perturb:
        ph = rng.uniform(0, 2 * np.pi, 2)
        Y[FUEL9] *= 1.0 + 0.2 * np.sin(2 * np.pi * x / nx + ph[0])
        Y[INERT9] = 0.0
        Y[INERT9] = 1.0 - Y.sum(axis=0)
        T = 1200.0 * (1.0 + 0.1 * np.sin(2 * np.pi * x / nx + ph[1]))
        u = 1e-3 * rng.uniform(-1.0, 1.0, size=(3, N))
    rho = _rho_from_state(mech, mech["P0"], T, Y)
    bb = {"type": "bounceback"}
    faces = [{"type": "periodic"}, {"type": "periodic"}, dict(bb), dict(bb), dict(bb), dict(bb)]
    return {"mech": mech, "nx": nx, "ny": ny, "nz": nz, "faces": faces,
            "substeps": substeps, "slaved": _slaved_auto(Y), "steps": steps,
            "init": {"rho": rho, "u": u, "T": T, "Y": Y}}


def _case_tube(seed=0, nx=None, steps=10000, substeps=2, mech=None, **kw):
    """Quasi-1D flame tube: inlet at x=0, outlet at x=nx-1, y/z periodic.
    Length U{64..2048}, fuel mole fraction U[0.05, 0.15], inlet speed
    U[0.2, 1.0] m/s; the left 80% is unburnt premix at 300 K, the right 20%
    the same premix at a seeded hot temperature (an ignition kernel standing in
    for the burnt state)."""
    mech = mech or mechanism_h2air9(substeps=substeps)
    rng = _rng(40, seed)
    L = int(nx) if nx is not None else int(rng.integers(64, 2049))
    X_fuel = rng.uniform(0.05, 0.15)
    u_ms = rng.uniform(0.2, 1.0)
    T_hot = rng.uniform(1500.0, 1700.0)
    units = mech["units"]
    u_in = u_ms / units["c_unit"]
    Yin = _premix_Y(mech, X_fuel)
    x = np.arange(L, dtype=float)
    T = np.where(x < 0.8 * L, 300.0, T_hot)
    Y = np.repeat(Yin[:, None], L, axis=1)
    rho = _rho_from_state(mech, mech["P0"], T, Y)
    u = np.zeros((3, L))
    u[0] = u_in
    rho_in = float(_rho_from_state(mech, mech["P0"], np.array([300.0]), Yin[:, None])[0])
    faces = [
        {"type": "inlet", "rho": rho_in, "u": u_in, "T": 300.0, "Y": Yin.tolist()},
        {"type": "outlet", "P_inf": mech["P0"], "sigma": 0.25},
        {"type": "periodic"}, {"type": "periodic"},
        {"type": "periodic"}, {"type": "periodic"},
    ]
    return {"mech": mech, "nx": L, "ny": 1, "nz": 1, "faces": faces,
            "substeps": substeps, "slaved": _slaved_auto(Y), "steps": steps,
            "init": {"rho": rho, "u": u, "T": T, "Y": Y},
            "meta": {"X_fuel": X_fuel, "u_ms": u_ms, "T_hot": T_hot}}


def _case_binary(seed=0, nx=64, ny=1, nz=1, steps=200, substeps=1, mech=None,
                 amp=1e-3, T0=300.0, masses=(2.0, 28.0), **kw):
    """Two non-reacting species (default masses 2 and 28) in a periodic box
    with a small sinusoidal composition mode at uniform pressure and
    temperature."""
    if mech is None:
        mech = _binary_mech(masses)
    x, _, _ = _coords(nx, ny, nz)
    X1 = 0.5 + amp * np.sin(2 * np.pi * x / nx)
    m = np.asarray(mech["molar_mass"])
    Y1 = X1 * m[0] / (X1 * m[0] + (1 - X1) * m[1])
    Y = np.stack([Y1, 1 - Y1])
    T = np.full(x.size, T0)
    rho = _rho_from_state(mech, mech["P0"], T, Y)
    return {"mech": mech, "nx": nx, "ny": ny, "nz": nz, "faces": periodic_faces(),
            "substeps": substeps, "slaved": _slaved_auto(Y), "steps": steps,
            "init": {"rho": rho, "u": np.zeros((3, x.size)), "T": T, "Y": Y}}


def _binary_mech(masses=(2.0, 28.0)):
    masses = [float(m) for m in masses]
    units = UnitMap(m_min=min(masses), rho_scale=1.0, dt_phys=1e-9, dx_phys=0.0)
    R_U = units.R_univ
    T_ref = 300.0
    m_ref = 0.5 * masses[0] + 0.5 * masses[1]   # molar mass at X = (0.5, 0.5)
    P0 = R_U * T_ref / m_ref
    mech = {
        "name": "binary non-reacting",
        "species": ["L", "Hv"], "M": 2, "molar_mass": masses,
        "elements": ["H", "N"], "composition": [[2, 0], [0, 2]],
        "nasa": [[3.5, 0, 0, 0, 0, -3.5 * T0_STD, 10.0],
                 [3.5, 0, 0, 0, 0, -3.5 * T0_STD, 20.0]],
        "R_univ": R_U, "P0": P0, "ln_cstd": math.log(P0 / R_U),
        "nu_f": [], "nu_r": [], "lnA": [], "beta": [], "Ta": [], "reversible": [],
        "units": units.__dict__ | {"R_univ": R_U, "c_unit": units.c_unit},
    }
    _transport(mech, T_ref=T_ref, rho_ref=1.0, P_ref=P0, pair_ref=(0, 1))
    mech["capped"] = []
    return mech


def scaled_rates(mech, factor: float):
    """Copy of a mechanism with every pre-exponential factor multiplied by
    `factor` (after the stiffness screen): a stiff variant for the linearly
    implicit reaction update."""
    out = copy.deepcopy(mech)
    out["lnA"] = [a + math.log(factor) for a in mech["lnA"]]
    out["name"] = "%s, rates x%g" % (mech["name"], factor)
    return out


def tube_batch(n: int = 256, seed: int = 0, mech=None, substeps: int = 2):
    """The uneven flame-tube batch: n independent tubes, lengths U{64..2048}."""
    mech = mech or mechanism_h2air9(substeps=substeps)
    return [make_case("tube", seed=seed * 100003 + k, mech=mech, substeps=substeps)
            for k in range(n)]


def serving_trace(n: int = 200, rate_hz: float = 20.0, seed: int = 0):
    """Seeded Poisson arrival trace of solve requests.  Each request is
    (arrival_s, kind, case_seed, steps) with kind drawn uniformly from
    reactor 16^3, flame tube 1024x1x1, channel 512x64x1, channel 256x64x64
    and a step budget U{1000..5000}."""
    rng = _rng(50, seed)
    t = np.cumsum(rng.exponential(1.0 / rate_hz, size=n))
    kinds = ["reactor16", "tube1024", "channel2d_512x64", "channel3d_256x64x64"]
    out = []
    for k in range(n):
        out.append({"arrival_s": float(t[k]), "kind": kinds[int(rng.integers(0, 4))],
                    "seed": int(rng.integers(0, 2**31 - 1)),
                    "steps": int(rng.integers(1000, 5001))})
    return out


def request_case(req, mech=None, scale_steps: float = 1.0):
    mech = mech or mechanism_h2air9()
    kind, seed = req["kind"], req["seed"]
    if kind == "reactor16":
        c = make_case("reactor", seed=seed, mech=mech,
                      T0=float(_rng(51, seed).uniform(1100.0, 1400.0)))
    elif kind == "tube1024":
        c = make_case("tube", seed=seed, nx=1024, mech=mech)
    elif kind == "channel2d_512x64":
        c = make_case("channel2d", seed=seed, nx=512, ny=64, nz=1, mech=mech)
    else:
        c = make_case("channel3d", seed=seed, nx=256, ny=64, nz=64, mech=mech)
    c["steps"] = max(1, int(req["steps"] * scale_steps))
    return c
