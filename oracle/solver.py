"""One time step of the M+2 coupled lattice Boltzmann equations, in order.

Per step (dt = dx = 1, lattice units, T in kelvin):

 1. Advection of every stored lattice (eq. advection); periodic faces wrap.
 2. Boundary reconstruction at interface nodes (section 4): Tamm-Mott-Smith
    walls, bounce-back walls, inlet (full or simplified), outlet, on
    disjoint node sets.
 3. Moments: rho, u (f lattice), rho_a, u_a (species; the slaved species by
    difference, eq. strongest), rho E (g lattice), P = sum f c c, q = sum g c;
    T from eq. temperature.
 4. Same-time gradients d_a = d/dx_a [rho u_a (1 - 3 R T) - rho u_a^3]
    (eqs. Pex, qex) and grad Y_a (eq. corrFourier) with the isotropic D3Q27
    stencil  d phi/dx_a = 3 sum_i w_i c_ia phi(x + c_i)  (reading: the paper
    cites isotropic lattice operators without printing them; ghost values
    beyond a non-periodic face repeat the nearest in-domain node).
 5. Relaxation parameters and the Stefan-Maxwell system (eq. transform1),
    solved for each Cartesian component.
 6. Reaction increment by l sub-steps (eq. R3), forward Euler or the
    linearly implicit variant.
 7. Species collision (eq. finalNumericalEquationsReactive with eqs. fStar,
    xiPstar2, and eq. R3 read with rho_a^{-1} f_ai^eq, since with the printed
    rho^{-1} the source would not carry mass rho_dot_a as eq. Dotfr requires).
 8. Momentum collision with the extended equilibrium (eqs. f, feqmix, Pex).
 9. Energy collision (eqs. g, geq_i, gstar, gstareq1mom, qdiff,
    corrFourier, qex).  Reading: P^eq in eq. gstareq1mom is the equilibrium
    pressure tensor rho (R T I + u u).  The update is evaluated in the
    algebraically identical form
        g' = g + omega (g^eq - g) + (1/2) c_i . Q   on |c_i|^2 = 1,
        Q  = (omega - omega_1)(q - u.(P - P^eq) + q^ex - q^eq)
             + omega_1 rho sum_a H_a Y_a V_a
             + (1/2)(2 - omega_1) P sum_a H_a grad Y_a,
    which is finite when omega = omega_1 (eqs. qdiff and corrFourier
    individually divide by omega - omega_1).

Initial populations are the equilibria f_a^eq (unslaved species), f^eq and
g^eq at the given (rho, u, T, Y).

Weakly coupled storage (case["coupling"] = "weak"; the system before the
slaving of eq. strongest, section 3.4): all M species lattices are stored
beside f and g, so the step advances M+2 independent lattices.  The two
subsystems exchange fields but not populations.  Reading: the species
subsystem supplies the composition Y_a = rho_a / sum_b rho_b; the mixture
subsystem supplies rho, u (from f) and, with rho E, the temperature.  The
species take u in their quasi-equilibria and in the Stefan-Maxwell
right-hand sides u_a - u, and every species collides with its own rho_a.
sum_a rho_a and rho are then two conserved densities that may drift apart,
which is the redundancy the slaving removes.
"""
import numpy as np

from . import boundary as bc
from .chemistry import reaction_increment
from .equilibria import energy_eq, extended_eq, mixture_eq, species_W, species_eq
from .lattice import C, C2, OPP, Q, W
from .thermo import H_species, U_species, gas_constants, mixture_R, solve_temperature
from .transport import inv_tau_ab, mixture_omegas, species_beta, stefan_maxwell

FACES = ("x-", "x+", "y-", "y+", "z-", "z+")


class Oracle:
    def __init__(self, case):
        self.mech = case["mech"]
        self.M = self.mech["M"]
        self.nx, self.ny, self.nz = case["nx"], case["ny"], case["nz"]
        self.N = self.nx * self.ny * self.nz
        self.faces = case["faces"]
        self.l = int(case.get("substeps", 2))
        self.reaction = case.get("reaction", "explicit")
        coupling = case.get("coupling", "strong")
        if coupling not in ("strong", "weak"):
            raise ValueError("unknown coupling %r" % (coupling,))
        self.s = None if coupling == "weak" else int(case["slaved"])
        self.stored = [a for a in range(self.M) if a != self.s]
        self._geometry()
        self.set_state(case["init"])

    # ------------------------------------------------------------------
    # geometry: periodic axes, interface nodes, incoming sets D
    # ------------------------------------------------------------------
    def _geometry(self):
        nx, ny, nz = self.nx, self.ny, self.nz
        types = [f["type"] for f in self.faces]
        self.periodic = []
        for ax in range(3):
            a, b = types[2 * ax], types[2 * ax + 1]
            if (a == "periodic") != (b == "periodic"):
                raise ValueError("an axis must be periodic on both faces or neither")
            self.periodic.append(a == "periodic")
        z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
        self.x, self.y, self.z = x.ravel(), y.ravel(), z.ravel()
        pos = [self.x, self.y, self.z]
        n_ax = [nx, ny, nz]
        on = {}
        for ax in range(3):
            on[FACES[2 * ax]] = (pos[ax] == 0) & (not self.periodic[ax])
            on[FACES[2 * ax + 1]] = (pos[ax] == n_ax[ax] - 1) & (not self.periodic[ax])
        self.on_face = on
        D = np.zeros((Q, self.N), dtype=bool)
        for i in range(Q):
            for ax in range(3):
                if self.periodic[ax]:
                    continue
                src = pos[ax] - C[i, ax]
                D[i] |= (src < 0) | (src >= n_ax[ax])
        self.D = D
        wall = np.zeros(self.N, dtype=bool)
        bb = np.zeros(self.N, dtype=bool)
        inlet = np.zeros(self.N, dtype=bool)
        outlet = np.zeros(self.N, dtype=bool)
        for k, name in enumerate(FACES):
            t = types[k]
            if t == "wall":
                wall |= on[name]
            elif t == "bounceback":
                bb |= on[name]
            elif t in ("inlet", "inlet_local"):
                inlet |= on[name]
            elif t == "outlet":
                outlet |= on[name]
        bb &= ~wall
        inlet &= ~(wall | bb)
        outlet &= ~(wall | bb)
        self.wall_nodes = np.nonzero(wall)[0]
        self.bb_nodes = np.nonzero(bb)[0]
        self.inlet_nodes = np.nonzero(inlet)[0]
        self.outlet_nodes = np.nonzero(outlet)[0]
        for name, t in zip(FACES, types):
            if t in ("inlet", "inlet_local") and name != "x-":
                raise ValueError("inlets are supported on the x- face only")
            if t == "outlet" and name != "x+":
                raise ValueError("outlets are supported on the x+ face only")
        # wall target temperature: first wall face touched in y-, y+, z-, z+, x-, x+
        T_tgt = np.full(self.N, np.nan)
        order = ("x+", "x-", "z+", "z-", "y+", "y-")   # later assignments win
        for name in order:
            f = self.faces[FACES.index(name)]
            if f["type"] == "wall":
                m = on[name]
                T_tgt[m] = f["T_lo"] + (f["T_hi"] - f["T_lo"]) * 0.5 * (
                    1.0 + np.tanh((self.x[m] - f["x0"]) / f["width"]))
        self.T_wall = T_tgt[self.wall_nodes]
        # neighbour indices for the gradient stencil (wrap or clamp per axis)
        self.nbr = np.zeros((Q, self.N), dtype=np.int64)
        for i in range(Q):
            q = []
            for ax in range(3):
                p = pos[ax] + C[i, ax]
                if self.periodic[ax]:
                    p = np.mod(p, n_ax[ax])
                else:
                    p = np.clip(p, 0, n_ax[ax] - 1)
                q.append(p)
            self.nbr[i] = (q[2] * ny + q[1]) * nx + q[0]
        # outlet: first interior neighbour along -x
        self.outlet_inner = self.outlet_nodes - 1
        self.inlet_face = self.faces[0] if types[0] in ("inlet", "inlet_local") else None
        self.outlet_face = self.faces[1] if types[1] == "outlet" else None

    # ------------------------------------------------------------------
    # state
    # ------------------------------------------------------------------
    def set_state(self, init):
        mech = self.mech
        rho = np.asarray(init["rho"], dtype=np.float64).copy()
        u = np.asarray(init["u"], dtype=np.float64).reshape(3, self.N).copy()
        T = np.asarray(init["T"], dtype=np.float64).copy()
        Y = np.asarray(init["Y"], dtype=np.float64).reshape(self.M, self.N).copy()
        Ra = gas_constants(mech)
        theta = mixture_R(mech, Y) * T
        U = (Y * U_species(mech, T)).sum(axis=0)
        self.fa = np.stack([species_eq(rho * Y[a], u, Ra[a] * T) for a in self.stored])
        self.f = mixture_eq(rho, u, theta)
        self.g = energy_eq(rho, u, theta, U)
        self.T = T.copy()
        # previous-step post-boundary moments (outlet LODI) and outlet state
        self.aux = {"rho": rho.copy(), "u": u.copy(), "T": T.copy(), "Y": Y.copy()}
        o = self.outlet_nodes
        self.out_state = {"rho": rho[o].copy(), "u": u[:, o].copy(), "T": T[o].copy(),
                          "Y": Y[:, o].copy()}
        self.time = 0

    def populations(self):
        """All stored populations, [L, 27, N], ordered: stored species in
        ascending species index, then f, then g (L = M + 1, or M + 2 in the
        weakly coupled storage)."""
        return np.concatenate([self.fa, self.f[None], self.g[None]], axis=0)

    def set_populations(self, pops):
        pops = np.asarray(pops, dtype=np.float64)
        ns = len(self.stored)
        self.fa = pops[:ns].copy()
        self.f = pops[ns].copy()
        self.g = pops[ns + 1].copy()

    # ------------------------------------------------------------------
    # step
    # ------------------------------------------------------------------
    def _stream(self, arr):
        """f_i(x) <- f_i(x - c_i) (eq. advection), periodic wrap."""
        shp = (self.nz, self.ny, self.nx)
        out = np.empty_like(arr)
        for i in range(Q):
            cx, cy, cz = C[i]
            out[..., i, :] = np.roll(arr[..., i, :].reshape(arr.shape[:-2] + shp),
                                     shift=(cz, cy, cx), axis=(-3, -2, -1)
                                     ).reshape(arr.shape[:-2] + (self.N,))
        return out

    def _grad(self, phi, axis):
        acc = 0.0
        for i in range(Q):
            if C[i, axis] != 0:
                acc = acc + W[i] * C[i, axis] * phi[self.nbr[i]]
        return 3.0 * acc

    def step(self, n=1):
        for _ in range(int(n)):
            self._step()

    def _step(self):
        mech, M, l = self.mech, self.M, self.l
        stored, s = self.stored, self.s
        fa_prev, f_prev, g_prev = self.fa, self.f, self.g
        # 1. advection
        fa = self._stream(fa_prev)
        f = self._stream(f_prev)
        g = self._stream(g_prev)
        # 2. boundaries
        w = self.wall_nodes
        if w.size:
            Dw = self.D[:, w]
            r = bc.tms_wall(mech, stored, s, Dw, fa[:, :, w], f[:, w], g[:, w],
                            fa_prev[:, :, w], f_prev[:, w], g_prev[:, w], OPP,
                            self.T_wall)
            fa[:, :, w], f[:, w], g[:, w] = r
        b = self.bb_nodes
        if b.size:
            r = bc.bounce_back_wall(self.D[:, b], fa[:, :, b], f[:, b], g[:, b],
                                    fa_prev[:, :, b], f_prev[:, b], g_prev[:, b], OPP)
            fa[:, :, b], f[:, b], g[:, b] = r
        k = self.inlet_nodes
        if k.size:
            fi = self.inlet_face
            inlet = bc.flux_inlet_local if fi["type"] == "inlet_local" else bc.flux_inlet
            r = inlet(mech, stored, s, self.D[:, k], fa[:, :, k], f[:, k],
                      g[:, k], fi["rho"], fi["u"], fi["T"], fi["Y"])
            fa[:, :, k], f[:, k], g[:, k] = r
        o = self.outlet_nodes
        if o.size:
            fo = self.outlet_face
            inner = {key: (v[..., self.outlet_inner]) for key, v in self.aux.items()}
            out = bc.lodi_outlet_state(mech, self.out_state, inner, fo["P_inf"],
                                       fo["sigma"], float(self.nx))
            r = bc.lodi_outlet(mech, stored, s, self.D[:, o], fa[:, :, o], f[:, o],
                               g[:, o], out)
            fa[:, :, o], f[:, o], g[:, o] = r
            self.out_state = out
        # 3. moments
        mo = bc.mixed_moments(mech, stored, s, fa, f, g, self.T)
        rho, u, rho_a, u_a, Y, U, T, rho_Y = (mo[k_] for k_ in
                                              ("rho", "u", "rho_a", "u_a", "Y", "U", "T", "rho_Y"))
        R = mixture_R(mech, Y)
        theta = R * T
        P = rho * theta
        Ra = gas_constants(mech)
        Pt = np.zeros((3, 3, self.N))
        for a_ in range(3):
            for b_ in range(3):
                Pt[a_, b_] = (f * (C[:, a_] * C[:, b_])[:, None]).sum(axis=0)
        q = np.stack([(g * C[:, d][:, None]).sum(axis=0) for d in range(3)])
        # 4. same-time gradients
        Phi = rho * u * (1.0 - 3.0 * theta) - rho * u ** 3
        d = np.stack([self._grad(Phi[a_], a_) for a_ in range(3)])
        G = np.stack([np.stack([self._grad(Y[a], ax) for ax in range(3)]) for a in range(M)])
        # 5. relaxation parameters and Stefan-Maxwell diffusion velocities
        itab = inv_tau_ab(mech, Y, T, P)
        beta, inv_tau = species_beta(mech, Y, itab)
        omega, omega1 = mixture_omegas(mech, T, P)
        V = stefan_maxwell(Y, itab, inv_tau, u_a, u)
        # 6. reactions
        drho = reaction_increment(mech, rho_a, rho_Y, U, T, l, self.reaction)
        # 7. species collision
        Wsp = [species_W(u, Ra[b] * T) for b in range(M)]
        feq_b = [rho_a[b] * Wsp[b] for b in range(M)]
        fstar_b = [species_eq(rho_a[b], u + V[b], Ra[b] * T) for b in range(M)]
        fa_new = np.empty_like(fa)
        for k_, a in enumerate(stored):
            F = np.zeros((Q, self.N))
            for b in range(M):
                if b != a:
                    F = F + itab[a, b] * (feq_b[b] - fstar_b[b])
            F = Y[a] * F
            fa_new[k_] = (fa[k_] + 2.0 * beta[a] * (feq_b[a] - fa[k_])
                          + (beta[a] - 1.0) * F + Wsp[a] * drho[a])
        # 8. momentum collision with the extended equilibrium
        Pex = theta + u ** 2 + (2.0 - omega) / (2.0 * rho * omega) * d
        f_new = f + omega * (extended_eq(rho, u, Pex) - f)
        # 9. energy collision
        Ha = H_species(mech, T)
        H = (Y * Ha).sum(axis=0)
        geq = energy_eq(rho, u, theta, U)
        qeq = rho * u * (H + 0.5 * (u ** 2).sum(axis=0))
        Peq = np.zeros((3, 3, self.N))
        for a_ in range(3):
            for b_ in range(3):
                Peq[a_, b_] = rho * ((theta if a_ == b_ else 0.0) + u[a_] * u[b_])
        uP = np.stack([sum(u[b_] * (Pt[b_, a_] - Peq[b_, a_]) for b_ in range(3))
                       for a_ in range(3)])
        qex = -0.5 * u * d
        diff = sum(Ha[a] * Y[a] * V[a] for a in range(M))
        corr = sum(Ha[a] * G[a] for a in range(M))
        Qv = ((omega - omega1) * (q - uP + qex - qeq) + omega1 * rho * diff
              + 0.5 * (2.0 - omega1) * P * corr)
        g_new = g + omega * (geq - g)
        for i in range(Q):
            if C2[i] == 1:
                g_new[i] = g_new[i] + 0.5 * (C[i, 0] * Qv[0] + C[i, 1] * Qv[1]
                                             + C[i, 2] * Qv[2])
        self.fa, self.f, self.g = fa_new, f_new, g_new
        self.T = T
        self.aux = {"rho": rho, "u": u, "T": T, "Y": Y}
        self.time += 1
        self.last = {"rho": rho, "u": u, "u_a": u_a, "T": T, "Y": Y, "P": P, "V": V,
                     "d": d, "G": G, "drho": drho, "beta": beta, "omega": omega,
                     "omega1": omega1, "itab": itab, "inv_tau": inv_tau, "U": U}

    # ------------------------------------------------------------------
    # read-out
    # ------------------------------------------------------------------
    def fields(self):
        """Macroscopic fields of the stored (post-collision) populations:
        rho, u [3,N], T, Y [M,N], P."""
        mo = bc.mixed_moments(self.mech, self.stored, self.s, self.fa, self.f, self.g,
                              self.T)
        P = mo["rho"] * mixture_R(self.mech, mo["Y"]) * mo["T"]
        return {"rho": mo["rho"], "u": mo["u"], "T": mo["T"], "Y": mo["Y"], "P": P}

    def invariants(self):
        """sum rho, sum rho u (3), sum rho E, element totals (moles), and a
        non-finite flag."""
        rho = self.f.sum(axis=0)
        j = [(self.f * C[:, k][:, None]).sum(axis=0).sum() for k in range(3)]
        rhoE = self.g.sum()
        m = np.asarray(self.mech["molar_mass"], dtype=np.float64)
        comp = np.asarray(self.mech["composition"], dtype=np.float64)
        rho_a = np.zeros((self.M, self.N))
        for k, a in enumerate(self.stored):
            rho_a[a] = self.fa[k].sum(axis=0)
        if self.s is not None:
            rho_a[self.s] = rho - rho_a.sum(axis=0)
        elem = ((rho_a / m[:, None]).sum(axis=1)[:, None] * comp).sum(axis=0)
        bad = not (np.isfinite(self.fa).all() and np.isfinite(self.f).all()
                   and np.isfinite(self.g).all())
        return np.array([rho.sum(), *j, rhoE, *elem, float(bad)])
