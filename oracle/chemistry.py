"""Mass-action reaction sources and the explicit sub-steps (paper section 2.3).

The paper takes the production rates rho_dot_a^r(U, rho_1..rho_M) from a
kinetics package.  Here they are the textbook mass-action law for the seeded
mechanism (all quantities in lattice units, T in kelvin):

    c_b   = max(rho_b, 0) / m_b                         (molar concentrations)
    k_f   = A T^beta exp(-T_a / T)
    K_c   = exp(-sum_a dnu_a g_a/(R_U T)) (c_std)^(sum_a dnu_a),
            c_std = P_atm / (R_U T)
    q_r   = k_f prod_b c_b^nu'_b - [reversible] (k_f / K_c) prod_b c_b^nu''_b
    rho_dot_a = m_a sum_r (nu''_ar - nu'_ar) q_r

Concentrations are clipped at zero inside the rate law only; stored densities
are never clipped.

Sub-steps (eq. R3): with dt^r = dt / l, the densities are advanced by forward
Euler l times at frozen specific internal energy U; the temperature is
re-solved from (U, Y) before every sub-step after the first.  The node update
uses Delta rho_a = rho_a^(l) - rho_a^(0).

Linearly implicit variant (not in the paper, which only offers smaller
sub-steps against stiffness): each sub-step solves
    (I - dt^r J) Delta = dt^r rho_dot(rho^(s), T_s),   rho^(s+1) = rho^(s) + Delta,
with J_ab = d rho_dot_a / d rho_b the Jacobian of the mass-action law at the
sub-step's temperature.  Readings: J holds T fixed (the change of T with
composition at frozen U is left out of J and picked up by the re-solve before
the next sub-step); the clip max(c, 0) is differentiated as the identity.
Since every column of J sums to zero (mass) and is orthogonal to the element
vectors, the update conserves mass and elements exactly like eq. R3; for a
linear network it is backward Euler.
"""
import numpy as np

from .thermo import gibbs_RT, solve_temperature


def production_rates(mech, rho_a, T):
    """rho_dot_a for all species, [M, N]."""
    m = np.asarray(mech["molar_mass"], dtype=np.float64)[:, None]
    M = rho_a.shape[0]
    conc = np.maximum(rho_a, 0.0) / m
    out = np.zeros_like(rho_a)
    R = len(mech["lnA"])
    if R == 0:
        return out
    gRT = gibbs_RT(mech, T)
    lnT = np.log(T)
    for r in range(R):
        nu_f = np.asarray(mech["nu_f"][r])
        nu_r = np.asarray(mech["nu_r"][r])
        kf = np.exp(mech["lnA"][r] + mech["beta"][r] * lnT - mech["Ta"][r] / T)
        fwd = kf.copy()
        for b in range(M):
            for _ in range(int(nu_f[b])):
                fwd = fwd * conc[b]
        q = fwd
        if mech["reversible"][r]:
            dnu = nu_r - nu_f
            lnKc = -(dnu[:, None] * gRT).sum(axis=0) + dnu.sum() * (mech["ln_cstd"] - lnT)
            rev = kf / np.exp(lnKc)
            for b in range(M):
                for _ in range(int(nu_r[b])):
                    rev = rev * conc[b]
            q = fwd - rev
        for a in range(M):
            d = int(nu_r[a]) - int(nu_f[a])
            if d != 0:
                out[a] += m[a] * d * q
    return out


def rate_jacobian(mech, rho_a, T):
    """J[a, b, n] = d rho_dot_a / d rho_b at fixed T (power rule on each
    mass-action product), [M, M, N]."""
    m = np.asarray(mech["molar_mass"], dtype=np.float64)
    M, N = rho_a.shape
    conc = np.maximum(rho_a, 0.0) / m[:, None]
    J = np.zeros((M, M, N))
    R = len(mech["lnA"])
    if R == 0:
        return J
    gRT = gibbs_RT(mech, T)
    lnT = np.log(T)

    def d_product(nu, b):
        """d/dc_b of prod_d c_d^nu_d."""
        if nu[b] == 0:
            return np.zeros(N)
        out = nu[b] * conc[b] ** (nu[b] - 1)
        for d in range(M):
            if d != b and nu[d] > 0:
                out = out * conc[d] ** nu[d]
        return out

    for r in range(R):
        nu_f = np.asarray(mech["nu_f"][r], dtype=np.int64)
        nu_r = np.asarray(mech["nu_r"][r], dtype=np.int64)
        kf = np.exp(mech["lnA"][r] + mech["beta"][r] * lnT - mech["Ta"][r] / T)
        kr = None
        if mech["reversible"][r]:
            dnu = nu_r - nu_f
            lnKc = -(dnu[:, None] * gRT).sum(axis=0) + dnu.sum() * (mech["ln_cstd"] - lnT)
            kr = kf / np.exp(lnKc)
        for b in range(M):
            dq = kf * d_product(nu_f, b)
            if kr is not None:
                dq = dq - kr * d_product(nu_r, b)
            dq = dq / m[b]                     # dc_b / drho_b = 1 / m_b
            for a in range(M):
                dn = int(nu_r[a]) - int(nu_f[a])
                if dn != 0:
                    J[a, b] += m[a] * dn * dq
    return J


def linearly_implicit_substep(mech, rho_a, T, h):
    """Delta of one linearly implicit sub-step of length h: solve
    (I - h J) Delta = h rho_dot at every node."""
    M, N = rho_a.shape
    w = production_rates(mech, rho_a, T)
    J = rate_jacobian(mech, rho_a, T)
    A = np.eye(M)[None, :, :] - h * np.moveaxis(J, 2, 0)        # [N, M, M]
    return np.linalg.solve(A, (h * w).T[:, :, None])[:, :, 0].T


def reaction_increment(mech, rho_a, rho, U, T, substeps, scheme="explicit"):
    """Delta rho_a over one lattice time step by l sub-steps at frozen U:
    forward Euler (eq. R3) or the linearly implicit variant.  T is the
    temperature at the start of the step; rho normalises the composition,
    Y = rho_a / rho, in the temperature solves between sub-steps."""
    if scheme not in ("explicit", "implicit"):
        raise ValueError("unknown reaction scheme %r" % (scheme,))
    cur = rho_a.copy()
    Tcur = T.copy()
    for s in range(substeps):
        if s > 0:
            Tcur = solve_temperature(mech, cur / rho, U, Tcur)
        if scheme == "explicit":
            cur = cur + production_rates(mech, cur, Tcur) / substeps
        else:
            cur = cur + linearly_implicit_substep(mech, cur, Tcur, 1.0 / substeps)
    return cur - rho_a
