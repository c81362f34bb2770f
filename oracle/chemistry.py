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


def reaction_increment(mech, rho_a, rho, U, T, substeps):
    """Delta rho_a over one lattice time step by l forward-Euler sub-steps at
    frozen U (eq. R3).  T is the temperature at the start of the step."""
    cur = rho_a.copy()
    Tcur = T.copy()
    for s in range(substeps):
        if s > 0:
            Tcur = solve_temperature(mech, cur / rho, U, Tcur)
        cur = cur + production_rates(mech, cur, Tcur) / substeps
    return cur - rho_a
