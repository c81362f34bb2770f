"""Relaxation times and parameters (paper sections 2.3 and 3.4).

The paper obtains mu, lambda and the Stefan-Maxwell diffusivities D_ab from a
kinetics package.  Here they follow the synthetic power laws carried by the
mechanism's "transport" block:

    mu     = mu_ref (T/T_ref)^mu_exp,        lambda = mu C_p / Pr
    D_ab   = D_ref[a][b] (T/T_ref)^D_exp (P_ref / P)

Reading of eq. taua's companion (the characteristic time tau_ab): the paper
prints tau_ab = m R_U T / (D_ab m_a m_b), which has units of inverse time and
contradicts the kinetic equation (eq. stefanMaxwell), whose relaxation
coefficient P X_a X_b / (D_ab rho_a) equals Y_b m R_U T / (D_ab m_a m_b).  The
consistent reading, used here, is

    1/tau_ab = m R_U T / (D_ab m_a m_b),     1/tau_a = sum_{b != a} Y_b / tau_ab.
"""
import numpy as np

from .thermo import mixture_R


def inv_tau_ab(mech, Y, T, P):
    """1/tau_ab for all pairs, [M, M, N] (diagonal left at zero)."""
    tr = mech["transport"]
    m = np.asarray(mech["molar_mass"], dtype=np.float64)
    M = len(m)
    D_ref = np.asarray(tr["D_ref"], dtype=np.float64)
    inv_m = (Y / m[:, None]).sum(axis=0)                  # 1/m (mixture)
    scale = (T / tr["T_ref"]) ** tr["D_exp"] * (tr["P_ref"] / P)
    out = np.zeros((M, M) + np.shape(T))
    for a in range(M):
        for b in range(M):
            if a == b:
                continue
            D_ab = D_ref[a, b] * scale
            out[a, b] = (1.0 / inv_m) * mech["R_univ"] * T / (D_ab * m[a] * m[b])
    return out


def species_beta(mech, Y, itab):
    """beta_a = dt/(2 tau_a + dt) with dt = 1 (eqs. betaa, taua).  [M, N]."""
    M = Y.shape[0]
    inv_tau = np.zeros_like(Y)
    for a in range(M):
        for b in range(M):
            if b != a:
                inv_tau[a] += Y[b] * itab[a, b]
    tau = 1.0 / inv_tau
    return 1.0 / (2.0 * tau + 1.0), inv_tau


def mixture_omegas(mech, T, P):
    """omega from mu = (1/omega - 1/2) P dt (eq. mu) and omega_1 from
    lambda = (1/omega_1 - 1/2) P C_p dt (eq. lambda) with lambda = mu C_p/Pr."""
    tr = mech["transport"]
    mu = tr["mu_ref"] * (T / tr["T_ref"]) ** tr["mu_exp"]
    omega = 1.0 / (mu / P + 0.5)
    omega1 = 1.0 / (mu / (tr["Pr"] * P) + 0.5)
    return omega, omega1


def mixture_pressure(mech, rho, Y, T):
    return rho * mixture_R(mech, Y) * T


def stefan_maxwell(Y, itab, inv_tau, u_a, u):
    """Diffusion velocities V_a from eq. transform1 (dt = 1), for each
    Cartesian component:
        (1 + 1/(2 tau_a)) V_a - (1/2) sum_{b != a} Y_b V_b / tau_ab = u_a - u.
    Y [M,N], itab [M,M,N], inv_tau [M,N], u_a [M,3,N], u [3,N] -> V [M,3,N].
    Solved with numpy's LU (partial pivoting)."""
    M, N = Y.shape
    A = np.zeros((N, M, M))
    for a in range(M):
        A[:, a, a] = 1.0 + 0.5 * inv_tau[a]
        for b in range(M):
            if b != a:
                A[:, a, b] = -0.5 * Y[b] * itab[a, b]
    V = np.zeros((M, 3, N))
    for ax in range(3):
        rhs = np.stack([u_a[a, ax] - u[ax] for a in range(M)], axis=1)   # [N, M]
        V[:, ax] = np.linalg.solve(A, rhs[..., None])[..., 0].T
    return V
