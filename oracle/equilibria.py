"""Equilibria and quasi-equilibria (paper sections 2.2, 3.2 and 3.3).

Species (eqs. 27eq, 27qeq with the parameters of eq. xiPstar2):
    f_ai^eq = rho_a Psi_i(u, u^2 + R_a T)
    f_bi^*  = rho_b Psi_i(u + V_b, (u + V_b)^2 + R_b T)
Momentum lattice (eqs. feq, feqmix, Peq):
    f_i^eq  = rho Psi_i(u, u^2 + R T),   f_i^ex = rho Psi_i(u, P^ex)
Energy lattice (eqs. oalpha, Oa, OaOa, geq_i): the product form with the
operator symbols xi_a = O_a, P_aa = O_a^2, O_a A = R T dA/du_a + u_a A, applied
to the generating function E(u) = U + u^2/2 at fixed temperature.  The
operator algebra is carried out literally on polynomials in (u_x, u_y, u_z)
whose coefficients are node arrays, then evaluated at the node velocity.
Quasi-equilibrium (eq. gstar): g_i^* = g_i^eq + (1/2) c_i . (q^* - q^eq) on the
six links with |c_i|^2 = 1, g_i^eq elsewhere.
"""
import numpy as np

from .lattice import C, C2, Q, product_form


def species_W(u, theta_a):
    """W_ai = Psi_i(u, u^2 + theta_a): the species equilibrium per unit
    density (and the shape of the reaction source, eq. fsource)."""
    return product_form(u, u ** 2 + theta_a)


def species_eq(rho_a, u, theta_a):
    return rho_a * species_W(u, theta_a)


def mixture_eq(rho, u, theta):
    return rho * product_form(u, u ** 2 + theta)


def extended_eq(rho, u, Pex):
    return rho * product_form(u, Pex)


# --- energy equilibrium by the operator product form -----------------------
def _poly_add(p, q, scale=1.0):
    out = dict(p)
    for k, v in q.items():
        out[k] = out[k] + scale * v if k in out else scale * v
    return out


def _poly_scale(p, s):
    return {k: s * v for k, v in p.items()}


def _op(p, axis, theta):
    """O_axis A = theta dA/du_axis + u_axis A on a polynomial A."""
    out = {}
    for powers, coef in p.items():
        n = powers[axis]
        if n > 0:
            k = list(powers)
            k[axis] -= 1
            k = tuple(k)
            term = theta * coef * n
            out[k] = out[k] + term if k in out else term
        k = list(powers)
        k[axis] += 1
        k = tuple(k)
        out[k] = out[k] + coef if k in out else coef
    return out


def _psi_op(c, p, axis, theta):
    """Psi_c(O, O^2) applied to p: Psi_0 = 1 - O^2, Psi_{+-1} = (+-O + O^2)/2."""
    o1 = _op(p, axis, theta)
    o2 = _op(o1, axis, theta)
    if c == 0:
        return _poly_add(p, o2, -1.0)
    sign = 1.0 if c == 1 else -1.0
    return _poly_scale(_poly_add(_poly_scale(o1, sign), o2), 0.5)


def _poly_eval(p, pw):
    """Evaluate p at the node velocity; pw[axis][k] = u_axis^k."""
    val = 0.0
    for (px, py, pz), coef in p.items():
        val = val + coef * pw[0][px] * pw[1][py] * pw[2][pz]
    return val


def energy_eq(rho, u, theta, U):
    """g_i^eq = rho Psi_cx(O_x,O_x^2) Psi_cy(O_y,O_y^2) Psi_cz(O_z,O_z^2) E,
    E = U + (u_x^2 + u_y^2 + u_z^2)/2 (eqs. geq_i, totalE).  [27, N]."""
    ones = np.ones_like(theta)
    E = {(0, 0, 0): U * ones, (2, 0, 0): 0.5 * ones, (0, 2, 0): 0.5 * ones,
         (0, 0, 2): 0.5 * ones}
    pw = []
    for ax in range(3):
        powers = [ones]
        for _ in range(8):
            powers.append(powers[-1] * u[ax])
        pw.append(powers)
    out = []
    for i in range(Q):
        cx, cy, cz = C[i]
        p = _psi_op(cz, E, 2, theta)
        p = _psi_op(cy, p, 1, theta)
        p = _psi_op(cx, p, 0, theta)
        out.append(rho * _poly_eval(p, pw))
    return np.stack(out)


def energy_quasi_eq(geq, dq):
    """g^* of eq. gstar given dq = q^* - q^eq ([3, N])."""
    gs = geq.copy()
    for i in range(Q):
        if C2[i] == 1:
            gs[i] = gs[i] + 0.5 * (C[i, 0] * dq[0] + C[i, 1] * dq[1] + C[i, 2] * dq[2])
    return gs
