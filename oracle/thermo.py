"""Species thermochemistry and the temperature equation (paper section 3.1).

Species data are one-range NASA-7 polynomials (the usual input form of a
kinetics package; the paper takes them from one).  With R_a = R_U / m_a:

    C_{a,p}(T) = R_a (a0 + a1 T + a2 T^2 + a3 T^3 + a4 T^4)
    H_a(T)     = R_a (a0 T + a1 T^2/2 + a2 T^3/3 + a3 T^4/4 + a4 T^5/5 + a5)
    U_a(T)     = H_a(T) - R_a T                 (Mayer relation, C_p - C_v = R_a)
    S_a(T)/R_a = a0 ln T + a1 T + a2 T^2/2 + a3 T^3/3 + a4 T^4/4 + a6

so U_a(T) = U_a^0 + int_{T0}^{T} C_{a,v} dT' (eq. specUa) and likewise for H_a
(eq. specHa); the formation energy U_a^0 = U_a(T0) is carried by a5.
"""
import numpy as np


def _coef(mech):
    return np.asarray(mech["nasa"], dtype=np.float64)          # [M, 7]


def gas_constants(mech):
    return mech["R_univ"] / np.asarray(mech["molar_mass"], dtype=np.float64)


def cp_species(mech, T):
    a = _coef(mech)[:, :, None]
    R = gas_constants(mech)[:, None]
    return R * (a[:, 0] + a[:, 1] * T + a[:, 2] * T ** 2 + a[:, 3] * T ** 3 + a[:, 4] * T ** 4)


def cv_species(mech, T):
    return cp_species(mech, T) - gas_constants(mech)[:, None]


def H_species(mech, T):
    """Specific enthalpy H_a(T), eq. specHa.  Returns [M, N]."""
    a = _coef(mech)[:, :, None]
    R = gas_constants(mech)[:, None]
    return R * (a[:, 0] * T + a[:, 1] * T ** 2 / 2 + a[:, 2] * T ** 3 / 3
                + a[:, 3] * T ** 4 / 4 + a[:, 4] * T ** 5 / 5 + a[:, 5])


def U_species(mech, T):
    """Specific internal energy U_a(T), eq. specUa.  Returns [M, N]."""
    return H_species(mech, T) - gas_constants(mech)[:, None] * T


def gibbs_RT(mech, T):
    """Dimensionless molar Gibbs energy g_a/(R_U T) = h/(R T) - s/R, [M, N]."""
    a = _coef(mech)[:, :, None]
    h = (a[:, 0] + a[:, 1] * T / 2 + a[:, 2] * T ** 2 / 3 + a[:, 3] * T ** 3 / 4
         + a[:, 4] * T ** 4 / 5 + a[:, 5] / T)
    s = (a[:, 0] * np.log(T) + a[:, 1] * T + a[:, 2] * T ** 2 / 2 + a[:, 3] * T ** 3 / 3
         + a[:, 4] * T ** 4 / 4 + a[:, 6])
    return h - s


def mixture_R(mech, Y):
    """R = R_U / m with 1/m = sum_a Y_a / m_a (section 2.1)."""
    m = np.asarray(mech["molar_mass"], dtype=np.float64)[:, None]
    return mech["R_univ"] * (Y / m).sum(axis=0)


def solve_temperature(mech, Y, U, T_guess, rtol=1e-12, max_iter=100):
    """Solve sum_a Y_a U_a(T) = U for T (eq. temperature) by Newton's method,
    starting from T_guess, until |dT| <= rtol * T.  Raises if it does not
    converge."""
    T = np.array(T_guess, dtype=np.float64, copy=True)
    for _ in range(max_iter):
        F = (Y * U_species(mech, T)).sum(axis=0) - U
        dF = (Y * cv_species(mech, T)).sum(axis=0)
        dT = F / dF
        T = T - dT
        if np.all(np.abs(dT) <= rtol * np.abs(T)):
            return T
    raise RuntimeError("temperature Newton iteration did not converge")
