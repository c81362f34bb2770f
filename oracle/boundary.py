"""Boundary conditions at interface nodes (paper section 4).

Notation of section 4.1: D is the set of incoming velocities at an interface
node (populations whose pre-advection source lies outside the domain through
a non-periodic face).  All three constructions share one pattern: build an
equilibrium from imposed data, mix it into the incoming links to obtain a
"local" state, and combine equilibria so that the node's moments equal the
imposed values.

Stored lattices are the M-1 unslaved species, the momentum lattice f and the
energy lattice g; the slaved species (eq. strongest) is implied by
f - sum_a f_a and is not reconstructed separately.  In the weakly coupled
storage (slaved = None) all M species are stored and reconstructed, and the
composition of a population set is Y_a = rho_a / sum_b rho_b.

Readings where the paper is silent:
  * A node touching several non-periodic faces takes the union of their
    incoming links; a node touching any wall face is a wall node (walls take
    precedence over the inlet and the outlet; Tamm-Mott-Smith walls over
    bounce-back walls).
  * The simplified inlet ("apply the local equilibria") sets every
    population of the inlet node, incoming and outgoing, to the local
    equilibria.
  * Aligned walls take the target temperature at the node's own x position,
    T^tgt = T_w(x) (the ramp is tanh-shaped, centred at x0, width w), and
    u^tgt = u_a^tgt = 0 (stationary impermeable wall).
  * Local species velocities are replaced by the local mixture velocity when a
    species density is below 1e-14 of the mixture density.
  * LODI (outlet): the single-component Poinsot-Lele relations, one-sided in
    x, with a partially non-reflecting incoming wave L1 = K (P - P_inf),
    K = sigma (1 - Ma^2) c / L_x, explicit in time from the previous step's
    outlet state and the previous step's post-boundary moments at the first
    interior node.  The composition follows eq. convectiveBC with the
    backward difference along the outlet normal.
"""
import numpy as np

from .equilibria import energy_eq, mixture_eq, species_eq
from .lattice import C
from .thermo import (U_species, cv_species, gas_constants, mixture_R,
                     solve_temperature)

RHO_GUARD = 1e-14


def mixed_moments(mech, stored, slaved, fa, f, g, T_guess):
    """Moments of a population set (eqs. density1, momentum1, fdensity,
    f1momMomentum, g0momTotalEnergy) and the temperature (eq. temperature).
    fa: [len(stored), 27, n] stored species.  Returns rho [n], u [3, n],
    rho_a [M, n], u_a [M, 3, n], Y [M, n], U [n], T [n] and rho_Y [n], the
    density that normalises Y (rho when a species is slaved, sum_a rho_a in
    the weakly coupled storage, slaved = None)."""
    M = mech["M"]
    rho = f.sum(axis=0)
    j = np.stack([(f * C[:, k][:, None]).sum(axis=0) for k in range(3)])
    u = j / rho
    n = rho.shape[0]
    rho_a = np.zeros((M, n))
    j_a = np.zeros((M, 3, n))
    for k, a in enumerate(stored):
        rho_a[a] = fa[k].sum(axis=0)
        for d in range(3):
            j_a[a, d] = (fa[k] * C[:, d][:, None]).sum(axis=0)
    if slaved is None:
        rho_Y = rho_a.sum(axis=0)
    else:
        rho_a[slaved] = rho - sum(rho_a[a] for a in stored)
        j_a[slaved] = j - sum(j_a[a] for a in stored)
        rho_Y = rho
    Y = rho_a / rho_Y
    u_a = np.empty_like(j_a)
    for a in range(M):
        small = rho_a[a] <= RHO_GUARD * rho
        safe = np.where(small, 1.0, rho_a[a])
        u_a[a] = np.where(small, u, j_a[a] / safe)
    rhoE = g.sum(axis=0)
    U = rhoE / rho - 0.5 * (u ** 2).sum(axis=0)
    T = solve_temperature(mech, Y, U, T_guess)
    return {"rho": rho, "u": u, "rho_a": rho_a, "u_a": u_a, "Y": Y, "U": U, "T": T,
            "rho_Y": rho_Y}


def equilibria_set(mech, stored, rho, Y, u, T, u_species=None):
    """(f^eq, g^eq, f_a^eq) at (rho, Y, u, T) (eqs. faEqGeneral, fEqGeneral,
    gEqGeneral).  Species use u_species[a] if given, else the mixture u."""
    R = mixture_R(mech, Y)
    theta = R * T
    Ra = gas_constants(mech)
    U = (Y * U_species(mech, T)).sum(axis=0)
    feq = mixture_eq(rho, u, theta)
    geq = energy_eq(rho, u, theta, U)
    faeq = np.stack([species_eq(rho * Y[a], u if u_species is None else u_species[a],
                                Ra[a] * T) for a in stored])
    return feq, geq, faeq


def _mix(D, inc, out):
    return np.where(D, inc, out)


def tms_wall(mech, stored, slaved, D, fa, f, g, fa_prev, f_prev, g_prev, opp,
             T_tgt):
    """Tamm-Mott-Smith isothermal wall (section 4.2.2, eqs. BBrho, BBY,
    tgtf/tgtg/tgtfa, locRho..locT, ftms, gtms, fatms).  Arrays are restricted
    to the wall nodes; *_prev are the pre-advection populations at the same
    nodes (bounce-back source, eq. bb)."""
    M = mech["M"]
    n = f.shape[1]
    # step 1: bounce-back density and mass fractions
    f_bb = _mix(D, f_prev[opp], f)
    fa_bb = np.stack([_mix(D, fa_prev[k][opp], fa[k]) for k in range(len(stored))])
    rho_bb = f_bb.sum(axis=0)
    rhoY = np.zeros((M, n))
    for k, a in enumerate(stored):
        rhoY[a] = fa_bb[k].sum(axis=0)
    if slaved is None:
        Y_bb = rhoY / rhoY.sum(axis=0)
    else:
        rhoY[slaved] = rho_bb - sum(rhoY[a] for a in stored)
        Y_bb = rhoY / rho_bb
    # step 2: target equilibria with u^tgt = u_a^tgt = 0, T^tgt
    u0 = np.zeros((3, n))
    f_t, g_t, fa_t = equilibria_set(mech, stored, rho_bb, Y_bb, u0, T_tgt)
    # step 3: local state with incoming links at the target
    loc = mixed_moments(mech, stored, slaved, _mix(D, fa_t, fa), _mix(D, f_t, f),
                        _mix(D, g_t, g), T_tgt)
    f_l, g_l, fa_l = equilibria_set(mech, stored, loc["rho"], loc["Y"], loc["u"],
                                    loc["T"], u_species=loc["u_a"])
    # step 4
    f_new = np.where(D, 2 * f_t - f_l, f_t + f - f_l)
    g_new = np.where(D, 2 * g_t - g_l, g_t + g - g_l)
    fa_new = np.where(D[None], 2 * fa_t - fa_l, fa_t + fa - fa_l)
    return fa_new, f_new, g_new


def bounce_back_wall(D, fa, f, g, fa_prev, f_prev, g_prev, opp):
    """Bounce-back wall (section 4.2.1, eq. bb): every incoming population of
    every stored lattice takes the pre-advection value of the opposite
    velocity at the same node.  No slip half-way between the interface node
    and the wall on the momentum lattice, zero heat flux (adiabatic) on the
    energy lattice; nothing is imposed."""
    fa_new = np.where(D[None], fa_prev[:, opp], fa)
    f_new = np.where(D, f_prev[opp], f)
    g_new = np.where(D, g_prev[opp], g)
    return fa_new, f_new, g_new


def flux_inlet(mech, stored, slaved, D, fa, f, g, rho_in, u_in, T_in, Y_in):
    """Flux inlet (section 4.3, eqs. in_f..in_fa, inletlocRho..inletlocT,
    in_loc_*, in_tgt_*, f_inlet, g_inlet, fa_inlet)."""
    n = f.shape[1]
    ones = np.ones(n)
    uin = np.stack([u_in * ones, 0 * ones, 0 * ones])
    Yin = np.asarray(Y_in, dtype=np.float64)[:, None] * ones
    f_i, g_i, fa_i = equilibria_set(mech, stored, rho_in * ones, Yin, uin, T_in * ones)
    loc = mixed_moments(mech, stored, slaved, _mix(D, fa_i, fa), _mix(D, f_i, f),
                        _mix(D, g_i, g), T_in * ones)
    f_l, g_l, fa_l = equilibria_set(mech, stored, loc["rho"], loc["Y"], loc["u"], loc["T"])
    f_t, g_t, fa_t = equilibria_set(mech, stored, loc["rho"], loc["Y"], uin, T_in * ones)
    f_new = np.where(D, f_t + f_i - f_l, f_t + f - f_l)
    g_new = np.where(D, g_t + g_i - g_l, g_t + g - g_l)
    fa_new = np.where(D[None], fa_t + fa_i - fa_l, fa_t + fa - fa_l)
    return fa_new, f_new, g_new


def flux_inlet_local(mech, stored, slaved, D, fa, f, g, rho_in, u_in, T_in, Y_in):
    """Simplified flux inlet (section 4.3, closing remarks): the construction
    stops at the local state of step 2 (incoming links at the inlet
    equilibrium, eqs. inletlocRho..inletlocT) and every population of the
    node takes the local equilibria (eqs. in_loc_f, in_loc_g, in_loc_fa), so
    velocity and temperature keep their local values instead of u^in, T^in."""
    n = f.shape[1]
    ones = np.ones(n)
    uin = np.stack([u_in * ones, 0 * ones, 0 * ones])
    Yin = np.asarray(Y_in, dtype=np.float64)[:, None] * ones
    f_i, g_i, fa_i = equilibria_set(mech, stored, rho_in * ones, Yin, uin, T_in * ones)
    loc = mixed_moments(mech, stored, slaved, _mix(D, fa_i, fa), _mix(D, f_i, f),
                        _mix(D, g_i, g), T_in * ones)
    f_l, g_l, fa_l = equilibria_set(mech, stored, loc["rho"], loc["Y"], loc["u"], loc["T"])
    return fa_l, f_l, g_l


def lodi_outlet_state(mech, prev, inner, P_inf, sigma, Lx):
    """Outlet state (rho, u, T, Y) at time t from the outlet state at t-1
    (`prev`) and the post-boundary moments at t-1 of the first interior node
    (`inner`); see the module docstring for the LODI reading and
    eq. convectiveBC for the composition."""
    rho0, u0, T0, Y0 = prev["rho"], prev["u"], prev["T"], prev["Y"]
    rho1, u1, T1, Y1 = inner["rho"], inner["u"], inner["T"], inner["Y"]
    R0 = mixture_R(mech, Y0)
    P0 = rho0 * R0 * T0
    P1 = rho1 * mixture_R(mech, Y1) * T1
    Cv = (Y0 * cv_species(mech, T0)).sum(axis=0)
    gamma = (Cv + R0) / Cv
    c = np.sqrt(gamma * P0 / rho0)
    un = u0[0]
    d_rho = rho0 - rho1
    d_P = P0 - P1
    d_u = u0 - u1
    Ma = un / c
    L1 = sigma * (1.0 - Ma ** 2) * c / Lx * (P0 - P_inf)
    L2 = un * (c ** 2 * d_rho - d_P)
    L3 = un * d_u[1]
    L4 = un * d_u[2]
    L5 = (un + c) * (d_P + rho0 * c * d_u[0])
    rho_o = rho0 - (L2 + 0.5 * (L5 + L1)) / c ** 2
    P_o = P0 - 0.5 * (L5 + L1)
    u_o = np.stack([un - (L5 - L1) / (2.0 * rho0 * c), u0[1] - L3, u0[2] - L4])
    Y_o = Y0 - un * (Y0 - Y1)
    T_o = P_o / (rho_o * mixture_R(mech, Y_o))
    return {"rho": rho_o, "u": u_o, "T": T_o, "Y": Y_o}


def lodi_outlet(mech, stored, slaved, D, fa, f, g, out):
    """Outlet populations (section 4.4, eqs. out_f..out_fa,
    outletlocRho..outletlocT, f_outlet, g_outlet, fa_outlet)."""
    f_o, g_o, fa_o = equilibria_set(mech, stored, out["rho"], out["Y"], out["u"], out["T"])
    loc = mixed_moments(mech, stored, slaved, _mix(D, fa_o, fa), _mix(D, f_o, f),
                        _mix(D, g_o, g), out["T"])
    f_l, g_l, fa_l = equilibria_set(mech, stored, loc["rho"], loc["Y"], loc["u"], loc["T"])
    f_new = np.where(D, 2 * f_o - f_l, f_o + f - f_l)
    g_new = np.where(D, 2 * g_o - g_l, g_o + g - g_l)
    fa_new = np.where(D[None], 2 * fa_o - fa_l, fa_o + fa - fa_l)
    return fa_new, f_new, g_new
