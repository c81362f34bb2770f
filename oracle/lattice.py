"""D3Q27 velocity set and product-form factors (paper section 2.2).

Velocity ordering (an interface convention shared with the library's
population read/write calls): i = 9 (c_z + 1) + 3 (c_y + 1) + (c_x + 1), so
the rest velocity is i = 13 and the opposite of i is 26 - i.
"""
import numpy as np

Q = 27

C = np.array([[cx, cy, cz]
              for cz in (-1, 0, 1) for cy in (-1, 0, 1) for cx in (-1, 0, 1)],
             dtype=np.int64)                      # eq. d3q27vel
OPP = np.array([int(np.where((C == -C[i]).all(axis=1))[0][0]) for i in range(Q)])
C2 = (C ** 2).sum(axis=1)                         # |c_i|^2

# Lattice weights used by the isotropic gradient (the product of the 1D
# weights 2/3 for c = 0 and 1/6 for c = +-1); also the zero-velocity
# equilibrium at theta = 1/3.
_W1 = {0: 2.0 / 3.0, 1: 1.0 / 6.0, -1: 1.0 / 6.0}
W = np.array([_W1[cx] * _W1[cy] * _W1[cz] for cx, cy, cz in C])


def psi(c, xi, P):
    """One-dimensional factor Psi_c(xi, P) of eqs. phi0, phiPlus, phis:
    Psi_0 = 1 - P, Psi_{+1} = (xi + P)/2, Psi_{-1} = (-xi + P)/2."""
    if c == 0:
        return 1.0 - P
    if c == 1:
        return 0.5 * (xi + P)
    return 0.5 * (-xi + P)


def product_form(xi, P):
    """Psi_i of eq. prod for all 27 velocities.

    xi, P: arrays [3, ...] (components x, y, z).  Returns [27, ...]."""
    out = []
    for i in range(Q):
        cx, cy, cz = C[i]
        out.append(psi(cx, xi[0], P[0]) * psi(cy, xi[1], P[1]) * psi(cz, xi[2], P[2]))
    return np.stack(out)
