"""Plain FP64 CPU oracle for the reactive-mixture lattice Boltzmann step.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path imports, calls or
executes this package; only the test-suite, the smoke check and the CPU
baseline leg of the benchmark use it.  It shares no code with the HIP
library: both consume the same seeded inputs (the workload generator, which
holds none of the method's arithmetic) and nothing else.

The oracle follows Sawant, Dorschner & Karlin, "Consistent lattice Boltzmann
model for reactive mixtures" (arXiv 2108.07605), in the paper's order and
notation, vectorised over lattice nodes with explicit loops over species and
discrete velocities.  Section and equation references use the paper's own
labels.  Where the paper is silent or its printed formula is inconsistent the
reading taken is stated at the point of use.

Modules
    lattice    D3Q27 velocities and the product-form factors (section 2.2)
    thermo     species energy/enthalpy and the temperature equation (3.1)
    transport  relaxation times and parameters (sections 2.3, 3.4)
    chemistry  mass-action sources with explicit sub-steps (section 2.3)
    equilibria species, momentum and energy equilibria (sections 2.2, 3.2, 3.3)
    boundary   TMS wall, flux inlet and LODI outlet (section 4)
    solver     the time step and read-out

Parity unpinned: which boundary a node on faces of different kinds follows
(a wall face before an inlet or outlet face, a TMS face before a
bounce-back one) has no independent check; the synthetic thermo, transport
and mechanism laws are inputs, not method.  Every other part is pinned in
tests/test_oracle_pins.py, the union of incoming links at edges and corners
by causality in a box closed by walls.
"""
from .solver import Oracle  # noqa: F401
