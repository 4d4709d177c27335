"""Reference oracle for the Enskog-Vlasov finite-difference lattice Boltzmann
(EV-FDLB) time step of Busuioc & Sofonea, "Thermal Enskog-Vlasov Lattice
Boltzmann model with phase separation" (arXiv:2503.15187).

THIS PACKAGE IS TEST INFRASTRUCTURE.  It is a plain, slow, single-threaded
FP64 numpy implementation of what one time step computes, written from the
paper (Sec. II, eqs. (eq:sutherland)-(eq:prandtl), and the numerical
methods named in Sec. III) so that the HIP path can be checked against it.
Only the test-suite, the smoke check and the CPU-baseline leg of the bench
may import it.  It shares no code with the HIP path and imports nothing
from the product package.

Every array routine is generic in dtype: it runs in float64 and in
complex128 (complex-step differentiation of the whole step).

Modules
-------
quadrature : full-range Gauss-Hermite velocity set and the Hermite tables
model      : contact value, transport coefficients, force and averaging
             kernels, equation of state, critical point, Maxwell construction
step1d     : one TVD-RK3 time step of the reduced 1D model
step2d     : one TVD-RK3 time step of the 2D extension
loss       : the scalar objectives used for gradient checks

Pins: every function is checked in tests/test_oracle_pins.py (1D) and
tests/test_oracle2d_pins.py (2D) against
closed forms, library routines, invariants or values printed in the paper.
Functions without such a check say "parity unpinned" in their docstring.
"""

from .quadrature import gauss_hermite, hermite_table, equilibrium_matrix, \
    momentum_derivative_matrix
from .model import Params
from . import model, step1d, step2d

__all__ = ["gauss_hermite", "hermite_table", "equilibrium_matrix",
           "momentum_derivative_matrix", "Params", "model", "step1d", "step2d"]
