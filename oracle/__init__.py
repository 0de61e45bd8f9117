"""Plain FP64 CPU oracle for the D2Q37 thermal lattice Boltzmann step.

TEST INFRASTRUCTURE ONLY.  This package is the independent reference that the
HIP path is checked against.  Only ``tests/``, ``__graft_entry__.smoke()`` and
the ``cpu_baseline`` leg of ``bench.py`` may import it; the product library
(``paper_1405_1253_amd``) never imports, links or calls anything here, and this
package imports nothing from the product.

Everything is written in numpy, vectorised over lattice sites, in float64 (or
complex128 when a test drives it with a complex step).  The arithmetic follows
the paper's definitions in their own form -- explicit Hermite tensors for the
equilibrium, the central-moment form of the temperature, ``np.roll`` for the
streaming -- so that it can be checked against the paper by eye.  A library
matrix product is used for tensor contractions.

Modules
-------
lattice   velocity set, quadrature solve, Hermite tensors      (Sec. III.A, Fig. 2)
lbm       equilibrium, moments, pull/walls, collide, init, diagnostics
          (Sec. I eq. seteq, Sec. III.A eq. LBE and the forcing/renormalisation
          formulas, Sec. III.B, Sec. IV eqs. L(t) and 3L)
adjoint   hand-written reverse-mode derivative of N steps and of the init
"""
