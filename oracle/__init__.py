"""FP64 CPU oracle for the contour-deformation G0W0 hot path.

TEST INFRASTRUCTURE ONLY.  This package is a plain, slow, obviously correct
restatement of the paper's formulas (Mejia-Rodriguez, Kunitsa, Apra, Govind,
"Scalable Molecular GW Calculations: Valence and Core Spectra").  It exists to
check the HIP path; it is imported, called or executed only by tests/,
__graft_entry__.smoke() and the cpu_baseline leg of bench.py.  It shares no
code with the HIP path: the only thing both sides consume is the seeded input
generator `gwgen`, which holds no GW arithmetic.

Everything is float64 numpy.  Dielectric matrices are inverted explicitly with
numpy.linalg.inv (no Cholesky, no iterative solver, no blocking or fusion).

Modules
  grid  - modified Gauss-Legendre imaginary-frequency grid
  cd    - polarizability, screened interaction, contour-deformation Sigma_c
  sd    - spectral-decomposition (Casida RPA) route, used as an independent pin
  qp    - quasiparticle step tree and the graphical (scan) solver

Pins: every function here is checked by tests/test_oracle_pins.py against
closed forms, invariants, the independent spectral-decomposition route and
brute force on tiny inputs.  The one result without an external pin (which of
several quasiparticle roots the step tree returns when a scan window holds
more than one) is marked "parity unpinned" in qp.py.
"""
from . import grid, cd, sd, qp  # noqa: F401
