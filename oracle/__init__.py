"""FP64 CPU oracle of the dual-resolution phase-field step -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of ``bench.py``
may import this package. The product path (the HIP library and its Python binding) never
imports, calls or falls back to it; the two share no code. Inputs come from ``workloads``.

The oracle follows the paper (Bazesefidpar, Brandt, Tammisola, "A dual resolution
phase-field solver for wetting of viscoelastic droplets") step by step, in plain NumPy /
SciPy with FP64 arithmetic:

* Sec. 3.1 -- dual grid, prolongation (eq. dual1), restriction (eq. dual2) and mixture
  properties (eq. dual3): ``discrete.prolong``, ``discrete.restrict``.
* Sec. 3.2.1 -- Cahn-Hilliard with the Dong stabilised splitting (eqs. NS25-NS34): two
  constant-coefficient Helmholtz solves, Psi then phi: ``step.cahn_hilliard``.
* Sec. 3.2.2 -- Navier-Stokes with the constant-coefficient projection (eqs. NS35-NS39):
  three velocity Helmholtz solves, one pressure Poisson solve, correction:
  ``step.navier_stokes``.
* Sec. 3.2.3 -- polymer stress with second-order TVD Runge-Kutta (eqs. NS40-NS44), here in
  stress form for the Oldroyd-B model (eq. NS4 with alpha = 0): ``step.polymer``.

Every constant-coefficient solve is done exactly by FFT in the periodic x and y directions
and by the DCT-II / DST-II / DST-I that diagonalise the wall-normal second difference
(``discrete.helmholtz``): a different algorithm from the GPU path's batched tridiagonal
solve, reaching the same discrete solution.
"""
from . import model, discrete, step  # noqa: F401
