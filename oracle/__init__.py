"""Plain FP64 CPU oracle for the NSFR right-hand side (Cicchino & Nadarajah,
"Discretely Nonlinearly Stable Weight-Adjusted Flux Reconstruction High-Order
Method for Compressible Flows on Curvilinear Grids", arXiv 2312.07725).

THIS PACKAGE IS TEST INFRASTRUCTURE. Only the test-suite, the smoke check and
the CPU-baseline leg of the benchmark may import it. The GPU library never
calls, links or imports anything here, and nothing here imports the GPU
library: the two implementations share no code.

Everything is written with plain PyTorch CPU tensor operations in float64 (or
complex128, for complex-step derivatives), following the paper's equations
step by step, so that each function can be checked against the paper by eye.
The modules are:

  operators   1D LGL reference operators, SBP, ESFR K and the FR projection
  mesh        warped periodic hexahedral mesh and conservative-curl metrics
  flux        Euler flux, entropy variables, the entropy-conserving two-point flux
  residual    NSFR residual: line-wise (sum-factorised) and dense (definition) forms
  gl          NSFR with Gauss-Legendre (and overintegrated) quadrature: entropy
              projection, hybrid surface-volume terms, weight-adjusted and exact mass
  mass        weight-adjusted and exact inverses of the FR-modified mass
  timestep    classical RK4, CFL time step
  problems    manufactured-solution state and source term
  diagnostics entropy / conservation / kinetic-energy rates
  adjoint     vector-Jacobian products (reverse mode) and complex-step JVPs

Functions whose result is not pinned by an independent test say "parity
unpinned" in their docstring.
"""

from . import operators, mesh, flux, residual, mass, timestep, problems, diagnostics, adjoint, gl  # noqa: F401
from .scheme import Scheme  # noqa: F401
