"""Plain FP64 CPU reference for the semiclassical nonlinear Poisson solve.

TEST INFRASTRUCTURE ONLY.  This package exists to check the GPU library: only
the test suite, the package smoke check and the CPU-baseline leg of the
benchmark may import it.  The product path never calls it and shares no code,
constants or helpers with it.

What it computes (all in FP64, NumPy/SciPy):

* carrier statistics of Sec. II.A.1 -- Thomas-Fermi (0 K limit of Eq.
  FDstatistics), and Fermi-Dirac through the Bednarczyk form of Eq.
  FDIntApprox with the exp(x) switch below x = -50;
* the Galerkin weak form of Eq. PoissonWeakForm on a rectilinear Q1
  hexahedral mesh with 2x2x2 Gauss quadrature, gate Dirichlet values of
  Eq. ContOnIns and the default zero-flux Neumann faces;
* an assembled sparse Newton iteration with backtracking on the residual
  norm, the linear (charge-free) initial guess, nodal densities, the electron
  count in a region (Sec. III) and the adjoint gradient of that count.

Pinned by the ``-m "not gpu"`` tests (closed forms, quadrature, asymptotes,
brute force); see each function's docstring for what it follows.
"""
from . import physics, fem, solver  # noqa: F401
