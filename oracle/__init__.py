"""FP64 CPU oracle of the space-time least-squares heat solver.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call,
link or execute this package; only the test suite, the smoke check and the
CPU-baseline leg of the benchmark use it.  It shares no code with the GPU
library: the only common dependency is the seeded input generator module
``stls_inputs``, which holds none of the method's arithmetic.

Plain, slow, obviously correct: numpy/scipy in float64, dense matrices,
no blocking or fusion beyond what the paper's definitions state.

Paper: Montardini, Negri, Sangalli, Tani, "Space-time least-squares
isogeometric method and efficient solver for parabolic problems"
(arXiv:1809.10026).  Sections are numbered as in the paper's source
(2 Preliminaries, 3 Model problem, 4 Linear solver, 5 Numerical benchmarks).

Modules
  bspline   Cox-de Boor basis and derivatives (§2.1)
  assemble  Gauss quadrature, univariate matrices, loads (§4.1, eq. A_kron)
  system    Kronecker-sum system matrix, matvec, preconditioner (§4.1-4.2)
  fd        fast diagonalization, Algorithm 1 (§4.3)
  pcg       preconditioned conjugate gradient (§4.2, §5)
  grad      adjoint gradients of a space-time misfit (extension, see module)
  norms     error norms of the manufactured-solution study (§5.1)
  geometry  mapped domains: pulled-back spatial matrices, the geometry
            coefficients, Algorithm 2 and the preconditioner P^G (§4.4,
            Appendix A.3), loads and error norms on the mapped domain

Parity status: every function is pinned by a test in tests/test_oracle_*.py
except where its docstring says "parity unpinned".
"""
from . import bspline, assemble, system, fd, pcg, norms, geometry  # noqa: F401
