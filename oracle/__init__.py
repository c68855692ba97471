"""Plain FP64 CPU oracle for the implicit soft-body step and its adjoint.

TEST INFRASTRUCTURE ONLY. Only the tests, the smoke check and the benchmark's
CPU-baseline leg may import this package; the product path (the HIP library and
its Python binding) never does, and this package never imports the product.
It shares no code with the GPU path: energies, derivatives and the assembled
Hessian are written out from the paper's definitions (fem.py), and the step and
adjoint use direct sparse solves (solve.py), not CG.

Parity status: every function here is pinned by the CPU tests in
tests/test_oracle_pins.py, tests/test_oracle_springs.py and tests/test_oracle_models.py (closed forms,
invariants, finite differences, independent automatic differentiation and brute
force); none is "parity unpinned".
"""
from .fem import Mesh, Problem  # noqa: F401
from . import fem, solve  # noqa: F401
