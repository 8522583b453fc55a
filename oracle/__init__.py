"""FP64 CPU oracle for the MCS Stokes method with its auxiliary-space preconditioner.

TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the CPU
baseline leg of the benchmark may import this package.  The GPU product path
never imports, calls or links anything here, and this package imports nothing
from the product path.

Reference: Kogler, Lederer, Schoeberl, "A conforming auxiliary space
preconditioner for the mass conserving mixed stress method" (arXiv 2207.08481).
Every function cites the section / equation it follows.  The oracle is written
for clarity, not speed: per-element dense numpy linear algebra, scipy sparse
global matrices, sequential Gauss-Seidel loops.
"""
from .poly import multi_indices  # noqa: F401
from .topology import Topology  # noqa: F401
from .element import ElementData, element_system  # noqa: F401
from .system import GlobalSystem  # noqa: F401
# precond and minres are imported lazily by users

