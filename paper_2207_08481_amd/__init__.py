"""MI355X solver for the hybridised mass conserving mixed stress (MCS) Stokes
discretisation with its conforming auxiliary-space preconditioner
(Kogler, Lederer, Schoeberl, arXiv 2207.08481).

The numerical path lives in libmcs.so (HIP kernels for gfx950 behind the C ABI
of include/mcs.h); `mcs.Problem` is its Python binding.
"""
from .mcs import Batch, Problem, Server, load_library, MCSError, OP, PC  # noqa: F401
