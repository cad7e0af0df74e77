"""MI355X-native matrix-free weighted-quadrature (MF-WQ) isogeometric solver.

Hot path (all in libwqfd.so, HIP for gfx950): the MF-WQ stiffness operator of
Section 3.2 (Algorithm 2) and its transpose, the Fast Diagonalization
preconditioner of Section 4, right-preconditioned BiCGStab, mixed-precision
iterative refinement, and adjoint gradients.  ``wqfd`` is the torch binding of
the C ABI declared in include/wqfd.h; ``problem`` builds handles from a
synthetic workload; ``autograd`` wraps the solve in a torch.autograd.Function.
"""
from ._lib import LIB_PATH, lib  # noqa: F401

__all__ = ["LIB_PATH", "lib"]
