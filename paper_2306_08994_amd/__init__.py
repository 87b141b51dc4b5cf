"""paper_2306_08994_amd -- Foata-level multifrontal LU of FEM systems on AMD MI355X (gfx950).

The solver is a C ABI library (libmf.so, include/mf.h) of hand-written HIP kernels; this
package holds its sources (csrc/), its build step (build.py), a ctypes binding (solver.py) and a
torch.autograd.Function over it (autograd.py).  Importing the package does not load the
library; the first Plan does, and raises if it has not been built.
"""
from .solver import MFError, Plan, analyse  # noqa: F401


def __getattr__(name):
    # the autograd wrapper needs torch; import it on first use only
    if name in ("MFSolve", "mf_solve"):
        from . import autograd
        return getattr(autograd, name)
    raise AttributeError(name)


__all__ = ["Plan", "analyse", "MFError", "MFSolve", "mf_solve"]
