"""MI355X (gfx950) solver for the CN-WSGD discretisation of 2-D two-sided space-fractional diffusion
equations: flexible GMRES preconditioned by a multigrid V-cycle, after Moghaderi, Dehghan, Donatelli
and Mazza, "Spectral analysis and multigrid preconditioners for two-dimensional space-fractional
diffusion equations".

The computation lives in libfde.so (hand-written HIP kernels behind the C ABI of include/fde.h);
`fde` is its Python binding with the same function names.
"""
from . import _lib  # noqa: F401

__all__ = ["_lib"]
