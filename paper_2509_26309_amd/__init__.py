"""MI355X (gfx950) TBPM propagation library: Chebyshev time evolution of
random-phase states under a sparse tight-binding Hamiltonian, the correlation
function C(t) = <psi0|e^{-iHt}|psi0> and the density of states.

The compute path is libtbpm.so (hand-written HIP, C ABI in include/tbpm.h);
`tbpm` is its ctypes binding.
"""
from . import tbpm  # noqa: F401
from .tbpm import Context, TBPMError  # noqa: F401
