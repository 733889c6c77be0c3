"""MI355X-native differentiable XPBD (DiffXPBD): forward Gauss-Seidel
projections and their exact adjoint as hand-written HIP kernels for gfx950
behind a C ABI (``include/xpbd.h``).

Importing the package loads nothing; ``paper_2301_01396_amd.lib`` opens the
shared library on first use and fails loudly if it is not built.
"""
__all__ = ["scenes"]
