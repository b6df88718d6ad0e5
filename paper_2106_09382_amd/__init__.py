"""CONCORD-PCD on MI355X: edge-coloured parallel coordinate descent for sparse
precision-matrix estimation (Choi, Lee & Yu, arXiv 2106.09382), as HIP
kernels for gfx950 behind a C ABI (include/concord.h).

The solver entry points live in ``paper_2106_09382_amd._lib`` (loaded on first
use; importing this package does not touch the GPU)::

    from paper_2106_09382_amd import fit, gram
    omega, info = fit(S, lam=0.2, tol=1e-7)      # S: p x p CUDA tensor

``datagen`` draws the seeded synthetic workloads.
"""
__version__ = "0.1.0"


def __getattr__(name):
    if name in ("fit", "gram", "schedule", "strerror", "ConcordError", "NotConvergedWarning",
                "load"):
        from . import _lib
        return getattr(_lib, name)
    raise AttributeError(name)
