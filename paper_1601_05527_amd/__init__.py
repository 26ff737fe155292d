"""Algebraic-distance network sparsification on MI355X (gfx950).

The compute path lives in the HIP library ``libad.so`` (C ABI declared in
``include/ad.h``); ``api`` marshals torch tensors into it.  ``graphs`` builds
symmetric CSR inputs and seeded synthetic graphs.
"""
__all__ = ["graphs", "api"]


def __getattr__(name):
    if name == "api":
        from . import api
        return api
    if name == "graphs":
        from . import graphs
        return graphs
    raise AttributeError(name)
