"""Algebraic-distance network sparsification on MI355X (gfx950).

The compute path lives in the HIP library ``libad.so`` (C ABI declared in
``include/ad.h``); ``paper_1601_05527_amd.api`` marshals torch tensors into
it.  ``paper_1601_05527_amd.graphs`` builds symmetric CSR inputs and seeded
synthetic graphs.  Submodules are imported explicitly.
"""
