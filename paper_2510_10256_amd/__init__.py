"""Barrier-filtered contact evaluation for thickened rods and shells on MI355X.

The compute path is the HIP library ``libbfc.so`` (C ABI in ``include/bfc.h``);
this package only marshals arguments to it, with PyTorch providing device
memory and streams.  Importing the package does not load the library; the
first call that needs it does, and raises if it is missing.
"""
from .binding import (lib, build, ContactScene, Batch, BF_FP64, BF_MIXED, BF_FILTER_PAPER, BF_FILTER_NONE,  # noqa: F401
                      BF_FILTER_CULL, BF_REFDIST_PARAM, BF_REFDIST_EUCLID_REST,
                      BF_S_CAND_OVERFLOW, BF_S_ACT_OVERFLOW, BF_S_INFEASIBLE, BF_S_BSR_OVERFLOW,
                      BF_S_CORE_OVERFLOW, BF_F_FILTERED, BF_F_INFEASIBLE, BF_F_CORE, EXPORTED)

__all__ = ["lib", "build", "ContactScene", "Batch"]
