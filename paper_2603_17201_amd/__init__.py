"""MI355X (gfx950) library for Sim3-corrected search-and-fuse (loop fusion)
and the Sim3 reprojection residual, after FastLoop (arXiv 2603.17201).

The compute lives in ``libfastloop.so`` (HIP, built by ``build.py``) behind
the C ABI of ``include/fastloop.h``; this package only marshals arguments.
"""
from ._abi import (ADD, FUSE, INVALID, MAX_KP, NO_DIST, NO_MATCH, NOT_VISIBLE, SKIP,  # noqa: F401
                   PGO_MAX_BAND_NODES, PGO_SOLVER_AUTO, PGO_SOLVER_CG, PGO_SOLVER_DIRECT, PGO_SOLVER_DIRECT_WIDE,
                   LIB_PATH, SIGNATURES, load, last_error)

__all__ = ["load", "last_error", "LIB_PATH", "SIGNATURES", "Context", "DeviceBatch", "FuseOutputs",
           "Sim3Residual", "FlError", "search_fuse_noalloc", "InversePairs"]


def __getattr__(name):
    # the torch-facing binding is imported lazily so that the ABI can be
    # inspected without importing torch
    if name in ("Context", "DeviceBatch", "FuseOutputs", "Sim3Residual", "FlError", "params_struct",
                "search_fuse_noalloc", "InversePairs"):
        from . import binding
        return getattr(binding, name)
    raise AttributeError(name)
