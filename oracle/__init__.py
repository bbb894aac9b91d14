"""CPU oracle for Sim3-corrected search-and-fuse and the Sim3 reprojection
residual.

TEST INFRASTRUCTURE ONLY.  Nothing in the GPU library imports, links or runs
anything in this package; only the tests, the smoke check and the benchmark's
CPU-baseline leg do.  It shares no code with the GPU path: the search-and-fuse
definition is plain C (``fl_oracle.c``), the Sim3 algebra and the residual are
float64 NumPy/SciPy written from their definitions.
"""
from .search import search_fuse, census_fp64, hamming256, project, build_grid, lib_path, build_oracle  # noqa: F401
from . import sim3, residual, pgo  # noqa: F401

# decision codes of the search-and-fuse outputs
NOT_VISIBLE, NO_MATCH, ADD, FUSE, SKIP, INVALID = 0, 1, 2, 3, 4, 5
NO_DIST = 0x7FFF
