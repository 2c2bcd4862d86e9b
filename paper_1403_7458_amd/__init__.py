"""MI355X (gfx950) SpAMM and SP2: the hot path of the O(N) SCF solver of
Bock, Challacombe & Kale, as HIP kernels behind a C ABI (include/spamm.h).

The Python names below are the C entry points, marshalled by `_lib`.
"""
from ._lib import (FP32, FP64, LIB_PATH, PENDING, SIGNATURES, Sp2Server, SpammError, SpammMatrix,
                   load, profile_enable, profile_phases, profile_read, profile_reset,
                   sp2_footprint_bytes, sp2_initial_guess, sp2_options, sp2_solve, spamm_cull,
                   spamm_matrix_norms, spamm_multiply, spamm_to_dense, spamm_tree_build, version)

__all__ = ["FP32", "FP64", "LIB_PATH", "PENDING", "SIGNATURES", "Sp2Server", "SpammError",
           "SpammMatrix", "load", "profile_enable", "profile_phases", "profile_read", "profile_reset",
           "sp2_footprint_bytes", "sp2_initial_guess", "sp2_options", "sp2_solve", "spamm_cull",
           "spamm_matrix_norms", "spamm_multiply", "spamm_to_dense", "spamm_tree_build",
           "version"]
