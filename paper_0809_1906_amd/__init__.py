"""Exact betweenness centrality on AMD Instinct MI355X (gfx950).

The computation lives in the HIP library libbc.so behind the C ABI of
include/bc.h; this package only binds it.  Importing never falls back to a
CPU path: without the built library, :func:`load` raises.
"""
from .binding import (BC, BCError, FORMS, bc_all_pairs, bc_sampled_distances, bc_create, bc_create_many, bc_destroy, bc_get_info, bc_get_timing,  # noqa: F401
                      bc_last_error, bc_options_init, bc_read, bc_read_edges, bc_read_sssp, bc_read_sssp_noalloc, bc_reset, bc_run,
                      bc_status_string, load, LIB_PATH, SIGNATURES)
from .binding import (BC_OK, BC_ERR_INVALID_ARG, BC_ERR_INVALID_GRAPH, BC_ERR_NOMEM,  # noqa: F401
                      BC_ERR_DEVICE, BC_ERR_OVERFLOW, BC_ERR_STATE, BC_ERR_UNSUPPORTED)
from .binding import (BC_FORM_AUTO, BC_FORM_PLAIN_FP64, BC_FORM_SPARSE, BC_FORM_ALGEBRAIC,  # noqa: F401
                      BC_FORM_HYBRID, BC_FORM_MANY, BC_TUNE_DEFAULT, BC_TUNE_MEASURED, BC_TUNE_CACHED,
                      BC_ALL_PAIRS_MAX_N, BC_ALGEBRAIC_MAX_WEIGHT, BC_ALGEBRAIC_MAX_DEGREE, BC_SAMPLED_MAX_S,
                      BC_NOALLOC_SCRATCH_BYTES)
