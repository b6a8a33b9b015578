"""MI355X (gfx950) transient-search hot path.

Brute-force incoherent dedispersion of 2-bit filterbank data, boxcar matched
filtering and exact sigma-cut peak finding (sections 2.2 and 2.3 of
"Spotting Radio Transients with the help of GPUs"), as hand-written HIP
kernels behind the C ABI in include/dedisp.h.  This package is the thin
Python binding (``_lib``): argument marshalling only.
"""
from ._lib import (  # noqa: F401
    Batch, DedispError, dedisp_autotune, dedisp_batch_create, dedisp_batch_execute,
    dedisp_batch_info, Model, Server, triage_create, triage_forward, triage_forward_backward, triage_score,
    triage_get_params, triage_num_params, triage_save, triage_set_params, triage_tiles,
    triage_train_step, dedisp_serve_create, dedisp_serve_submit, dedisp_serve_poll,
    dedisp_serve_stats, dedisp_now_ns, EVENT_DTYPE, OUT_I32, OUT_U16, Plan, boxcar_filter, dedisp_default_tile,
    dedisp_execute, dedisp_execute_repacked, dedisp_execute_tile, dedisp_repack, dedisp_last_error, dedisp_plan_copy_delays,
    dedisp_plan_create, dedisp_plan_info, dedisp_tile_candidates, dedisp_workspace_bytes,
    events_from_buffer, find_peaks, find_peaks_read_stats, find_peaks_workspace_bytes, lib,
)
