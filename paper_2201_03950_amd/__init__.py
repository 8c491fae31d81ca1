"""Batched tridiagonal line solves and ADI steps on MI355X (gfx950).

The compute path is the HIP library ``libtrid.so`` (C ABI in ``include/trid.h``);
this package is its thin torch-tensor binding.  Importing the package does not
load the library; the first call does, and raises if it is missing.
"""

from ._binding import (  # noqa: F401
    PREC_F32,
    PREC_F32_REFINE64,
    PREC_F64,
    TridError,
    adi_step,
    adi_step_adjoint,
    adi_step_adjoint_kept,
    adi_step_keep,
    adi_step_noalloc,
    gtsv,
    gtsv_adjoint,
    gtsv_const,
    gtsv_refine,
    gtsv_s,
    gtsv_s_adjoint,
    gtsv_s_refine,
    gtsv_varlen,
    gtsv_varlen_dev,
    cache_report,
    model_adi,
    model_gtsv,
    model_hv,
    autotune_report,
    TRID_FORM_ARRAYS,
    TRID_FORM_S,
    hv_step,
    load_library,
    plan_load,
    plan_save,
    set_tile,
    timing_enable,
    timing_read,
    timing_select,
)
