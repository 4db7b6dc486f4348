"""Sum-factorised local finite-element assembly on hexahedral cells for
MI355X (gfx950): HIP kernels behind a C ABI (include/sf.h), with this thin
ctypes binding.  Nothing here computes: every step runs in libsf.so.
"""
from .binding import (  # noqa: F401
    FAMILY, FORM, PRECISION, IO, SF_OK, SF_ERR_ARG, SF_ERR_UNSUPPORTED, SF_ERR_NOMEM, SF_ERR_HIP,
    SF_ERR_GEOMETRY, SF_ERR_CAPACITY, SF_FLAG_DETJ, SF_FLAG_NONAFFINE, SF_FLAG_NONBOX, SF_GEOM_AFFINE, SF_GEOM_BOX, SF_GEOM_TRILINEAR,
    SfOp, SfJob, SfError, Context, Batch, load, make_op, make_job, sf_set_geometry, sf_element_dims, assemble_action, assemble_action_box_noalloc, assemble_action_global_q,
    assemble_element_matrix, sf_check_errors, sf_dof_map_q, sf_concat_index, sf_block_layout,
    sf_rule_1d, sf_lagrange_table, sf_plan_axis_order, sf_autotune, sf_tuned_variant, sf_load_tuning,
)
