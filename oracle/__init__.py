"""Oracle: TEST INFRASTRUCTURE ONLY.

A plain FP64 CPU implementation (``sf_oracle.c``) of direct, non-factorised
quadrature assembly for the forms and elements of Homolya, Kirby & Ham,
"Exposing and exploiting structure: optimal code generation for high-order
finite element methods" (Sec. 1.1 eq. laplace_prefiat and the matrix-free
action; Secs. 1.2, 2.5-2.7 for the tensor-product, GL/GLL, enriched and
H(div)/H(curl) elements).  Only ``tests/``, ``__graft_entry__.smoke()`` and
the CPU-baseline leg of ``bench.py`` may import it.  It shares no code with
the GPU library and the GPU library never imports it.
"""
from .oracle import (  # noqa: F401
    FAMILIES, FORMS, build, load, gl_rule, gll_rule, lagrange, lagrange_deriv,
    ndof, tabulate, jacobian, element_matrix, action, dofmap_q, global_action_q, concat_index,
    num_threads, set_num_threads, svk_energy, svk_residual, svk_jacobian_action, svk_matrix,
)
