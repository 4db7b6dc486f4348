"""GPU parity of the scalar-family kernels (Q_p, dQ_p; mass, Laplace) against
the FP64 oracle, through the C ABI.

Tolerance: relative L2 over the whole output <= 1e-12 for FP64 (the oracle
is FP64 without FMA contraction; the kernels use FMAs and a different but
exact reordering of the same finite sum, so only rounding differs).  Sizes
span several workgroup tiles and a ragged last tile.
"""
import numpy as np
import pytest

import oracle
import paper_1711_02473_amd as sf
from paper_1711_02473_amd import synth
from tests.gpu_util import dev, empty, host, max_cell_rel, rel_l2

pytestmark = pytest.mark.gpu

TOL64 = 1e-12


@pytest.fixture(scope="module")
def ctx(lib):
    c = sf.Context(0)
    yield c
    c.close()


def mesh_for(p):
    return (5, 5, 7) if p <= 3 else (3, 4, 5)


def run_action(ctx, op, V, kap, u, io=np.float64):
    n = V.shape[0]
    nd, _ = sf.sf_element_dims(op)
    dV = dev(V)
    dk = dev(kap.astype(io)) if kap is not None else None
    du = dev(u.astype(io))
    dy = empty((n, nd), io)
    sf.assemble_action(ctx, op, n, dV, dk, du, dy)
    flags = sf.sf_check_errors(ctx)
    return host(dy), flags


def run_matrix(ctx, op, V, kap, io=np.float64):
    n = V.shape[0]
    nd, _ = sf.sf_element_dims(op)
    dV = dev(V)
    dk = dev(kap.astype(io)) if kap is not None else None
    dA = empty((n, nd, nd), io)
    sf.assemble_element_matrix(ctx, op, n, dV, dk, dA)
    flags = sf.sf_check_errors(ctx)
    return host(dA), flags


@pytest.mark.parametrize("family", ["Q", "DQ", "QGLL"])
@pytest.mark.parametrize("form", ["LAPLACE", "MASS"])
@pytest.mark.parametrize("p", range(1, 9))
def test_action_fp64_boxes(ctx, family, form, p):
    nx, ny, nz = mesh_for(p)
    V = synth.box_mesh(nx, ny, nz, 2)
    n = len(V)
    nd = (p + 1) ** 3
    kap = synth.kappa(n, nd, 2)
    u = synth.dof_vector(n, nd, 2)
    print("case", family, form, p, n, flush=True)
    y, flags = run_action(ctx, sf.make_op(family, p, form), V, kap, u)
    ref = oracle.action(family, p, form, V, u, kappa=kap)
    assert flags == 0
    assert rel_l2(y, ref) <= TOL64, (rel_l2(y, ref), max_cell_rel(y, ref))


@pytest.mark.parametrize("family,form,p", [("Q", "LAPLACE", 1), ("Q", "LAPLACE", 3), ("Q", "LAPLACE", 8),
                                           ("Q", "MASS", 5), ("DQ", "LAPLACE", 4), ("DQ", "MASS", 6)])
def test_action_fp64_affine_no_kappa(ctx, family, form, p):
    """Sheared parallelepipeds exercise every entry of the symmetric factor |J| G G^T."""
    V = synth.affine_cells(37, 5)
    nd = (p + 1) ** 3
    u = synth.dof_vector(len(V), nd, 5)
    y, flags = run_action(ctx, sf.make_op(family, p, form), V, None, u)
    ref = oracle.action(family, p, form, V, u)
    assert flags == 0
    assert rel_l2(y, ref) <= TOL64


def test_config1_q2_laplace(ctx):
    """4x4x4 box mesh, Q_2 on GLL nodes, 3^3 GL points, kappa per point, FP64:
    the 27-entry local action and the full 27x27 element matrices."""
    V = synth.box_mesh(4, 4, 4, 1)
    kap = synth.kappa(64, 27, 1)
    u = synth.dof_vector(64, 27, 1)
    op = sf.make_op("Q", 2, "LAPLACE")
    y, f1 = run_action(ctx, op, V, kap, u)
    A, f2 = run_matrix(ctx, op, V, kap)
    yr = oracle.action("Q", 2, "LAPLACE", V, u, kappa=kap)
    Ar = oracle.element_matrix("Q", 2, "LAPLACE", V, kappa=kap)
    assert f1 == 0 and f2 == 0
    assert rel_l2(y, yr) <= TOL64 and rel_l2(A, Ar) <= TOL64
    assert max_cell_rel(A, Ar) <= 10 * TOL64


@pytest.mark.parametrize("family", ["Q", "DQ", "QGLL"])
@pytest.mark.parametrize("form", ["LAPLACE", "MASS"])
@pytest.mark.parametrize("p", range(1, 9))
def test_element_matrix_fp64(ctx, family, form, p):
    n = {1: 70, 2: 40, 3: 20, 4: 9, 5: 5, 6: 3, 7: 2, 8: 2}[p]
    V = synth.box_mesh(1, 1, n, 3)
    nq = (p + 1) ** 3
    kap = synth.kappa(n, nq, 3)
    print("case", family, form, p, n, flush=True)
    A, flags = run_matrix(ctx, sf.make_op(family, p, form), V, kap)
    ref = oracle.element_matrix(family, p, form, V, kappa=kap)
    assert flags == 0
    assert rel_l2(A, ref) <= TOL64, rel_l2(A, ref)


@pytest.mark.parametrize("p", [2, 5, 8])
def test_action_equals_matrix_times_u(ctx, p):
    """GPU action = GPU element matrix applied to u (two independent kernels)."""
    V = synth.box_mesh(1, 2, 3, 4)
    nd = (p + 1) ** 3
    kap = synth.kappa(len(V), nd, 4)
    u = synth.dof_vector(len(V), nd, 4)
    op = sf.make_op("Q", p, "LAPLACE")
    y, _ = run_action(ctx, op, V, kap, u)
    A, _ = run_matrix(ctx, op, V, kap)
    assert rel_l2(y, np.einsum("cij,cj->ci", A, u)) <= TOL64


@pytest.mark.parametrize("prec,io,tol", [("fp32", "f64", 5e-6), ("fp64", "f32", 2e-6), ("fp32", "f32", 5e-6)])
@pytest.mark.parametrize("p", [1, 4, 8])
def test_action_fp32_variants(ctx, prec, io, tol, p):
    V = synth.box_mesh(3, 3, 4, 6)
    nd = (p + 1) ** 3
    kap = synth.kappa(len(V), nd, 6)
    u = synth.dof_vector(len(V), nd, 6)
    npio = np.float32 if io == "f32" else np.float64
    y, flags = run_action(ctx, sf.make_op("Q", p, "LAPLACE", precision=prec, io=io), V, kap, u, io=npio)
    # the oracle sees exactly the values the kernel read
    ref = oracle.action("Q", p, "LAPLACE", V, u.astype(npio).astype(np.float64),
                        kappa=kap.astype(npio).astype(np.float64))
    assert flags == 0
    assert rel_l2(y, ref) <= tol


@pytest.mark.parametrize("p", [2, 6])
def test_element_matrix_f32_output(ctx, p):
    V = synth.box_mesh(1, 1, 3, 7)
    kap = synth.kappa(3, (p + 1) ** 3, 7)
    A, _ = run_matrix(ctx, sf.make_op("Q", p, "LAPLACE", io="f32"), V, kap, io=np.float32)
    ref = oracle.element_matrix("Q", p, "LAPLACE", V, kappa=kap.astype(np.float32).astype(np.float64))
    assert rel_l2(A, ref) <= 1e-6


def test_determinism_and_zero_cells(ctx):
    V = synth.box_mesh(4, 4, 4, 8)
    kap = synth.kappa(64, 729, 8)
    u = synth.dof_vector(64, 729, 8)
    op = sf.make_op("Q", 8, "LAPLACE")
    y1, _ = run_action(ctx, op, V, kap, u)
    y2, _ = run_action(ctx, op, V, kap, u)
    assert np.array_equal(y1, y2)
    assert sf.assemble_action(ctx, op, 0, None, None, None, None) == 0


def test_geometry_flags(ctx):
    """det J <= 0, non-affine vertices and (for element matrices) non-box cells raise
    device flags that sf_check_errors reports and then clears."""
    op = sf.make_op("Q", 2, "LAPLACE")
    good = synth.box_mesh(2, 2, 2, 9)
    u = synth.dof_vector(8, 27, 9)
    _, f = run_action(ctx, op, good, None, u)
    assert f == 0
    flat = good.copy()
    flat[3, :, 2] = flat[3, 0, 2]  # collapse cell 3 in z: det J = 0
    _, f = run_action(ctx, op, flat, None, u)
    assert f & sf.SF_FLAG_DETJ
    assert sf.sf_check_errors(ctx) == 0
    tri = synth.trilinear_cells(8, 9)
    _, f = run_action(ctx, op, tri, None, u)
    assert f & sf.SF_FLAG_NONAFFINE
    aff = synth.affine_cells(8, 9)
    _, f = run_action(ctx, op, aff, None, u)
    assert f == 0
    # element matrices: exact on sheared cells in the default (affine) geometry; the
    # box-cell kernel of a context declared SF_GEOM_BOX flags them instead
    A, f = run_matrix(ctx, op, aff, None)
    assert f == 0 and rel_l2(A, oracle.element_matrix("Q", 2, "LAPLACE", aff)) <= TOL64
    cbox = sf.Context(0)
    try:
        sf.sf_set_geometry(cbox, "box")
        _, f = run_matrix(cbox, op, aff, None)
        assert f & sf.SF_FLAG_NONBOX
    finally:
        cbox.close()


@pytest.mark.parametrize("grid,p", [((3, 2, 4), 1), ((4, 4, 4), 2), ((2, 3, 5), 5), ((3, 3, 3), 8)])
def test_dof_map_bit_exact(ctx, grid, p):
    nx, ny, nz = grid
    m = empty((nx * ny * nz, (p + 1) ** 3), np.int32)
    sf.sf_dof_map_q(ctx, nx, ny, nz, p, m)
    ref, _ = oracle.dofmap_q(nx, ny, nz, p)
    assert np.array_equal(host(m), ref)
