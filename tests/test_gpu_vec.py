"""GPU parity of the H(div) (NCF) and H(curl) (NCE) kernels against the FP64
oracle, through the C ABI: actions on boxes and sheared affine cells,
element matrices on boxes, FP32 variants, and sampled cells of the full
48^3-cell workload.  Tolerance: relative L2 <= 1e-12 for FP64."""
import numpy as np
import pytest

import oracle
import paper_1711_02473_amd as sf
from paper_1711_02473_amd import synth
from tests.gpu_util import dev, empty, host, max_cell_rel, rel_l2

pytestmark = pytest.mark.gpu

TOL64 = 1e-12
FORM = {"NCF": "HDIV", "NCE": "HCURL"}


@pytest.fixture(scope="module")
def ctx(lib):
    c = sf.Context(0)
    yield c
    c.close()


def gpu_action(ctx, op, V, kap, u, io=np.float64):
    n = len(V)
    nd, _ = sf.sf_element_dims(op)
    dy = empty((n, nd), io)
    sf.assemble_action(ctx, op, n, dev(V), dev(kap.astype(io)) if kap is not None else None, dev(u.astype(io)), dy)
    return host(dy), sf.sf_check_errors(ctx)


def gpu_matrix(ctx, op, V, kap, io=np.float64):
    n = len(V)
    nd, _ = sf.sf_element_dims(op)
    dA = empty((n, nd, nd), io)
    sf.assemble_element_matrix(ctx, op, n, dev(V), dev(kap.astype(io)) if kap is not None else None, dA)
    return host(dA), sf.sf_check_errors(ctx)


@pytest.mark.parametrize("family", ["NCF", "NCE"])
@pytest.mark.parametrize("k", range(1, 7))
@pytest.mark.parametrize("form,alpha,beta", [("MASS", 1.0, 0.0), ("DIVCURL", 0.7, 1.3)])
def test_action_fp64_boxes(ctx, family, k, form, alpha, beta):
    f = FORM[family] if form == "DIVCURL" else "MASS"
    grid = (3, 3, 5) if k <= 3 else (2, 3, 4)
    V = synth.box_mesh(*grid, 40 + k)
    n = len(V)
    nd = oracle.ndof(family, k)
    kap = synth.kappa(n, (k + 1) ** 3, 40 + k)
    u = synth.dof_vector(n, nd, 40 + k)
    print("case", family, k, f, n, flush=True)
    y, flags = gpu_action(ctx, sf.make_op(family, k, f, alpha=alpha, beta=beta), V, kap, u)
    ref = oracle.action(family, k, f, V, u, kappa=kap, alpha=alpha, beta=beta)
    assert flags == 0
    assert rel_l2(y, ref) <= TOL64, (rel_l2(y, ref), max_cell_rel(y, ref))


@pytest.mark.parametrize("family", ["NCF", "NCE"])
@pytest.mark.parametrize("k", [1, 2, 4, 6])
def test_action_fp64_affine(ctx, family, k):
    """Sheared cells exercise the full Piola factors J^T J / |J| and |J| G G^T."""
    V = synth.affine_cells(19, 50 + k)
    nd = oracle.ndof(family, k)
    u = synth.dof_vector(len(V), nd, 50 + k)
    y, flags = gpu_action(ctx, sf.make_op(family, k, FORM[family], alpha=1.1, beta=0.6), V, None, u)
    ref = oracle.action(family, k, FORM[family], V, u, alpha=1.1, beta=0.6)
    assert flags == 0
    assert rel_l2(y, ref) <= TOL64


@pytest.mark.parametrize("family", ["NCF", "NCE"])
@pytest.mark.parametrize("k", range(1, 7))
def test_element_matrix_fp64(ctx, family, k):
    n = {1: 30, 2: 12, 3: 6, 4: 3, 5: 2, 6: 2}[k]
    V = synth.box_mesh(1, 1, n, 60 + k)
    kap = synth.kappa(n, (k + 1) ** 3, 60 + k)
    print("case", family, k, n, flush=True)
    A, flags = gpu_matrix(ctx, sf.make_op(family, k, FORM[family], alpha=0.9, beta=1.2), V, kap)
    ref = oracle.element_matrix(family, k, FORM[family], V, kappa=kap, alpha=0.9, beta=1.2)
    assert flags == 0
    assert rel_l2(A, ref) <= TOL64, rel_l2(A, ref)


@pytest.mark.parametrize("family", ["NCF", "NCE"])
@pytest.mark.parametrize("k", [2, 5])
def test_element_matrix_mass_and_action_consistency(ctx, family, k):
    V = synth.box_mesh(1, 2, 2, 70 + k)
    nd = oracle.ndof(family, k)
    u = synth.dof_vector(len(V), nd, 70 + k)
    op = sf.make_op(family, k, "MASS")
    A, _ = gpu_matrix(ctx, op, V, None)
    y, _ = gpu_action(ctx, op, V, None, u)
    assert rel_l2(A, oracle.element_matrix(family, k, "MASS", V)) <= TOL64
    assert rel_l2(y, np.einsum("cij,cj->ci", A, u)) <= TOL64


@pytest.mark.parametrize("family", ["NCF", "NCE"])
@pytest.mark.parametrize("k", range(1, 7))
@pytest.mark.parametrize("prec,io,tol", [("fp32", "f32", 5e-6), ("fp64", "f32", 2e-6), ("fp32", "f64", 5e-6)])
def test_action_fp32(ctx, family, k, prec, io, tol):
    """FP32 contractions and/or FP32 storage at every degree the benchmark times, on
    boxes (a ragged cell count) and on sheared cells; the oracle runs on the FP32-rounded
    inputs, so the error is the kernels' own."""
    grid = (3, 3, 5) if k <= 3 else (2, 3, 4)
    npio = np.float32 if io == "f32" else np.float64
    op = sf.make_op(family, k, FORM[family], precision=prec, io=io, alpha=1.2, beta=0.8)
    nd = oracle.ndof(family, k)
    for V in (synth.box_mesh(*grid, 80 + k)[:-1], synth.affine_cells(7, 81 + k)):
        u = synth.dof_vector(len(V), nd, 80 + k)
        y, flags = gpu_action(ctx, op, V, None, u, io=npio)
        ref = oracle.action(family, k, FORM[family], V, u.astype(npio).astype(np.float64), alpha=1.2, beta=0.8)
        assert flags == 0
        assert rel_l2(y, ref) <= tol, rel_l2(y, ref)


@pytest.mark.parametrize("family", ["NCF", "NCE"])
@pytest.mark.parametrize("k", [1, 3, 6])
@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_full_size_48cubed_f32_storage_sampled(ctx, family, k, prec):
    """The 48^3 workload with FP32 storage (the benchmark's FP32 rows), in its launch
    configuration: sampled cells against the oracle run on the FP32-rounded inputs."""
    V = synth.box_mesh(48, 48, 48, 4)
    n = len(V)
    nd = oracle.ndof(family, k)
    u = synth.dof_vector(n, nd, 4).astype(np.float32)
    dy = empty((n, nd), np.float32)
    dy.fill_(np.nan)
    sf.assemble_action(ctx, sf.make_op(family, k, FORM[family], precision=prec, io="f32"), n, dev(V), None, dev(u), dy)
    assert sf.sf_check_errors(ctx) == 0
    y = host(dy)
    assert np.isfinite(y).all()
    idx = np.unique(np.concatenate([np.linspace(0, n - 1, 40).astype(np.int64), [n - 1]]))
    ref = oracle.action(family, k, FORM[family], V[idx], u[idx].astype(np.float64))
    assert rel_l2(y[idx], ref) <= (2e-6 if prec == "fp64" else 5e-6)


@pytest.mark.parametrize("family", ["NCF", "NCE"])
@pytest.mark.parametrize("k", [1, 3, 6])
def test_full_size_48cubed_sampled(ctx, family, k):
    """The 48^3-cell H(div)/H(curl) workload (alpha = beta = 1, kappa = 1), in the
    launch configuration the benchmark uses: every output cell of a sample of 40
    evenly spaced cells (first and last included) against the oracle."""
    V = synth.box_mesh(48, 48, 48, 4)
    n = len(V)
    nd = oracle.ndof(family, k)
    u = synth.dof_vector(n, nd, 4)
    y, flags = gpu_action(ctx, sf.make_op(family, k, FORM[family]), V, None, u)
    assert flags == 0
    idx = np.unique(np.concatenate([np.linspace(0, n - 1, 40).astype(np.int64), [n - 1]]))
    ref = oracle.action(family, k, FORM[family], V[idx], u[idx])
    assert rel_l2(y[idx], ref) <= TOL64


@pytest.fixture(scope="module")
def ctx_box(lib):
    c = sf.Context(0)
    sf.sf_set_geometry(c, "box")
    yield c
    c.close()


BOX_PREC = [("fp64", "f64", TOL64), ("fp64", "f32", 2e-6), ("fp32", "f64", 5e-6), ("fp32", "f32", 5e-6)]


@pytest.mark.parametrize("family", ["NCF", "NCE"])
@pytest.mark.parametrize("k", range(1, 7))
@pytest.mark.parametrize("form,alpha,beta", [("MASS", 1.0, 0.0), ("DIVCURL", 0.7, 1.3)])
@pytest.mark.parametrize("prec,io,tol", BOX_PREC)
def test_action_box_context(ctx_box, family, k, form, alpha, beta, prec, io, tol):
    """Box-cell contexts run the kernel with diagonal Piola factors and the pointwise
    stage fused into the contractions: every degree, both forms, every precision and
    storage pair, kappa per point, a cell count that leaves the last group ragged."""
    f = FORM[family] if form == "DIVCURL" else "MASS"
    grid = (3, 3, 5) if k <= 3 else (2, 3, 4)
    V = synth.box_mesh(*grid, 240 + k)[:-1]
    n = len(V)
    npio = np.float32 if io == "f32" else np.float64
    nd = oracle.ndof(family, k)
    kap = synth.kappa(n, (k + 1) ** 3, 240 + k).astype(npio)
    u = synth.dof_vector(n, nd, 240 + k).astype(npio)
    print("case", family, k, f, prec, io, n, flush=True)
    op = sf.make_op(family, k, f, precision=prec, io=io, alpha=alpha, beta=beta)
    y, flags = gpu_action(ctx_box, op, V, kap, u, io=npio)
    ref = oracle.action(family, k, f, V, u.astype(np.float64), kappa=kap.astype(np.float64), alpha=alpha, beta=beta)
    assert flags == 0
    assert rel_l2(y, ref) <= tol, (rel_l2(y, ref), max_cell_rel(y, ref))


@pytest.mark.parametrize("family", ["NCF", "NCE"])
@pytest.mark.parametrize("k", [2, 5])
def test_box_context_flags_sheared_cells(ctx_box, family, k):
    """A box context applies only the diagonal Piola factors: sheared cells raise
    SF_FLAG_NONBOX, boxes do not."""
    nd = oracle.ndof(family, k)
    V = synth.affine_cells(5, 250 + k)
    u = synth.dof_vector(len(V), nd, 250 + k)
    _, flags = gpu_action(ctx_box, sf.make_op(family, k, FORM[family]), V, None, u)
    assert flags & sf.SF_FLAG_NONBOX
    V = synth.box_mesh(1, 2, 3, 251 + k)
    _, flags = gpu_action(ctx_box, sf.make_op(family, k, FORM[family]), V, None, synth.dof_vector(6, nd, 3))
    assert flags == 0


@pytest.mark.parametrize("family", ["NCF", "NCE"])
@pytest.mark.parametrize("k", range(1, 7))
@pytest.mark.parametrize("io", ["f64", "f32"])
def test_box_context_48cubed_sampled(ctx_box, family, k, io):
    """The 48^3-cell workload in the benchmark's launch (box context, alpha = beta = 1,
    kappa = 1, FP64 contractions, FP64 or FP32 storage): 40 evenly spaced cells (first
    and last included) against the oracle; outputs pre-filled with NaN."""
    V = synth.box_mesh(48, 48, 48, 4)
    n = len(V)
    nd = oracle.ndof(family, k)
    npio = np.float32 if io == "f32" else np.float64
    u = synth.dof_vector(n, nd, 4).astype(npio)
    dy = empty((n, nd), npio)
    dy.fill_(np.nan)
    sf.assemble_action(ctx_box, sf.make_op(family, k, FORM[family], io=io), n, dev(V), None, dev(u), dy)
    assert sf.sf_check_errors(ctx_box) == 0
    y = host(dy)
    assert np.isfinite(y).all()
    idx = np.unique(np.concatenate([np.linspace(0, n - 1, 40).astype(np.int64), [n - 1]]))
    ref = oracle.action(family, k, FORM[family], V[idx], u[idx].astype(np.float64))
    assert rel_l2(y[idx], ref) <= (TOL64 if io == "f64" else 2e-6)


@pytest.fixture(scope="module")
def ctx_tri(lib):
    c = sf.Context(0)
    sf.sf_set_geometry(c, "trilinear")
    yield c
    c.close()


@pytest.mark.parametrize("family", ["NCF", "NCE"])
@pytest.mark.parametrize("k", range(1, 7))
@pytest.mark.parametrize("form,alpha,beta", [("MASS", 1.0, 0.0), ("DIVCURL", 0.8, 1.4)])
def test_action_trilinear_cells(ctx_tri, family, k, form, alpha, beta):
    """General trilinear cells (SF_GEOM_TRILINEAR): the Piola factors J^T J / |J|,
    |J| G G^T and 1 / |J| at every quadrature point, against the oracle's direct
    quadrature with the trilinear map evaluated point by point."""
    f = FORM[family] if form == "DIVCURL" else "MASS"
    n = {1: 40, 2: 25, 3: 13, 4: 9, 5: 5, 6: 4}[k]
    V = synth.trilinear_cells(n, 190 + k)
    nd = oracle.ndof(family, k)
    kap = synth.kappa(n, (k + 1) ** 3, 190 + k)
    u = synth.dof_vector(n, nd, 190 + k)
    print("case trilinear", family, k, f, n, flush=True)
    y, flags = gpu_action(ctx_tri, sf.make_op(family, k, f, alpha=alpha, beta=beta), V, kap, u)
    ref = oracle.action(family, k, f, V, u, kappa=kap, alpha=alpha, beta=beta)
    assert flags == 0
    assert rel_l2(y, ref) <= TOL64, (rel_l2(y, ref), max_cell_rel(y, ref))


def test_trilinear_cells_flag_and_reject_low_precision(ctx_tri):
    V = synth.trilinear_cells(4, 199)
    V[1, 7] = V[1, 0] - 0.9 * (V[1, 7] - V[1, 0])
    nd = oracle.ndof("NCE", 2)
    _, flags = gpu_action(ctx_tri, sf.make_op("NCE", 2, "HCURL"), V, None, synth.dof_vector(4, nd, 199))
    assert flags & sf.SF_FLAG_DETJ
    for prec, io in (("fp32", "f64"), ("fp64", "f32")):
        with pytest.raises(sf.SfError) as e:
            gpu_action(ctx_tri, sf.make_op("NCF", 2, "HDIV", precision=prec, io=io), synth.trilinear_cells(2, 198),
                       None, synth.dof_vector(2, oracle.ndof("NCF", 2), 198),
                       io=np.float32 if io == "f32" else np.float64)
        assert e.value.code == sf.SF_ERR_UNSUPPORTED
