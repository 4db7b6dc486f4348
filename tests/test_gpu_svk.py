"""GPU parity of the Saint Venant-Kirchhoff hyperelastic actions on the vector
Q_p element (SF_SVK: the linearised residual applied to du at u0; SF_SVK_RESIDUAL:
the residual) against the oracle's direct quadrature, FP64, relative L2 <= 1e-12,
on affine cells and, in a trilinear-geometry context, on general trilinear cells;
plus argument checks, geometry flags and a full-size sampled check."""
import numpy as np
import pytest

import oracle
import paper_1711_02473_amd as sf
from paper_1711_02473_amd import synth
from tests.gpu_util import dev, empty, host, max_cell_rel, rel_l2

pytestmark = pytest.mark.gpu

LAM, MU = 1.3, 0.8
NCELLS = {1: 70, 2: 40, 3: 21, 4: 9, 5: 5, 6: 3, 7: 3, 8: 2}


@pytest.fixture(scope="module")
def ctxs(lib):
    a = sf.Context(0)
    t = sf.Context(0)
    sf.sf_set_geometry(t, "trilinear")
    yield {"affine": a, "trilinear": t}
    a.close()
    t.close()


def run(ctx, op, V, u0, u):
    nd, _ = sf.sf_element_dims(op)
    y = empty((len(V), nd), np.float64)
    sf.assemble_action(ctx, op, len(V), dev(V), dev(u0) if u0 is not None else None, dev(u), y)
    return host(y), sf.sf_check_errors(ctx)


def reference(family, p, form, V, u0, du):
    if form == "SVK":
        return oracle.svk_jacobian_action(family, p, V, u0 if u0 is not None else np.zeros_like(du), du, LAM, MU)
    return oracle.svk_residual(family, p, V, du, LAM, MU)


@pytest.mark.parametrize("geom", ["affine", "trilinear"])
@pytest.mark.parametrize("form", ["SVK", "SVK_RESIDUAL"])
@pytest.mark.parametrize("family", ["Q", "QGLL"])
@pytest.mark.parametrize("p", [1, 2, 3, 4, 5, 6, 7, 8])
def test_svk_action_matches_oracle(ctxs, geom, form, family, p):
    n = NCELLS[p]
    V = synth.affine_cells(n, 80 + p) if geom == "affine" else synth.trilinear_cells(n, 80 + p)
    nd = 3 * (p + 1) ** 3
    u0, du = synth.displacements(n, nd, 80 + p, amp=0.05)
    if form == "SVK_RESIDUAL":
        du = 0.05 * du  # the residual's displacement
    op = sf.make_op(family, p, form, alpha=LAM, beta=MU)
    print("case svk", geom, form, family, p, flush=True)
    y, f = run(ctxs[geom], op, V, u0 if form == "SVK" else None, du)
    assert f == 0
    ref = reference(family, p, form, V, u0, du)
    assert rel_l2(y, ref) <= 1e-12
    assert max_cell_rel(y, ref) <= 1e-11


def test_svk_without_linearisation_point_is_linear_elasticity(ctxs):
    p, n = 3, 11
    V = synth.affine_cells(n, 91)
    _, du = synth.displacements(n, 3 * 64, 91)
    y, f = run(ctxs["affine"], sf.make_op("Q", p, "SVK", alpha=LAM, beta=MU), V, None, du)
    assert f == 0
    assert rel_l2(y, reference("Q", p, "SVK", V, None, du)) <= 1e-12


def test_svk_flags_and_rejections(ctxs):
    p, n = 2, 5
    nd = 3 * 27
    u0, du = synth.displacements(n, nd, 92)
    op = sf.make_op("Q", p, "SVK", alpha=LAM, beta=MU)
    # a trilinear cell in an affine context is flagged
    _, f = run(ctxs["affine"], op, synth.trilinear_cells(n, 92), u0, du)
    assert f & sf.SF_FLAG_NONAFFINE
    # a folded cell in the trilinear context raises DETJ
    V = synth.trilinear_cells(n, 93)
    V[1, 7] = V[1, 0] - 0.9 * (V[1, 7] - V[1, 0])
    _, f = run(ctxs["trilinear"], op, V, u0, du)
    assert f & sf.SF_FLAG_DETJ
    # residual takes no coefficient; FP32 is not built; DQ has no vector form
    with pytest.raises(sf.SfError):
        run(ctxs["affine"], sf.make_op("Q", p, "SVK_RESIDUAL", alpha=LAM, beta=MU), synth.affine_cells(n, 94), u0, du)
    with pytest.raises(sf.SfError):
        run(ctxs["affine"], sf.make_op("Q", p, "SVK", precision="fp32"), synth.affine_cells(n, 94), u0, du)
    with pytest.raises(sf.SfError):
        sf.sf_element_dims(sf.make_op("DQ", p, "SVK"))


@pytest.mark.parametrize("p", [2, 4, 8])
def test_svk_full_size_sampled(ctxs, p):
    """The bench's SVK workload (64^3 box cells, u0 0.01 N(0,1), du N(0,1) drawn on the
    GPU) in the bench's launch; evenly spaced cells recomputed by the oracle."""
    import torch
    V = synth.box_mesh(64, 64, 64, 2)
    n = len(V)
    nd = 3 * (p + 1) ** 3
    u0, du = synth.device_displacements(n, nd, 1, p)
    y = torch.empty_like(du)
    Vd = dev(V)
    sf.assemble_action(ctxs["affine"], sf.make_op("Q", p, "SVK", alpha=LAM, beta=MU), n, Vd, u0, du, y)
    assert sf.sf_check_errors(ctxs["affine"]) == 0
    idx = np.linspace(0, n - 1, 6).astype(np.int64)
    it = torch.from_numpy(idx).cuda()
    ref = oracle.svk_jacobian_action("Q", p, V[idx], host(u0[it]), host(du[it]), LAM, MU)
    assert max_cell_rel(host(y[it]), ref) <= 1e-11


SVK_MATRIX_CASES = [(g, f, p) for g in ("affine", "trilinear") for f in ("Q", "QGLL") for p in (1, 2, 3, 4, 5)] + \
    [("trilinear", "Q", 6), ("affine", "QGLL", 6), ("trilinear", "Q", 7), ("affine", "Q", 8)]


@pytest.mark.parametrize("geom,family,p", SVK_MATRIX_CASES)
def test_svk_element_matrix_matches_oracle(ctxs, geom, family, p):
    """The oracle's direct quadrature of the tangent modulus costs O(n^9) per cell (30 s for
    one p = 8 cell), so the high degrees run on one or two cells."""
    n = {1: 9, 2: 5, 3: 3, 4: 2, 5: 2, 6: 2, 7: 1, 8: 1}[p]
    V = synth.affine_cells(n, 150 + p) if geom == "affine" else synth.trilinear_cells(n, 150 + p)
    nd = 3 * (p + 1) ** 3
    u0, du = synth.displacements(n, nd, 150 + p, amp=0.05)
    op = sf.make_op(family, p, "SVK", alpha=LAM, beta=MU)
    print("case svk matrix", geom, family, p, flush=True)
    A = empty((n, nd, nd), np.float64)
    sf.assemble_element_matrix(ctxs[geom], op, n, dev(V), dev(u0), A)
    assert sf.sf_check_errors(ctxs[geom]) == 0
    Ah = host(A)
    ref = oracle.svk_matrix(family, p, V, u0, LAM, MU)
    assert rel_l2(Ah, ref) <= 1e-12
    # the tangent of a hyperelastic energy is symmetric
    assert rel_l2(Ah, np.transpose(Ah, (0, 2, 1))) <= 1e-12
    # the matrix applied to du is the GPU's own linearised action
    y, f = run(ctxs[geom], op, V, u0, du)
    assert f == 0
    assert rel_l2(np.einsum("cij,cj->ci", Ah, du), y) <= 1e-12


def test_svk_element_matrix_limits(ctxs):
    V = synth.affine_cells(2, 160)
    for op in (sf.make_op("Q", 2, "SVK_RESIDUAL"),):
        nd, _ = sf.sf_element_dims(op)
        A = empty((2, nd, nd), np.float64)
        with pytest.raises(sf.SfError):
            sf.assemble_element_matrix(ctxs["affine"], op, 2, dev(V), None, A)


def test_svk_element_matrix_at_rest_and_empty(ctxs):
    """u0 = NULL is the linearisation at rest (linear elasticity); ncells = 0 is a no-op."""
    p, n = 2, 4
    V = synth.affine_cells(n, 170)
    nd = 3 * (p + 1) ** 3
    op = sf.make_op("Q", p, "SVK", alpha=LAM, beta=MU)
    A = empty((n, nd, nd), np.float64)
    sf.assemble_element_matrix(ctxs["affine"], op, n, dev(V), None, A)
    assert sf.sf_check_errors(ctxs["affine"]) == 0
    ref = oracle.svk_matrix("Q", p, V, np.zeros((n, nd)), LAM, MU)
    assert rel_l2(host(A), ref) <= 1e-12
    y = empty((1, nd), np.float64)
    sf.assemble_action(ctxs["affine"], op, 0, dev(V), None, dev(np.zeros((1, nd))), y)
    sf.assemble_element_matrix(ctxs["affine"], op, 0, dev(V), None, A)
    assert sf.sf_check_errors(ctxs["affine"]) == 0
