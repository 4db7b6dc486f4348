"""GPU parity of the Q_p / dQ_p / collocated actions on general trilinear
hexahedra (context geometry SF_GEOM_TRILINEAR: J, |J| and |J| G G^T evaluated
at every quadrature point) against the oracle, which evaluates the trilinear
map at every point by its own route.  Tolerance 1e-12 relative L2 (FP64)."""
import numpy as np
import pytest

import oracle
import paper_1711_02473_amd as sf
from paper_1711_02473_amd import synth
from tests.gpu_util import dev, empty, host, rel_l2

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx(lib):
    c = sf.Context(0)
    sf.sf_set_geometry(c, "trilinear")
    yield c
    c.close()


def launch(ctx, op, V, kap, u):
    nd, _ = sf.sf_element_dims(op)
    y = empty((len(V), nd), np.float64)
    sf.assemble_action(ctx, op, len(V), dev(V), dev(kap) if kap is not None else None, dev(u), y)
    return host(y), sf.sf_check_errors(ctx)


@pytest.mark.parametrize("family", ["Q", "DQ", "QGLL"])
@pytest.mark.parametrize("form", ["LAPLACE", "MASS"])
@pytest.mark.parametrize("p", [1, 2, 4, 6, 8])
def test_trilinear_action(ctx, family, form, p):
    n = {1: 150, 2: 90, 4: 25, 6: 9, 8: 4}[p]
    V = synth.trilinear_cells(n, 30 + p)
    nq = (p + 1) ** 3
    kap = synth.kappa(n, nq, 30 + p)
    u = synth.dof_vector(n, nq, 30 + p)
    print("case trilinear", family, form, p, flush=True)
    y, f = launch(ctx, sf.make_op(family, p, form), V, kap, u)
    assert f == 0
    ref = oracle.action(family, p, form, V, u, kappa=kap)
    assert rel_l2(y, ref) <= 1e-12


def test_trilinear_mode_on_boxes_and_affine_cells(ctx):
    """Boxes and parallelepipeds are trilinear maps too: same results as the oracle."""
    p = 3
    for V in (synth.box_mesh(2, 3, 2, 31), synth.affine_cells(12, 31)):
        u = synth.dof_vector(len(V), 64, 31)
        y, f = launch(ctx, sf.make_op("Q", p, "LAPLACE"), V, None, u)
        assert f == 0
        assert rel_l2(y, oracle.action("Q", p, "LAPLACE", V, u)) <= 1e-12


def test_trilinear_mode_flags_inverted_points_and_rejects_low_precision(ctx):
    V = synth.trilinear_cells(6, 32)
    V[2, 7] = V[2, 0] - 0.9 * (V[2, 7] - V[2, 0])  # fold one corner through the cell
    u = synth.dof_vector(6, 27, 32)
    _, f = launch(ctx, sf.make_op("Q", 2, "LAPLACE"), V, None, u)
    assert f & sf.SF_FLAG_DETJ
    with pytest.raises(sf.SfError):
        launch(ctx, sf.make_op("Q", 2, "LAPLACE", precision="fp32"), synth.trilinear_cells(2, 33), None,
               synth.dof_vector(2, 27, 33))
