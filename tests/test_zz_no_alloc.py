"""The allocation-free box-cell action (assemble_action_box_noalloc) through
the C ABI against the allocating entry point (assemble_action on a context
with SF_GEOM_BOX) on the same inputs, to the FP64 bar (relative L2 <= 1e-12;
FP32 contractions 5e-6 against the oracle): two calls in a row, the second
with a smaller input, into output buffers prefilled with NaN."""
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
    sf.sf_set_geometry(c, "box")
    yield c
    c.close()


def _inputs(n, p, seed):
    V = synth.box_mesh(n, 1, 1, seed) if n < 8 else synth.box_mesh(2, 4, (n + 7) // 8, seed)[:n]
    nd = (p + 1) ** 3
    return V, synth.kappa(len(V), nd, seed), synth.dof_vector(len(V), nd, seed)


@pytest.mark.parametrize("family,form,p", [("Q", "LAPLACE", 1), ("Q", "LAPLACE", 3), ("Q", "LAPLACE", 8),
                                           ("Q", "MASS", 5), ("DQ", "LAPLACE", 6), ("QGLL", "LAPLACE", 7)])
def test_noalloc_matches_allocating_entry_point(ctx, family, form, p):
    op = sf.make_op(family, p, form)
    nd = (p + 1) ** 3
    for n, seed in ((300 if p <= 4 else 90, 101), (37, 102)):  # second call smaller
        V, kap, u = _inputs(n, p, seed)
        dV, dk, du = dev(V), dev(kap), dev(u)
        y_ref = empty((len(V), nd), np.float64)
        y_ref.fill_(np.nan)
        sf.assemble_action(ctx, op, len(V), dV, dk, du, y_ref)
        y = empty((len(V), nd), np.float64)
        y.fill_(np.nan)
        print("case noalloc", family, form, p, len(V), flush=True)
        sf.assemble_action_box_noalloc(ctx, op, len(V), dV, dk, du, y)
        assert sf.sf_check_errors(ctx) == 0
        yh, rh = host(y), host(y_ref)
        assert np.isfinite(yh).all()
        assert rel_l2(yh, rh) <= 1e-12, rel_l2(yh, rh)


def test_noalloc_fp32_and_rejections(ctx):
    p = 4
    V, kap, u = _inputs(50, p, 103)
    op = sf.make_op("Q", p, "LAPLACE", precision="fp32")
    y = empty((50, (p + 1) ** 3), np.float64)
    sf.assemble_action_box_noalloc(ctx, op, 50, dev(V), dev(kap), dev(u), y)
    assert sf.sf_check_errors(ctx) == 0
    assert rel_l2(host(y), oracle.action("Q", p, "LAPLACE", V, u, kappa=kap)) <= 5e-6
    for bad in (sf.make_op("Q", p, "LAPLACE", precision="bf16"), sf.make_op("NCF", 2, "HDIV"),
                sf.make_op("VQ", 2, "LAPLACE")):
        nd, _ = sf.sf_element_dims(bad)
        with pytest.raises(sf.SfError) as e:
            sf.assemble_action_box_noalloc(ctx, bad, 2, dev(V[:2]), None, dev(np.zeros((2, nd))),
                                           empty((2, nd), np.float64))
        assert e.value.code == sf.SF_ERR_UNSUPPORTED
    assert sf.assemble_action_box_noalloc(ctx, op, 0, None, None, None, None) == 0
