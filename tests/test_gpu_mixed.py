"""Mixed-precision actions (MFMA contractions, FP32 accumulation, FP64 geometry)
against the FP64 oracle.  BF16X3 (three-term split operands) must reach
relative L2 <= 1e-6; single-term BF16 / FP16 have no accuracy target in the
paper and are checked against loose bounds derived from their unit roundoff
(2^-9 and 2^-12 relative per rounding, a dozen contractions deep)."""
import json

import numpy as np
import pytest

import oracle
import paper_1711_02473_amd as sf
from paper_1711_02473_amd import synth
from tests.gpu_util import dev, empty, host, rel_l2

pytestmark = pytest.mark.gpu

# relative L2 bounds of the actions: BF16x3 the precision target; the single-term modes
# about 20x their unit roundoff (BF16 2^-9, FP16 2^-11), which covers the four rounded
# contraction stages, the sum-factorised kernel (two to three times the dense kernels'
# error) and sheared cells (measured: BF16 2-9e-3, FP16 3-6e-4)
BOUND = {"bf16x3": 1e-6, "fp16": 1e-2, "bf16": 4e-2}


@pytest.fixture(scope="module")
def ctx(lib):
    c = sf.Context(0)
    yield c
    c.close()


def run(ctx, op, V, kap, u, io=np.float64):
    n = len(V)
    nd, _ = sf.sf_element_dims(op)
    dy = empty((n, nd), io)
    sf.assemble_action(ctx, op, n, dev(V), dev(kap.astype(io)) if kap is not None else None, dev(u.astype(io)), dy)
    return host(dy), sf.sf_check_errors(ctx)


@pytest.mark.parametrize("mode", ["bf16x3", "fp16", "bf16"])
@pytest.mark.parametrize("family,form", [("Q", "LAPLACE"), ("Q", "MASS"), ("DQ", "LAPLACE")])
@pytest.mark.parametrize("p", range(1, 9))
def test_mixed_action_error(ctx, mode, family, form, p):
    grid = (5, 5, 7) if p <= 3 else (3, 4, 5)
    V = synth.box_mesh(*grid, 90 + p)
    n = len(V)
    nd = (p + 1) ** 3
    kap = synth.kappa(n, nd, 90 + p)
    u = synth.dof_vector(n, nd, 90 + p)
    y, flags = run(ctx, sf.make_op(family, p, form, precision=mode), V, kap, u)
    ref = oracle.action(family, p, form, V, u, kappa=kap)
    err = rel_l2(y, ref)
    print("mixed", mode, family, form, p, "rel_l2 %.3e" % err, flush=True)
    assert flags == 0
    assert err <= BOUND[mode], err


@pytest.mark.parametrize("p", [2, 8])
def test_mixed_affine_f32_io(ctx, p):
    V = synth.affine_cells(33, 95)
    nd = (p + 1) ** 3
    u = synth.dof_vector(len(V), nd, 95)
    y, flags = run(ctx, sf.make_op("Q", p, "LAPLACE", precision="bf16x3", io="f32"), V, None, u, io=np.float32)
    ref = oracle.action("Q", p, "LAPLACE", V, u.astype(np.float32).astype(np.float64))
    assert flags == 0
    assert rel_l2(y, ref) <= 1e-6


def test_mixed_unsupported_for_vector_families(ctx):
    op = sf.make_op("NCF", 2, "HDIV", precision="bf16")
    V = synth.box_mesh(1, 1, 2, 96)
    nd, _ = sf.sf_element_dims(op)
    u = dev(synth.dof_vector(2, nd, 96))
    y = empty((2, nd), np.float64)
    with pytest.raises(sf.SfError) as e:
        sf.assemble_action(ctx, op, 2, dev(V), None, u, y)
    assert e.value.code == sf.SF_ERR_UNSUPPORTED


@pytest.fixture(scope="module")
def ctx_box(lib):
    c = sf.Context(0)
    sf.sf_set_geometry(c, "box")
    yield c
    c.close()


# only the final (q0) contraction of the element matrix runs in the lower precision:
# one rounding of each operand (2^-9 BF16, 2^-12 FP16 relative), about 2^-24 for BF16X3
MAT_BOUND = {"bf16x3": 1e-6, "fp16": 5e-3, "bf16": 2e-2}


@pytest.mark.parametrize("mode", ["bf16x3", "fp16", "bf16"])
@pytest.mark.parametrize("family,form", [("Q", "LAPLACE"), ("Q", "MASS"), ("DQ", "LAPLACE")])
@pytest.mark.parametrize("p", range(1, 9))
def test_mixed_element_matrix_error(ctx_box, mode, family, form, p):
    """Element matrices with the final contraction on MFMA (FP32 accumulation) on box
    cells, against the FP64 oracle; FP32 storage of the output for one case each."""
    n = {1: 45, 2: 14, 3: 9, 4: 5, 5: 3, 6: 2, 7: 2, 8: 2}[p]
    V = synth.box_mesh(1, 1, n, 210 + p)
    nd = (p + 1) ** 3
    kap = synth.kappa(n, nd, 210 + p)
    io = "f32" if (p == 3 and family == "Q") else "f64"
    npio = np.float32 if io == "f32" else np.float64
    op = sf.make_op(family, p, form, precision=mode, io=io)
    A = empty((n, nd, nd), npio)
    A.fill_(np.nan)
    sf.assemble_element_matrix(ctx_box, op, n, dev(V), dev(kap.astype(npio)), A)
    assert sf.sf_check_errors(ctx_box) == 0
    ref = oracle.element_matrix(family, p, form, V, kappa=kap.astype(npio).astype(np.float64))
    got = host(A)
    assert np.isfinite(got).all()
    err = rel_l2(got, ref)
    print("mixed matrix", mode, family, form, p, "rel_l2 %.3e" % err, flush=True)
    assert err <= max(MAT_BOUND[mode], 2e-7 if io == "f32" else 0.0), err


def test_mixed_element_matrix_rejections(ctx, ctx_box):
    V = dev(synth.box_mesh(1, 1, 2, 220))
    A = empty((2, 27, 27), np.float64)
    for c, op in ((ctx, sf.make_op("Q", 2, "LAPLACE", precision="bf16")),          # not a box context
                  (ctx_box, sf.make_op("QGLL", 2, "LAPLACE", precision="bf16")),   # collocated family
                  (ctx_box, sf.make_op("Q", 2, "LAPLACE", precision="fp32"))):     # no FP32 matrix kernel
        with pytest.raises(sf.SfError) as e:
            sf.assemble_element_matrix(c, op, 2, V, None, A)
        assert e.value.code == sf.SF_ERR_UNSUPPORTED


def force_variant(ctx, op, variant, tmp_path):
    key = "gfx950|fam%d|p%d|form%d|nq%d|prec%d|io%d|standalone" % (
        op.family, op.degree, op.form, op.degree + 1, op.precision, op.io_dtype)
    path = tmp_path / ("tune_%d.json" % variant)
    path.write_text(json.dumps({key: variant}))
    sf.sf_load_tuning(ctx, str(path))


@pytest.mark.parametrize("mode", ["bf16x3", "fp16", "bf16"])
@pytest.mark.parametrize("family,form", [("Q", "LAPLACE"), ("Q", "MASS"), ("DQ", "LAPLACE"), ("QGLL", "LAPLACE")])
@pytest.mark.parametrize("p", range(1, 9))
def test_mixed_dense_and_sumfact_kernels(ctx, tmp_path, mode, family, form, p):
    """The dense Kronecker kernels (variant 0, the default: one n^3 x n^3 product at
    p <= 3, plane x axis-0 products at p = 4..8, BF16x3 at p = 8 excepted) and the
    sum-factorised kernel (variant 1) on sheared affine cells, 117 cells (seven
    16-cell tiles and a ragged one; an odd count, so the last two-cell tile holds
    one cell), both against the oracle; FP32 storage too."""
    n = 117 if p <= 6 else 37
    V = synth.affine_cells(n, 230 + p)
    nd = (p + 1) ** 3
    kap = synth.kappa(n, nd, 230 + p)
    u = synth.dof_vector(n, nd, 230 + p)
    ref = oracle.action(family, p, form, V, u, kappa=kap)
    for io, npio in (("f64", np.float64), ("f32", np.float32)):
        op = sf.make_op(family, p, form, precision=mode, io=io)
        ref_io = ref if io == "f64" else oracle.action(
            family, p, form, V, u.astype(npio).astype(np.float64), kappa=kap.astype(npio).astype(np.float64))
        got = {}
        for v in (0, 1):
            print("case dense/sumfact", mode, family, form, p, io, "variant", v, flush=True)
            force_variant(ctx, op, v, tmp_path)
            y, flags = run(ctx, op, V, kap, u, io=npio)
            assert flags == 0
            assert np.isfinite(y).all()
            err = rel_l2(y, ref_io)
            assert err <= max(BOUND[mode], 3e-7 if io == "f32" else 0.0), (v, err)
            got[v] = y
        force_variant(ctx, op, 0, tmp_path)  # the module's context keeps the default
        # the two kernels round differently (operands of different contractions), both
        # within the bound; their difference is within twice the bound
        assert rel_l2(got[0], got[1]) <= 2 * BOUND[mode]


@pytest.mark.parametrize("io", ["f64", "f32"])
@pytest.mark.parametrize("mode", ["bf16x3", "bf16"])
@pytest.mark.parametrize("p", range(1, 9))
def test_mixed_dense_full_size_sampled(ctx, mode, p, io):
    """The mixed-precision benchmark configuration (64^3 box cells, kappa per point,
    FP64 and FP32 storage as the bench times them) on the default kernel; sampled cells
    against the oracle (on the FP32-rounded inputs for FP32 storage)."""
    import torch
    n1 = 64
    n, nd = n1 ** 3, (p + 1) ** 3
    Vh = synth.box_mesh(n1, n1, n1, 2)
    (kap, u), = synth.device_action_inputs(n, nd, 2, p)
    if io == "f32":
        kap, u = kap.float(), u.float()
    y = torch.empty_like(u)
    y.fill_(np.nan)
    op = sf.make_op("Q", p, "LAPLACE", precision=mode, io=io)
    print("case dense full-size", mode, "p", p, io, flush=True)
    sf.assemble_action(ctx, op, n, dev(Vh), kap, u, y)
    assert sf.sf_check_errors(ctx) == 0
    assert bool(torch.isfinite(y).all())
    idx = np.unique(np.concatenate([np.arange(0, n, 4099), np.arange(n - 9, n), [0, 1, 2, 3, n // 2]]))
    ti = torch.from_numpy(idx).cuda()
    ref = oracle.action("Q", p, "LAPLACE", Vh[idx], host(u[ti]).astype(np.float64),
                        kappa=host(kap[ti]).astype(np.float64))
    assert rel_l2(host(y[ti]).astype(np.float64), ref) <= max(BOUND[mode], 3e-7 if io == "f32" else 0.0)


@pytest.mark.parametrize("mode", ["bf16", "bf16x3"])
@pytest.mark.parametrize("p", [1, 2, 3, 4, 5, 6, 7, 8])
def test_mixed_dense_flags_and_small_counts(ctx, mode, p):
    """Geometry flags from the dense kernels' FP64 cell factor (one non-affine cell,
    one inverted cell, each alone in a batch of good cells), and tiny cell counts
    (1, 2, 5: tiles and batches mostly empty, so the next-tile prefetches of u and
    kappa stop early) with and without kappa, FP64 and FP32 storage, against the
    oracle (on the FP32-rounded inputs for FP32 storage)."""
    nd = (p + 1) ** 3
    op = sf.make_op("Q", p, "LAPLACE", precision=mode)
    for ncell in (1, 2, 5):
        V = synth.affine_cells(ncell, 240 + ncell)
        u = synth.dof_vector(ncell, nd, 240 + ncell)
        kap = synth.kappa(ncell, nd, 245 + ncell)
        for io, npio in (("f64", np.float64), ("f32", np.float32)):
            op_io = sf.make_op("Q", p, "LAPLACE", precision=mode, io=io)
            for k in (None, kap):
                print("case small count", mode, p, ncell, io, "kappa" if k is not None else "no kappa", flush=True)
                y, flags = run(ctx, op_io, V, k, u, io=npio)
                assert flags == 0
                r = lambda a: None if a is None else a.astype(npio).astype(np.float64)
                ref = oracle.action("Q", p, "LAPLACE", V, r(u), kappa=r(k))
                assert rel_l2(y, ref) <= max(BOUND[mode], 3e-7 if io == "f32" else 0.0)
    V = synth.affine_cells(40, 250)
    V_bad = V.copy()
    V_bad[17] = synth.trilinear_cells(1, 251)[0]  # not an affine image of its first four vertices
    u = synth.dof_vector(40, nd, 250)
    print("case flags", mode, p, flush=True)
    _, flags = run(ctx, op, V_bad, None, u)
    assert flags & sf.SF_FLAG_NONAFFINE
    V_inv = V.copy()
    V_inv[33] = V_inv[33][[4, 5, 6, 7, 0, 1, 2, 3]]  # mirrored along axis 0: det J < 0
    _, flags = run(ctx, op, V_inv, None, u)
    assert flags & sf.SF_FLAG_DETJ
    _, flags = run(ctx, op, V, None, u)
    assert flags == 0
