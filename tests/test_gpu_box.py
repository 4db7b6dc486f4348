"""GPU parity of the box-cell action kernels (context geometry SF_GEOM_BOX)
against the FP64 oracle, through the C ABI.

Under SF_GEOM_BOX the Q_p / dQ_p actions run kernels specialised to a
diagonal Jacobian (the factor |J| G G^T of the argument factorisation,
Sec. 3.2, is diagonal).  Every kernel variant the autotuner may pick is
checked: the variant is forced through a tuning file (sf_load_tuning).
Sizes leave a ragged last cell group; the full-size cases use the
benchmark's 64^3 mesh and launch configuration and compare sampled cells,
including cells that persistent workgroups reach after several groups.
"""
import json

import numpy as np
import pytest

import oracle
import paper_1711_02473_amd as sf
from paper_1711_02473_amd import synth
from tests.gpu_util import dev, empty, host, max_cell_rel, rel_l2

pytestmark = pytest.mark.gpu

TOL64 = 1e-12
VARIANTS = (0, 1, 2, 3, 4, 5)


def variants_for(p):
    """Every variant the autotuner may pick at degree p (6, one cell per thread, is p = 1 only)."""
    return VARIANTS + ((6,) if p == 1 else ())


@pytest.fixture(scope="module")
def ctx(lib):
    c = sf.Context(0)
    sf.sf_set_geometry(c, "box")
    yield c
    c.close()


def force_variant(ctx, op, variant, tmp_path):
    key = "gfx950|fam%d|p%d|form%d|nq%d|prec%d|io%d|standalone" % (
        op.family, op.degree, op.form, op.degree + 1, op.precision, op.io_dtype)
    path = tmp_path / ("tune_%d.json" % variant)
    path.write_text(json.dumps({key: variant}))
    sf.sf_load_tuning(ctx, str(path))


def cells_for(p):
    # 174 / 59 cells: neither is a multiple of the cells per workgroup group (256 // (p+1)^2)
    return synth.box_mesh(5, 5, 7, 11)[:174] if p <= 3 else synth.box_mesh(3, 4, 5, 11)[:59]


def launch(ctx, op, V, kap, u, io=np.float64):
    n = V.shape[0]
    nd, _ = sf.sf_element_dims(op)
    dy = empty((n, nd), io)
    sf.assemble_action(ctx, op, n, dev(V), dev(kap.astype(io)) if kap is not None else None, dev(u.astype(io)), dy)
    flags = sf.sf_check_errors(ctx)
    return host(dy), flags


@pytest.mark.parametrize("family", ["Q", "DQ", "QGLL"])
@pytest.mark.parametrize("form", ["LAPLACE", "MASS"])
@pytest.mark.parametrize("p", range(1, 9))
def test_box_action_fp64_all_variants(ctx, tmp_path, family, form, p):
    V = cells_for(p)
    n, nd = len(V), (p + 1) ** 3
    kap = synth.kappa(n, nd, 11)
    u = synth.dof_vector(n, nd, 11)
    ref = oracle.action(family, p, form, V, u, kappa=kap)
    op = sf.make_op(family, p, form)
    for v in variants_for(p):
        print("case", family, form, p, n, "variant", v, flush=True)
        force_variant(ctx, op, v, tmp_path)
        y, flags = launch(ctx, op, V, kap, u)
        assert flags == 0
        assert rel_l2(y, ref) <= TOL64, (v, rel_l2(y, ref), max_cell_rel(y, ref))


@pytest.mark.parametrize("family,form,p", [("Q", "LAPLACE", 2), ("Q", "MASS", 7), ("DQ", "LAPLACE", 5)])
def test_box_action_no_kappa(ctx, family, form, p):
    V = cells_for(p)
    u = synth.dof_vector(len(V), (p + 1) ** 3, 12)
    y, flags = launch(ctx, sf.make_op(family, p, form), V, None, u)
    assert flags == 0
    assert rel_l2(y, oracle.action(family, p, form, V, u)) <= TOL64


@pytest.mark.parametrize("prec,io,tol", [("fp32", "f64", 5e-6), ("fp64", "f32", 2e-6), ("fp32", "f32", 5e-6)])
@pytest.mark.parametrize("p", range(1, 9))
def test_box_action_fp32(ctx, tmp_path, prec, io, tol, p):
    V = cells_for(p)
    n, nd = len(V), (p + 1) ** 3
    npio = np.float32 if io == "f32" else np.float64
    kap = synth.kappa(n, nd, 13)
    u = synth.dof_vector(n, nd, 13)
    ref = oracle.action("Q", p, "LAPLACE", V, u.astype(npio).astype(np.float64),
                        kappa=kap.astype(npio).astype(np.float64))
    op = sf.make_op("Q", p, "LAPLACE", precision=prec, io=io)
    for v in variants_for(p):
        force_variant(ctx, op, v, tmp_path)
        y, flags = launch(ctx, op, V, kap, u, io=npio)
        assert flags == 0
        assert rel_l2(y, ref) <= tol, (v, rel_l2(y, ref))


def test_cell_kernel_flags_p1(ctx, tmp_path):
    """The one-cell-per-thread kernel (p = 1) raises the same flags as the group kernels:
    SF_FLAG_NONBOX on sheared cells, nothing on boxes, SF_FLAG_DETJ on a collapsed box."""
    op = sf.make_op("Q", 1, "LAPLACE")
    force_variant(ctx, op, 6, tmp_path)
    u = synth.dof_vector(16, 8, 15)
    _, f = launch(ctx, op, synth.affine_cells(16, 15), None, u)
    assert f & sf.SF_FLAG_NONBOX
    boxes = synth.box_mesh(2, 2, 4, 15)
    _, f = launch(ctx, op, boxes, None, u)
    assert f == 0
    flat = boxes.copy()
    flat[5, :, 0] = flat[5, 0, 0]
    _, f = launch(ctx, op, flat, None, u)
    assert f & sf.SF_FLAG_DETJ


@pytest.mark.parametrize("variant", VARIANTS)
def test_box_mode_flags_non_box_cells(ctx, tmp_path, variant):
    """Under SF_GEOM_BOX, sheared cells raise SF_FLAG_NONBOX in the box-cell kernels
    (the general kernel, variant 3, computes them exactly instead); boxes raise
    nothing; a collapsed box raises SF_FLAG_DETJ."""
    op = sf.make_op("Q", 3, "LAPLACE")
    force_variant(ctx, op, variant, tmp_path)
    u = synth.dof_vector(16, 64, 14)
    aff = synth.affine_cells(16, 14)
    y, f = launch(ctx, op, aff, None, u)
    if variant == 3:
        assert f == 0 and rel_l2(y, oracle.action("Q", 3, "LAPLACE", aff, u)) <= TOL64
    else:
        assert f & sf.SF_FLAG_NONBOX
    boxes = synth.box_mesh(2, 2, 4, 14)
    _, f = launch(ctx, op, boxes, None, u)
    assert f == 0
    flat = boxes.copy()
    flat[5, :, 0] = flat[5, 0, 0]
    _, f = launch(ctx, op, flat, None, u)
    assert f & sf.SF_FLAG_DETJ


def test_geometry_switch_back_to_affine(lib):
    """The geometry hint is per context; back on SF_GEOM_AFFINE sheared cells are exact again."""
    c = sf.Context(0)
    try:
        V = synth.affine_cells(23, 15)
        u = synth.dof_vector(23, 125, 15)
        op = sf.make_op("Q", 4, "LAPLACE")
        sf.sf_set_geometry(c, "box")
        sf.sf_set_geometry(c, "affine")
        y, f = launch(c, op, V, None, u)
        assert f == 0
        assert rel_l2(y, oracle.action("Q", 4, "LAPLACE", V, u)) <= TOL64
        with pytest.raises(sf.SfError):
            sf.sf_set_geometry(c, 7)
    finally:
        c.close()


@pytest.mark.parametrize("form,p", [("LAPLACE", 1), ("LAPLACE", 2), ("LAPLACE", 5), ("LAPLACE", 8),
                                    ("MASS", 1), ("MASS", 5), ("MASS", 8)])
def test_box_full_size_sampled(ctx, tmp_path, form, p):
    """The benchmark configurations (Laplace headline and mass leg): 64^3 box cells,
    kappa per Gauss point, FP64, every variant; sampled cells (first, last, spread,
    and a run at the end) checked against the oracle cell by cell."""
    import torch
    n1 = 64
    n, nd = n1 ** 3, (p + 1) ** 3
    Vh = synth.box_mesh(n1, n1, n1, 2)
    V = dev(Vh)
    (kap, u), = synth.device_action_inputs(n, nd, 2, p)
    y = torch.empty_like(u)
    idx = np.unique(np.concatenate([np.arange(0, n, 4099), np.arange(n - 9, n), [0, 1, 2, 3, n // 2]]))
    ti = torch.from_numpy(idx).cuda()
    kh, uh = host(kap[ti]), host(u[ti])
    ref = oracle.action("Q", p, form, Vh[idx], uh, kappa=kh)
    op = sf.make_op("Q", p, form)
    for v in variants_for(p):
        print("case full-size", form, "p", p, "variant", v, flush=True)
        force_variant(ctx, op, v, tmp_path)
        y.fill_(np.nan)
        sf.assemble_action(ctx, op, n, V, kap, u, y)
        assert sf.sf_check_errors(ctx) == 0
        yh = host(y[ti])
        assert rel_l2(yh, ref) <= TOL64, (v, rel_l2(yh, ref), max_cell_rel(yh, ref))
        assert bool(torch.isfinite(y).all())


def test_box_launches_on_two_streams(ctx, tmp_path):
    """Persistent box-cell launches claim cell groups from per-launch counters; several
    launches in flight on different streams, and many in a row on one stream, must each
    cover every cell exactly once.  At p = 8 (nine points per axis) a quarter of the cell
    groups are claimed dynamically once every workgroup has been dealt two rounds; the
    meshes here are large enough for that claimed tail, so the counters, their slot ring
    and their reset are all exercised.  Every cell's result is the same arithmetic
    whichever workgroup computes it, so the outputs must equal a lone launch's bit for
    bit; sampled cells are also checked against the oracle."""
    import torch
    p = 8
    op = sf.make_op("Q", p, "LAPLACE")
    force_variant(ctx, op, 0, tmp_path)
    nd = (p + 1) ** 3
    cases = []
    for k in range(2):
        V = synth.box_mesh(22, 22, 22 + k, 16 + k)
        cases.append((V, synth.kappa(len(V), nd, 16 + k), synth.dof_vector(len(V), nd, 16 + k)))
    # enough cell groups (3 cells each) for a claimed tail, ngroups * 3/4 >= 2 * grid,
    # with up to four resident workgroups on each of the 256 compute units
    assert len(cases[0][0]) // 3 * 3 // 4 >= 2 * 256 * 4
    dev_in = [(dev(V), dev(kap), dev(u)) for V, kap, u in cases]
    lone = []
    for k in range(2):
        y = empty((len(cases[k][0]), nd), np.float64)
        sf.assemble_action(ctx, op, len(cases[k][0]), *dev_in[k], y)
        lone.append(host(y))
    assert sf.sf_check_errors(ctx) == 0
    for k in range(2):
        V, kap, u = cases[k]
        idx = np.unique(np.concatenate([np.linspace(0, len(V) - 1, 12).astype(np.int64), [len(V) - 1]]))
        ref = oracle.action("Q", p, "LAPLACE", V[idx], u[idx], kappa=kap[idx])
        assert rel_l2(lone[k][idx], ref) <= TOL64
    streams = [torch.cuda.Stream(), torch.cuda.Stream()]
    outs = [empty((len(V), nd), np.float64) for V, _, _ in cases]
    for o in outs:
        o.fill_(np.nan)
    torch.cuda.synchronize()
    for rep in range(6):
        for k in range(2):
            sf.assemble_action(ctx, op, len(cases[k][0]), *dev_in[k], outs[k], streams[k])
    torch.cuda.synchronize()
    assert sf.sf_check_errors(ctx) == 0
    for k in range(2):
        yk = host(outs[k])
        assert np.isfinite(yk).all()
        assert np.array_equal(yk, lone[k])
