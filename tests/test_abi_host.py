"""Host-only checks of the C-ABI library (no GPU): it loads, exports every
symbol include/sf.h declares, validates arguments before touching HIP, and
its host-side tables and index maps agree with the oracle."""
import itertools
import os
import re

import numpy as np
import pytest

import oracle
import paper_1711_02473_amd as sf
from tests.test_golden import load_rtcf2

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def header_functions():
    txt = open(os.path.join(ROOT, "include", "sf.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[a-z_0-9]+\s*\**\s*([a-z_0-9]+)\s*\(", txt, flags=re.M)
    return sorted(set(names))


def test_library_exports_every_declared_symbol():
    lib = sf.load()
    names = header_functions()
    assert "assemble_action" in names and "assemble_element_matrix" in names and len(names) >= 20
    for n in names:
        assert hasattr(lib, n), n


def test_element_dims_and_validation():
    for fam, degs in (("Q", range(1, 9)), ("DQ", range(1, 9))):
        for p in degs:
            for form in ("MASS", "LAPLACE"):
                assert sf.sf_element_dims(sf.make_op(fam, p, form)) == ((p + 1) ** 3, (p + 1) ** 3)
    for k in range(1, 7):
        assert sf.sf_element_dims(sf.make_op("NCF", k, "HDIV")) == (3 * k * k * (k + 1), (k + 1) ** 3)
        assert sf.sf_element_dims(sf.make_op("NCE", k, "HCURL")) == (3 * k * (k + 1) ** 2, (k + 1) ** 3)
    bad = [sf.make_op("Q", 0, "MASS"), sf.make_op("Q", 9, "MASS"), sf.make_op("NCF", 7, "HDIV"),
           sf.make_op("Q", 2, "HDIV"), sf.make_op("NCF", 2, "LAPLACE"), sf.make_op("NCE", 2, "HDIV"),
           sf.make_op("Q", 2, "MASS", nq1=5)]
    for op in bad:
        with pytest.raises(sf.SfError) as e:
            sf.sf_element_dims(op)
        assert e.value.code == sf.SF_ERR_UNSUPPORTED
    op = sf.make_op("Q", 2, "MASS")
    op.io_dtype = 7
    with pytest.raises(sf.SfError):
        sf.sf_element_dims(op)
    op = sf.make_op("Q", 2, "MASS", nq1=-1)
    with pytest.raises(sf.SfError) as e:
        sf.sf_element_dims(op)
    assert e.value.code == sf.SF_ERR_ARG


def test_entry_points_reject_bad_arguments_before_hip():
    lib = sf.load()
    op = sf.make_op("Q", 2, "LAPLACE")
    import ctypes
    assert lib.assemble_action(None, ctypes.byref(op), 10, 1, None, 1, 2, None) == sf.SF_ERR_ARG
    assert lib.assemble_element_matrix(None, ctypes.byref(op), 10, 1, None, 1, None) == sf.SF_ERR_ARG
    assert lib.sf_check_errors(None, None, None) == sf.SF_ERR_ARG
    assert lib.sf_dof_map_q(None, 2, 2, 2, 1, 1, None) == sf.SF_ERR_ARG
    assert lib.sf_context_destroy(None) == sf.SF_ERR_ARG
    assert lib.sf_batch_launch(None, None) < 0


@pytest.mark.parametrize("kind,m", [(0, m) for m in range(1, 13)] + [(1, m) for m in range(2, 13)])
def test_rules_match_oracle(kind, m):
    x, w = sf.sf_rule_1d(kind, m)
    xo, wo = oracle.gl_rule(m) if kind == 0 else oracle.gll_rule(m)
    assert np.abs(np.array(x) - xo).max() <= 2e-16 * 4
    assert np.abs(np.array(w) - wo).max() <= 1e-15


@pytest.mark.parametrize("nn,npt,kind", [(n, m, k) for n in range(1, 11) for m in (n, n + 1) for k in (0, 1)])
def test_lagrange_tables_match_oracle(nn, npt, kind):
    if kind == 1 and nn < 2:
        return
    nodes = (oracle.gl_rule(nn) if kind == 0 else oracle.gll_rule(nn))[0]
    pts = oracle.gl_rule(npt)[0]
    B, D = sf.sf_lagrange_table(list(nodes), list(pts))
    for p, x in enumerate(pts):
        for i in range(nn):
            assert abs(B[p][i] - oracle.lagrange(nodes, i, x)) < 1e-14
            assert abs(D[p][i] - oracle.lagrange_deriv(nodes, i, x)) < 1e-12 * max(1.0, nn * nn)


def test_concat_index_rtcf2_and_oracle():
    """Paper's RTCF_2 example (Sec. 3.5) and random layouts against the oracle's enumeration."""
    for num, blk, ia, ib, _, _ in load_rtcf2():
        assert sf.sf_concat_index([[3, 2], [2, 3]], blk, [ia - 1, ib - 1]) + 1 == num
    g = np.random.default_rng(3)
    for _ in range(30):
        ndim = int(g.integers(1, 4))
        nb = int(g.integers(1, 4))
        ext = g.integers(1, 4, (nb, ndim)).tolist()
        b = int(g.integers(0, nb))
        multi = [int(g.integers(0, e)) for e in ext[b]]
        assert sf.sf_concat_index(ext, b, multi) == oracle.concat_index(ext, b, multi)


@pytest.mark.parametrize("fam", ["NCF", "NCE", "Q"])
@pytest.mark.parametrize("k", [1, 2, 3, 6])
def test_block_layout(fam, k):
    form = {"NCF": "HDIV", "NCE": "HCURL", "Q": "LAPLACE"}[fam]
    ext, off = sf.sf_block_layout(sf.make_op(fam, k, form))
    nd, _ = sf.sf_element_dims(sf.make_op(fam, k, form))
    assert off[0] == 0 and sum(int(np.prod(e)) for e in ext) == nd
    if fam == "NCF":
        assert ext == [[k + 1, k, k], [k, k + 1, k], [k, k, k + 1]]
    if fam == "NCE":
        assert ext == [[k, k + 1, k + 1], [k + 1, k, k + 1], [k + 1, k + 1, k]]
    for c in range(len(ext)):
        assert sf.sf_concat_index(ext, c, [0, 0, 0]) == off[c]


def test_plan_axis_order_is_cheapest():
    """Alg. 1 restricted to three axis contractions: the chosen order costs no more than any other."""
    g = np.random.default_rng(5)
    for _ in range(50):
        ein = g.integers(1, 10, 3).tolist()
        eout = g.integers(1, 10, 3).tolist()
        order, flops = sf.sf_plan_axis_order(ein, eout)
        costs = {}
        for perm in itertools.permutations(range(3)):
            cur = list(ein)
            f = 0
            for a in perm:
                f += 2 * eout[a] * int(np.prod(cur))
                cur[a] = eout[a]
            costs[perm] = f
        assert flops == min(costs.values()) == costs[tuple(order)]
        assert tuple(order) == min(p for p, c in costs.items() if c == flops)


def test_svk_vector_element_dims_layout_and_validation():
    """The hyperelastic forms act on the vector Q_p element: 3 (p+1)^3 DOFs in three
    component blocks; FP64 only, family Q or QGLL only, no element matrices."""
    for fam in ("Q", "QGLL"):
        for p in range(1, 9):
            for form in ("SVK", "SVK_RESIDUAL"):
                op = sf.make_op(fam, p, form, alpha=1.0, beta=0.5)
                n = p + 1
                assert sf.sf_element_dims(op) == (3 * n ** 3, n ** 3)
                ext, off = sf.sf_block_layout(op)
                assert ext == [[n, n, n]] * 3 and off == [0, n ** 3, 2 * n ** 3]
    for bad in (sf.make_op("DQ", 2, "SVK"), sf.make_op("NCF", 2, "SVK"), sf.make_op("Q", 2, "SVK", precision="fp32"),
                sf.make_op("Q", 2, "SVK", io="f32"), sf.make_op("Q", 9, "SVK"), sf.make_op("Q", 2, "SVK", nq1=4)):
        with pytest.raises(sf.SfError):
            sf.sf_element_dims(bad)


def test_vector_family_dims_and_layout():
    for p in range(1, 9):
        n = p + 1
        for form in ("MASS", "LAPLACE"):
            op = sf.make_op("VQ", p, form)
            assert sf.sf_element_dims(op) == (3 * n ** 3, n ** 3)
            ext, off = sf.sf_block_layout(op)
            assert ext == [[n, n, n]] * 3 and off == [0, n ** 3, 2 * n ** 3]
    for bad in (sf.make_op("VQ", 2, "HDIV"), sf.make_op("VQ", 2, "MASS", precision="fp32"),
                sf.make_op("VQ", 2, "MASS", io="f32"), sf.make_op("VQ", 9, "LAPLACE")):
        with pytest.raises(sf.SfError):
            sf.sf_element_dims(bad)
