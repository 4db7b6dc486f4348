"""Parity at the benchmark's full sizes, in the launch configurations bench.py
times, on sampled outputs the oracle computes cell by cell: element matrices on
the first cells of the 64^3 mesh, the lower-precision actions on the 64^3 mesh,
and the 2048-mesh batched launch.

Tolerances: FP64 1e-12 (relative L2 over the sampled outputs); FP32
contractions 5e-6; BF16 x3 split MFMA contractions 1e-6 (the mixed-precision
target; FP32 accumulation over about a dozen stages).
"""
import numpy as np
import pytest

import bench
import oracle
import paper_1711_02473_amd as sf
from paper_1711_02473_amd import synth
from tests.gpu_util import dev, host, rel_l2

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx(lib):
    c = sf.Context(0)
    sf.sf_set_geometry(c, "box")
    yield c
    c.close()


@pytest.fixture(scope="module")
def mesh64():
    Vh = synth.box_mesh(64, 64, 64, 2)
    return Vh, dev(Vh)


@pytest.mark.parametrize("p", [2, 5, 8])
def test_element_matrix_leg_sampled(ctx, mesh64, p):
    import torch
    Vh, V = mesh64
    n3 = (p + 1) ** 3
    nc = bench.matrix_leg_cells(p, len(Vh))
    kap = synth.device_kappa(nc, n3, 2, p)
    A = torch.empty((nc, n3, n3), device="cuda", dtype=torch.float64)
    print("case element-matrix leg p", p, "cells", nc, flush=True)
    sf.assemble_element_matrix(ctx, sf.make_op("Q", p, "LAPLACE"), nc, V, kap, A)
    assert sf.sf_check_errors(ctx) == 0
    idx = np.unique([0, nc // 3, nc // 2, nc - 1] if p < 8 else [0, nc - 1])
    ti = torch.from_numpy(idx).cuda()
    Ah, kh = host(A[ti]), host(kap[ti])
    del A
    ref = oracle.element_matrix("Q", p, "LAPLACE", Vh[idx], kappa=kh)
    assert rel_l2(Ah, ref) <= 1e-12


@pytest.mark.parametrize("mode,tol", [("fp32", 5e-6), ("bf16x3", 1e-6)])
@pytest.mark.parametrize("p", [4, 8])
def test_mixed_leg_sampled(ctx, mesh64, mode, tol, p):
    """The mixed-precision leg: FP64 storage, lower-precision contractions."""
    import torch
    Vh, V = mesh64
    n = len(Vh)
    n3 = (p + 1) ** 3
    (kap, u), = synth.device_action_inputs(n, n3, 2, p)
    y = torch.empty_like(u)
    print("case mixed leg", mode, "p", p, flush=True)
    sf.assemble_action(ctx, sf.make_op("Q", p, "LAPLACE", precision=mode), n, V, kap, u, y)
    assert sf.sf_check_errors(ctx) == 0
    idx = np.unique(np.concatenate([np.arange(0, n, 8191), [n - 1]]))
    ti = torch.from_numpy(idx).cuda()
    ref = oracle.action("Q", p, "LAPLACE", Vh[idx], host(u[ti]), kappa=host(kap[ti]))
    assert rel_l2(host(y[ti]), ref) <= tol


@pytest.mark.parametrize("mode,tol", [("fp64", 1e-12), ("bf16x3", 1e-6)])
def test_batched_leg_sampled(ctx, mode, tol):
    """The batched workload as bench.py builds it (2048 meshes, degrees 2..8, one
    persistent launch from a captured graph); one cell from every 97th mesh and the
    last cell of the last mesh checked against the oracle."""
    import torch
    wl = synth.batched_workload(2048)
    verts = [synth.batch_mesh(m, n) for m, (n, p) in enumerate(wl)]
    off = np.concatenate([[0], np.cumsum([n ** 3 for n, p in wl])])
    Vh = np.concatenate(verts)
    V = dev(Vh)
    slabs, slab_off = synth.batched_device_inputs(wl)
    ys = {p: torch.empty_like(u) for p, (k, u) in slabs.items()}
    jobs = []
    for m, (n, p) in enumerate(wl):
        n3 = (p + 1) ** 3
        kap, u = slabs[p]
        jobs.append(sf.make_job(sf.make_op("Q", p, "LAPLACE", precision=mode), n ** 3,
                                V.data_ptr() + int(off[m]) * 24 * 8, kap.data_ptr() + slab_off[m] * n3 * 8,
                                u.data_ptr() + slab_off[m] * n3 * 8, ys[p].data_ptr() + slab_off[m] * n3 * 8))
    print("case batched leg", mode, flush=True)
    b = sf.Batch(ctx, jobs)
    b.launch()
    torch.cuda.synchronize()
    assert sf.sf_check_errors(ctx) == 0
    num = den = 0.0
    for m in list(range(0, len(wl), 97)) + [len(wl) - 1]:
        n, p = wl[m]
        c = (m * 7919) % (n ** 3) if m != len(wl) - 1 else n ** 3 - 1
        kap, u = slabs[p]
        r = slab_off[m] + c
        ref = oracle.action("Q", p, "LAPLACE", Vh[int(off[m]) + c][None], host(u[r:r + 1]), kappa=host(kap[r:r + 1]))
        got = host(ys[p][r:r + 1])
        num += float(np.sum((got - ref) ** 2))
        den += float(np.sum(ref ** 2))
    b.close()
    assert (num / den) ** 0.5 <= tol
