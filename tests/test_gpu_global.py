"""GPU parity of the global C0 Q_p action (gather through the lattice numbering,
box-cell action, FP64 atomic scatter-add) against the oracle's global action
(brute-force numbering, direct-quadrature local actions, scatter-add).

Tolerance 1e-12 relative L2 (FP64; the order of the atomic additions varies).
The full-size case uses the benchmark's 64^3 mesh and compares sampled global
DOFs, each recomputed from the oracle's local actions of the cells that share
it (numbered by the lattice rule of the interface, which the DOF-map tests pin
to the oracle's brute-force numbering).
"""
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
    yield c
    c.close()


def run_global(ctx, op, nx, ny, nz, V, kap, ug):
    y = empty((len(ug),), np.float64)
    sf.assemble_action_global_q(ctx, op, nx, ny, nz, dev(V), dev(kap) if kap is not None else None, dev(ug), y)
    return host(y), sf.sf_check_errors(ctx)


@pytest.mark.parametrize("form", ["LAPLACE", "MASS"])
@pytest.mark.parametrize("p", range(1, 9))
def test_global_action_small_grid(ctx, form, p):
    nx, ny, nz = (3, 2, 4) if p <= 4 else (2, 2, 3)
    V = synth.box_mesh(nx, ny, nz, 24)
    kap = synth.kappa(len(V), (p + 1) ** 3, 24)
    _, nu = oracle.dofmap_q(nx, ny, nz, p)
    ug = np.random.default_rng([24, p]).standard_normal(nu)
    print("case global", form, p, flush=True)
    y, f = run_global(ctx, sf.make_op("Q", p, form), nx, ny, nz, V, kap, ug)
    assert f == 0
    ref = oracle.global_action_q(nx, ny, nz, p, form, V, ug, kappa=kap)
    assert rel_l2(y, ref) <= 1e-12


def test_global_action_rejects_other_ops(ctx):
    V = synth.box_mesh(1, 1, 1, 25)
    u = dev(np.zeros(27))
    y = empty((27,), np.float64)
    for op in (sf.make_op("DQ", 2, "LAPLACE"), sf.make_op("Q", 2, "LAPLACE", precision="fp32"),
               sf.make_op("Q", 2, "LAPLACE", io="f32")):
        with pytest.raises(sf.SfError):
            sf.assemble_action_global_q(ctx, op, 1, 1, 1, dev(V), None, u, y)


@pytest.mark.parametrize("grid", [(1, 1, 1), (1, 3, 2), (5, 1, 1), (2, 5, 3)])
@pytest.mark.parametrize("p", [1, 3, 6])
def test_global_action_grid_shapes(ctx, grid, p):
    """Grids with one-cell-wide axes and odd extents against the oracle; a second
    launch on the same inputs agrees to the rounding of the atomic additions' order."""
    nx, ny, nz = grid
    V = synth.box_mesh(nx, ny, nz, 26)
    n = nx * ny * nz
    _, nu = oracle.dofmap_q(nx, ny, nz, p)
    kap = synth.kappa(n, (p + 1) ** 3, 26)
    ug = synth.dof_vector(1, nu, 26)[0]
    op = sf.make_op("Q", p, "LAPLACE")
    print("case global grid", grid, "p", p, flush=True)
    y1, f = run_global(ctx, op, nx, ny, nz, V, kap, ug)
    assert f == 0
    y2, _ = run_global(ctx, op, nx, ny, nz, V, kap, ug)
    assert rel_l2(y2, y1) <= 1e-14
    ref = oracle.global_action_q(nx, ny, nz, p, "LAPLACE", V, ug, kappa=kap)
    assert rel_l2(y1, ref) <= 1e-12


@pytest.mark.parametrize("p", [2, 5, 8])
def test_global_action_full_size_sampled(ctx, p):
    import torch
    n1 = 64
    Vh = synth.box_mesh(n1, n1, n1, 2)
    n3 = (p + 1) ** 3
    L = n1 * p + 1
    ng = L ** 3
    kap = synth.device_kappa(n1 ** 3, n3, 2, p)
    g = torch.Generator(device="cuda")
    g.manual_seed(synth.SEED * 1000 + 230 + p)
    ug = torch.randn((ng,), generator=g, device="cuda", dtype=torch.float64)
    y = torch.empty_like(ug)
    print("case global full size p", p, flush=True)
    sf.assemble_action_global_q(ctx, sf.make_op("Q", p, "LAPLACE"), n1, n1, n1, dev(Vh), kap, ug, y)
    assert sf.sf_check_errors(ctx) == 0
    rng = np.random.default_rng([25, p])
    pts = [(0, 0, 0), (L - 1, L - 1, L - 1), (p, p, p), (L // 2, L // 3, L // 5)]
    pts += [tuple(int(v) for v in rng.integers(0, L, 3)) for _ in range(4)]
    loc = [(a, b, c) for a in range(p + 1) for b in range(p + 1) for c in range(p + 1)]
    uh = host(ug)
    num = den = 0.0
    for (A, B, Cc) in pts:
        # the cells that contain lattice point (A, B, Cc) and its local index in each
        ref = 0.0
        for i in {max(0, (A - 1) // p), min(n1 - 1, A // p)}:
            for j in {max(0, (B - 1) // p), min(n1 - 1, B // p)}:
                for k in {max(0, (Cc - 1) // p), min(n1 - 1, Cc // p)}:
                    a0, b0, c0 = A - i * p, B - j * p, Cc - k * p
                    if not (0 <= a0 <= p and 0 <= b0 <= p and 0 <= c0 <= p):
                        continue
                    cell = (i * n1 + j) * n1 + k
                    idx = [((i * p + a) * L + (j * p + b)) * L + (k * p + c) for (a, b, c) in loc]
                    yl = oracle.action("Q", p, "LAPLACE", Vh[cell][None], uh[idx][None],
                                       kappa=host(kap[cell:cell + 1]))
                    ref += yl[0, (a0 * (p + 1) + b0) * (p + 1) + c0]
        got = float(host(y[(A * L + B) * L + Cc:(A * L + B) * L + Cc + 1])[0])
        num += (got - ref) ** 2
        den += ref ** 2
    assert (num / den) ** 0.5 <= 1e-12
