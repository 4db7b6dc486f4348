"""Seeded synthetic inputs (meshes, coefficients, DOF vectors).

This module only draws random numbers and lays out mesh geometry; it holds
none of the assembly arithmetic.  It is the one piece of code that both the
GPU path's callers and the oracle's callers use, so that both see identical
bytes.

Recipe: ``numpy.random.default_rng([171102473, config_id, stream])`` with
stream 0 = cell spacings, 1 = kappa, 2 = DOF vectors, 3 = batched-workload
mesh sizes and degrees, 4 = geometric perturbations.  Spacings are
U[0.5, 1.5], kappa U[0.5, 2] per quadrature point, DOF vectors N(0, 1).

Meshes are conforming tensor grids of axis-aligned boxes: per-axis spacings
drawn independently, vertex coordinates at their cumulative sums from 0.
Cell (i, j, k) is number (i*ny + j)*nz + k; its reference vertex
(v0, v1, v2) in {0,1}^3 is stored at index 4*v0 + 2*v1 + v2.
"""
import numpy as np

SEED = 171102473


def rng(config_id, stream):
    return np.random.default_rng([SEED, int(config_id), int(stream)])


def grid_vertices(xs, ys, zs):
    """Per-cell vertex array [ncells][8][3] of the tensor grid with node coordinates xs, ys, zs."""
    xs = np.asarray(xs, dtype=np.float64)
    ys = np.asarray(ys, dtype=np.float64)
    zs = np.asarray(zs, dtype=np.float64)
    nx, ny, nz = len(xs) - 1, len(ys) - 1, len(zs) - 1
    V = np.empty((nx, ny, nz, 8, 3), dtype=np.float64)
    for v0 in (0, 1):
        for v1 in (0, 1):
            for v2 in (0, 1):
                v = 4 * v0 + 2 * v1 + v2
                V[:, :, :, v, 0] = xs[v0:nx + v0][:, None, None]
                V[:, :, :, v, 1] = ys[v1:ny + v1][None, :, None]
                V[:, :, :, v, 2] = zs[v2:nz + v2][None, None, :]
    return V.reshape(nx * ny * nz, 8, 3)


def box_spacings(nx, ny, nz, config_id):
    g = rng(config_id, 0)
    hx = g.uniform(0.5, 1.5, nx)
    hy = g.uniform(0.5, 1.5, ny)
    hz = g.uniform(0.5, 1.5, nz)
    return hx, hy, hz


def box_mesh(nx, ny, nz, config_id):
    """Box cells with edge lengths U[0.5, 1.5]: vertices [nx*ny*nz][8][3]."""
    hx, hy, hz = box_spacings(nx, ny, nz, config_id)
    cum = lambda h: np.concatenate([[0.0], np.cumsum(h)])
    return grid_vertices(cum(hx), cum(hy), cum(hz))


def kappa(ncells, nq, config_id, dtype=np.float64):
    """Coefficient per quadrature point, U[0.5, 2], [ncells][nq]."""
    return rng(config_id, 1).uniform(0.5, 2.0, (ncells, nq)).astype(dtype)


def dof_vector(ncells, ndof, config_id, dtype=np.float64):
    """Cell-major local DOF vector, N(0, 1), [ncells][ndof]."""
    return rng(config_id, 2).standard_normal((ncells, ndof)).astype(dtype)


def batched_workload(nmeshes=2048, config_id=5, nmin=4, nmax=16, pmin=2, pmax=8):
    """Sizes and degrees of the batched mixed workload: list of (n_m, p_m),
    n_m uniform in {nmin..nmax} (n_m^3 cells), p_m uniform in {pmin..pmax}."""
    g = rng(config_id, 3)
    ns = g.integers(nmin, nmax + 1, nmeshes)
    ps = g.integers(pmin, pmax + 1, nmeshes)
    return [(int(a), int(b)) for a, b in zip(ns, ps)]


def batch_mesh(m, n, config_id=5):
    """Mesh m of the batched workload: an n x n x n box grid whose spacings are
    drawn from default_rng([SEED, config_id, 0, m]), U[0.5, 1.5]."""
    g = np.random.default_rng([SEED, int(config_id), 0, int(m)])
    cum = lambda h: np.concatenate([[0.0], np.cumsum(h)])
    return grid_vertices(cum(g.uniform(0.5, 1.5, n)), cum(g.uniform(0.5, 1.5, n)), cum(g.uniform(0.5, 1.5, n)))


def affine_cells(ncells, config_id, shear=0.3):
    """Parallelepiped cells x = x0 + J xi with J = diag(U[0.5,1.5]) + U[-shear, shear]
    off the diagonal (det J > 0 for shear <= 0.3)."""
    g = rng(config_id, 4)
    x0 = g.uniform(-1.0, 1.0, (ncells, 3))
    J = g.uniform(-shear, shear, (ncells, 3, 3))
    d = g.uniform(0.5, 1.5, (ncells, 3))
    for a in range(3):
        J[:, a, a] = d[:, a]
    V = np.empty((ncells, 8, 3))
    for v0 in (0, 1):
        for v1 in (0, 1):
            for v2 in (0, 1):
                xi = np.array([v0, v1, v2], dtype=np.float64)
                V[:, 4 * v0 + 2 * v1 + v2, :] = x0 + J @ xi
    return V


def trilinear_cells(ncells, config_id, amp=0.15):
    """Unit-ish boxes with every vertex moved by U[-amp, amp] per coordinate
    (a genuinely trilinear, non-affine map; det J > 0 for amp <= 0.15)."""
    g = rng(config_id, 4)
    V = box_mesh(1, 1, 1, config_id).repeat(ncells, axis=0)
    return V + g.uniform(-amp, amp, V.shape)


def device_action_inputs(ncells, n3, config_id, degree, nsets=1):
    """Full-size action inputs drawn on the GPU (torch's Philox generator on
    "cuda", seeded from (config_id, degree)): nsets tuples (kappa, u) of
    [ncells][n3] FP64 tensors, kappa U[0.5, 2], u N(0, 1).  Used where the
    host-side generators would take too long; the same seed gives the same
    values on every run, and tests copy sampled cells back to the host."""
    import torch
    g = torch.Generator(device="cuda")
    g.manual_seed(SEED * 100 + int(config_id) * 10 + int(degree))
    out = []
    for _ in range(nsets):
        kap = torch.rand((ncells, n3), generator=g, device="cuda", dtype=torch.float64) * 1.5 + 0.5
        u = torch.randn((ncells, n3), generator=g, device="cuda", dtype=torch.float64)
        out.append((kap, u))
    return out


def displacements(ncells, ndof, config_id, amp=0.01):
    """Host-side displacement pair (u0, du) for the hyperelastic forms, [ncells][ndof] each:
    u0 = amp N(0, 1) (the linearisation point), du N(0, 1) (the direction); stream 2."""
    g = rng(config_id, 2)
    u0 = amp * g.standard_normal((ncells, ndof))
    du = g.standard_normal((ncells, ndof))
    return u0, du


def device_displacements(ncells, ndof, config_id, degree, amp=0.01):
    """Full-size (u0, du) on "cuda" from torch's generator seeded with (config_id, degree):
    u0 = amp N(0, 1), du N(0, 1), [ncells][ndof] FP64."""
    import torch
    g = torch.Generator(device="cuda")
    g.manual_seed(SEED * 1000 + int(config_id) * 100 + 20 + int(degree))
    u0 = torch.randn((ncells, ndof), generator=g, device="cuda", dtype=torch.float64) * amp
    du = torch.randn((ncells, ndof), generator=g, device="cuda", dtype=torch.float64)
    return u0, du


def device_kappa(ncells, nq, config_id, degree):
    """kappa U[0.5, 2], [ncells][nq] FP64 on "cuda", from torch's generator seeded with
    (config_id, degree) (stream 1 of the recipe)."""
    import torch
    g = torch.Generator(device="cuda")
    g.manual_seed(SEED * 1000 + int(config_id) * 100 + 10 + int(degree))
    return torch.rand((ncells, nq), generator=g, device="cuda", dtype=torch.float64) * 1.5 + 0.5


def batched_device_inputs(workload, config_id=5):
    """Inputs of the batched workload on "cuda": per degree p, one slab of kappa and one of
    u holding that degree's meshes back to back (mesh order), drawn from torch's generator
    seeded with (config_id, p).  Returns ({p: (kappa, u)}, offset) where offset[m] is mesh
    m's first row in its degree's slab."""
    import torch
    count, offset = {}, []
    for n, p in workload:
        offset.append(count.get(p, 0))
        count[p] = count.get(p, 0) + n ** 3
    out = {}
    for p in sorted(count):
        n3 = (p + 1) ** 3
        g = torch.Generator(device="cuda")
        g.manual_seed(SEED * 1000 + int(config_id) * 100 + 20 + p)
        kap = torch.rand((count[p], n3), generator=g, device="cuda", dtype=torch.float64) * 1.5 + 0.5
        u = torch.randn((count[p], n3), generator=g, device="cuda", dtype=torch.float64)
        out[p] = (kap, u)
    return out, offset
