"""Exact 1-D building blocks for pinning the oracle (test helper).

Lagrange polynomials are formed as coefficient arrays with numpy's
polynomial routines and integrated exactly (polyint), so nothing here shares
the oracle's product-formula evaluation or its quadrature.  Box-cell element
matrices of every form are then Kronecker products of these 1-D matrices
(the tensor-product structure of Sec. 1.2, eq. limits_tpe), a textbook
construction independent of both 3-D assembly paths.
"""
import itertools

import numpy as np
from numpy.polynomial import polynomial as P


def lagrange_coeffs(nodes):
    """Coefficient arrays (ascending powers) of the Lagrange basis on ``nodes``."""
    nodes = np.asarray(nodes, dtype=np.float64)
    out = []
    for i, xi in enumerate(nodes):
        others = np.delete(nodes, i)
        c = P.polyfromroots(others) if len(others) else np.array([1.0])
        out.append(c / P.polyval(xi, c))
    return out


def integrate01(c):
    ci = P.polyint(c)
    return P.polyval(1.0, ci) - P.polyval(0.0, ci)


def matrix1d(nodes_test, d_test, nodes_trial, d_trial, weight=None):
    """M[i, j] = int_0^1 w(x) (l_i^(d_test))(x) (l_j^(d_trial))(x) dx, exactly;
    ``weight`` is an optional coefficient array of a polynomial w."""
    lt = lagrange_coeffs(nodes_test)
    ls = lagrange_coeffs(nodes_trial)
    if d_test:
        lt = [P.polyder(c) for c in lt]
    if d_trial:
        ls = [P.polyder(c) for c in ls]
    M = np.zeros((len(lt), len(ls)))
    for i, a in enumerate(lt):
        for j, b in enumerate(ls):
            prod = P.polymul(a, b)
            if weight is not None:
                prod = P.polymul(prod, weight)
            M[i, j] = integrate01(prod)
    return M


def kron3(a, b, c):
    return np.kron(np.kron(a, b), c)


EPS = np.zeros((3, 3, 3))
for _a, _b, _c in itertools.permutations(range(3)):
    EPS[_a, _b, _c] = np.linalg.det(np.eye(3)[[_a, _b, _c]])


def blocks(family, degree, gl, gll):
    """Per-block per-axis node sets (the oracle's element reading, restated):
    Q -> GLL_{p+1}^3; DQ -> GL_{p+1}^3; NCF_k block c -> GLL_{k+1} on axis c,
    GL_k elsewhere; NCE_k block c -> GL_k on axis c, GLL_{k+1} elsewhere."""
    if family == "Q":
        return [[gll(degree + 1)] * 3]
    if family == "DQ":
        return [[gl(degree + 1)] * 3]
    k = degree
    out = []
    for c in range(3):
        axes = []
        for a in range(3):
            pk = (a == c) if family == "NCF" else (a != c)
            axes.append(gll(k + 1) if pk else gl(k))
        out.append(axes)
    return out


def box_matrix(family, degree, form, h, gl, gll, alpha=1.0, beta=1.0, kappa_poly=None):
    """Exact element matrix on the box [0,h0]x[0,h1]x[0,h2] (kappa = 1, or a
    polynomial of one reference coordinate given as (axis, coeffs))."""
    h = np.asarray(h, dtype=np.float64)
    S = float(np.prod(h))
    bl = blocks(family, degree, gl, gll)
    sizes = [int(np.prod([len(ax) for ax in b])) for b in bl]
    offs = np.concatenate([[0], np.cumsum(sizes)]).astype(int)
    N = offs[-1]
    A = np.zeros((N, N))

    def term(c, dt, cp, ds):
        mats = []
        for a in range(3):
            w = kappa_poly[1] if (kappa_poly is not None and kappa_poly[0] == a) else None
            mats.append(matrix1d(bl[c][a], dt[a], bl[cp][a], ds[a], weight=w))
        return kron3(*mats)

    e = np.eye(3, dtype=int)
    z = (0, 0, 0)
    for c in range(len(bl)):
        for cp in range(len(bl)):
            blk = np.zeros((sizes[c], sizes[cp]))
            if family in ("Q", "DQ"):
                if form == "MASS":
                    blk += S * term(c, z, cp, z)
                else:
                    for a in range(3):
                        blk += S / h[a] ** 2 * term(c, e[a], cp, e[a])
            elif family == "NCF":
                am = alpha if form == "HDIV" else 1.0
                bd = beta if form == "HDIV" else 0.0
                if c == cp:
                    blk += am * h[c] ** 2 / S * term(c, z, cp, z)
                if bd:
                    blk += bd / S * term(c, e[c], cp, e[cp])
            else:  # NCE
                am = alpha if form == "HCURL" else 1.0
                bc = beta if form == "HCURL" else 0.0
                if c == cp:
                    blk += am * S / h[c] ** 2 * term(c, z, cp, z)
                if bc:
                    for a in range(3):
                        for b in range(3):
                            for bp in range(3):
                                coef = EPS[a, b, c] * EPS[a, bp, cp]
                                if coef:
                                    blk += bc * coef * h[a] ** 2 / S * term(c, e[b], cp, e[bp])
            A[offs[c]:offs[c + 1], offs[cp]:offs[cp + 1]] = blk
    return A


def box_vertices(h, x0=(0.0, 0.0, 0.0)):
    V = np.zeros((8, 3))
    for v0 in (0, 1):
        for v1 in (0, 1):
            for v2 in (0, 1):
                V[4 * v0 + 2 * v1 + v2] = np.asarray(x0) + np.asarray(h) * np.array([v0, v1, v2])
    return V
