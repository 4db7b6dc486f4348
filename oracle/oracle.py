"""ctypes wrapper of the FP64 CPU oracle (test infrastructure only).

Every function here marshals numpy arrays into ``sf_oracle.c`` and back; the
arithmetic is in the C file.  Family / form names are strings so that the
oracle and the GPU library share no constant tables.
"""
import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "sf_oracle.c")
_LIB = os.path.join(_HERE, "liborc.so")
# a separately built copy (e.g. an AddressSanitizer / UBSan build made by the
# sanitizer test) may be named here; it is loaded as is, never rebuilt
_LIB_OVERRIDE = os.environ.get("SF_ORACLE_LIB", "")

FAMILIES = {"Q": 0, "DQ": 1, "NCF": 2, "NCE": 3, "QGLL": 4, "VQ": 5}
FORMS = {"MASS": 0, "LAPLACE": 1, "HDIV": 2, "HCURL": 3}

_lib = None


def build(force=True):
    """Compile the oracle with gcc: FP64, no fast-math, no FMA contraction."""
    if not force and os.path.exists(_LIB) and os.path.getmtime(_LIB) >= os.path.getmtime(_SRC):
        return _LIB
    tmp = _LIB + ".tmp%d" % os.getpid()
    cmd = ["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fopenmp", "-shared", "-fPIC",
           "-std=c11", "-Wall", "-o", tmp, _SRC, "-lm"]
    subprocess.check_call(cmd)
    os.replace(tmp, _LIB)
    return _LIB


def load():
    global _lib
    if _lib is not None:
        return _lib
    if _LIB_OVERRIDE:
        lib = ctypes.CDLL(_LIB_OVERRIDE)
    else:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build()
        lib = ctypes.CDLL(_LIB)
    dp = ctypes.POINTER(ctypes.c_double)
    ip = ctypes.POINTER(ctypes.c_int)
    lib.orc_gauss_legendre.argtypes = [ctypes.c_int, dp, dp]
    lib.orc_gauss_lobatto.argtypes = [ctypes.c_int, dp, dp]
    lib.orc_lagrange.argtypes = [dp, ctypes.c_int, ctypes.c_int, ctypes.c_double]
    lib.orc_lagrange.restype = ctypes.c_double
    lib.orc_lagrange_deriv.argtypes = [dp, ctypes.c_int, ctypes.c_int, ctypes.c_double]
    lib.orc_lagrange_deriv.restype = ctypes.c_double
    lib.orc_element_ndof.argtypes = [ctypes.c_int, ctypes.c_int]
    lib.orc_tabulate.argtypes = [ctypes.c_int, ctypes.c_int, dp, dp, dp]
    lib.orc_jacobian.argtypes = [dp, dp, dp]
    lib.orc_element_matrix.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                       ctypes.c_double, ctypes.c_double, ctypes.c_long, dp, dp, dp]
    lib.orc_action.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                               ctypes.c_double, ctypes.c_double, ctypes.c_long, dp, dp, dp, dp]
    lib.orc_svk.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_double, ctypes.c_double,
                            ctypes.c_int, ctypes.c_long, dp, dp, dp, dp]
    lib.orc_svk_matrix.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_double, ctypes.c_double,
                                   ctypes.c_long, dp, dp, dp]
    lib.orc_dofmap_q.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int, ip]
    lib.orc_dofmap_q.restype = ctypes.c_long
    lib.orc_concat_index.argtypes = [ctypes.c_int, ctypes.c_int, ip, ctypes.c_int, ip]
    lib.orc_concat_index.restype = ctypes.c_long
    _lib = lib
    return lib


def _dp(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _ip(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_int))


def gl_rule(m):
    """m-point Gauss-Legendre nodes and weights on [0,1]."""
    x = np.zeros(m)
    w = np.zeros(m)
    if load().orc_gauss_legendre(m, _dp(x), _dp(w)):
        raise ValueError("bad GL size %d" % m)
    return x, w


def gll_rule(m):
    """m-point Gauss-Lobatto-Legendre nodes and weights on [0,1]."""
    x = np.zeros(m)
    w = np.zeros(m)
    if load().orc_gauss_lobatto(m, _dp(x), _dp(w)):
        raise ValueError("bad GLL size %d" % m)
    return x, w


def lagrange(nodes, i, x):
    nodes = np.ascontiguousarray(nodes, dtype=np.float64)
    return load().orc_lagrange(_dp(nodes), len(nodes), i, float(x))


def lagrange_deriv(nodes, i, x):
    nodes = np.ascontiguousarray(nodes, dtype=np.float64)
    return load().orc_lagrange_deriv(_dp(nodes), len(nodes), i, float(x))


def ndof(family, degree):
    n = load().orc_element_ndof(FAMILIES[family], degree)
    if n < 0:
        raise ValueError("unsupported element %s%d" % (family, degree))
    return n


def tabulate(family, degree, xi):
    """Reference values [ndof][3] and derivatives [ndof][3][3] (d v_c / d xi_b)."""
    nd = ndof(family, degree)
    xi = np.ascontiguousarray(xi, dtype=np.float64)
    val = np.zeros((nd, 3))
    grad = np.zeros((nd, 3, 3))
    load().orc_tabulate(FAMILIES[family], degree, _dp(xi), _dp(val), _dp(grad))
    return val, grad


def jacobian(X, xi):
    X = np.ascontiguousarray(X, dtype=np.float64).reshape(8, 3)
    xi = np.ascontiguousarray(xi, dtype=np.float64)
    J = np.zeros((3, 3))
    load().orc_jacobian(_dp(X), _dp(xi), _dp(J))
    return J


def _prep(vertices, kappa, nq):
    vertices = np.ascontiguousarray(vertices, dtype=np.float64)
    ncells = vertices.shape[0]
    assert vertices.shape[1:] == (8, 3)
    kp = None
    if kappa is not None:
        kappa = np.ascontiguousarray(kappa, dtype=np.float64)
        assert kappa.shape == (ncells, nq), (kappa.shape, (ncells, nq))
        kp = _dp(kappa)
    return vertices, kappa, kp, ncells


def _nq1(family, degree, nq1):
    return nq1 if nq1 and nq1 > 0 else degree + 1


def element_matrix(family, degree, form, vertices, kappa=None, nq1=0, alpha=1.0, beta=1.0,
                   check_geometry=True):
    """Direct-quadrature element matrices [ncells][ndof][ndof] (row = test)."""
    m = _nq1(family, degree, nq1)
    vertices, kappa, kp, ncells = _prep(vertices, kappa, m ** 3)
    nd = ndof(family, degree)
    A = np.zeros((ncells, nd, nd))
    rc = load().orc_element_matrix(FAMILIES[family], degree, FORMS[form], m, alpha, beta, ncells,
                                   _dp(vertices), kp, _dp(A))
    if rc < 0:
        raise ValueError("oracle rejected arguments (%d)" % rc)
    if rc > 0 and check_geometry:
        raise ValueError("det J <= 0 in cell %d" % (rc - 1))
    return A


def action(family, degree, form, vertices, u, kappa=None, nq1=0, alpha=1.0, beta=1.0,
           check_geometry=True):
    """Direct-quadrature operator action y[ncells][ndof] = a(psi_i, u)."""
    m = _nq1(family, degree, nq1)
    vertices, kappa, kp, ncells = _prep(vertices, kappa, m ** 3)
    nd = ndof(family, degree)
    u = np.ascontiguousarray(u, dtype=np.float64)
    assert u.shape == (ncells, nd)
    y = np.zeros((ncells, nd))
    rc = load().orc_action(FAMILIES[family], degree, FORMS[form], m, alpha, beta, ncells,
                           _dp(vertices), kp, _dp(u), _dp(y))
    if rc < 0:
        raise ValueError("oracle rejected arguments (%d)" % rc)
    if rc > 0 and check_geometry:
        raise ValueError("det J <= 0 in cell %d" % (rc - 1))
    return y


def _svk(mode, family, degree, vertices, u0, du, lam, mu, nq1, check_geometry):
    m = _nq1(family, degree, nq1)
    vertices = np.ascontiguousarray(vertices, dtype=np.float64)
    ncells = vertices.shape[0]
    assert vertices.shape[1:] == (8, 3)
    nd = 3 * ndof(family, degree)
    u0 = np.ascontiguousarray(u0, dtype=np.float64)
    assert u0.shape == (ncells, nd), (u0.shape, (ncells, nd))
    dp = None
    if du is not None:
        du = np.ascontiguousarray(du, dtype=np.float64)
        assert du.shape == (ncells, nd)
        dp = _dp(du)
    out = np.zeros(ncells if mode == 0 else (ncells, nd))
    rc = load().orc_svk(FAMILIES[family], degree, m, float(lam), float(mu), mode, ncells, _dp(vertices),
                        _dp(u0), dp, _dp(out))
    if rc < 0:
        raise ValueError("oracle rejected arguments (%d)" % rc)
    if rc > 0 and check_geometry:
        raise ValueError("det J <= 0 in cell %d" % (rc - 1))
    return out


def svk_energy(family, degree, vertices, u0, lam, mu, nq1=0, check_geometry=True):
    """Saint Venant-Kirchhoff strain energy per cell, sum_q w |J| W(E(u0)) (family Q or QGLL;
    u0 [ncells][3 ndof], component-major: DOF (c, i) at c * ndof + i)."""
    return _svk(0, family, degree, vertices, u0, None, lam, mu, nq1, check_geometry)


def svk_residual(family, degree, vertices, u0, lam, mu, nq1=0, check_geometry=True):
    """Residual action y[c][(c', i)] = int P(u0) : grad(psi_i e_c') (no body force)."""
    return _svk(1, family, degree, vertices, u0, None, lam, mu, nq1, check_geometry)


def svk_jacobian_action(family, degree, vertices, u0, du, lam, mu, nq1=0, check_geometry=True):
    """Action of the linearised residual at u0 on du: int dP(u0; du) : grad(psi_i e_c')."""
    return _svk(2, family, degree, vertices, u0, du, lam, mu, nq1, check_geometry)


def svk_matrix(family, degree, vertices, u0, lam, mu, nq1=0, check_geometry=True):
    """Element matrices of the linearised residual at u0, [ncells][3 ndof][3 ndof] (row = test),
    from the tangent modulus of P at every point."""
    m = _nq1(family, degree, nq1)
    vertices = np.ascontiguousarray(vertices, dtype=np.float64)
    ncells = vertices.shape[0]
    nd = 3 * ndof(family, degree)
    u0 = np.ascontiguousarray(u0, dtype=np.float64)
    assert u0.shape == (ncells, nd)
    A = np.zeros((ncells, nd, nd))
    rc = load().orc_svk_matrix(FAMILIES[family], degree, m, float(lam), float(mu), ncells, _dp(vertices), _dp(u0),
                               _dp(A))
    if rc < 0:
        raise ValueError("oracle rejected arguments (%d)" % rc)
    if rc > 0 and check_geometry:
        raise ValueError("det J <= 0 in cell %d" % (rc - 1))
    return A


def dofmap_q(nx, ny, nz, p):
    """Brute-force global C0 Q_p numbering, int32 [ncells][(p+1)^3], and the DOF count."""
    n = p + 1
    m = np.zeros((nx * ny * nz, n ** 3), dtype=np.int32)
    nu = load().orc_dofmap_q(nx, ny, nz, p, _ip(m))
    if nu < 0:
        raise ValueError("bad grid")
    return m, int(nu)


def global_action_q(nx, ny, nz, p, form, vertices, u_global, kappa=None):
    """Global C0 Q_p operator action on an nx x ny x nz cell grid (Sec. 1.1: the global
    operator is the sum over cells of P_K^T A_K P_K): gather each cell's local DOFs
    through the brute-force numbering (dofmap_q), apply the direct-quadrature local
    action, and add every local result into the global vector."""
    m, nu = dofmap_q(nx, ny, nz, p)
    u_global = np.ascontiguousarray(u_global, dtype=np.float64)
    assert u_global.shape == (nu,)
    y_loc = action("Q", p, form, vertices, u_global[m], kappa=kappa)
    y = np.zeros(nu)
    np.add.at(y, m.ravel(), y_loc.ravel())
    return y


def concat_index(extents, block, multi):
    """Flat number of (block, multi-index) in a concatenation of row-major blocks."""
    ext = np.ascontiguousarray(np.asarray(extents, dtype=np.int32))
    nblocks, ndim = ext.shape
    mi = np.ascontiguousarray(np.asarray(multi, dtype=np.int32))
    return int(load().orc_concat_index(ndim, nblocks, _ip(ext), block, _ip(mi)))


def num_threads():
    return int(load().orc_num_threads())


def set_num_threads(n):
    """OpenMP thread count of later oracle calls (the GNU OpenMP runtime the
    oracle is linked against)."""
    load()
    ctypes.CDLL("libgomp.so.1").omp_set_num_threads(int(n))
