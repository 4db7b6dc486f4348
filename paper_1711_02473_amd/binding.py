"""ctypes binding of libsf.so (include/sf.h): argument marshalling only.

Every call goes straight to the C ABI; tensors are passed as device
pointers (``tensor.data_ptr()``) and streams as ``hipStream_t`` handles
(``torch.cuda.current_stream().cuda_stream`` by default).  If the compiled
library is missing, loading raises: there is no fallback path.
"""
import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libsf.so")

FAMILY = {"Q": 0, "DQ": 1, "NCF": 2, "NCE": 3, "QGLL": 4, "VQ": 5}
FORM = {"MASS": 0, "LAPLACE": 1, "HDIV": 2, "HCURL": 3, "SVK": 4, "SVK_RESIDUAL": 5}
PRECISION = {"fp64": 0, "fp32": 1, "bf16": 2, "fp16": 3, "bf16x3": 4}
IO = {"f64": 0, "f32": 1}

SF_OK = 0
SF_ERR_ARG = -1
SF_ERR_UNSUPPORTED = -2
SF_ERR_NOMEM = -3
SF_ERR_HIP = -4
SF_ERR_GEOMETRY = -5
SF_ERR_CAPACITY = -6
SF_FLAG_DETJ, SF_FLAG_NONAFFINE, SF_FLAG_NONBOX = 1, 2, 4
SF_GEOM_AFFINE, SF_GEOM_BOX, SF_GEOM_TRILINEAR = 0, 1, 2


class SfOp(ctypes.Structure):
    _fields_ = [("family", ctypes.c_int32), ("degree", ctypes.c_int32), ("form", ctypes.c_int32),
                ("nq1", ctypes.c_int32), ("precision", ctypes.c_int32), ("io_dtype", ctypes.c_int32),
                ("alpha", ctypes.c_double), ("beta", ctypes.c_double)]


class SfJob(ctypes.Structure):
    _fields_ = [("op", SfOp), ("ncells", ctypes.c_int64), ("vertices", ctypes.c_void_p),
                ("kappa", ctypes.c_void_p), ("u", ctypes.c_void_p), ("y", ctypes.c_void_p),
                ("A", ctypes.c_void_p), ("A_arena_cells", ctypes.c_int64)]


class SfError(RuntimeError):
    def __init__(self, code, where):
        self.code = code
        super().__init__("%s: %s (%d)" % (where, _lib().sf_status_string(code).decode(), code))


_LIB = None


def load(path=LIB_PATH):
    """Load the compiled library; raises OSError if it was not built."""
    global _LIB
    if _LIB is not None:
        return _LIB
    if not os.path.exists(path):
        raise OSError("libsf.so not built: run python -m paper_1711_02473_amd.build_lib (%s)" % path)
    L = ctypes.CDLL(path)
    vp, i32, i64, dp = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.POINTER(ctypes.c_double)
    ip = ctypes.POINTER(ctypes.c_int32)
    opp = ctypes.POINTER(SfOp)
    sig = {
        "sf_context_create": ([ctypes.c_int, ctypes.POINTER(vp)], ctypes.c_int),
        "sf_context_destroy": ([vp], ctypes.c_int),
        "sf_status_string": ([ctypes.c_int], ctypes.c_char_p),
        "sf_element_dims": ([opp, ip, ip], ctypes.c_int),
        "sf_set_geometry": ([vp, i32], ctypes.c_int),
        "assemble_action": ([vp, opp, i64, vp, vp, vp, vp, vp], ctypes.c_int),
        "assemble_element_matrix": ([vp, opp, i64, vp, vp, vp, vp], ctypes.c_int),
        "assemble_action_box_noalloc": ([vp, opp, i64, vp, vp, vp, vp, vp], ctypes.c_int),
        "assemble_action_global_q": ([vp, opp, i32, i32, i32, vp, vp, vp, vp, vp], ctypes.c_int),
        "sf_check_errors": ([vp, vp, ip], ctypes.c_int),
        "sf_dof_map_q": ([vp, i32, i32, i32, i32, vp, vp], ctypes.c_int),
        "sf_concat_index": ([i32, i32, ip, i32, ip], i64),
        "sf_block_layout": ([opp, ip, ip, ip], ctypes.c_int),
        "sf_rule_1d": ([i32, i32, dp, dp], ctypes.c_int),
        "sf_lagrange_table": ([i32, dp, i32, dp, dp, dp], ctypes.c_int),
        "sf_plan_axis_order": ([ip, ip, ip], i64),
        "sf_batch_create": ([vp, ctypes.POINTER(SfJob), i32, ctypes.POINTER(vp)], ctypes.c_int),
        "sf_batch_launch": ([vp, vp], ctypes.c_int),
        "sf_batch_destroy": ([vp], ctypes.c_int),
        "sf_batch_info": ([vp, ctypes.POINTER(i64), ip], ctypes.c_int),
        "sf_autotune": ([vp, opp, i64, ctypes.c_char_p], ctypes.c_int),
        "sf_tuned_variant": ([vp, opp, ip], ctypes.c_int),
        "sf_load_tuning": ([vp, ctypes.c_char_p], ctypes.c_int),
    }
    for name, (args, res) in sig.items():
        f = getattr(L, name)
        f.argtypes = args
        f.restype = res
    _LIB = L
    return L


def _lib():
    return load()


def _check(rc, where):
    if rc < 0:
        raise SfError(rc, where)
    return rc


def make_op(family, degree, form, nq1=0, precision="fp64", io="f64", alpha=1.0, beta=1.0):
    return SfOp(FAMILY[family], int(degree), FORM[form], int(nq1), PRECISION[precision], IO[io],
                float(alpha), float(beta))


def _ptr(x):
    if x is None:
        return None
    if isinstance(x, int):
        return x
    return x.data_ptr()


def _stream(s):
    if s is None:
        import torch
        return torch.cuda.current_stream().cuda_stream
    if isinstance(s, int):
        return s
    return s.cuda_stream


class Context:
    """Owns an sf_context (tables, device error flag, tuning cache)."""

    def __init__(self, device=0):
        h = ctypes.c_void_p()
        _check(_lib().sf_context_create(int(device), ctypes.byref(h)), "sf_context_create")
        self.handle = h

    def close(self):
        if self.handle:
            _lib().sf_context_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def sf_set_geometry(ctx, geometry):
    """SF_GEOM_AFFINE (default), SF_GEOM_BOX (the caller guarantees axis-aligned boxes) or
    SF_GEOM_TRILINEAR (general trilinear hexahedra, geometry per quadrature point)."""
    g = {"affine": SF_GEOM_AFFINE, "box": SF_GEOM_BOX, "trilinear": SF_GEOM_TRILINEAR}.get(geometry, geometry)
    return _check(_lib().sf_set_geometry(ctx.handle, int(g)), "sf_set_geometry")


def sf_element_dims(op):
    nd, nq = ctypes.c_int32(), ctypes.c_int32()
    _check(_lib().sf_element_dims(ctypes.byref(op), ctypes.byref(nd), ctypes.byref(nq)), "sf_element_dims")
    return nd.value, nq.value


def assemble_action(ctx, op, ncells, vertices, kappa, u, y, stream=None):
    return _check(_lib().assemble_action(ctx.handle, ctypes.byref(op), int(ncells), _ptr(vertices), _ptr(kappa),
                                         _ptr(u), _ptr(y), _stream(stream)), "assemble_action")


def assemble_action_box_noalloc(ctx, op, ncells, vertices, kappa, u, y, stream=None):
    return _check(_lib().assemble_action_box_noalloc(ctx.handle, ctypes.byref(op), int(ncells), _ptr(vertices),
                                                     _ptr(kappa), _ptr(u), _ptr(y), _stream(stream)),
                  "assemble_action_box_noalloc")


def assemble_action_global_q(ctx, op, nx, ny, nz, vertices, kappa, u_global, y_global, stream=None):
    return _check(_lib().assemble_action_global_q(ctx.handle, ctypes.byref(op), int(nx), int(ny), int(nz),
                                                  _ptr(vertices), _ptr(kappa), _ptr(u_global), _ptr(y_global),
                                                  _stream(stream)), "assemble_action_global_q")


def assemble_element_matrix(ctx, op, ncells, vertices, kappa, A, stream=None):
    return _check(_lib().assemble_element_matrix(ctx.handle, ctypes.byref(op), int(ncells), _ptr(vertices),
                                                 _ptr(kappa), _ptr(A), _stream(stream)), "assemble_element_matrix")


def sf_check_errors(ctx, stream=None):
    """Returns the device flag bits raised since the last check (0 = none)."""
    f = ctypes.c_int32()
    rc = _lib().sf_check_errors(ctx.handle, _stream(stream), ctypes.byref(f))
    if rc not in (SF_OK, SF_ERR_GEOMETRY):
        raise SfError(rc, "sf_check_errors")
    return f.value


def sf_dof_map_q(ctx, nx, ny, nz, p, map_device, stream=None):
    return _check(_lib().sf_dof_map_q(ctx.handle, nx, ny, nz, p, _ptr(map_device), _stream(stream)), "sf_dof_map_q")


def sf_concat_index(extents, block, multi):
    ext = [int(e) for row in extents for e in row]
    ndim = len(extents[0])
    E = (ctypes.c_int32 * len(ext))(*ext)
    M = (ctypes.c_int32 * ndim)(*[int(m) for m in multi])
    return _check(_lib().sf_concat_index(ndim, len(extents), E, int(block), M), "sf_concat_index")


def sf_block_layout(op):
    nb = ctypes.c_int32()
    ext = (ctypes.c_int32 * 9)()
    off = (ctypes.c_int32 * 3)()
    _check(_lib().sf_block_layout(ctypes.byref(op), ctypes.byref(nb), ext, off), "sf_block_layout")
    n = nb.value
    return [list(ext[3 * b:3 * b + 3]) for b in range(n)], list(off[:n])


def sf_rule_1d(kind, m):
    x = (ctypes.c_double * m)()
    w = (ctypes.c_double * m)()
    _check(_lib().sf_rule_1d(int(kind), int(m), x, w), "sf_rule_1d")
    return list(x), list(w)


def sf_lagrange_table(nodes, pts):
    nn, npt = len(nodes), len(pts)
    N = (ctypes.c_double * nn)(*nodes)
    P = (ctypes.c_double * npt)(*pts)
    B = (ctypes.c_double * (nn * npt))()
    D = (ctypes.c_double * (nn * npt))()
    _check(_lib().sf_lagrange_table(nn, N, npt, P, B, D), "sf_lagrange_table")
    return ([list(B[p * nn:(p + 1) * nn]) for p in range(npt)], [list(D[p * nn:(p + 1) * nn]) for p in range(npt)])


def sf_plan_axis_order(ext_in, ext_out):
    I = (ctypes.c_int32 * 3)(*ext_in)
    O = (ctypes.c_int32 * 3)(*ext_out)
    order = (ctypes.c_int32 * 3)()
    flops = _check(_lib().sf_plan_axis_order(I, O, order), "sf_plan_axis_order")
    return list(order), flops


class Batch:
    """A captured persistent batched launch (sf_batch_*)."""

    def __init__(self, ctx, jobs):
        arr = (SfJob * len(jobs))(*jobs)
        h = ctypes.c_void_p()
        _check(_lib().sf_batch_create(ctx.handle, arr, len(jobs), ctypes.byref(h)), "sf_batch_create")
        self.handle = h
        self._jobs = arr

    def launch(self, stream=None):
        return _check(_lib().sf_batch_launch(self.handle, _stream(stream)), "sf_batch_launch")

    def info(self):
        nt, nw = ctypes.c_int64(), ctypes.c_int32()
        _check(_lib().sf_batch_info(self.handle, ctypes.byref(nt), ctypes.byref(nw)), "sf_batch_info")
        return nt.value, nw.value

    def close(self):
        if self.handle:
            _lib().sf_batch_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def make_job(op, ncells, vertices, kappa=None, u=None, y=None, A=None, A_arena_cells=0):
    return SfJob(op, int(ncells), _ptr(vertices), _ptr(kappa), _ptr(u), _ptr(y), _ptr(A), int(A_arena_cells))


def sf_autotune(ctx, op, ncells_hint, cache_json_path=None):
    p = cache_json_path.encode() if cache_json_path else None
    return _check(_lib().sf_autotune(ctx.handle, ctypes.byref(op), int(ncells_hint), p), "sf_autotune")


def sf_tuned_variant(ctx, op):
    v = ctypes.c_int32()
    _check(_lib().sf_tuned_variant(ctx.handle, ctypes.byref(op), ctypes.byref(v)), "sf_tuned_variant")
    return v.value


def sf_load_tuning(ctx, path):
    return _check(_lib().sf_load_tuning(ctx.handle, path.encode()), "sf_load_tuning")
