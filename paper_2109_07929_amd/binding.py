"""ctypes binding of libmca.so: the C ABI of include/mca.h, argument marshalling only.

Every function keeps the C name and order of arguments.  Array arguments are
torch float64 tensors on the GPU (contiguous, m x n, or length m for v_in);
the binding passes their device pointers and the current HIP stream.  All
computation happens inside libmca.so.  If the library is missing, every call
raises: there is no fallback path.
"""

from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libmca.so")

MCA_OK = 0
MCA_ERR_INVALID_ARG = 1
MCA_ERR_NONFINITE = 2
MCA_ERR_WORKSPACE = 3
MCA_ERR_NOT_CONVERGED = 4
MCA_ERR_BREAKDOWN = 5
MCA_ERR_HIP = 6

MCA_DEVICE_SINH = 0
MCA_DEVICE_LINEAR = 1
MCA_PREC_FP64 = 0
MCA_PREC_FP32 = 1
MCA_PREC_BF16X3 = 2
MCA_PREC_BF16 = 3
MCA_PRECOND_LITERAL = 0
MCA_PRECOND_PERMODE = 1
MCA_PRECOND_NONE = 2
MCA_PRECOND_APPROX = 3
MCA_PRECOND_JACOBI = 4
MCA_FLAG_INITIAL_GUESS = 1
MCA_FLAG_TIMING = 2
MCA_FLAG_GUESS_FALLBACK = 4
MCA_FLAG_SWEEP_START = 8
MCA_FLAG_GRAPH = 16
MCA_FLAG_MGS_PASSES = 32
MCA_FLAG_TIMING_SAMPLED = 64
MCA_KCLASS_GEMM = 0
MCA_KCLASS_JACOBIAN = 1
MCA_KCLASS_ORTHO = 2
MCA_KCLASS_RESIDUAL = 3
MCA_NUM_KCLASS = 4
MCA_MAX_RESTART = 64
MCA_MAX_NEWTON = 64

# every entry point include/mca.h declares
ABI_SYMBOLS = (
    "mca_options_default", "mca_status_string", "mca_last_error", "mca_abi_struct_size",
    "mca_plan_create", "mca_plan_destroy", "mca_plan_host_eigen",
    "mca_plan_device_bytes", "mca_plan_upload", "mca_workspace_bytes",
    "mca_precond_workspace_bytes", "mca_residual", "mca_jacobian_apply",
    "mca_precond_apply", "mca_precond_apply_noalloc", "mca_solve",
    "mca_batch_create", "mca_batch_destroy", "mca_batch_offsets", "mca_batch_device_bytes",
    "mca_batch_product_tile", "mca_batch_upload", "mca_batch_workspace_bytes", "mca_solve_batched",
    "mca_cnn_param_count", "mca_cnn_workspace_bytes", "mca_cnn_predict", "mca_cnn_gradient",
    "mca_cnn_adam",
)


class mca_geometry(C.Structure):
    _fields_ = [("m", C.c_int32), ("n", C.c_int32), ("device_model", C.c_int32),
                ("reserved", C.c_int32), ("g_top", C.c_double), ("g_bot", C.c_double),
                ("g_src", C.c_double), ("g_top_end", C.c_double), ("g_bot_end0", C.c_double),
                ("g_bot_end1", C.c_double), ("v0", C.c_double)]


class mca_options(C.Structure):
    _fields_ = [("newton_tol", C.c_double), ("gmres_tol", C.c_double), ("restart", C.c_int32),
                ("max_newton", C.c_int32), ("max_krylov", C.c_int32), ("precision", C.c_int32),
                ("precond", C.c_int32), ("flags", C.c_int32)]


class mca_stats(C.Structure):
    _fields_ = [("newton_iters", C.c_int32), ("krylov_iters", C.c_int32),
                ("backtracks", C.c_int32), ("restarts", C.c_int32),
                ("rel_residual", C.c_double), ("a_last", C.c_double),
                ("residual_history", C.c_double * (MCA_MAX_NEWTON + 1)),
                ("krylov_history", C.c_int32 * MCA_MAX_NEWTON),
                ("kernel_ms", C.c_double * MCA_NUM_KCLASS),
                ("kernel_launches", C.c_int32 * MCA_NUM_KCLASS), ("start", C.c_int32),
                ("err_bound", C.c_double)]

    def history(self):
        k = self.newton_iters
        return (list(self.residual_history[: k + 1]), list(self.krylov_history[:k]))


class MCAError(RuntimeError):
    def __init__(self, status: int, what: str):
        self.status = status
        super().__init__(f"{what}: {status_string(status)} ({status})"
                         + (f" [{last_error()}]" if status == MCA_ERR_HIP else ""))


_lib = None


def lib():
    """The loaded libmca.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with "
                          "`python -m paper_2109_07929_amd.build` (there is no CPU fallback)")
    L = C.CDLL(LIB_PATH)
    vp, sz, i32, dbl = C.c_void_p, C.c_size_t, C.c_int32, C.c_double
    PP = C.POINTER(C.c_void_p)
    L.mca_options_default.argtypes = [C.POINTER(mca_options)]
    L.mca_options_default.restype = None
    L.mca_status_string.argtypes = [i32]
    L.mca_status_string.restype = C.c_char_p
    L.mca_last_error.argtypes = []
    L.mca_last_error.restype = C.c_char_p
    L.mca_abi_struct_size.argtypes = [C.c_int32]
    L.mca_abi_struct_size.restype = C.c_size_t
    for which, st in enumerate((mca_geometry, mca_options, mca_stats)):
        if L.mca_abi_struct_size(which) != C.sizeof(st):
            raise ImportError(f"{LIB_PATH}: {st.__name__} is {L.mca_abi_struct_size(which)} bytes "
                              f"in the library and {C.sizeof(st)} in the binding")
    L.mca_plan_create.argtypes = [C.POINTER(mca_geometry), PP]
    L.mca_plan_create.restype = i32
    L.mca_plan_destroy.argtypes = [vp]
    L.mca_plan_destroy.restype = None
    L.mca_plan_host_eigen.argtypes = [vp, i32, vp, vp]
    L.mca_plan_host_eigen.restype = i32
    L.mca_plan_device_bytes.argtypes = [vp]
    L.mca_plan_device_bytes.restype = sz
    L.mca_plan_upload.argtypes = [vp, vp, sz, vp]
    L.mca_plan_upload.restype = i32
    L.mca_workspace_bytes.argtypes = [vp, C.POINTER(mca_options)]
    L.mca_workspace_bytes.restype = sz
    L.mca_precond_workspace_bytes.argtypes = [vp, i32, i32]
    L.mca_precond_workspace_bytes.restype = sz
    L.mca_residual.argtypes = [vp, vp, vp, vp, vp, vp, vp, vp, vp]
    L.mca_residual.restype = i32
    L.mca_jacobian_apply.argtypes = [vp, vp, vp, vp, vp, vp, vp]
    L.mca_jacobian_apply.restype = i32
    L.mca_precond_apply.argtypes = [vp, i32, i32, dbl, dbl, vp, vp, vp, vp, vp, sz, vp]
    L.mca_precond_apply.restype = i32
    L.mca_precond_apply_noalloc.argtypes = [vp, i32, i32, dbl, dbl, vp, vp, vp, vp, vp]
    L.mca_precond_apply_noalloc.restype = i32
    L.mca_solve.argtypes = [vp, vp, vp, vp, vp, C.POINTER(mca_options), vp, sz,
                            C.POINTER(mca_stats), vp]
    L.mca_solve.restype = i32
    L.mca_batch_create.argtypes = [i32, C.POINTER(mca_geometry), PP]
    L.mca_batch_create.restype = i32
    L.mca_batch_destroy.argtypes = [vp]
    L.mca_batch_destroy.restype = None
    L.mca_batch_offsets.argtypes = [vp, vp, vp]
    L.mca_batch_offsets.restype = i32
    L.mca_batch_device_bytes.argtypes = [vp]
    L.mca_batch_device_bytes.restype = sz
    L.mca_batch_upload.argtypes = [vp, vp, sz, vp]
    L.mca_batch_upload.restype = i32
    L.mca_batch_product_tile.argtypes = [vp]
    L.mca_batch_product_tile.restype = i32
    L.mca_batch_workspace_bytes.argtypes = [vp, C.POINTER(mca_options)]
    L.mca_batch_workspace_bytes.restype = sz
    L.mca_solve_batched.argtypes = [vp, vp, vp, vp, vp, C.POINTER(mca_options), vp, sz,
                                    C.POINTER(mca_stats), vp]
    L.mca_solve_batched.restype = i32
    L.mca_cnn_param_count.argtypes = []
    L.mca_cnn_param_count.restype = C.c_int64
    L.mca_cnn_workspace_bytes.argtypes = [i32, i32, i32]
    L.mca_cnn_workspace_bytes.restype = sz
    L.mca_cnn_predict.argtypes = [vp, i32, C.POINTER(mca_geometry), vp, vp, vp, vp, vp, sz, vp]
    L.mca_cnn_predict.restype = i32
    L.mca_cnn_gradient.argtypes = [vp, i32, C.POINTER(mca_geometry), vp, vp, vp, vp, vp, vp, vp,
                                   sz, vp]
    L.mca_cnn_gradient.restype = i32
    L.mca_cnn_adam.argtypes = [vp, vp, vp, vp, i32, C.c_float, vp]
    L.mca_cnn_adam.restype = i32
    _lib = L
    return L


def status_string(status: int) -> str:
    return lib().mca_status_string(int(status)).decode()


def last_error() -> str:
    return lib().mca_last_error().decode()


def _check(status: int, what: str) -> int:
    if status != MCA_OK:
        raise MCAError(status, what)
    return status


# ------------------------------------------------------------- marshalling
def _stream(stream):
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return C.c_void_p(stream.cuda_stream if hasattr(stream, "cuda_stream") else int(stream))


def _ptr(t, numel=None, what="array"):
    """Device pointer of a contiguous float64 GPU tensor (None -> NULL)."""
    import torch
    if t is None:
        return None
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{what}: expected a torch tensor")
    if not t.is_cuda or t.dtype != torch.float64 or not t.is_contiguous():
        raise ValueError(f"{what}: expected a contiguous float64 GPU tensor")
    if numel is not None and t.numel() != numel:
        raise ValueError(f"{what}: expected {numel} elements, got {t.numel()}")
    return C.c_void_p(t.data_ptr())


def _buf(t, what="buffer"):
    import torch
    if t is None:
        return None, 0
    if not isinstance(t, torch.Tensor) or not t.is_cuda or not t.is_contiguous():
        raise ValueError(f"{what}: expected a contiguous GPU tensor")
    return C.c_void_p(t.data_ptr()), t.numel() * t.element_size()


def geometry(m, n, g_top=0.4, g_bot=0.4, g_src=0.4, g_top_end=1e-3, g_bot_end0=0.1,
             g_bot_end1=0.1, v0=0.25, device=MCA_DEVICE_SINH) -> mca_geometry:
    return mca_geometry(int(m), int(n), int(device), 0, float(g_top), float(g_bot),
                        float(g_src), float(g_top_end), float(g_bot_end0), float(g_bot_end1),
                        float(v0))


def geometry_from(g) -> mca_geometry:
    """mca_geometry from any object with the synth.Geometry attributes."""
    return geometry(g.m, g.n, g.g_top, g.g_bot, g.g_src, g.g_top_end, g.g_bot_end0,
                    g.g_bot_end1, g.v0, getattr(g, "device", MCA_DEVICE_SINH))


def options(**kw) -> mca_options:
    o = mca_options()
    lib().mca_options_default(C.byref(o))
    for k, v in kw.items():
        if not hasattr(o, k):
            raise AttributeError(k)
        setattr(o, k, v)
    return o


# ------------------------------------------------------------ the C ABI
def mca_options_default() -> mca_options:
    return options()


def mca_plan_create(geom: mca_geometry) -> C.c_void_p:
    out = C.c_void_p()
    _check(lib().mca_plan_create(C.byref(geom), C.byref(out)), "mca_plan_create")
    return out


def mca_plan_destroy(plan) -> None:
    lib().mca_plan_destroy(plan)


def mca_plan_host_eigen(plan, layer: int, length: int):
    lam = np.zeros(length)
    q = np.zeros((length, length))
    _check(lib().mca_plan_host_eigen(plan, int(layer), lam.ctypes.data_as(C.c_void_p),
                                     q.ctypes.data_as(C.c_void_p)), "mca_plan_host_eigen")
    return lam, q


def mca_plan_device_bytes(plan) -> int:
    return int(lib().mca_plan_device_bytes(plan))


def mca_plan_upload(plan, dev_buf, stream=None) -> None:
    p, nbytes = _buf(dev_buf, "dev_buf")
    _check(lib().mca_plan_upload(plan, p, nbytes, _stream(stream)), "mca_plan_upload")


def mca_workspace_bytes(plan, opts: mca_options | None = None) -> int:
    return int(lib().mca_workspace_bytes(plan, C.byref(opts) if opts is not None else None))


def mca_precond_workspace_bytes(plan, form: int, precision: int = MCA_PREC_FP64) -> int:
    return int(lib().mca_precond_workspace_bytes(plan, int(form), int(precision)))


def mca_residual(plan, m, n, g_dev, v_in, v_t, v_b, f_t, f_b, d=None, stream=None) -> None:
    mn = m * n
    _check(lib().mca_residual(plan, _ptr(g_dev, mn, "g_dev"), _ptr(v_in, m, "v_in"),
                              _ptr(v_t, mn, "v_t"), _ptr(v_b, mn, "v_b"), _ptr(f_t, mn, "f_t"),
                              _ptr(f_b, mn, "f_b"), _ptr(d, mn, "d"), _stream(stream)),
           "mca_residual")


def mca_jacobian_apply(plan, m, n, d, x_t, x_b, y_t, y_b, stream=None) -> None:
    mn = m * n
    _check(lib().mca_jacobian_apply(plan, _ptr(d, mn, "d"), _ptr(x_t, mn, "x_t"),
                                    _ptr(x_b, mn, "x_b"), _ptr(y_t, mn, "y_t"),
                                    _ptr(y_b, mn, "y_b"), _stream(stream)),
           "mca_jacobian_apply")


def mca_precond_apply(plan, m, n, form, precision, a1, a2, r_t, r_b, z_t, z_b, ws,
                      stream=None) -> None:
    mn = m * n
    wp, wbytes = _buf(ws, "ws")
    _check(lib().mca_precond_apply(plan, int(form), int(precision), float(a1), float(a2),
                                   _ptr(r_t, mn, "r_t"), _ptr(r_b, mn, "r_b"),
                                   _ptr(z_t, mn, "z_t"), _ptr(z_b, mn, "z_b"), wp, wbytes,
                                   _stream(stream)), "mca_precond_apply")


MCA_NOALLOC_SCRATCH_BYTES = 32 << 20


def mca_precond_apply_noalloc(plan, m, n, form, precision, a1, a2, r_t, r_b, z_t, z_b,
                              stream=None) -> None:
    mn = m * n
    _check(lib().mca_precond_apply_noalloc(plan, int(form), int(precision), float(a1), float(a2),
                                           _ptr(r_t, mn, "r_t"), _ptr(r_b, mn, "r_b"),
                                           _ptr(z_t, mn, "z_t"), _ptr(z_b, mn, "z_b"),
                                           _stream(stream)), "mca_precond_apply_noalloc")


def mca_solve(plan, m, n, g_dev, v_in, v_t, v_b, opts: mca_options | None, ws, stream=None,
              check: bool = True):
    """Returns (status, mca_stats); raises on any status but MCA_OK when check is set."""
    mn = m * n
    wp, wbytes = _buf(ws, "ws")
    st = mca_stats()
    status = lib().mca_solve(plan, _ptr(g_dev, mn, "g_dev"), _ptr(v_in, m, "v_in"),
                             _ptr(v_t, mn, "v_t"), _ptr(v_b, mn, "v_b"),
                             C.byref(opts) if opts is not None else None, wp, wbytes,
                             C.byref(st), _stream(stream))
    if check:
        _check(status, "mca_solve")
    return status, st


# ---------------------------------------------------------------- batches
def mca_batch_create(geoms) -> C.c_void_p:
    arr = (mca_geometry * len(geoms))(*geoms)
    out = C.c_void_p()
    _check(lib().mca_batch_create(len(geoms), arr, C.byref(out)), "mca_batch_create")
    return out


def mca_batch_destroy(batch) -> None:
    lib().mca_batch_destroy(batch)


def mca_batch_offsets(batch, count: int):
    """(cross_offsets, row_offsets): int64 arrays of count + 1 entries."""
    cross = np.zeros(count + 1, dtype=np.int64)
    rows = np.zeros(count + 1, dtype=np.int64)
    _check(lib().mca_batch_offsets(batch, cross.ctypes.data_as(C.c_void_p),
                                   rows.ctypes.data_as(C.c_void_p)), "mca_batch_offsets")
    return cross, rows


def mca_batch_device_bytes(batch) -> int:
    return int(lib().mca_batch_device_bytes(batch))


def mca_batch_product_tile(batch) -> int:
    return int(lib().mca_batch_product_tile(batch))


def mca_batch_upload(batch, dev_buf, stream=None) -> None:
    p, nbytes = _buf(dev_buf, "dev_buf")
    _check(lib().mca_batch_upload(batch, p, nbytes, _stream(stream)), "mca_batch_upload")


def mca_batch_workspace_bytes(batch, opts: mca_options | None = None) -> int:
    return int(lib().mca_batch_workspace_bytes(batch, C.byref(opts) if opts is not None else None))


def mca_solve_batched(batch, count, total, rows, g_dev, v_in, v_t, v_b, opts, ws, stream=None,
                      check: bool = True):
    """Returns (status, [mca_stats] * count); total = sum m n, rows = sum m."""
    wp, wbytes = _buf(ws, "ws")
    st = (mca_stats * count)()
    status = lib().mca_solve_batched(batch, _ptr(g_dev, total, "g_dev"), _ptr(v_in, rows, "v_in"),
                                     _ptr(v_t, total, "v_t"), _ptr(v_b, total, "v_b"),
                                     C.byref(opts) if opts is not None else None, wp, wbytes,
                                     st, _stream(stream))
    if check:
        _check(status, "mca_solve_batched")
    return status, list(st)


# ------------------------------------------------------- warm-start network
def _f32(t, numel, what):
    import torch
    if not isinstance(t, torch.Tensor) or not t.is_cuda or t.dtype != torch.float32 or \
            not t.is_contiguous() or t.numel() != numel:
        raise ValueError(f"{what}: expected a contiguous float32 GPU tensor of {numel} values")
    return C.c_void_p(t.data_ptr())


def mca_cnn_param_count() -> int:
    return int(lib().mca_cnn_param_count())


def mca_cnn_workspace_bytes(batch, m, n) -> int:
    return int(lib().mca_cnn_workspace_bytes(int(batch), int(m), int(n)))


def _geoms(geoms):
    geoms = [g if isinstance(g, mca_geometry) else geometry_from(g) for g in geoms]
    return (mca_geometry * len(geoms))(*geoms), len(geoms), geoms[0].m, geoms[0].n


def mca_cnn_predict(params, geoms, g_dev, v_in, v_t, v_b, ws, stream=None):
    """geoms: one geometry (mca_geometry or synth.Geometry) per crossbar of the batch."""
    arr, batch, m, n = _geoms(geoms)
    P = batch * m * n
    wp, wbytes = _buf(ws, "ws")
    _check(lib().mca_cnn_predict(_f32(params, mca_cnn_param_count(), "params"), batch, arr,
                                 _ptr(g_dev, P, "g_dev"), _ptr(v_in, batch * m, "v_in"),
                                 _ptr(v_t, P, "v_t"), _ptr(v_b, P, "v_b"), wp, wbytes,
                                 _stream(stream)), "mca_cnn_predict")


def mca_cnn_gradient(params, geoms, g_dev, v_in, v_t, v_b, grad, loss, ws, stream=None):
    arr, batch, m, n = _geoms(geoms)
    P = batch * m * n
    wp, wbytes = _buf(ws, "ws")
    npar = mca_cnn_param_count()
    _check(lib().mca_cnn_gradient(_f32(params, npar, "params"), batch, arr,
                                  _ptr(g_dev, P, "g_dev"), _ptr(v_in, batch * m, "v_in"),
                                  _ptr(v_t, P, "v_t"), _ptr(v_b, P, "v_b"),
                                  _f32(grad, npar, "grad"), _f32(loss, 1, "loss"), wp, wbytes,
                                  _stream(stream)), "mca_cnn_gradient")


def mca_cnn_adam(params, grad, adam_m, adam_v, step, lr, stream=None):
    npar = mca_cnn_param_count()
    _check(lib().mca_cnn_adam(_f32(params, npar, "params"), _f32(grad, npar, "grad"),
                              _f32(adam_m, npar, "adam_m"), _f32(adam_v, npar, "adam_v"),
                              int(step), float(lr), _stream(stream)), "mca_cnn_adam")
