"""Python access to the plain FP64 CPU oracle (``mca_oracle.c``).

TEST INFRASTRUCTURE: only the tests, the smoke check and the CPU-baseline leg
of the benchmark use this package.  It imports nothing from the HIP solver
package and the solver imports nothing from here.

Each wrapper takes numpy float64 arrays (m x n row-major) and a geometry-like
object with the attributes m, n, g_top, g_bot, g_src, g_top_end, g_bot_end0,
g_bot_end1, v0, device.
"""

from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "mca_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")


def build() -> str:
    """Compile the oracle with gcc (plain -O2, single thread)."""
    cmd = ["gcc", "-O2", "-Wall", "-fPIC", "-shared", "-o", _LIB, _SRC, "-lm"]
    subprocess.run(cmd, check=True)
    return _LIB


class _Geom(C.Structure):
    _fields_ = [("m", C.c_int), ("n", C.c_int), ("device", C.c_int), ("pad_", C.c_int),
                ("g_top", C.c_double), ("g_bot", C.c_double), ("g_src", C.c_double),
                ("g_top_end", C.c_double), ("g_bot_end0", C.c_double),
                ("g_bot_end1", C.c_double), ("v0", C.c_double)]


_lib = None
_P = np.ctypeslib.ndpointer(dtype=np.float64, flags="C_CONTIGUOUS")


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        build()
    lib = C.CDLL(_LIB)
    G = C.POINTER(_Geom)
    d = C.c_double
    lib.orc_wire_matrix.argtypes = [C.c_int, d, d, d, _P, _P]
    lib.orc_residual.argtypes = [G, _P, _P, _P, _P, _P, _P, _P]
    lib.orc_source_norm.argtypes = [G, _P]
    lib.orc_source_norm.restype = d
    lib.orc_jacobian_apply.argtypes = [G, _P, _P, _P, _P, _P]
    lib.orc_dense_jacobian.argtypes = [G, _P, _P]
    lib.orc_dense_precond.argtypes = [G, d, d, _P]
    lib.orc_dense_solve.argtypes = [C.c_int, _P, _P]
    lib.orc_precond_apply_dense.argtypes = [G, d, d, _P, _P, _P, _P]
    lib.orc_precond_apply_band.argtypes = [G, d, d, _P, _P, _P, _P]
    lib.orc_jacobian_solve_band.argtypes = [G, _P, _P, _P, _P, _P]
    lib.orc_jacobian_solve_cg.argtypes = [G, _P, _P, _P, _P, _P, d, C.c_int]
    lib.orc_solve.argtypes = [G, _P, _P, _P, _P, d, C.c_int, C.c_int, _P]
    lib.orc_mhat_inverse_apply.argtypes = [G, d, d, _P, _P]
    lib.orc_mhat_inverse_apply.restype = None
    lib.orc_precond_apply_approx.argtypes = [G, d, d, _P, _P, _P, _P]
    lib.orc_precond_apply_approx.restype = None
    lib.orc_jacobi_apply.argtypes = [G, _P, _P, _P, _P, _P]
    lib.orc_jacobi_apply.restype = None
    lib.orc_sweep_guess.argtypes = [G, _P, _P, _P, _P]
    lib.orc_sweep_guess.restype = None
    _lib = lib
    return lib


def _geom(g) -> _Geom:
    return _Geom(int(g.m), int(g.n), int(getattr(g, "device", 0)), 0,
                 float(g.g_top), float(g.g_bot), float(g.g_src), float(g.g_top_end),
                 float(g.g_bot_end0), float(g.g_bot_end1), float(g.v0))


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.float64)


def wire_matrix(length: int, g: float, end0: float, end1: float):
    """(diag, off) of one wire's tridiagonal conductance matrix, eq. (G)."""
    diag = np.zeros(length)
    off = np.zeros(max(length, 1))
    _load().orc_wire_matrix(length, g, end0, end1, diag, off)
    return diag, off[: length - 1]


def residual(geom, g_dev, v_in, v_t, v_b):
    """(F_t, F_b, D) of eqs. (MNA)/(F) at (v_t, v_b)."""
    m, n = geom.m, geom.n
    ft, fb, d = np.zeros((m, n)), np.zeros((m, n)), np.zeros((m, n))
    _load().orc_residual(C.byref(_geom(geom)), _f64(g_dev), _f64(v_in), _f64(v_t),
                         _f64(v_b), ft, fb, d)
    return ft, fb, d


def source_norm(geom, v_in) -> float:
    return float(_load().orc_source_norm(C.byref(_geom(geom)), _f64(v_in)))


def jacobian_apply(geom, d, x_t, x_b):
    """(y_t, y_b) = J(D) [x_t; x_b], eq. (J)."""
    m, n = geom.m, geom.n
    yt, yb = np.zeros((m, n)), np.zeros((m, n))
    _load().orc_jacobian_apply(C.byref(_geom(geom)), _f64(d), _f64(x_t), _f64(x_b), yt, yb)
    return yt, yb


def dense_jacobian(geom, d) -> np.ndarray:
    N = 2 * geom.m * geom.n
    A = np.zeros((N, N))
    _load().orc_dense_jacobian(C.byref(_geom(geom)), _f64(d), A)
    return A


def dense_precond(geom, a1: float, a2: float) -> np.ndarray:
    N = 2 * geom.m * geom.n
    A = np.zeros((N, N))
    _load().orc_dense_precond(C.byref(_geom(geom)), float(a1), float(a2), A)
    return A


def dense_solve(A, b) -> np.ndarray:
    """The oracle's own Gaussian elimination with partial pivoting."""
    A = _f64(A).copy()
    x = _f64(b).copy()
    if _load().orc_dense_solve(A.shape[0], A, x) != 0:
        raise np.linalg.LinAlgError("zero pivot")
    return x


def precond_apply(geom, a1: float, a2: float, r_t, r_b, method: str = "auto"):
    """(z_t, z_b) = P^{-1} [r_t; r_b] for P of eq. (P)."""
    m, n = geom.m, geom.n
    zt, zb = np.zeros((m, n)), np.zeros((m, n))
    if method == "auto":
        method = "dense" if 2 * m * n <= 1024 else "band"
    fn = _load().orc_precond_apply_dense if method == "dense" else _load().orc_precond_apply_band
    rc = fn(C.byref(_geom(geom)), float(a1), float(a2), _f64(r_t), _f64(r_b), zt, zb)
    if rc != 0:
        raise RuntimeError(f"oracle precond_apply failed ({rc})")
    return zt, zb


def mhat_inverse_apply(geom, a1: float, a2: float, w):
    """Mhat^{-1} w of eqs. (Mhat), (M-1hat), (2matrix4): G2hat^{-1} W G1^{-1}."""
    out = np.zeros((geom.m, geom.n))
    _load().orc_mhat_inverse_apply(C.byref(_geom(geom)), float(a1), float(a2), _f64(w), out)
    return out


def precond_apply_approx(geom, a1: float, a2: float, r_t, r_b):
    """(z_t, z_b) = eq. (block) with the paper's approximation M ~ Mhat."""
    zt, zb = np.zeros((geom.m, geom.n)), np.zeros((geom.m, geom.n))
    _load().orc_precond_apply_approx(C.byref(_geom(geom)), float(a1), float(a2), _f64(r_t),
                                     _f64(r_b), zt, zb)
    return zt, zb


def jacobi_apply(geom, d, r_t, r_b):
    """(z_t, z_b) = r ./ diag(J(d)): the point-Jacobi baseline."""
    zt, zb = np.zeros((geom.m, geom.n)), np.zeros((geom.m, geom.n))
    _load().orc_jacobi_apply(C.byref(_geom(geom)), _f64(d), _f64(r_t), _f64(r_b), zt, zb)
    return zt, zb


def sweep_guess(geom, g_dev, v_in):
    """(V_t, V_b) of one block Gauss-Seidel sweep on J(0) V = Y."""
    vt, vb = np.zeros((geom.m, geom.n)), np.zeros((geom.m, geom.n))
    _load().orc_sweep_guess(C.byref(_geom(geom)), _f64(g_dev), _f64(v_in), vt, vb)
    return vt, vb


def jacobian_solve(geom, d, b_t, b_b, method: str = "band", rel_tol: float = 1e-13):
    m, n = geom.m, geom.n
    xt, xb = np.zeros((m, n)), np.zeros((m, n))
    if method == "band":
        rc = _load().orc_jacobian_solve_band(C.byref(_geom(geom)), _f64(d), _f64(b_t),
                                             _f64(b_b), xt, xb)
    else:
        rc = _load().orc_jacobian_solve_cg(C.byref(_geom(geom)), _f64(d), _f64(b_t),
                                           _f64(b_b), xt, xb, float(rel_tol), 100000)
        rc = 0 if rc >= 0 else rc
    if rc != 0:
        raise RuntimeError(f"oracle jacobian_solve failed ({rc})")
    return xt, xb


def solve(geom, g_dev, v_in, tol: float = 1e-14, max_it: int = 50,
          method: str = "auto", guess=None):
    """Steady state by Newton's method with direct (band) or CG linear steps.

    Returns (v_t, v_b, newton_steps, history of ||F||/||Y||).
    """
    m, n = geom.m, geom.n
    if method == "auto":
        # band storage (p+1) * 2mn doubles, p = 2 min(m, n)
        method = "band" if (2 * min(m, n) + 1) * 2 * m * n * 8 <= (1 << 30) else "cg"
    vt = np.zeros((m, n)) if guess is None else _f64(guess[0]).copy()
    vb = np.zeros((m, n)) if guess is None else _f64(guess[1]).copy()
    hist = np.zeros(max_it + 1)
    k = _load().orc_solve(C.byref(_geom(geom)), _f64(g_dev), _f64(v_in), vt, vb,
                          float(tol), int(max_it), 1 if method == "cg" else 0, hist)
    if k < 0:
        raise RuntimeError("oracle Newton did not converge")
    return vt, vb, k, hist[: k + 1]
