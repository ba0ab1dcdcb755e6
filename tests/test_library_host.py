"""Host-side checks of libmca.so that need no GPU.

* the library loads and exports every entry point include/mca.h declares;
* geometry and option validation;
* the plan's host eigen-decomposition of the wire matrices (eq. (G) with
  terminations), pinned by the DST-I closed form of the paper's uniform G,
  by orthogonality, and by G Q = Q diag(lambda) against numpy's assembly.
"""

import ctypes as C
import os
import re

import numpy as np
import pytest

from paper_2109_07929_amd import binding as B
from paper_2109_07929_amd import synth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_header_symbols_are_exported():
    header = open(os.path.join(ROOT, "include", "mca.h")).read()
    declared = set(re.findall(r"\b(mca_[a-z_]+)\s*\(", header))
    assert declared == set(B.ABI_SYMBOLS)
    lib = B.lib()
    for name in declared:
        assert hasattr(lib, name), name


def test_struct_layouts_match_the_library():
    lib = B.lib()
    for which, st in enumerate((B.mca_geometry, B.mca_options, B.mca_stats)):
        assert lib.mca_abi_struct_size(which) == C.sizeof(st), st.__name__
    assert lib.mca_abi_struct_size(3) == 0


def test_status_strings():
    assert B.status_string(B.MCA_OK) == "ok"
    assert "converged" in B.status_string(B.MCA_ERR_NOT_CONVERGED)


def test_options_default():
    o = B.options()
    assert o.restart == 30 and o.gmres_tol == 1e-8 and o.newton_tol == 1e-10
    assert o.precision == B.MCA_PREC_FP64 and o.precond == B.MCA_PRECOND_LITERAL


@pytest.mark.parametrize("bad", [
    dict(m=0), dict(n=0), dict(g_top=0.0), dict(g_bot=-1.0), dict(g_src=float("nan")),
    dict(g_src=0.0, g_top_end=0.0), dict(g_bot_end0=0.0, g_bot_end1=0.0), dict(v0=0.0),
    dict(device=7),
])
def test_invalid_geometry_rejected(bad):
    kw = dict(m=4, n=5)
    kw.update(bad)
    g = B.geometry(**kw)
    with pytest.raises(B.MCAError) as e:
        B.mca_plan_create(g)
    assert e.value.status == B.MCA_ERR_INVALID_ARG


def test_linear_device_needs_no_v0():
    P = B.mca_plan_create(B.geometry(3, 3, v0=0.0, device=B.MCA_DEVICE_LINEAR))
    B.mca_plan_destroy(P)


def test_workspace_bytes_reject_bad_options():
    P = B.mca_plan_create(B.geometry(8, 8))
    try:
        assert B.mca_workspace_bytes(P, B.options(restart=0)) == 0
        assert B.mca_workspace_bytes(P, B.options(restart=65)) == 0
        ok = B.mca_workspace_bytes(P, B.options())
        assert ok > 31 * 2 * 64 * 8
        assert B.mca_workspace_bytes(P, B.options(restart=10)) < ok
    finally:
        B.mca_plan_destroy(P)


def _tri(length, g, e0, e1):
    T = np.zeros((length, length))
    for k in range(length - 1):
        T[k, k] += g
        T[k + 1, k + 1] += g
        T[k, k + 1] = T[k + 1, k] = -g
    T[0, 0] += e0
    T[-1, -1] += e1
    return T


@pytest.mark.parametrize("n", [1, 2, 3, 8, 31, 64, 257])
def test_eigen_matches_dst1_closed_form(n):
    """Both ends tied through g: G is eq. (G), lambda_k = 2g(1 - cos(k pi/(n+1))),
    eigenvectors sqrt(2/(n+1)) sin(j k pi/(n+1)) (the DST-I basis)."""
    g = 0.7
    P = B.mca_plan_create(B.geometry(2, n, g_top=g, g_src=g, g_top_end=g))
    try:
        lam, Q = B.mca_plan_host_eigen(P, 0, n)
    finally:
        B.mca_plan_destroy(P)
    k = np.arange(1, n + 1)
    ref = 2 * g * (1 - np.cos(k * np.pi / (n + 1)))
    np.testing.assert_allclose(lam, ref, rtol=0, atol=4e-15 * 4 * g)
    j = np.arange(1, n + 1)[:, None]
    S = np.sqrt(2.0 / (n + 1)) * np.sin(j * k[None, :] * np.pi / (n + 1))
    # equal up to the sign of each column
    signs = np.sign(np.sum(S * Q, axis=0))
    np.testing.assert_allclose(Q * signs, S, rtol=0, atol=2e-13)


@pytest.mark.parametrize("m,n", [(1, 1), (5, 3), (33, 17), (128, 96)])
def test_eigen_of_terminated_wires(m, n):
    geo = synth.Geometry(m, n)
    P = B.mca_plan_create(B.geometry_from(geo))
    try:
        for layer, L, (g, e0, e1) in ((0, n, (geo.g_top, geo.g_src, geo.g_top_end)),
                                      (1, m, (geo.g_bot, geo.g_bot_end0, geo.g_bot_end1))):
            lam, Q = B.mca_plan_host_eigen(P, layer, L)
            T = _tri(L, g, e0, e1)
            assert np.all(np.diff(lam) > 0)
            np.testing.assert_allclose(Q.T @ Q, np.eye(L), rtol=0, atol=1e-13)
            np.testing.assert_allclose(T @ Q, Q * lam, rtol=0, atol=1e-14)
            np.testing.assert_allclose(lam, np.linalg.eigvalsh(T), rtol=0, atol=4e-15)
    finally:
        B.mca_plan_destroy(P)


@pytest.mark.slow
def test_eigen_1024_orthogonal():
    geo = synth.Geometry(1024, 1024)
    P = B.mca_plan_create(B.geometry_from(geo))
    try:
        lam, Q = B.mca_plan_host_eigen(P, 0, 1024)
    finally:
        B.mca_plan_destroy(P)
    T = _tri(1024, geo.g_top, geo.g_src, geo.g_top_end)
    assert np.abs(Q.T @ Q - np.eye(1024)).max() < 2e-14
    assert np.abs(T @ Q - Q * lam).max() < 1e-14


def test_batch_host_setup():
    """mca_batch_create: offsets of the concatenated arrays, per-crossbar eigen data,
    option validation of the batched solve (host only)."""
    geoms = [B.geometry(3, 5), B.geometry(64, 17, g_top=0.3), B.geometry(1, 1)]
    h = B.mca_batch_create(geoms)
    try:
        cross, rows = B.mca_batch_offsets(h, 3)
        assert list(cross) == [0, 15, 15 + 64 * 17, 15 + 64 * 17 + 1]
        assert list(rows) == [0, 3, 67, 68]
        assert B.mca_batch_device_bytes(h) > 0
        ok = B.options(precond=B.MCA_PRECOND_PERMODE, precision=B.MCA_PREC_BF16X3)
        n_ok = B.mca_batch_workspace_bytes(h, ok)
        assert n_ok > 0 and n_ok % 256 == 0
        assert B.mca_batch_workspace_bytes(h, None) == n_ok
        # FP64 and the literal form are single-crossbar only
        assert B.mca_batch_workspace_bytes(h, B.options()) == 0
        assert B.mca_batch_workspace_bytes(
            h, B.options(precond=B.MCA_PRECOND_LITERAL, precision=B.MCA_PREC_FP32)) == 0
        assert B.mca_batch_workspace_bytes(h, B.options(
            precond=B.MCA_PRECOND_PERMODE, precision=B.MCA_PREC_FP32, restart=0)) == 0
        # larger restart -> more Krylov storage
        big = B.options(precond=B.MCA_PRECOND_PERMODE, precision=B.MCA_PREC_BF16X3, restart=40)
        assert B.mca_batch_workspace_bytes(h, big) > n_ok
    finally:
        B.mca_batch_destroy(h)


def test_batch_create_rejects_bad_geometry():
    with pytest.raises(B.MCAError) as e:
        B.mca_batch_create([B.geometry(4, 4), B.geometry(0, 4)])
    assert e.value.status == B.MCA_ERR_INVALID_ARG
    with pytest.raises(B.MCAError):
        B.mca_batch_create([])


def test_approx_and_jacobi_forms_validation():
    """The approximate (paper's Mhat) and Jacobi forms are FP64-only."""
    P = B.mca_plan_create(B.geometry(8, 8))
    try:
        for form in (B.MCA_PRECOND_APPROX, B.MCA_PRECOND_JACOBI):
            assert B.mca_workspace_bytes(P, B.options(precond=form)) > 0
            assert B.mca_workspace_bytes(P, B.options(precond=form,
                                                      precision=B.MCA_PREC_FP32)) == 0
        assert B.mca_workspace_bytes(P, B.options(precond=5)) == 0
        # the approximate form needs its multiplier tables; Jacobi no workspace
        assert B.mca_precond_workspace_bytes(P, B.MCA_PRECOND_APPROX) > 0
    finally:
        B.mca_plan_destroy(P)


def test_batch_shares_set_up_of_equal_geometries():
    """Crossbars with the same geometry share one eigen set-up and one copy of the
    device eigenbases."""
    same = B.mca_batch_create([B.geometry(40, 30)] * 3)
    diff = B.mca_batch_create([B.geometry(40, 30, g_top=0.3 + 0.1 * k) for k in range(3)])
    one = B.mca_batch_create([B.geometry(40, 30)])
    try:
        per_plan = B.mca_batch_device_bytes(diff) - B.mca_batch_device_bytes(same)
        assert per_plan > 2 * 4 * (40 * 40 + 30 * 30)       # two plans' FP32 + bf16 planes
        assert B.mca_batch_device_bytes(same) - B.mca_batch_device_bytes(one) < 8192
    finally:
        for h in (same, diff, one):
            B.mca_batch_destroy(h)


@pytest.mark.parametrize("sizes,count,tile", [
    ((1024, 1024), 4, 128),        # 4 x 64 tiles of 128: 256
    ((300, 520), 4, 64),           # 4 x 15 = 60 tiles of 128: too few
    ((300, 520), 18, 128),         # 18 x 15 = 270
    ((255, 1024), 8, 64),          # a side below 256
    ((64, 64), 300, 64),
])
def test_batch_product_tile_choice(sizes, count, tile):
    """128 x 128 product tiles only when every side is >= 256 and a product has
    at least 256 of them (host query, no GPU)."""
    h = B.mca_batch_create([B.geometry(*sizes)] * count)
    try:
        assert B.mca_batch_product_tile(h) == tile
    finally:
        B.mca_batch_destroy(h)
