"""Pins of the CPU oracle against facts that do not come from the oracle.

Each test checks one oracle routine against an independent fact: a netlist
stamped element by element, dense LU from numpy, central finite differences,
a closed form, Kirchhoff's current law, a symmetry of the circuit, or the
exactness of the paper's preconditioner for uniform linear devices.  A
plausible slip anywhere in the oracle (a dropped termination, a sign, a
transposed layer, a wrong band index) fails at least one of them.
"""

import math
import os

import numpy as np
import pytest

import oracle
from paper_2109_07929_amd import synth

SHAPES = [(1, 1), (1, 5), (4, 1), (3, 4), (5, 3), (6, 6)]


def _geom(m, n, **kw):
    base = dict(g_top=0.4, g_bot=0.3, g_src=0.35, g_top_end=1e-3,
                g_bot_end0=0.1, g_bot_end1=0.07, v0=0.25)
    base.update(kw)
    return synth.Geometry(m, n, **base)


def _dev_i(geom, g, u):
    if geom.device == synth.DEVICE_LINEAR:
        return g * u
    return g * geom.v0 * math.sinh(u / geom.v0)


def netlist_residual(geom, g_dev, v_in, vt, vb):
    """KCL at every node, stamped from an explicit element list.

    Each two-terminal element adds the current it draws out of a node; the
    residual of a node is the total current leaving it.  This formulation
    never forms a wire matrix or a Kronecker product.
    """
    m, n = geom.m, geom.n
    volt = {}
    for i in range(m):
        for j in range(n):
            volt[("t", i, j)] = vt[i, j]
            volt[("b", i, j)] = vb[i, j]
        volt[("src", i)] = v_in[i]
    volt["gnd"] = 0.0
    res = {key: 0.0 for key in volt if key[0] in ("t", "b")}
    elements = []                                   # (node a, node b, conductance)
    for i in range(m):
        for j in range(n - 1):
            elements.append((("t", i, j), ("t", i, j + 1), geom.g_top))
        elements.append((("src", i), ("t", i, 0), geom.g_src))
        elements.append((("t", i, n - 1), "gnd", geom.g_top_end))
    for j in range(n):
        for i in range(m - 1):
            elements.append((("b", i, j), ("b", i + 1, j), geom.g_bot))
        elements.append((("b", 0, j), "gnd", geom.g_bot_end0))
        elements.append((("b", m - 1, j), "gnd", geom.g_bot_end1))
    for a, b, g in elements:
        cur = g * (volt[a] - volt[b])               # from a to b
        if a in res:
            res[a] += cur
        if b in res:
            res[b] -= cur
    for i in range(m):
        for j in range(n):
            cur = _dev_i(geom, g_dev[i, j], vt[i, j] - vb[i, j])   # top -> bottom
            res[("t", i, j)] += cur
            res[("b", i, j)] -= cur
    ft = np.array([[res[("t", i, j)] for j in range(n)] for i in range(m)])
    fb = np.array([[res[("b", i, j)] for j in range(n)] for i in range(m)])
    return ft, fb


@pytest.mark.parametrize("m,n", SHAPES)
@pytest.mark.parametrize("device", [synth.DEVICE_SINH, synth.DEVICE_LINEAR])
def test_residual_matches_netlist(m, n, device):
    geom = _geom(m, n, device=device)
    rng = np.random.default_rng(m * 100 + n)
    g_dev = np.exp(rng.uniform(np.log(1e-6), np.log(1e-3), (m, n)))
    v_in = rng.uniform(-0.3, 0.3, m)
    vt, vb = rng.uniform(-0.4, 0.4, (m, n)), rng.uniform(-0.2, 0.2, (m, n))
    ft, fb, d = oracle.residual(geom, g_dev, v_in, vt, vb)
    nt, nb = netlist_residual(geom, g_dev, v_in, vt, vb)
    scale = 0.4 * 0.4
    np.testing.assert_allclose(ft, nt, rtol=0, atol=1e-15 * scale * 10)
    np.testing.assert_allclose(fb, nb, rtol=0, atol=1e-15 * scale * 10)


def test_wire_matrix_is_paper_G_when_ends_equal_g():
    # eq. (G): 2g on the diagonal, -g off it, when both wire ends are tied through g
    diag, off = oracle.wire_matrix(7, 0.8, 0.8, 0.8)
    np.testing.assert_array_equal(diag, np.full(7, 1.6))
    np.testing.assert_array_equal(off, np.full(6, -0.8))


@pytest.mark.parametrize("m,n", [(3, 4), (5, 2), (1, 6)])
def test_device_slope_by_finite_differences(m, n):
    geom = _geom(m, n)
    rng = np.random.default_rng(7)
    g_dev = rng.uniform(1e-5, 1e-4, (m, n))
    vt, vb = rng.uniform(0, 0.3, (m, n)), rng.uniform(0, 0.1, (m, n))
    _, _, d = oracle.residual(geom, g_dev, np.zeros(m), vt, vb)
    h = 1e-5
    u = vt - vb
    i_plus = g_dev * geom.v0 * np.sinh((u + h) / geom.v0)
    i_minus = g_dev * geom.v0 * np.sinh((u - h) / geom.v0)
    np.testing.assert_allclose(d, (i_plus - i_minus) / (2 * h), rtol=1e-8)


@pytest.mark.parametrize("m,n", [(1, 1), (3, 4), (5, 3), (4, 4)])
def test_jacobian_is_derivative_of_residual(m, n):
    """J x against central differences of the (netlist-pinned) residual."""
    geom = _geom(m, n)
    rng = np.random.default_rng(11)
    g_dev = np.exp(rng.uniform(np.log(1e-5), np.log(1e-3), (m, n)))
    v_in = rng.uniform(0, 0.3, m)
    vt, vb = rng.uniform(0, 0.3, (m, n)), rng.uniform(0, 0.15, (m, n))
    xt, xb = rng.standard_normal((m, n)), rng.standard_normal((m, n))
    _, _, d = oracle.residual(geom, g_dev, v_in, vt, vb)
    yt, yb = oracle.jacobian_apply(geom, d, xt, xb)
    eps = 1e-6
    fpt, fpb, _ = oracle.residual(geom, g_dev, v_in, vt + eps * xt, vb + eps * xb)
    fmt, fmb, _ = oracle.residual(geom, g_dev, v_in, vt - eps * xt, vb - eps * xb)
    np.testing.assert_allclose(yt, (fpt - fmt) / (2 * eps), rtol=0, atol=1e-9)
    np.testing.assert_allclose(yb, (fpb - fmb) / (2 * eps), rtol=0, atol=1e-9)


@pytest.mark.parametrize("m,n", [(3, 4), (5, 3), (6, 6)])
def test_dense_jacobian_symmetric_positive_definite(m, n):
    geom = _geom(m, n)
    rng = np.random.default_rng(3)
    d = rng.uniform(1e-6, 1e-3, (m, n))
    J = oracle.dense_jacobian(geom, d)
    np.testing.assert_array_equal(J, J.T)
    assert np.linalg.eigvalsh(J).min() > 0
    x = rng.standard_normal(2 * m * n)
    yt, yb = oracle.jacobian_apply(geom, d, x[: m * n].reshape(m, n), x[m * n:].reshape(m, n))
    np.testing.assert_allclose(np.concatenate([yt.ravel(), yb.ravel()]), J @ x,
                               rtol=0, atol=1e-14)


def test_dense_solve_matches_numpy():
    rng = np.random.default_rng(5)
    A = rng.standard_normal((40, 40))
    b = rng.standard_normal(40)
    np.testing.assert_allclose(oracle.dense_solve(A, b), np.linalg.solve(A, b), rtol=1e-10)


@pytest.mark.parametrize("m,n", [(1, 1), (2, 7), (7, 2), (6, 5), (9, 12), (12, 9)])
def test_band_cholesky_solve_matches_dense(m, n):
    """Band Cholesky (both interleaved orderings, m > n and m < n) vs numpy LU."""
    geom = _geom(m, n)
    rng = np.random.default_rng(m * 13 + n)
    d = rng.uniform(1e-6, 1e-2, (m, n))
    bt, bb = rng.standard_normal((m, n)), rng.standard_normal((m, n))
    xt, xb = oracle.jacobian_solve(geom, d, bt, bb, method="band")
    J = oracle.dense_jacobian(geom, d)
    x = np.linalg.solve(J, np.concatenate([bt.ravel(), bb.ravel()]))
    scale = np.abs(x).max()
    np.testing.assert_allclose(np.concatenate([xt.ravel(), xb.ravel()]), x, rtol=0,
                               atol=1e-11 * scale)


@pytest.mark.parametrize("m,n", [(4, 4), (6, 9), (9, 6)])
def test_cg_solve_matches_band(m, n):
    geom = _geom(m, n)
    rng = np.random.default_rng(m * 7 + n)
    d = rng.uniform(1e-6, 1e-3, (m, n))
    bt, bb = rng.standard_normal((m, n)), rng.standard_normal((m, n))
    xt, xb = oracle.jacobian_solve(geom, d, bt, bb, method="band")
    ct, cb = oracle.jacobian_solve(geom, d, bt, bb, method="cg", rel_tol=1e-14)
    scale = max(np.abs(xt).max(), np.abs(xb).max())
    np.testing.assert_allclose(ct, xt, rtol=0, atol=1e-10 * scale)
    np.testing.assert_allclose(cb, xb, rtol=0, atol=1e-10 * scale)


def _kron_P(geom, a1, a2):
    """eq. (P) assembled with numpy Kronecker products from eqs. (Gt)/(Gb)."""
    m, n = geom.m, geom.n
    def tri(length, g, e0, e1):
        A = np.zeros((length, length))
        for k in range(length - 1):                  # one segment between k, k+1
            A[k, k] += g
            A[k + 1, k + 1] += g
            A[k, k + 1] -= g
            A[k + 1, k] -= g
        A[0, 0] += e0
        A[-1, -1] += e1
        return A
    Gtop = tri(n, geom.g_top, geom.g_src, geom.g_top_end)
    Gbot = tri(m, geom.g_bot, geom.g_bot_end0, geom.g_bot_end1)
    Gt = np.kron(np.eye(m), Gtop)
    Gb = np.kron(Gbot, np.eye(n))
    I = np.eye(m * n)
    return np.block([[Gt + a1 * I, -a1 * I], [-a2 * I, Gb + a2 * I]])


@pytest.mark.parametrize("m,n", [(1, 1), (1, 4), (3, 1), (3, 4), (5, 3)])
@pytest.mark.parametrize("a1,a2", [(2e-5, 2e-5), (3e-4, 7e-5)])
def test_precond_apply_matches_kron_definition(m, n, a1, a2):
    geom = _geom(m, n)
    rng = np.random.default_rng(17)
    rt, rb = rng.standard_normal((m, n)), rng.standard_normal((m, n))
    P = _kron_P(geom, a1, a2)
    np.testing.assert_allclose(oracle.dense_precond(geom, a1, a2), P, rtol=0, atol=0)
    z = np.linalg.solve(P, np.concatenate([rt.ravel(), rb.ravel()]))
    scale = np.abs(z).max()
    for method in ("dense", "band"):
        zt, zb = oracle.precond_apply(geom, a1, a2, rt, rb, method=method)
        np.testing.assert_allclose(np.concatenate([zt.ravel(), zb.ravel()]), z,
                                   rtol=0, atol=1e-10 * scale)


@pytest.mark.parametrize("m,n", [(4, 6), (7, 5)])
def test_precond_is_exact_for_uniform_devices(m, n):
    """With every device slope equal to a, P(a, a) equals J (Section III-A)."""
    geom = _geom(m, n)
    a = 4e-5
    d = np.full((m, n), a)
    np.testing.assert_array_equal(oracle.dense_jacobian(geom, d), oracle.dense_precond(geom, a, a))
    rng = np.random.default_rng(2)
    xt, xb = rng.standard_normal((m, n)), rng.standard_normal((m, n))
    yt, yb = oracle.jacobian_apply(geom, d, xt, xb)
    zt, zb = oracle.precond_apply(geom, a, a, yt, yb, method="band")
    np.testing.assert_allclose(zt, xt, rtol=0, atol=1e-9)
    np.testing.assert_allclose(zb, xb, rtol=0, atol=1e-9)


# ---------------------------------------------------------------- whole solve

def _bisect_1x1(geom, g, vin):
    gt1 = geom.g_src + geom.g_top_end
    gb1 = geom.g_bot_end0 + geom.g_bot_end1
    rhs = geom.g_src * vin / gt1
    f = lambda u: u + _dev_i(geom, g, u) * (1 / gt1 + 1 / gb1) - rhs
    lo, hi = min(0.0, rhs), max(0.0, rhs)
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        if mid == lo or mid == hi:
            break
        if f(mid) > 0:
            hi = mid
        else:
            lo = mid
    u = 0.5 * (lo + hi)
    cur = _dev_i(geom, g, u)
    return (geom.g_src * vin - cur) / gt1, cur / gb1


@pytest.mark.parametrize("g", [1e-6, 1e-4, 0.05])
@pytest.mark.parametrize("device", [synth.DEVICE_SINH, synth.DEVICE_LINEAR])
def test_solve_1x1_closed_form(g, device):
    geom = _geom(1, 1, device=device)
    vin = 0.27
    t, b = _bisect_1x1(geom, g, vin)
    vt, vb, k, hist = oracle.solve(geom, np.array([[g]]), np.array([vin]))
    assert abs(vt[0, 0] - t) <= 1e-14 * abs(t)
    assert abs(vb[0, 0] - b) <= 1e-14 * abs(t)
    if device == synth.DEVICE_LINEAR:
        gt1 = geom.g_src + geom.g_top_end
        gb1 = geom.g_bot_end0 + geom.g_bot_end1
        u = (geom.g_src * vin / gt1) / (1 + g * (1 / gt1 + 1 / gb1))
        assert abs((vt[0, 0] - vb[0, 0]) - u) <= 1e-14 * u


def _kcl_balance(geom, v_in, vt, vb, g_dev):
    """Current into the array from the sources, out through the terminations,
    and the total current through the devices vs out of the bottom ends."""
    i_in = np.sum(geom.g_src * (v_in - vt[:, 0]))
    i_top_out = np.sum(geom.g_top_end * vt[:, -1])
    i_bot_out = np.sum(geom.g_bot_end0 * vb[0, :] + geom.g_bot_end1 * vb[-1, :])
    u = vt - vb
    i_dev = np.sum(g_dev * geom.v0 * np.sinh(u / geom.v0))
    return i_in, i_top_out + i_bot_out, i_dev, i_bot_out


@pytest.mark.parametrize("m,n,method", [(32, 32, "band"), (16, 24, "band"), (24, 16, "band"),
                                        (32, 32, "cg")])
def test_solve_kirchhoff_and_zero_residual(m, n, method):
    cb = synth.crossbar(m, n, seed=0)
    vt, vb, k, hist = oracle.solve(cb.geom, cb.g_dev, cb.v_in, method=method)
    ft, fb, _ = netlist_residual(cb.geom, cb.g_dev, cb.v_in, vt, vb) if m * n <= 64 else \
        oracle.residual(cb.geom, cb.g_dev, cb.v_in, vt, vb)
    ynorm = np.linalg.norm(cb.geom.g_src * cb.v_in)
    assert np.sqrt(np.sum(ft ** 2) + np.sum(fb ** 2)) <= 1e-13 * ynorm
    i_in, i_out, i_dev, i_bot = _kcl_balance(cb.geom, cb.v_in, vt, vb, cb.g_dev)
    assert abs(i_in - i_out) <= 1e-12 * abs(i_in)
    assert abs(i_dev - i_bot) <= 1e-12 * abs(i_dev)
    assert 2 <= k <= 8


@pytest.mark.parametrize("m,n", [(1, 1), (1, 6), (5, 1), (4, 7), (7, 4)])
def test_source_norm_is_netlist_residual_at_zero(m, n):
    """||Y||_2 (the oracle's Newton scale) equals ||F(0)||_2 of the netlist.

    At V = 0 only the drive elements carry current, so the node residuals of
    the element-by-element netlist are minus the source currents: their norm
    is ||Y||.  g_src differs from g_top and from every termination here, so a
    norm built from the wrong element (or with v_in squared twice, or from one
    row only) fails.
    """
    geom = _geom(m, n)
    rng = np.random.default_rng(100 * m + n)
    v_in = rng.uniform(-0.3, 0.3, m)
    g_dev = rng.uniform(1e-6, 1e-4, (m, n))
    z = np.zeros((m, n))
    ft, fb = netlist_residual(geom, g_dev, v_in, z, z)
    ref = math.sqrt(float(np.sum(ft ** 2) + np.sum(fb ** 2)))
    assert abs(oracle.source_norm(geom, v_in) - ref) <= 1e-15 * ref
    # one driven row: the closed form g_src |v|
    one = np.zeros(m)
    one[m - 1] = -0.2
    assert abs(oracle.source_norm(geom, one) - geom.g_src * 0.2) <= 1e-16


def test_newton_history_starts_at_one():
    """The oracle's first recorded ratio is ||F(0)|| / ||Y|| = 1 (zero start)."""
    cb = synth.crossbar(6, 9, seed=11)
    _, _, _, hist = oracle.solve(cb.geom, cb.g_dev, cb.v_in)
    assert abs(hist[0] - 1.0) <= 1e-15


def _wire_lambda_min(length, g, e0, e1):
    from scipy.linalg import eigvalsh_tridiagonal
    if length == 1:
        return e0 + e1
    diag = np.full(length, 2.0 * g)
    diag[0], diag[-1] = g + e0, g + e1
    return float(eigvalsh_tridiagonal(diag, np.full(length - 1, -g), select="i",
                                      select_range=(0, 0))[0])


def _certified_rel_error(geom, g_dev, v_in, vt, vb):
    """||V - V*||_2 / max|V| bound from the residual alone.

    F is the gradient of a strongly convex energy: J(V) >= blkdiag(G_t, G_b)
    because dI/du >= 0, so ||V - V*|| <= ||F(V)|| / lambda_min with
    lambda_min = min(lambda_min(G_top), lambda_min(G_bot)) (scipy's
    tridiagonal eigenvalue routine on wire matrices written out here).
    """
    ft, fb, _ = oracle.residual(geom, g_dev, v_in, vt, vb)
    fn = math.sqrt(float(np.sum(ft ** 2) + np.sum(fb ** 2)))
    lam = min(_wire_lambda_min(geom.n, geom.g_top, geom.g_src, geom.g_top_end),
              _wire_lambda_min(geom.m, geom.g_bot, geom.g_bot_end0, geom.g_bot_end1))
    return fn / lam / max(np.abs(vt).max(), np.abs(vb).max())


@pytest.mark.slow
def test_band_and_cg_newton_agree_256():
    """Oracle A (band Cholesky Newton) and oracle B (CG Newton), 256 x 256.

    Two unrelated linear solvers inside the same Newton iteration reach the
    same steady state; the CG form is what the large-size GPU tests compare
    against.  About a minute (the band factorisation is O(mn min(m,n)^2)).
    """
    cb = synth.crossbar(256, 256, seed=0)
    a_t, a_b, ka, _ = oracle.solve(cb.geom, cb.g_dev, cb.v_in, method="band")
    c_t, c_b, kc, _ = oracle.solve(cb.geom, cb.g_dev, cb.v_in, method="cg")
    scale = max(np.abs(a_t).max(), np.abs(a_b).max())
    assert max(np.abs(a_t - c_t).max(), np.abs(a_b - c_b).max()) <= 1e-12 * scale
    assert ka == kc


@pytest.mark.slow
@pytest.mark.skipif(os.environ.get("MCA_ORACLE_XL") != "1",
                    reason="512 x 512 band factorisations take about 15 minutes on one core "
                           "and 4.3 GB; set MCA_ORACLE_XL=1 to run")
def test_band_and_cg_newton_agree_512():
    cb = synth.crossbar(512, 512, seed=0)
    a_t, a_b, ka, _ = oracle.solve(cb.geom, cb.g_dev, cb.v_in, method="band")
    c_t, c_b, kc, _ = oracle.solve(cb.geom, cb.g_dev, cb.v_in, method="cg")
    scale = max(np.abs(a_t).max(), np.abs(a_b).max())
    diff = max(np.abs(a_t - c_t).max(), np.abs(a_b - c_b).max()) / scale
    print(f"512x512 band vs CG Newton: max rel difference {diff:.3e}, steps {ka} / {kc}")
    assert diff <= 1e-12
    assert ka == kc


@pytest.mark.slow
@pytest.mark.parametrize("size,bound", [(512, 1e-8), (1024, 2e-8)])
def test_cg_newton_within_certified_bound(size, bound):
    """Oracle B at the large parity sizes, checked without any linear solver.

    The certified bound holds for any V, so it pins the CG-Newton steady state
    to the exact one: about 5e-9 (512^2) and 1.1e-8 (1024^2) of max|V| at the
    rounding floor of the residual.
    """
    cb = synth.crossbar(size, size, seed=0)
    vt, vb, k, hist = oracle.solve(cb.geom, cb.g_dev, cb.v_in, method="cg")
    assert hist[-1] <= 1e-14
    assert _certified_rel_error(cb.geom, cb.g_dev, cb.v_in, vt, vb) <= bound


def test_solve_small_netlist_zero_residual():
    cb = synth.crossbar(4, 5, seed=3, g_lo=1e-3, g_hi=5e-2)
    vt, vb, k, hist = oracle.solve(cb.geom, cb.g_dev, cb.v_in)
    ft, fb = netlist_residual(cb.geom, cb.g_dev, cb.v_in, vt, vb)
    assert max(np.abs(ft).max(), np.abs(fb).max()) <= 1e-15


def test_solve_band_and_cg_agree():
    cb = synth.crossbar(40, 28, seed=4)
    a_t, a_b, _, _ = oracle.solve(cb.geom, cb.g_dev, cb.v_in, method="band")
    c_t, c_b, _, _ = oracle.solve(cb.geom, cb.g_dev, cb.v_in, method="cg")
    scale = np.abs(a_t).max()
    assert np.abs(a_t - c_t).max() <= 1e-12 * scale
    assert np.abs(a_b - c_b).max() <= 1e-12 * scale


def test_solve_symmetries():
    cb = synth.crossbar(9, 7, seed=5)
    z_t, z_b, k, _ = oracle.solve(cb.geom, cb.g_dev, np.zeros(9))
    assert k == 0 and not z_t.any() and not z_b.any()
    p_t, p_b, _, _ = oracle.solve(cb.geom, cb.g_dev, cb.v_in)
    n_t, n_b, _, _ = oracle.solve(cb.geom, cb.g_dev, -cb.v_in)
    np.testing.assert_allclose(n_t, -p_t, rtol=0, atol=1e-15)
    np.testing.assert_allclose(n_b, -p_b, rtol=0, atol=1e-15)


def test_solve_linear_device_is_one_linear_solve():
    """For linear devices F is affine, so V* = J^{-1} Y (numpy dense solve)."""
    cb = synth.crossbar(6, 5, seed=6, device=synth.DEVICE_LINEAR)
    vt, vb, k, _ = oracle.solve(cb.geom, cb.g_dev, cb.v_in)
    J = oracle.dense_jacobian(cb.geom, cb.g_dev)
    y = np.zeros(2 * 30)
    y[0:30:5] = cb.geom.g_src * cb.v_in                  # Y_t[i, 0]
    x = np.linalg.solve(J, y)
    np.testing.assert_allclose(np.concatenate([vt.ravel(), vb.ravel()]), x, rtol=0,
                               atol=1e-14 * np.abs(x).max())
    assert k <= 2


def test_certified_bound_holds():
    """||V - V*|| <= ||F(V)|| / lambda_min(G) for any V (F strongly monotone)."""
    cb = synth.crossbar(8, 6, seed=8)
    vt, vb, _, _ = oracle.solve(cb.geom, cb.g_dev, cb.v_in)
    rng = np.random.default_rng(1)
    pt, pb = vt + 1e-3 * rng.standard_normal(vt.shape), vb + 1e-3 * rng.standard_normal(vb.shape)
    ft, fb, _ = oracle.residual(cb.geom, cb.g_dev, cb.v_in, pt, pb)
    P = _kron_P(cb.geom, 0.0, 0.0)
    mu = np.linalg.eigvalsh(P).min()
    err = np.sqrt(np.sum((pt - vt) ** 2) + np.sum((pb - vb) ** 2))
    assert err <= np.sqrt(np.sum(ft ** 2) + np.sum(fb ** 2)) / mu


# --------------------------------------------- identities the paper relies on

def test_block_inversion_identity_and_M():
    """eq. (block) with B = -a1 I, C = -a2 I and eq. (M) on a small crossbar."""
    geom = _geom(3, 4)
    a1, a2 = 2e-5, 3e-5
    P = _kron_P(geom, a1, a2)
    mn = 12
    A, B, Cb, D = P[:mn, :mn], P[:mn, mn:], P[mn:, :mn], P[mn:, mn:]
    Binv = np.linalg.inv(B)
    M = Cb - D @ Binv @ A
    Minv = np.linalg.inv(M)
    blk = np.block([[-Minv @ D @ Binv, Minv],
                    [Binv + Binv @ A @ Minv @ D @ Binv, -Binv @ A @ Minv]])
    Pinv = np.linalg.inv(P)
    np.testing.assert_allclose(blk, Pinv, rtol=0, atol=1e-9 * np.abs(Pinv).max())
    # eq. (M): M = -a2 I + (1/a1) (G2 (x) G1), G1 = G_top + a1 I, G2 = G_bot + a2 I
    Gt = P[:mn, :mn] - a1 * np.eye(mn)
    Gb = P[mn:, mn:] - a2 * np.eye(mn)
    Gtop = Gt[:4, :4]
    Gbot = Gb[::4, ::4]
    M2 = -a2 * np.eye(mn) + np.kron(Gbot + a2 * np.eye(3), Gtop + a1 * np.eye(4)) / a1
    np.testing.assert_allclose(M, M2, rtol=1e-12, atol=0)


def test_row_major_kronecker_vec_identity():
    """(A (x) B) vec_r(X) = vec_r(A X B^T): the reshaping behind eq. (2matrix4)."""
    rng = np.random.default_rng(0)
    A, B, X = rng.standard_normal((3, 3)), rng.standard_normal((5, 5)), rng.standard_normal((3, 5))
    np.testing.assert_allclose(np.kron(A, B) @ X.ravel(), (A @ X @ B.T).ravel(), rtol=1e-13)


# ------------------------------------ the paper's approximation M ~ Mhat

def _wire_dense(length, g, e0, e1):
    A = np.zeros((length, length))
    for k in range(length - 1):
        A[k, k] += g
        A[k + 1, k + 1] += g
        A[k, k + 1] -= g
        A[k + 1, k] -= g
    A[0, 0] += e0
    A[-1, -1] += e1
    return A


@pytest.mark.parametrize("m,n", [(1, 1), (1, 4), (3, 1), (3, 4), (5, 3)])
def test_mhat_inverse_is_kron_of_tridiagonal_inverses(m, n):
    """eqs. (Mhat), (G2hat), (M-1hat): Mhat = G2hat (x) G1 with G2hat = (G_bot + a2 I)/a1
    and G1 = G_top + a1 I; its inverse applied through eq. (2matrix4) equals a dense
    numpy solve with the assembled Kronecker product."""
    geom = _geom(m, n)
    a1, a2 = 3e-3, 5e-4
    G1 = _wire_dense(n, geom.g_top, geom.g_src, geom.g_top_end) + a1 * np.eye(n)
    G2hat = (_wire_dense(m, geom.g_bot, geom.g_bot_end0, geom.g_bot_end1) + a2 * np.eye(m)) / a1
    w = np.random.default_rng(4).standard_normal((m, n))
    ref = np.linalg.solve(np.kron(G2hat, G1), w.ravel()).reshape(m, n)
    out = oracle.mhat_inverse_apply(geom, a1, a2, w)
    np.testing.assert_allclose(out, ref, rtol=0, atol=1e-11 * np.abs(ref).max())


@pytest.mark.parametrize("m,n", [(1, 1), (2, 5), (4, 3), (6, 6)])
def test_approx_precond_equals_exact_when_a2_is_zero(m, n):
    """Mhat drops only the -a2 I term of eq. (M): with a2 = 0 the approximate
    preconditioner is exactly P^{-1} (dense LU of the assembled eq. (P))."""
    geom = _geom(m, n)
    a1 = 0.02
    rng = np.random.default_rng(9)
    rt, rb = rng.standard_normal((m, n)), rng.standard_normal((m, n))
    P = _kron_P(geom, a1, 0.0)
    z = np.linalg.solve(P, np.concatenate([rt.ravel(), rb.ravel()]))
    zt, zb = oracle.precond_apply_approx(geom, a1, 0.0, rt, rb)
    np.testing.assert_allclose(np.concatenate([zt.ravel(), zb.ravel()]), z, rtol=0,
                               atol=1e-11 * np.abs(z).max())


@pytest.mark.parametrize("m,n", [(3, 4), (5, 3), (6, 6)])
@pytest.mark.parametrize("a", [2e-5, 1e-2])
def test_approx_precond_inverts_P_without_its_lower_coupling(m, n, a):
    """The Schur complement of [[G_t + a1 I, -a1 I], [0, G_b + a2 I]] is exactly
    (G_b + a2 I)(G_t + a1 I)/a1 = Mhat, so eq. (block) with Mhat inverts P with its
    -a2 I block removed.  Also: it differs from P^{-1} by O(a2)."""
    geom = _geom(m, n)
    a1 = a2 = a
    rng = np.random.default_rng(5)
    rt, rb = rng.standard_normal((m, n)), rng.standard_normal((m, n))
    Phat = _kron_P(geom, a1, a2)
    mn = m * n
    Phat[mn:, :mn] = 0.0
    zt, zb = oracle.precond_apply_approx(geom, a1, a2, rt, rb)
    z = np.concatenate([zt.ravel(), zb.ravel()])
    r = np.concatenate([rt.ravel(), rb.ravel()])
    # the paper's order divides by a1: about log10(lambda_max / a1) digits are lost
    lam_max = 4 * max(geom.g_top, geom.g_bot) + 1.0          # >= ||Phat||
    tol = 64 * 2.2e-16 * (lam_max / a1) * lam_max * np.abs(z).max()
    np.testing.assert_allclose(Phat @ z, r, rtol=0, atol=tol)
    ze = np.linalg.solve(_kron_P(geom, a1, a2), r)
    assert np.abs(z - ze).max() <= 0.5 * np.abs(ze).max()   # a different operator, but close
    assert not np.allclose(z, ze, rtol=1e-12, atol=0)


def test_jacobi_matches_dense_diagonal():
    geom = _geom(4, 5)
    rng = np.random.default_rng(6)
    d = rng.uniform(1e-6, 1e-4, (4, 5))
    rt, rb = rng.standard_normal((4, 5)), rng.standard_normal((4, 5))
    diag = np.diag(oracle.dense_jacobian(geom, d))
    zt, zb = oracle.jacobi_apply(geom, d, rt, rb)
    np.testing.assert_allclose(np.concatenate([zt.ravel(), zb.ravel()]),
                               np.concatenate([rt.ravel(), rb.ravel()]) / diag, rtol=1e-15)


@pytest.mark.parametrize("m,n", [(1, 1), (1, 5), (4, 1), (3, 4), (5, 6)])
def test_sweep_guess_is_one_block_gauss_seidel_step(m, n):
    """V_t = A11^{-1} Y_t, V_b = A22^{-1}(D V_t) with the diagonal blocks of the
    dense J(D = g_dev) (the linearisation at V = 0) and numpy's dense solver."""
    geom = _geom(m, n)
    rng = np.random.default_rng(m + 7 * n)
    g = 10 ** rng.uniform(-3, -1, (m, n))       # strong devices: every term matters
    v_in = rng.uniform(0, 0.3, m)
    J = oracle.dense_jacobian(geom, g)
    mn = m * n
    yt = np.zeros((m, n))
    yt[:, 0] = geom.g_src * v_in
    vt = np.linalg.solve(J[:mn, :mn], yt.ravel())
    vb = np.linalg.solve(J[mn:, mn:], g.ravel() * vt)
    st, sb = oracle.sweep_guess(geom, g, v_in)
    np.testing.assert_allclose(st.ravel(), vt, rtol=1e-12, atol=1e-15)
    np.testing.assert_allclose(sb.ravel(), vb, rtol=1e-12, atol=1e-15)


def test_golden_32x32_seed0_unchanged():
    """The stored oracle steady state (tests/golden/make_golden.py) still holds."""
    import json
    import os
    path = os.path.join(os.path.dirname(__file__), "golden", "oracle_32x32_seed0.json")
    ref = json.load(open(path))
    cb = synth.crossbar(32, 32, seed=0)
    vt, vb, k, _ = oracle.solve(cb.geom, cb.g_dev, cb.v_in, method="band")
    assert k == ref["newton_steps"]
    assert abs(vt.sum() - ref["sum_vt"]) <= 1e-12 * abs(ref["sum_vt"])
    assert abs(vb.sum() - ref["sum_vb"]) <= 1e-12 * abs(ref["sum_vb"])
    for i, j, t, b in ref["samples"]:
        assert abs(vt[i, j] - t) <= 1e-14 and abs(vb[i, j] - b) <= 1e-14
