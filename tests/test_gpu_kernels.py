"""Parity of the HIP kernels (through the C ABI) with the CPU oracle.

Each case draws seeded inputs from paper_2109_07929_amd.synth, runs one entry
point of libmca.so on the GPU and the oracle's routine on the same inputs,
and compares element by element.  Shapes span several 64 x 64 GEMM tiles with
ragged tails, plus the degenerate single-row / single-column crossbars.

Tolerances (FP64):
  residual / Jacobian: 1e-14 x (sum of the branch conductances at a node x the
    largest voltage): both sides sum the same few terms in different orders.
  preconditioner, per-mode form: 1e-11 relative to max|z| -- four dense
    transforms of an orthonormal basis, each accurate to ~n eps.
  preconditioner, literal form: the paper's evaluation order divides by a1 and
    so loses about log10(lambda_max / a1) digits; the bound used is
    2e-16 x 64 x (lambda_max / a1) relative to max|z|.
"""

import numpy as np
import pytest
import torch

import oracle
from paper_2109_07929_amd import Plan, synth
from paper_2109_07929_amd import binding as B

pytestmark = pytest.mark.gpu

SHAPES = [(1, 1), (1, 7), (6, 1), (5, 3), (16, 24), (33, 65), (64, 64), (100, 130), (130, 70),
          (256, 128)]


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).to("cuda")


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def say(*a):
    print(*a, flush=True)


@pytest.mark.parametrize("m,n", SHAPES)
@pytest.mark.parametrize("device", [synth.DEVICE_SINH, synth.DEVICE_LINEAR])
def test_residual_parity(m, n, device):
    say(f"residual {m}x{n} device={device}")
    cb = synth.crossbar(m, n, seed=m * 1000 + n, device=device)
    vt, vb = synth.voltages(m, n, seed=m + 7 * n)
    ft, fb, d = oracle.residual(cb.geom, cb.g_dev, cb.v_in, vt, vb)
    plan = Plan(cb.geom)
    gft, gfb, gd = plan.residual(dev(cb.g_dev), dev(cb.v_in), dev(vt), dev(vb))
    g = cb.geom
    scale = (2 * max(g.g_top, g.g_bot) + g.g_src) * 0.3
    np.testing.assert_allclose(host(gft), ft, rtol=0, atol=1e-14 * scale)
    np.testing.assert_allclose(host(gfb), fb, rtol=0, atol=1e-14 * scale)
    np.testing.assert_allclose(host(gd), d, rtol=4e-15, atol=0)


@pytest.mark.parametrize("m,n", SHAPES)
def test_jacobian_parity(m, n):
    say(f"jacobian {m}x{n}")
    geom = synth.Geometry(m, n, g_top=0.4, g_bot=0.3, g_src=0.35, g_bot_end1=0.07)
    rng = np.random.default_rng(m * 31 + n)
    d = np.exp(rng.uniform(np.log(1e-6), np.log(1e-3), (m, n)))
    xt, xb = synth.vector(m, n, seed=m * 17 + n)
    yt, yb = oracle.jacobian_apply(geom, d, xt, xb)
    plan = Plan(geom)
    gyt, gyb = plan.jacobian_apply(dev(d), dev(xt), dev(xb))
    scale = 4 * 0.4 * max(np.abs(xt).max(), np.abs(xb).max())
    np.testing.assert_allclose(host(gyt), yt, rtol=0, atol=1e-14 * scale)
    np.testing.assert_allclose(host(gyb), yb, rtol=0, atol=1e-14 * scale)


def _literal_tol(plan, a1):
    lam_max = max(plan.lt_max, plan.lb_max)
    return 2.2e-16 * 64 * lam_max / a1


def _plan_with_eigs(geom):
    plan = Plan(geom)
    lt, _ = B.mca_plan_host_eigen(plan.handle, 0, geom.n)
    lb, _ = B.mca_plan_host_eigen(plan.handle, 1, geom.m)
    plan.lt_max, plan.lb_max = lt.max(), lb.max()
    return plan


@pytest.mark.parametrize("m,n", SHAPES)
@pytest.mark.parametrize("form", [B.MCA_PRECOND_LITERAL, B.MCA_PRECOND_PERMODE])
@pytest.mark.parametrize("a1,a2", [(2.2e-5, 2.2e-5), (3e-4, 4e-5)])
def test_precond_parity(m, n, form, a1, a2):
    say(f"precond {m}x{n} form={form} a=({a1},{a2})")
    geom = synth.Geometry(m, n)
    rt, rb = synth.vector(m, n, seed=m * 13 + n)
    zt, zb = oracle.precond_apply(geom, a1, a2, rt, rb)
    plan = _plan_with_eigs(geom)
    gzt, gzb = plan.precond_apply(a1, a2, dev(rt), dev(rb), form=form)
    scale = max(np.abs(zt).max(), np.abs(zb).max())
    tol = 1e-11 if form == B.MCA_PRECOND_PERMODE else max(1e-11, _literal_tol(plan, min(a1, a2)))
    err = max(np.abs(host(gzt) - zt).max(), np.abs(host(gzb) - zb).max()) / scale
    say(f"  rel err {err:.3e} (tol {tol:.1e})")
    assert err <= tol


@pytest.mark.parametrize("m,n,ends", [(64, 48, (0.1, 0.1)), (64, 48, (0.1, 0.07)),
                                      (2, 5, (0.1, 0.1)), (130, 70, (0.2, 0.2)),
                                      (7, 9, (0.1, 0.1)), (128, 256, (0.1, 0.07))])
def test_precond_literal_persymmetric_fold(m, n, ends):
    """Equal bottom terminations with m even take the folded Q_m transforms
    (symmetric / antisymmetric eigenvector halves); unequal ends or odd m the
    full ones.  Both must match the oracle."""
    a1 = a2 = 2.2e-5
    geom = synth.Geometry(m, n, g_bot_end0=ends[0], g_bot_end1=ends[1])
    rt, rb = synth.vector(m, n, seed=m + 3 * n)
    zt, zb = oracle.precond_apply(geom, a1, a2, rt, rb)
    plan = _plan_with_eigs(geom)
    gzt, gzb = plan.precond_apply(a1, a2, dev(rt), dev(rb), form=B.MCA_PRECOND_LITERAL)
    scale = max(np.abs(zt).max(), np.abs(zb).max())
    err = max(np.abs(host(gzt) - zt).max(), np.abs(host(gzb) - zb).max()) / scale
    tol = max(1e-11, _literal_tol(plan, a1))
    say(f"  {m}x{n} ends {ends}: rel err {err:.2e} (tol {tol:.1e})")
    assert err <= tol


def test_precond_none_is_identity():
    m, n = 9, 11
    rt, rb = synth.vector(m, n, seed=1)
    plan = Plan(synth.Geometry(m, n))
    zt, zb = plan.precond_apply(1e-5, 1e-5, dev(rt), dev(rb), form=B.MCA_PRECOND_NONE)
    np.testing.assert_array_equal(host(zt), rt)
    np.testing.assert_array_equal(host(zb), rb)


@pytest.mark.parametrize("m,n,form", [(1024, 1024, B.MCA_PRECOND_LITERAL),
                                      (1024, 1024, B.MCA_PRECOND_PERMODE),
                                      (1152, 1024, B.MCA_PRECOND_LITERAL)])
def test_precond_inverts_P_at_1024(m, n, form):
    """Full size (1024 x 1024, the solver's launch shape; 1152 x 1024 puts the
    literal form's last product over more than 256 tiles, the register-staged
    kernel with the unfold fused): ||P z - r|| / ||r||, with P z from the
    oracle's Jacobian product at uniform slope a (P(a,a) = J)."""
    a = 2.2e-5
    say(f"precond {m}x{n} form={form}")
    geom = synth.Geometry(m, n)
    rt, rb = synth.vector(m, n, seed=5)
    plan = _plan_with_eigs(geom)
    gzt, gzb = plan.precond_apply(a, a, dev(rt), dev(rb), form=form)
    zt, zb = host(gzt), host(gzb)
    pt, pb = oracle.jacobian_apply(geom, np.full((m, n), a), zt, zb)
    rel = np.sqrt(np.sum((pt - rt) ** 2) + np.sum((pb - rb) ** 2)) / np.sqrt(
        np.sum(rt ** 2) + np.sum(rb ** 2))
    say(f"  ||Pz - r||/||r|| = {rel:.3e}")
    assert rel <= (1e-10 if form == B.MCA_PRECOND_PERMODE else 1e-6)
    # sampled entries against the direct CG solve of the oracle
    ct, cb = oracle.jacobian_solve(geom, np.full((m, n), a), rt, rb, method="cg", rel_tol=1e-13)
    scale = max(np.abs(ct).max(), np.abs(cb).max())
    err = max(np.abs(zt - ct).max(), np.abs(zb - cb).max()) / scale
    say(f"  max rel err vs oracle CG {err:.3e}")
    assert err <= (1e-9 if form == B.MCA_PRECOND_PERMODE else 1e-5)


# line lengths across the solver's forms: chunks of 8 (up to 1024), chunks of
# 16 (up to 2048, ragged last chunk), cyclic reduction (longer)
APPROX_SHAPES = SHAPES + [(300, 77), (40, 3000), (3, 8192), (8192, 3), (1500, 37), (20, 1100),
                          (2048, 6), (1024, 9)]


@pytest.mark.parametrize("m,n", APPROX_SHAPES)
@pytest.mark.parametrize("a1,a2", [(2.2e-5, 2.2e-5), (3e-4, 4e-5)])
def test_precond_approx_parity(m, n, a1, a2):
    """The paper's approximation M ~ Mhat: GPU block back-substitution by line
    solves against the oracle's literal order (eq. (block) with Mhat^{-1} by eq. (2matrix4))."""
    say(f"precond approx {m}x{n} a=({a1},{a2})")
    geom = synth.Geometry(m, n)
    rt, rb = synth.vector(m, n, seed=m * 7 + n)
    zt, zb = oracle.precond_apply_approx(geom, a1, a2, rt, rb)
    plan = _plan_with_eigs(geom)
    gzt, gzb = plan.precond_apply(a1, a2, dev(rt), dev(rb), form=B.MCA_PRECOND_APPROX)
    scale = max(np.abs(zt).max(), np.abs(zb).max())
    # the oracle's order divides by a1 (the GPU's does not): its rounding sets the bar
    tol = max(1e-11, _literal_tol(plan, a1))
    err = max(np.abs(host(gzt) - zt).max(), np.abs(host(gzb) - zb).max()) / scale
    say(f"  rel err {err:.3e} (tol {tol:.1e})")
    assert err <= tol


def test_precond_approx_inverts_P_without_lower_coupling_at_1024():
    """Full size: the approximate z solves [[G_t + a1 I, -a1 I], [0, G_b + a2 I]] z = r
    (P with its -a2 I block dropped), checked with the oracle's Jacobian product at
    uniform slope a (P(a, a) = J):  P z + [0; a z_t] = r."""
    m = n = 1024
    a = 2.2e-5
    geom = synth.Geometry(m, n)
    rt, rb = synth.vector(m, n, seed=6)
    plan = Plan(geom)
    gzt, gzb = plan.precond_apply(a, a, dev(rt), dev(rb), form=B.MCA_PRECOND_APPROX)
    zt, zb = host(gzt), host(gzb)
    pt, pb = oracle.jacobian_apply(geom, np.full((m, n), a), zt, zb)
    pb = pb + a * zt
    rel = np.sqrt(np.sum((pt - rt) ** 2) + np.sum((pb - rb) ** 2)) / np.sqrt(
        np.sum(rt ** 2) + np.sum(rb ** 2))
    # backward-stable solves: ||Phat z - r|| <= c eps ||Phat|| ||z||, ||Phat|| <= 2
    zr = np.sqrt(np.sum(zt ** 2) + np.sum(zb ** 2)) / np.sqrt(np.sum(rt ** 2) + np.sum(rb ** 2))
    bound = 64 * 2.2e-16 * 2.0 * zr
    say(f"  ||Phat z - r||/||r|| = {rel:.3e} (bound {bound:.1e})")
    assert rel <= bound
    ot, ob = oracle.precond_apply_approx(geom, a, a, rt, rb)
    scale = max(np.abs(ot).max(), np.abs(ob).max())
    err = max(np.abs(zt - ot).max(), np.abs(zb - ob).max()) / scale
    say(f"  max rel err vs oracle {err:.3e}")
    assert err <= max(1e-11, 2.2e-16 * 64 * 2.0 / a)


def test_precond_jacobi_only_in_the_solver():
    m, n = 6, 5
    rt, rb = synth.vector(m, n, seed=2)
    plan = Plan(synth.Geometry(m, n))
    with pytest.raises(B.MCAError):
        plan.precond_apply(1e-5, 1e-5, dev(rt), dev(rb), form=B.MCA_PRECOND_JACOBI)


def test_errors_and_validation():
    m, n = 8, 8
    plan = Plan(synth.Geometry(m, n))
    rt, rb = synth.vector(m, n, seed=2)
    with pytest.raises(B.MCAError) as e:
        plan.precond_apply(0.0, 1e-5, dev(rt), dev(rb))
    assert e.value.status == B.MCA_ERR_INVALID_ARG
    small = torch.empty(16, dtype=torch.uint8, device="cuda")
    with pytest.raises(B.MCAError) as e:
        plan.precond_apply(1e-5, 1e-5, dev(rt), dev(rb), ws=small)
    assert e.value.status == B.MCA_ERR_WORKSPACE
    # a plan that was never uploaded
    h = B.mca_plan_create(B.geometry(m, n))
    try:
        z = torch.zeros((m, n), dtype=torch.float64, device="cuda")
        with pytest.raises(B.MCAError) as e:
            B.mca_jacobian_apply(h, m, n, z, z, z, z.clone(), z.clone())
        assert e.value.status == B.MCA_ERR_WORKSPACE
    finally:
        B.mca_plan_destroy(h)


LOWPREC = [(B.MCA_PREC_FP32, 1e-4), (B.MCA_PREC_BF16X3, 1e-3), (B.MCA_PREC_BF16, 3e-2)]


@pytest.mark.parametrize("m,n", [(1, 1), (5, 3), (33, 65), (64, 64), (130, 70)])
@pytest.mark.parametrize("prec,tol", LOWPREC)
def test_precond_lowprec_parity(m, n, prec, tol):
    """Reduced-precision per-mode P^{-1} r against the oracle's direct solve.

    Bound: FP32 transforms carry ~sqrt(K) 2^-24 relative rounding per product and
    four products chain; split-BF16 keeps ~16 bits per operand; plain BF16 8 bits.
    The bounds below leave a factor >= 10 over those estimates at these sizes."""
    a1, a2 = 2.2e-5, 3e-5
    say(f"precond lowprec {m}x{n} prec={prec}")
    geom = synth.Geometry(m, n)
    rt, rb = synth.vector(m, n, seed=m * 13 + n)
    zt, zb = oracle.precond_apply(geom, a1, a2, rt, rb)
    plan = Plan(geom)
    gzt, gzb = plan.precond_apply(a1, a2, dev(rt), dev(rb), form=B.MCA_PRECOND_PERMODE,
                                  precision=prec)
    scale = max(np.abs(zt).max(), np.abs(zb).max())
    err = max(np.abs(host(gzt) - zt).max(), np.abs(host(gzb) - zb).max()) / scale
    say(f"  rel err {err:.3e} (tol {tol:.0e})")
    assert err <= tol


@pytest.mark.parametrize("m,n", [(2112, 2080), (2144, 2016)])
@pytest.mark.parametrize("prec,tol", [(B.MCA_PREC_FP32, 1e-4), (B.MCA_PREC_BF16X3, 2e-4),
                                      (B.MCA_PREC_BF16, 3e-2)])
def test_precond_lowprec_large_tiles(m, n, prec, tol):
    """Products of 2048-class sizes take the 128 x 128 tiles; ragged sizes (not a
    multiple of 128) against the FP64 per-mode path (itself oracle-checked above).
    The split-BF16 interior tiles run the software-pipelined loop, which takes
    whole rounds of six 32-deep slices and then the rest one by one: depths of
    66, 65, 67 and 63 slices leave 0, 5, 1 and 3 (the batch tests' 1024-class
    depths leave 2 and 4).  Bounds as in the folded 1024 test (measured 4.6e-6 and
    1.2e-5); plain BF16 (one plane, 8 bits per operand) as in the small-size test
    above; an indexing slip gives errors of order one."""
    a1, a2 = 2.2e-5, 3e-5
    say(f"precond lowprec large tiles {m}x{n} prec={prec}")
    geom = synth.Geometry(m, n)
    rt, rb = synth.vector(m, n, seed=11)
    plan = Plan(geom)
    ft, fb = plan.precond_apply(a1, a2, dev(rt), dev(rb), form=B.MCA_PRECOND_PERMODE)
    gt, gb = plan.precond_apply(a1, a2, dev(rt), dev(rb), form=B.MCA_PRECOND_PERMODE,
                                precision=prec)
    zt, zb = host(ft), host(fb)
    scale = max(np.abs(zt).max(), np.abs(zb).max())
    err = max(np.abs(host(gt) - zt).max(), np.abs(host(gb) - zb).max()) / scale
    say(f"  rel err vs FP64 {err:.3e} (tol {tol:.0e})")
    assert err <= tol


@pytest.mark.parametrize("prec,tol", [(B.MCA_PREC_FP32, 1e-4), (B.MCA_PREC_BF16X3, 2e-4)])
def test_precond_lowprec_folded_1024(prec, tol):
    """The standard 1024 x 1024 crossbar (persymmetric bottom wires, m/2 a multiple
    of 128): the reduced-precision chain folds and runs on 128 x 128 tiles through
    the direct-to-LDS loop.  Element by element against the FP64 per-mode path
    (oracle-checked above).  Rounding: four chained products of depth <= 1024,
    ~sqrt(K) 2^-24 each in FP32 (~1e-5 in all), ~2^-16 per operand in split-BF16
    (~2e-5); the bounds leave a factor of ten over those (measured 2.5e-6 and 1.2e-5),
    and an indexing slip in the fold, the interleave or the unfold gives errors of
    order one."""
    m = n = 1024
    a1, a2 = 2.2e-5, 3e-5
    say(f"precond lowprec folded {m}x{n} prec={prec}")
    geom = synth.Geometry(m, n)
    rt, rb = synth.vector(m, n, seed=17)
    plan = Plan(geom)
    ft, fb = plan.precond_apply(a1, a2, dev(rt), dev(rb), form=B.MCA_PRECOND_PERMODE)
    gt, gb = plan.precond_apply(a1, a2, dev(rt), dev(rb), form=B.MCA_PRECOND_PERMODE,
                                precision=prec)
    zt, zb = host(ft), host(fb)
    scale = max(np.abs(zt).max(), np.abs(zb).max())
    err = max(np.abs(host(gt) - zt).max(), np.abs(host(gb) - zb).max()) / scale
    say(f"  rel err vs FP64 {err:.3e} (tol {tol:.0e})")
    assert err <= tol


@pytest.mark.parametrize("prec,tol", [(B.MCA_PREC_FP32, 1e-2), (B.MCA_PREC_BF16X3, 5e-2),
                                      (B.MCA_PREC_BF16, 10.0)])
def test_precond_lowprec_residual_at_1024(prec, tol):
    """||P z - r|| / ||r|| of the reduced-precision preconditioner at 1024 x 1024,
    with P z from the oracle's Jacobian product at uniform slope (P(a,a) = J).

    This is what flexible GMRES sees.  The inverse transform rounds the large
    low-mode components (|x_hat| up to ||r|| / det_min ~ 1e5 ||r||) at the
    operand precision, and P maps that error back with its largest eigenvalues,
    so the residual is ~ eps_op x 1e5 x (a few): about 1e-3 in FP32, 1e-2 in
    split-BF16, and above 1 in plain BF16 (a weak preconditioner at this size)."""
    m = n = 1024
    a = 2.2e-5
    say(f"precond lowprec 1024^2 prec={prec}")
    geom = synth.Geometry(m, n)
    rt, rb = synth.vector(m, n, seed=5)
    plan = Plan(geom)
    gzt, gzb = plan.precond_apply(a, a, dev(rt), dev(rb), form=B.MCA_PRECOND_PERMODE,
                                  precision=prec)
    zt, zb = host(gzt), host(gzb)
    pt, pb = oracle.jacobian_apply(geom, np.full((m, n), a), zt, zb)
    rel = np.sqrt(np.sum((pt - rt) ** 2) + np.sum((pb - rb) ** 2)) / np.sqrt(
        np.sum(rt ** 2) + np.sum(rb ** 2))
    say(f"  ||Pz - r||/||r|| = {rel:.3e}")
    assert rel <= tol


def test_lowprec_needs_permode():
    m, n = 8, 8
    plan = Plan(synth.Geometry(m, n))
    rt, rb = synth.vector(m, n, seed=2)
    with pytest.raises(B.MCAError) as e:
        plan.precond_apply(1e-5, 1e-5, dev(rt), dev(rb), form=B.MCA_PRECOND_LITERAL,
                           precision=B.MCA_PREC_FP32)
    assert e.value.status == B.MCA_ERR_INVALID_ARG
