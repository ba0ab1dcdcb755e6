"""The learned warm start: the guess fallback of both solvers, and what the
trained network (paper_2109_07929_amd/warmstart_512.npy, made by
`python -m paper_2109_07929_amd.warmstart train`) gains on held-out 512 x 512
crossbars.  A warm start may only change iteration counts: the voltages match
the cold solve to the solver's bar."""

import os

import numpy as np
import pytest
import torch

import oracle
from paper_2109_07929_amd import Batch, Plan, synth, warmstart
from paper_2109_07929_amd import binding as B

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)


def test_guess_fallback_single_solve():
    cb = synth.crossbar(40, 30, seed=2)
    plan = Plan(cb.geom)
    g = torch.from_numpy(cb.g_dev).cuda()
    v = torch.from_numpy(cb.v_in).cuda()
    vt0, vb0, s0, st0 = plan.solve(g, v, B.options())
    bad = (torch.full_like(vt0, 5.0), torch.full_like(vb0, -5.0))
    o = B.options(flags=B.MCA_FLAG_GUESS_FALLBACK)
    vt1, vb1, s1, st1 = plan.solve(g, v, o, guess=bad)
    assert s1 == B.MCA_OK and st1.start == 0 and st1.newton_iters == st0.newton_iters
    assert torch.equal(vt1, vt0) and torch.equal(vb1, vb0)
    vt2, vb2, s2, st2 = plan.solve(g, v, o, guess=(vt0.clone(), vb0.clone()))
    assert s2 == B.MCA_OK and st2.start == 1 and st2.newton_iters == 0


def test_guess_fallback_batched():
    cbs = synth.mc_batch(4, seed=4, sizes=(24, 40))
    bt = Batch([c.geom for c in cbs])
    g = bt.concat([c.g_dev for c in cbs])
    v = bt.concat([c.v_in for c in cbs])
    o = B.options(precond=B.MCA_PRECOND_PERMODE, precision=B.MCA_PREC_BF16X3)
    vt0, vb0, s0, st0 = bt.solve(g, v, o)
    assert s0 == B.MCA_OK
    # crossbars 0, 2 get a useless guess, 1, 3 their solution
    gt, gb = vt0.clone(), vb0.clone()
    for b in (0, 2):
        gt[int(bt.cross[b]):int(bt.cross[b + 1])] = 7.0
    ow = B.options(precond=B.MCA_PRECOND_PERMODE, precision=B.MCA_PREC_BF16X3,
                   flags=B.MCA_FLAG_GUESS_FALLBACK)
    vt1, vb1, s1, st1 = bt.solve(g, v, ow, guess=(gt, gb))
    assert s1 == B.MCA_OK
    assert [s.start for s in st1] == [0, 1, 0, 1]
    assert [s.newton_iters for s in st1] == [st0[0].newton_iters, 0, st0[2].newton_iters, 0]
    scale = float(torch.maximum(vt0.abs().max(), vb0.abs().max()))
    assert float((vt1 - vt0).abs().max()) <= 1e-12 * scale


@pytest.mark.skipif(not os.path.exists(warmstart.DEFAULT_PARAMS), reason="no trained network")
def test_trained_network_gains_on_held_out_crossbars():
    """At the workload's Newton tolerance (||F|| <= 1e-10 ||Y||, both starts)
    the network's guesses save Newton steps and GMRES iterations."""
    params = warmstart.load_params()
    res = warmstart.evaluate(params, count=64, size=512, seed=424242)
    s = warmstart.summary(res)
    say(f"  {s}")
    assert s["max_relres_warm"] <= 1e-10
    assert s["guess_used_fraction"] >= 0.9
    assert s["newton_warm"] < s["newton_cold"]
    assert s["krylov_warm"] < s["krylov_cold"]


@pytest.mark.skipif(not os.path.exists(warmstart.DEFAULT_PARAMS), reason="no trained network")
def test_warm_started_voltages_match_cold_and_oracle():
    """A warm start changes only the path: run to ||F|| <= 1e-12 ||Y|| (a
    1e-10 stop certifies far less than the voltage bar: the certified bound
    ||F|| / lambda_min is then about 1e-4 of max |V| at 512^2), warm and cold
    voltages agree to 1e-8 and four warm-started crossbars match the oracle's
    steady state to 1e-8."""
    params = warmstart.load_params()
    res = warmstart.evaluate(params, count=64, size=512, seed=424243, newton_tol=1e-12, keep=4)
    s = warmstart.summary(res)
    say(f"  {s}")
    assert s["max_relres_warm"] <= 1e-12
    assert s["max_rel_dv_warm_vs_cold"] <= 1e-8
    assert len(res["kept"]) == 4
    for geom, g, v, vt, vb in res["kept"]:
        rt, rb, _, _ = oracle.solve(geom, g, v, method="cg")
        scale = max(np.abs(rt).max(), np.abs(rb).max())
        err = max(np.abs(vt - rt).max(), np.abs(vb - rb).max()) / scale
        say(f"  warm-started {geom.m}x{geom.n} vs oracle: {err:.1e}")
        assert err <= 1e-8


# A Newton tolerance no start can miss: the solve returns its starting point.
RETURN_START = 1e300


@pytest.mark.parametrize("m,n", [(1, 1), (5, 3), (40, 70), (300, 129), (1024, 1024)])
def test_sweep_start_single(m, n):
    """MCA_FLAG_SWEEP_START: the starting voltages equal the oracle's block
    Gauss-Seidel sweep element by element, and the solve from them reaches the
    oracle's steady state."""
    cb = synth.crossbar(m, n, seed=m + n)
    plan = Plan(cb.geom)
    g = torch.from_numpy(cb.g_dev).cuda()
    v = torch.from_numpy(cb.v_in).cuda()
    gt, gb = oracle.sweep_guess(cb.geom, cb.g_dev, cb.v_in)
    st_t, st_b, s, st = plan.solve(g, v, B.options(flags=B.MCA_FLAG_SWEEP_START,
                                                   newton_tol=RETURN_START))
    assert s == B.MCA_OK and st.start == 1 and st.newton_iters == 0
    scale = max(np.abs(gt).max(), np.abs(gb).max())
    d0 = max(np.abs(st_t.cpu().numpy() - gt).max(), np.abs(st_b.cpu().numpy() - gb).max()) / scale
    say(f"  {m}x{n}: sweep start vs oracle {d0:.1e}")
    assert d0 <= 1e-12
    if m * n > 300 * 129:
        return
    vt, vb, s, st = plan.solve(g, v, B.options(flags=B.MCA_FLAG_SWEEP_START))
    assert s == B.MCA_OK and st.start == 1
    ft, fb, _ = oracle.residual(cb.geom, cb.g_dev, cb.v_in, gt, gb)
    r0 = np.sqrt((ft ** 2).sum() + (fb ** 2).sum()) / oracle.source_norm(cb.geom, cb.v_in)
    say(f"  {m}x{n}: start residual gpu {st.residual_history[0]:.6e} oracle {r0:.6e}, "
        f"newton {st.newton_iters}")
    assert abs(st.residual_history[0] - r0) <= 1e-6 * r0 + 1e-15
    rt, rb, _, _ = oracle.solve(cb.geom, cb.g_dev, cb.v_in, method="band" if m * n < 5000 else "cg")
    scale = max(np.abs(rt).max(), np.abs(rb).max())
    err = max(np.abs(vt.cpu().numpy() - rt).max(), np.abs(vb.cpu().numpy() - rb).max()) / scale
    assert err <= 1e-8
    with pytest.raises(B.MCAError):
        plan.solve(g, v, B.options(flags=B.MCA_FLAG_SWEEP_START), guess=(vt, vb))


def test_sweep_start_batched_saves_a_newton_step():
    cbs = synth.mc_batch(6, seed=9, sizes=(64, 128, 256))
    bt = Batch([c.geom for c in cbs])
    g = bt.concat([c.g_dev for c in cbs])
    v = bt.concat([c.v_in for c in cbs])
    o = B.options(precond=B.MCA_PRECOND_PERMODE, precision=B.MCA_PREC_BF16X3)
    _, _, s0, st0 = bt.solve(g, v, o)
    flags = B.MCA_FLAG_SWEEP_START | B.MCA_FLAG_GUESS_FALLBACK
    ow = B.options(precond=B.MCA_PRECOND_PERMODE, precision=B.MCA_PREC_BF16X3, flags=flags)
    vt, vb, s1, st1 = bt.solve(g, v, ow)
    o_start = B.options(precond=B.MCA_PRECOND_PERMODE, precision=B.MCA_PREC_BF16X3, flags=flags,
                        newton_tol=RETURN_START)
    pt, pb, s2, st2 = bt.solve(g, v, o_start)
    assert s0 == B.MCA_OK and s1 == B.MCA_OK and s2 == B.MCA_OK
    pts = [t.cpu().numpy() for t in bt.split(pt)]
    pbs = [t.cpu().numpy() for t in bt.split(pb)]
    for b, c in enumerate(cbs):
        gt, gb = oracle.sweep_guess(c.geom, c.g_dev, c.v_in)
        scale = max(np.abs(gt).max(), np.abs(gb).max())
        assert st2[b].start == 1 and st2[b].newton_iters == 0
        assert max(np.abs(pts[b] - gt).max(), np.abs(pbs[b] - gb).max()) <= 1e-12 * scale
        ft, fb, _ = oracle.residual(c.geom, c.g_dev, c.v_in, gt, gb)
        r0 = np.sqrt((ft ** 2).sum() + (fb ** 2).sum()) / oracle.source_norm(c.geom, c.v_in)
        assert st1[b].start == 1
        assert abs(st1[b].residual_history[0] - r0) <= 1e-6 * r0
        assert st1[b].rel_residual <= 1e-10
    say(f"  newton cold {[s.newton_iters for s in st0]} sweep {[s.newton_iters for s in st1]}")
    assert sum(s.newton_iters for s in st1) < sum(s.newton_iters for s in st0)
