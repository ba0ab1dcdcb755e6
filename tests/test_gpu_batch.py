"""Parity of mca_solve_batched (many crossbars of different sizes in the same
launches) with the CPU oracle, crossbar by crossbar, and with mca_solve.

The bar is the solver's: every crossbar's voltages match the oracle's steady
state to 1e-8 relative error (max over both layers of |V - V_ref| / max |V_ref|).
"""

import numpy as np
import pytest
import torch

import oracle
from paper_2109_07929_amd import Batch, Plan, synth
from paper_2109_07929_amd import binding as B

pytestmark = pytest.mark.gpu

TOL = 1e-8
PRECS = [B.MCA_PREC_FP32, B.MCA_PREC_BF16X3, B.MCA_PREC_BF16]


def say(*a):
    print(*a, flush=True)


def rel_err(gt, gb, rt, rb):
    scale = max(np.abs(rt).max(), np.abs(rb).max())
    return max(np.abs(gt - rt).max(), np.abs(gb - rb).max()) / scale


def batch_solve(cbs, check=False, **opt):
    bt = Batch([c.geom for c in cbs])
    g = bt.concat([c.g_dev for c in cbs])
    v = bt.concat([c.v_in for c in cbs])
    kw = dict(precond=B.MCA_PRECOND_PERMODE, precision=B.MCA_PREC_BF16X3)
    kw.update(opt)
    vt, vb, status, stats = bt.solve(g, v, B.options(**kw), check=check)
    torch.cuda.synchronize()
    return bt, [t.cpu().numpy() for t in bt.split(vt)], [t.cpu().numpy() for t in bt.split(vb)], \
        status, stats


def ragged_batch(seed=3):
    # sizes off the 64-tile grid and odd products (unaligned offsets in the batch)
    return synth.mc_batch(7, seed=seed, sizes=(5, 20, 33, 64, 72))


@pytest.mark.parametrize("prec", PRECS)
def test_batch_ragged_vs_oracle(prec):
    cbs = ragged_batch()
    say(f"batch ragged prec={prec}: " + " ".join(f"{c.geom.m}x{c.geom.n}" for c in cbs))
    bt, vts, vbs, status, stats = batch_solve(cbs, precision=prec)
    assert status == B.MCA_OK
    for b, c in enumerate(cbs):
        rt, rb, _, _ = oracle.solve(c.geom, c.g_dev, c.v_in, method="band")
        err = rel_err(vts[b], vbs[b], rt, rb)
        st = stats[b]
        say(f"  {c.geom.m}x{c.geom.n}: newton {st.newton_iters} krylov "
            f"{list(st.krylov_history[:st.newton_iters])} relres {st.rel_residual:.1e} err {err:.1e}")
        assert st.rel_residual <= 1e-10
        assert err <= TOL
        # certified bound on the 2-norm error
        e2 = np.sqrt(np.sum((vts[b] - rt) ** 2) + np.sum((vbs[b] - rb) ** 2))
        assert e2 <= st.err_bound * (1 + 1e-6) + 1e-13 * np.abs(rt).max()


def test_batch_matches_single_solves():
    """Each crossbar of a batch follows mca_solve's iteration (same options)."""
    cbs = synth.mc_batch(3, seed=11, sizes=(48, 64, 96))
    _, vts, vbs, status, stats = batch_solve(cbs, precision=B.MCA_PREC_FP32)
    assert status == B.MCA_OK
    for b, c in enumerate(cbs):
        plan = Plan(c.geom)
        o = B.options(precond=B.MCA_PRECOND_PERMODE, precision=B.MCA_PREC_FP32)
        g = torch.from_numpy(c.g_dev).cuda()
        v = torch.from_numpy(c.v_in).cuda()
        vt, vb, s1, st1 = plan.solve(g, v, o)
        torch.cuda.synchronize()
        err = rel_err(vts[b], vbs[b], vt.cpu().numpy(), vb.cpu().numpy())
        say(f"  {c.geom.m}x{c.geom.n}: batch newton {stats[b].newton_iters} single "
            f"{st1.newton_iters}; krylov {stats[b].krylov_iters} vs {st1.krylov_iters}; diff {err:.1e}")
        assert stats[b].newton_iters == st1.newton_iters
        assert abs(stats[b].krylov_iters - st1.krylov_iters) <= 2
        assert err <= TOL


def nonlinear_batch():
    # drives of 2-3 V against v0 = 0.25 V and devices up to 1e-2 S: the full
    # Newton step overshoots the sinh devices, so the line search halves it
    cases = [(24, 20, 1e-3, 2.0, 5), (40, 36, 1e-2, 3.0, 6), (64, 64, 1e-2, 2.0, 7),
             (33, 70, 1e-3, 2.0, 8), (48, 40, 1e-2, 5.0, 9), (20, 24, 3e-2, 4.0, 10),
             (32, 32, 1e-2, 6.0, 11), (28, 52, 5e-2, 3.0, 12)]
    return [synth.crossbar(m, n, seed=sd, g_lo=1e-5, g_hi=ghi, v_hi=vhi)
            for m, n, ghi, vhi, sd in cases]


@pytest.mark.parametrize("prec", [B.MCA_PREC_FP32, B.MCA_PREC_BF16X3])
def test_batch_line_search_backtracks(prec):
    """Crossbars whose Newton steps are damped: the trial voltages go to the
    buffer that does not hold the current ones and accepted crossbars switch
    buffers, so halved trials, crossbars accepting at different rounds and
    crossbars that stopped earlier must all end at the oracle's steady state
    (1e-8) and agree with the single-crossbar solver."""
    cbs = nonlinear_batch()
    say(f"batch line search prec={prec}: " + " ".join(f"{c.geom.m}x{c.geom.n}" for c in cbs))
    _, vts, vbs, status, stats = batch_solve(cbs, precision=prec)
    assert status == B.MCA_OK
    # several crossbars halve, some more than once, and they stop at different steps
    assert sum(s.backtracks > 0 for s in stats) >= 2
    assert max(s.backtracks for s in stats) >= 2
    assert len({s.newton_iters for s in stats}) > 1
    for b, c in enumerate(cbs):
        rt, rb, _, _ = oracle.solve(c.geom, c.g_dev, c.v_in, method="band")
        err = rel_err(vts[b], vbs[b], rt, rb)
        st = stats[b]
        plan = Plan(c.geom)
        o = B.options(precond=B.MCA_PRECOND_PERMODE, precision=prec)
        vt1, vb1, s1, st1 = plan.solve(torch.from_numpy(c.g_dev).cuda(),
                                       torch.from_numpy(c.v_in).cuda(), o)
        torch.cuda.synchronize()
        err1 = rel_err(vts[b], vbs[b], vt1.cpu().numpy(), vb1.cpu().numpy())
        say(f"  {c.geom.m}x{c.geom.n}: newton {st.newton_iters} backtracks {st.backtracks} "
            f"(single: {st1.newton_iters}, {st1.backtracks}) err {err:.1e} vs single {err1:.1e}")
        assert s1 == B.MCA_OK
        assert st.rel_residual <= 1e-10
        assert err <= TOL
        assert err1 <= TOL
        assert st.newton_iters == st1.newton_iters and st.backtracks == st1.backtracks


@pytest.mark.parametrize("restart", [1, 3])
def test_batch_restarts(restart):
    cbs = ragged_batch(seed=5)
    say(f"batch restart={restart}")
    _, vts, vbs, status, stats = batch_solve(cbs, restart=restart, max_krylov=600)
    assert status == B.MCA_OK
    assert sum(s.restarts for s in stats) > 0
    for b, c in enumerate(cbs):
        rt, rb, _, _ = oracle.solve(c.geom, c.g_dev, c.v_in, method="band")
        assert rel_err(vts[b], vbs[b], rt, rb) <= TOL


def test_batch_mixed_outcomes():
    """A non-finite crossbar and a zero-drive crossbar do not disturb the others."""
    cbs = synth.mc_batch(4, seed=2, sizes=(16, 40))
    cbs[1].g_dev[3, 2] = np.nan
    cbs[2].v_in[:] = 0.0
    _, vts, vbs, status, stats = batch_solve(cbs)
    assert status == B.MCA_ERR_NONFINITE
    assert np.all(vts[2] == 0.0) and np.all(vbs[2] == 0.0)
    for b in (0, 3):
        c = cbs[b]
        rt, rb, _, _ = oracle.solve(c.geom, c.g_dev, c.v_in, method="band")
        assert rel_err(vts[b], vbs[b], rt, rb) <= TOL


def test_batch_initial_guess_at_solution():
    cbs = ragged_batch(seed=8)
    bt, vts, vbs, status, stats = batch_solve(cbs)
    assert status == B.MCA_OK
    g = bt.concat([c.g_dev for c in cbs])
    v = bt.concat([c.v_in for c in cbs])
    guess = (bt.concat(vts), bt.concat(vbs))
    o = B.options(precond=B.MCA_PRECOND_PERMODE, precision=B.MCA_PREC_BF16X3)
    vt, vb, status, stats = bt.solve(g, v, o, guess=guess)
    assert status == B.MCA_OK
    assert all(s.newton_iters == 0 for s in stats)
    torch.cuda.synchronize()
    assert torch.equal(vt, guess[0]) and torch.equal(vb, guess[1])


def test_batch_of_one_and_unsupported_options():
    c = synth.crossbar(24, 20, seed=4)
    _, vts, vbs, status, stats = batch_solve([c])
    assert status == B.MCA_OK
    rt, rb, _, _ = oracle.solve(c.geom, c.g_dev, c.v_in, method="band")
    assert rel_err(vts[0], vbs[0], rt, rb) <= TOL
    bt = Batch([c.geom])
    g = bt.concat([c.g_dev])
    v = bt.concat([c.v_in])
    with pytest.raises(B.MCAError):
        bt.solve(g, v, B.options())          # FP64 / literal: single-crossbar only


def test_batch_monte_carlo_256():
    """The Monte-Carlo workload: 256 crossbars with m, n drawn from {64, ..., 512}.
    Every crossbar's final residual is recomputed by the oracle on the host; four
    sampled crossbars are compared with the oracle's steady state."""
    cbs = synth.mc_batch(256, seed=0)
    say(f"batch MC 256: {sum(c.geom.m * c.geom.n for c in cbs)} crosspoints")
    bt, vts, vbs, status, stats = batch_solve(cbs)
    assert status == B.MCA_OK
    worst = 0.0
    for b, c in enumerate(cbs):
        ft, fb = oracle.residual(c.geom, c.g_dev, c.v_in, vts[b], vbs[b])[:2]
        rel = np.sqrt((ft ** 2).sum() + (fb ** 2).sum()) / oracle.source_norm(c.geom, c.v_in)
        worst = max(worst, rel)
    say(f"  worst oracle residual {worst:.2e}; newton "
        f"{min(s.newton_iters for s in stats)}..{max(s.newton_iters for s in stats)}")
    assert worst <= 2e-10
    for b in (0, 1, 100, 255):
        c = cbs[b]
        rt, rb, _, _ = oracle.solve(c.geom, c.g_dev, c.v_in, method="cg")
        err = rel_err(vts[b], vbs[b], rt, rb)
        say(f"  sample {b} {c.geom.m}x{c.geom.n}: err {err:.1e}")
        assert err <= TOL


def test_batch_more_than_1024_crossbars():
    """Over 1024 crossbars the per-crossbar control kernels run in several blocks
    (counters summed across them): every crossbar still converges, each matches
    its own residual check, and a sample matches the oracle."""
    cbs = synth.mc_batch(1100, seed=21, sizes=(4, 6, 8, 12))
    say(f"batch of {len(cbs)}")
    bt, vts, vbs, status, stats = batch_solve(cbs)
    assert status == B.MCA_OK
    assert all(s.rel_residual <= 1e-10 for s in stats)
    for b in (0, 511, 1023, 1024, 1099):
        c = cbs[b]
        rt, rb, _, _ = oracle.solve(c.geom, c.g_dev, c.v_in, method="band")
        assert rel_err(vts[b], vbs[b], rt, rb) <= TOL


_CG_CACHE = {}


def _oracle_cg(c, key):
    """Oracle B's steady state of crossbar c, computed once per module."""
    if key not in _CG_CACHE:
        _CG_CACHE[key] = oracle.solve(c.geom, c.g_dev, c.v_in, method="cg")[:2]
    return _CG_CACHE[key]


@pytest.mark.parametrize("prec", [B.MCA_PREC_FP32, B.MCA_PREC_BF16X3])
def test_batch_large_tiles_ragged(prec):
    """18 crossbars of 300 x 520 give 18 x 15 = 270 tiles of 128 per product, so
    the grouped products run 128 x 128 tiles (checked through the library's
    tile query), with edge tiles cut at 300 = 2 x 128 + 44 and 520 = 4 x 128 + 8
    and more than one tile per CU.  Every crossbar against the oracle."""
    cbs = [synth.crossbar(300, 520, seed=s) for s in range(18)]
    bt, vts, vbs, status, stats = batch_solve(cbs, precision=prec)
    assert bt.product_tile == 128
    assert status == B.MCA_OK
    worst = 0.0
    for b, c in enumerate(cbs):
        rt, rb = _oracle_cg(c, ("300x520", b))
        err = rel_err(vts[b], vbs[b], rt, rb)
        worst = max(worst, err)
        assert err <= TOL, (b, err)
    say(f"  18 x 300x520 prec {prec}: newton {[s.newton_iters for s in stats[:4]]}..., "
        f"worst err {worst:.1e}")


@pytest.mark.parametrize("prec", [B.MCA_PREC_FP32, B.MCA_PREC_BF16X3])
def test_batch_folded_and_full_chains(prec):
    """64-tile batch mixing crossbars whose chain folds (persymmetric G_bot, m/2 a
    multiple of 64: m = 128, 256) with ones that keep the full chain (m/2 off the
    tile, or unequal bottom ends), n off the tile grid.  Every crossbar against the
    oracle."""
    shapes = [(128, 100, 0.1), (192, 72, 0.1), (256, 136, 0.1), (256, 136, 0.07), (320, 64, 0.1),
              (128, 200, 0.1), (256, 135, 0.1)]
    cbs = [synth.crossbar(m, n, seed=20 + k, g_bot_end1=e1) for k, (m, n, e1) in enumerate(shapes)]
    bt, vts, vbs, status, stats = batch_solve(cbs, precision=prec)
    assert bt.product_tile == 64
    assert status == B.MCA_OK
    for b, c in enumerate(cbs):
        rt, rb, _, _ = oracle.solve(c.geom, c.g_dev, c.v_in, method="cg")
        err = rel_err(vts[b], vbs[b], rt, rb)
        say(f"  {c.geom.m}x{c.geom.n} ends {c.geom.g_bot_end0},{c.geom.g_bot_end1}: "
            f"newton {stats[b].newton_iters} err {err:.1e}")
        assert err <= TOL


@pytest.mark.parametrize("prec", [B.MCA_PREC_BF16X3])
def test_batch_folded_large_tiles_ragged(prec):
    """22 crossbars of 512 x 300 give 22 x 12 = 264 tiles of 128 per product: the
    folded chain on 128 x 128 tiles with the products' other side cut at
    300 = 2 x 128 + 44.  Four crossbars against the oracle, every residual checked."""
    cbs = [synth.crossbar(512, 300, seed=40 + s) for s in range(22)]
    bt, vts, vbs, status, stats = batch_solve(cbs, precision=prec)
    assert bt.product_tile == 128
    assert status == B.MCA_OK
    assert all(st.rel_residual <= 1e-10 for st in stats)
    for b in (0, 7, 14, 21):
        rt, rb = _oracle_cg(cbs[b], ("512x300", b))
        err = rel_err(vts[b], vbs[b], rt, rb)
        say(f"  512x300 #{b}: newton {stats[b].newton_iters} err {err:.1e}")
        assert err <= TOL


def test_batch_folded_short_depth_large_tiles():
    """16 crossbars of 256 x 1024 give 16 x 16 = 256 tiles of 128: the folded chain
    contracts over m / 2 = 128 (four 32-deep slices, fewer than one whole round of
    the software-pipelined loop, so only its tail steps run) and over n = 1024.
    Every residual recomputed by the oracle, four crossbars against its steady
    state element by element."""
    cbs = [synth.crossbar(256, 1024, seed=60 + s) for s in range(16)]
    bt, vts, vbs, status, stats = batch_solve(cbs)
    assert bt.product_tile == 128
    assert status == B.MCA_OK
    for b, c in enumerate(cbs):
        ft, fb = oracle.residual(c.geom, c.g_dev, c.v_in, vts[b], vbs[b])[:2]
        rel = np.sqrt((ft ** 2).sum() + (fb ** 2).sum()) / oracle.source_norm(c.geom, c.v_in)
        assert rel <= 1e-10, (b, rel)
    for b in (0, 5, 10, 15):
        rt, rb = _oracle_cg(cbs[b], ("256x1024", b))
        err = rel_err(vts[b], vbs[b], rt, rb)
        say(f"  256x1024 #{b}: newton {stats[b].newton_iters} krylov {stats[b].krylov_iters} "
            f"err {err:.1e}")
        assert err <= TOL


@pytest.mark.parametrize("count", [4, 5])
def test_batch_large_tiles_1024(count):
    """1024 x 1024 crossbars on 128 x 128 tiles, split-BF16: 4 crossbars give
    256 tiles per product (one per CU), 5 give 320 (some CUs take two); interior
    tiles take the direct-to-LDS loop either way.  Every crossbar's
    residual is recomputed by the oracle; crossbars 0 and 1 are compared with
    the oracle's steady state element by element."""
    cbs = [synth.crossbar(1024, 1024, seed=s) for s in range(count)]
    bt, vts, vbs, status, stats = batch_solve(cbs)
    assert bt.product_tile == 128
    assert status == B.MCA_OK
    for b, c in enumerate(cbs):
        ft, fb = oracle.residual(c.geom, c.g_dev, c.v_in, vts[b], vbs[b])[:2]
        rel = np.sqrt((ft ** 2).sum() + (fb ** 2).sum()) / oracle.source_norm(c.geom, c.v_in)
        assert rel <= 1e-10, (b, rel)
    for b in (0, 1):
        rt, rb = _oracle_cg(cbs[b], ("1024", b))
        err = rel_err(vts[b], vbs[b], rt, rb)
        say(f"  {count} x 1024^2 crossbar {b}: newton {stats[b].newton_iters} krylov "
            f"{stats[b].krylov_iters} err {err:.1e}")
        assert err <= TOL


@pytest.mark.parametrize("flag,stride", [(B.MCA_FLAG_TIMING, 1), (B.MCA_FLAG_TIMING_SAMPLED, 4)])
def test_batch_timing_of_the_products(flag, stride):
    """MCA_FLAG_TIMING(_SAMPLED) on a batch: HIP events around the four grouped
    products of every (every fourth) preconditioner application; the solution
    and the counts are those of the untimed solve bit for bit, stats[0] holds a
    positive time and four launches per timed application, the other records
    none; under MCA_FLAG_GRAPH nothing is timed."""
    cbs = ragged_batch(seed=8)
    bt, vt0, vb0, s0, st0 = batch_solve(cbs)
    _, vt1, vb1, s1, st1 = batch_solve(cbs, flags=flag)
    assert s0 == s1 == B.MCA_OK
    for b in range(len(cbs)):
        assert np.array_equal(vt0[b], vt1[b]) and np.array_equal(vb0[b], vb1[b])
        assert st0[b].krylov_iters == st1[b].krylov_iters
    ms = st1[0].kernel_ms[B.MCA_KCLASS_GEMM]
    n = st1[0].kernel_launches[B.MCA_KCLASS_GEMM]
    say(f"  timed {n // 4} applications, {ms:.3f} ms")
    assert ms > 0 and n > 0 and n % 4 == 0
    # every application of the batch is enqueued once per Arnoldi step; at least
    # the steps of the longest-running crossbar
    assert n // 4 >= max(s.krylov_iters for s in st1) // stride
    assert all(s.kernel_ms[B.MCA_KCLASS_GEMM] == 0 for s in st1[1:])
    _, _, _, s2, st2 = batch_solve(cbs, flags=flag | B.MCA_FLAG_GRAPH)
    assert s2 == B.MCA_OK and st2[0].kernel_launches[B.MCA_KCLASS_GEMM] == 0


def test_batch_graph_replays_match_eager():
    """Arnoldi steps captured as HIP graphs (MCA_FLAG_GRAPH) reproduce the eager
    launches bit for bit: at capture, on replays in later cycles (restart 5) and
    later solves, with eager solves and other inputs in between, and after a
    change of workspace (which drops the captured steps)."""
    cbs = ragged_batch(seed=5)
    bt = Batch([c.geom for c in cbs])
    kw = dict(precond=B.MCA_PRECOND_PERMODE, precision=B.MCA_PREC_BF16X3, restart=5)
    eager = B.options(**kw)
    graph = B.options(flags=B.MCA_FLAG_GRAPH, **kw)
    ws = bt.workspace(eager)
    ws2 = bt.workspace(eager)
    inputs = {
        "a": (bt.concat([c.g_dev for c in cbs]), bt.concat([c.v_in for c in cbs])),
        "b": (bt.concat([c.g_dev[::-1].copy() for c in cbs]),
              bt.concat([0.5 * c.v_in for c in cbs])),
    }

    def run(key, opts, w):
        g, v = inputs[key]
        vt, vb, status, stats = bt.solve(g, v, opts, ws=w)
        torch.cuda.synchronize()
        return (vt.cpu().numpy(), vb.cpu().numpy(), status,
                [(s.newton_iters, s.krylov_iters, s.restarts) for s in stats])

    ref = {k: run(k, eager, ws) for k in inputs}
    for k, r in ref.items():
        say(f"graph batch eager {k}: status {r[2]} iterations {r[3]}")
        assert r[2] == B.MCA_OK
    assert any(it[2] > 0 for it in ref["a"][3]), "restart 5 should restart some crossbar"
    for i, (k, w) in enumerate([("a", ws), ("b", ws), ("a", ws), ("b", ws2), ("a", ws2)]):
        if i == 2:
            run("b", eager, ws)          # eager work between the replays
        got = run(k, graph, w)
        say(f"graph replay {i} ({k}): status {got[2]} iterations {got[3]}")
        assert got[2] == ref[k][2]
        assert got[3] == ref[k][3]
        assert np.array_equal(got[0], ref[k][0]) and np.array_equal(got[1], ref[k][1])


def test_batch_graph_follows_gram_schmidt_form():
    """Captured Arnoldi steps depend on the Gram-Schmidt form: graph solves that
    alternate between the two-pass form and one pass per basis vector on one
    workspace each reproduce the eager solve of their own form bit for bit."""
    cbs = ragged_batch(seed=5)
    bt = Batch([c.geom for c in cbs])
    g = bt.concat([c.g_dev for c in cbs])
    v = bt.concat([c.v_in for c in cbs])
    kw = dict(precond=B.MCA_PRECOND_PERMODE, precision=B.MCA_PREC_BF16X3, restart=5)
    ws = bt.workspace(B.options(**kw))
    ref = {}
    for name, flags in (("two-pass", 0), ("per-vector", B.MCA_FLAG_MGS_PASSES)):
        vt, vb, status, stats = bt.solve(g, v, B.options(flags=flags, **kw), ws=ws)
        torch.cuda.synchronize()
        assert status == B.MCA_OK
        ref[name] = (vt.cpu().numpy(), vb.cpu().numpy(), [s.krylov_iters for s in stats])
    for name, flags in (("two-pass", 0), ("per-vector", B.MCA_FLAG_MGS_PASSES),
                        ("two-pass", 0), ("per-vector", B.MCA_FLAG_MGS_PASSES)):
        vt, vb, status, stats = bt.solve(g, v, B.options(flags=flags | B.MCA_FLAG_GRAPH, **kw),
                                         ws=ws)
        torch.cuda.synchronize()
        say(f"graph {name}: status {status} krylov {[s.krylov_iters for s in stats]}")
        assert status == B.MCA_OK
        assert [s.krylov_iters for s in stats] == ref[name][2]
        assert np.array_equal(vt.cpu().numpy(), ref[name][0])
        assert np.array_equal(vb.cpu().numpy(), ref[name][1])


def test_single_solve_rejects_graph_flag():
    c = synth.crossbar(16, 16, seed=0)
    plan = Plan(c.geom)
    o = B.options(flags=B.MCA_FLAG_GRAPH)
    with pytest.raises(Exception):
        plan.solve(torch.from_numpy(c.g_dev).cuda(), torch.from_numpy(c.v_in).cuda(), o)


@pytest.mark.parametrize("restart", [5, 30])
def test_batch_two_pass_gram_schmidt_matches_one_pass_per_vector(restart):
    """The batched solver's default orthogonalisation (modified Gram-Schmidt in
    compact WY form, two passes per step, per-crossbar reductions by each
    crossbar's last block) against MGS with one pass per basis vector: same
    Newton counts, GMRES counts within one per Newton step, and both within the
    bar of the oracle's steady state."""
    cbs = ragged_batch(seed=9)
    runs = {}
    for name, flags in (("two-pass", 0), ("per-vector", B.MCA_FLAG_MGS_PASSES)):
        _, vts, vbs, status, stats = batch_solve(cbs, restart=restart, flags=flags)
        assert status == B.MCA_OK
        runs[name] = (vts, vbs, stats)
    for b, c in enumerate(cbs):
        rt, rb, _, _ = oracle.solve(c.geom, c.g_dev, c.v_in, method="band")
        sa, sb = runs["two-pass"][2][b], runs["per-vector"][2][b]
        ka = list(sa.krylov_history[:sa.newton_iters])
        kb = list(sb.krylov_history[:sb.newton_iters])
        ea = rel_err(runs["two-pass"][0][b], runs["two-pass"][1][b], rt, rb)
        eb = rel_err(runs["per-vector"][0][b], runs["per-vector"][1][b], rt, rb)
        say(f"  {c.geom.m}x{c.geom.n} restart {restart}: two-pass {ka} err {ea:.1e}, "
            f"per-vector {kb} err {eb:.1e}")
        assert sa.newton_iters == sb.newton_iters
        assert all(abs(x - y) <= 1 for x, y in zip(ka, kb))
        assert ea <= TOL and eb <= TOL


def test_batch_many_ragged_crossbars_shallow_slices():
    """Enough ragged crossbars that the grouped products run two tiles per CU
    (64 x 64 tiles with 32-deep K slices, 512 or more tiles per product): every
    crossbar converges, and a sample matches the oracle's steady state."""
    cbs = synth.mc_batch(420, seed=21, sizes=(20, 33, 64, 72, 100))
    tiles = sum(-(-c.geom.m // 64) * -(-c.geom.n // 64) for c in cbs)
    say(f"ragged batch of {len(cbs)} crossbars, {tiles} tiles per product")
    assert tiles >= 512
    bt, vts, vbs, status, stats = batch_solve(cbs)
    assert status == B.MCA_OK
    assert max(s.rel_residual for s in stats) <= 1e-10
    for b in range(0, len(cbs), 21):
        c = cbs[b]
        rt, rb, _, _ = oracle.solve(c.geom, c.g_dev, c.v_in, method="band")
        err = rel_err(vts[b], vbs[b], rt, rb)
        say(f"  {c.geom.m}x{c.geom.n}: newton {stats[b].newton_iters} krylov "
            f"{stats[b].krylov_iters} err {err:.1e}")
        assert err <= TOL
