#!/usr/bin/env python3
"""Throughput of the steady-state memristor-crossbar solver on one MI355X.

One step = one full mca_solve (Newton + preconditioned flexible GMRES) of the
standard 1024 x 1024 crossbar (about 2.1M unknowns, FP64) from V = 0 to the
Newton tolerance 1e-10 (||F|| / ||Y||) with GMRES(30) tolerance 1e-8, inputs
already resident in HBM.  Prints one JSON line.

  python bench.py [--gpus 1] [--steps K] [--warmup W] [--size 1024]

With --mc COUNT a step is instead one batched solve (mca_solve_batched) of
COUNT Monte-Carlo crossbars of uneven sizes (m, n drawn from {64, ..., 512},
16-level weights with lognormal device variation, wire conductance drawn per
crossbar); with --batch COUNT, of COUNT standard size x size crossbars (seeds
seed .. seed + COUNT - 1).  Both are timed beside a loop of per-crossbar
mca_solve calls with the same options.
"""

from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0          # MI355X HBM3E
FP64_MFMA_PEAK_TFLOPS = 78.6   # MI355X dense FP64 matrix


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=10)
    p.add_argument("--warmup", type=int, default=2)
    p.add_argument("--size", type=int, default=1024, help="crossbar is size x size")
    p.add_argument("--seed", type=int, default=0)
    p.add_argument("--precond", choices=["literal", "permode", "approx", "jacobi", "none"],
                   default=None, help="default: literal for fp64, permode otherwise")
    p.add_argument("--precision", choices=["fp64", "fp32", "bf16x3", "bf16"], default="fp64",
                   help="arithmetic of the preconditioner's eigenbasis transforms")
    p.add_argument("--no-cpu-baseline", action="store_true")
    p.add_argument("--no-timing", action="store_true",
                   help="do not time kernel classes with HIP events (no roofline object)")
    p.add_argument("--full-timing", action="store_true",
                   help="time every kernel group inside the timed solves (MCA_FLAG_TIMING; each "
                        "timed event idles the GPU for a few microseconds) instead of every 4th "
                        "preconditioner application (MCA_FLAG_TIMING_SAMPLED)")
    p.add_argument("--mc", type=int, default=0,
                   help="batched Monte-Carlo workload of this many crossbars instead")
    p.add_argument("--batch", type=int, default=0,
                   help="batched solve of this many size x size crossbars instead")
    p.add_argument("--mgs-passes", action="store_true",
                   help="orthogonalise with one pass per basis vector (MCA_FLAG_MGS_PASSES) "
                        "instead of the two-pass compact WY form")
    p.add_argument("--graph", action="store_true",
                   help="with --mc / --batch: replay the Arnoldi steps as captured HIP graphs "
                        "(the eager launches are timed beside them)")
    p.add_argument("--no-loop", action="store_true",
                   help="with --mc / --batch: skip the per-crossbar loop comparison")
    p.add_argument("--no-compare", action="store_true",
                   help="skip the batched + warm-started + mixed-precision comparison")
    p.add_argument("--no-extra-configs", action="store_true",
                   help="skip the 2048^2 mixed-precision and 256-crossbar Monte-Carlo legs")
    p.add_argument("--compare-batch", type=int, default=16,
                   help="crossbars per batch of the comparison forms")
    p.add_argument("--copy-calib", action="store_true",
                   help="after the timed solves, copy a 256 MiB float64 array device-to-device "
                        "three times: a kernel of known traffic that calibrates the "
                        "FETCH_SIZE / WRITE_SIZE counters")
    return p.parse_args()


def gemm_traffic():
    """HBM bytes of one preconditioner application's FP64 transforms at 1024^2,
    from the committed rocprofv3 counter summary, or None when the kernels
    changed since it was taken."""
    import hashlib
    prof = os.path.join(ROOT, "profiles", "solve_fp64_1024x1024.md")
    h = hashlib.sha256()
    try:
        text = open(prof).read()
        for f in ("gemm.hip", "kernels.hip"):
            h.update(open(os.path.join(ROOT, "paper_2109_07929_amd", "csrc", f), "rb").read())
    except OSError:
        return None
    digest = h.hexdigest()
    vals = dict(l.split(": ", 1) for l in text.splitlines()
                if l.startswith(("transform_traffic_bytes_per_application:",
                                 "transform_source_sha256:")))
    if vals.get("transform_source_sha256", "").strip() != digest:
        return None
    return int(vals["transform_traffic_bytes_per_application"])


def krylov_hbm(st, mn, opts, kms, steps):
    """HBM roofline of the Krylov part of a solve (the Jacobian products and the
    Arnoldi orthogonalisation), from the timed kernel classes of the last solve's
    iteration counts.  Algorithmic bytes per crosspoint at Arnoldi step j: the
    matvec 40 (read x, D; write y) plus MGS 16 (j + 1) + 32 (read the basis once,
    read and write w).  Kernel bytes: what the kernels must move, which reads the
    basis twice in the two-pass form (projections, then update), and once per
    projection pass in the one-pass-per-vector form.  The time is that of the
    Jacobian and orthogonalisation classes (HIP events around the streaming
    passes; the one-block Givens kernels are outside them)."""
    from paper_2109_07929_amd import binding as B
    R = opts.restart
    two_pass = not (opts.flags & B.MCA_FLAG_MGS_PASSES) and R <= 32
    # literal FP64 form, two passes: the Jacobian pass also forms the preconditioner's
    # last step z_b from z_t (reads r_t and writes z_b instead of reading z_b: +8 B)
    post = (two_pass and opts.precond == B.MCA_PRECOND_LITERAL
            and opts.precision == B.MCA_PREC_FP64)
    alg = kern = 0.0
    for k in st.krylov_history[:st.newton_iters]:
        while k > 0:
            c = min(R, k)
            for j in range(c):
                alg += 40 + 16 * (j + 1) + 32
                if two_pass:
                    kern += (40 + (8 if post else 0) + 16 * (j + 1)) + (32 + 16 * (j + 1))
                else:
                    # Jacobian with <y, v_0> (56), j + 1 fused MGS passes (64, the last
                    # without the next projection 48), normalisation (32)
                    kern += 56 + 64 * j + 48 + 32
            k -= c
    ms = (kms[B.MCA_KCLASS_JACOBIAN] + kms[B.MCA_KCLASS_ORTHO]) / steps
    if ms <= 0:
        return None
    a = alg * mn / (ms * 1e-3) / 1e9
    kb = kern * mn / (ms * 1e-3) / 1e9
    return {"bound": "hbm", "form": "two-pass MGS (compact WY)" if two_pass else "MGS, one pass per vector",
            "ms_per_solve": round(ms, 4), "algorithmic_bytes_per_solve": alg * mn,
            "achieved_algorithmic": round(a, 1), "kernel_bytes_per_solve": kern * mn,
            "achieved_kernel": round(kb, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac_algorithmic": round(a / HBM_PEAK_GBS, 4), "frac_kernel": round(kb / HBM_PEAK_GBS, 4),
            "timing": "HIP-event brackets around each Jacobian and orthogonalisation group; each "
                      "bracket also holds the few microseconds a timed event leaves the GPU idle, so "
                      "these rates sit below the kernels' own (rocprofv3 durations per Arnoldi step "
                      "in profiles/solve_fp64_1024x1024.md)"}


def hbm_copy(out, roofline, kry_hbm, ev0, ev1, stream, dev):
    import torch
    big = torch.empty(1 << 27, dtype=torch.float64, device=dev)
    big2 = torch.empty_like(big)
    for _ in range(2):
        big2.copy_(big)
    ev0.record(stream)
    for _ in range(5):
        big2.copy_(big)
    ev1.record(stream)
    torch.cuda.synchronize()
    out["hbm_copy_GBs"] = round(2 * big.numel() * 8 * 5 / (ev0.elapsed_time(ev1) * 1e-3) / 1e9, 1)
    if roofline is not None and roofline.get("unit") == "GB/s":
        roofline["frac_of_copy"] = round(roofline["achieved"] / out["hbm_copy_GBs"], 4)
    if kry_hbm is not None:
        kry_hbm["frac_kernel_of_copy"] = round(kry_hbm["achieved_kernel"] / out["hbm_copy_GBs"], 4)


def _cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def _oracle_solve_seconds(m, n, seed):
    """One oracle solve of the standard crossbar (run in a worker process)."""
    import oracle
    from paper_2109_07929_amd import synth
    cb = synth.crossbar(m, n, seed=seed)
    t0 = time.perf_counter()
    oracle.solve(cb.geom, cb.g_dev, cb.v_in, method="cg")
    return time.perf_counter() - t0


def cpu_baseline(cb, workers=16):
    """The CPU oracle (plain FP64 C, one thread per solve) on the same crossbar:
    one full Newton solve with CG linear steps (the oracle's large-size method),
    first alone, then as many independent solves side by side as there are
    workers (the host's all-cores throughput; this box's share of host cores is
    at most 16)."""
    import multiprocessing as mp
    m, n = cb.geom.m, cb.geom.n
    t1 = _oracle_solve_seconds(m, n, 0)
    nproc = os.cpu_count() or 1
    try:
        avail = len(os.sched_getaffinity(0))
    except AttributeError:
        avail = nproc
    k = max(1, min(workers, avail))
    ctx = mp.get_context("spawn")
    t0 = time.perf_counter()
    with ctx.Pool(k) as pool:
        times = pool.starmap(_oracle_solve_seconds, [(m, n, s) for s in range(k)])
    wall = time.perf_counter() - t0
    return {"value": round(k / wall, 4), "unit": "solves/s", "cores": k, "kind": "oracle",
            "sample": f"{k} independent {m}x{n} solves (Newton, CG linear steps, to the FP64 "
                      f"floor; seeds 0..{k - 1}), one per worker process, side by side: "
                      f"{wall:.2f} s wall (slowest solve {max(times):.2f} s)",
            "single_thread": {"value": round(1.0 / t1, 4), "cores": 1,
                              "sample": f"one {m}x{n} solve, seed 0: {t1:.2f} s"},
            "cpu_model": _cpu_model(), "nproc": nproc, "cpus_available": avail}


def bench_batched(args):
    """Batched workloads: one step = one mca_solve_batched of all the crossbars."""
    import numpy as np
    import torch

    from paper_2109_07929_amd import Batch, Plan, synth
    from paper_2109_07929_amd import binding as B

    torch.cuda.init()
    dev = torch.device("cuda:0")
    prec = {"fp32": B.MCA_PREC_FP32, "bf16x3": B.MCA_PREC_BF16X3, "bf16": B.MCA_PREC_BF16}.get(
        args.precision, B.MCA_PREC_BF16X3)
    pname = {B.MCA_PREC_FP32: "fp32", B.MCA_PREC_BF16X3: "bf16x3", B.MCA_PREC_BF16: "bf16"}[prec]
    if args.mc:
        cbs = synth.mc_batch(args.mc, seed=args.seed)
        what = (f"batched Monte-Carlo, {args.mc} crossbars with m, n in {{64..512}}")
    else:
        cbs = [synth.crossbar(args.size, args.size, seed=args.seed + i) for i in range(args.batch)]
        what = f"batched, {args.batch} crossbars of {args.size}x{args.size}"
    count = len(cbs)
    t0 = time.perf_counter()
    bt = Batch([c.geom for c in cbs], device=dev)
    setup_ms = 1e3 * (time.perf_counter() - t0)
    g = bt.concat([c.g_dev for c in cbs])
    v = bt.concat([c.v_in for c in cbs])
    vt = torch.zeros(bt.total, dtype=torch.float64, device=dev)
    vb = torch.zeros_like(vt)
    opts = B.options(precond=B.MCA_PRECOND_PERMODE, precision=prec,
                     flags=B.MCA_FLAG_GRAPH if args.graph else 0)
    ws = bt.workspace(opts)
    stream = torch.cuda.current_stream()
    rows = int(bt.rows[-1])

    def timed(o):
        def step():
            return B.mca_solve_batched(bt.handle, bt.count, bt.total, rows, g, v, vt, vb, o, ws,
                                       stream)[1]
        for _ in range(args.warmup):
            step()
        torch.cuda.synchronize()
        ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        ev0.record(stream)
        for _ in range(args.steps):
            st = step()
        ev1.record(stream)
        torch.cuda.synchronize()
        return ev0.elapsed_time(ev1) / args.steps, st

    ms_per_step, stats = timed(opts)
    value = count * 1e3 / ms_per_step
    eager = None
    if args.graph:
        ems, _ = timed(B.options(precond=B.MCA_PRECOND_PERMODE, precision=prec))
        eager = {"ms_per_batch": round(ems, 3), "solves_per_s": round(count * 1e3 / ems, 2)}
        print(f"# eager launches: {ems:.2f} ms per batch", file=sys.stderr, flush=True)
    newton = [s.newton_iters for s in stats]
    krylov = [s.krylov_iters for s in stats]
    print(f"# batched: {ms_per_step:.2f} ms per batch", file=sys.stderr, flush=True)

    loop = None
    if not args.no_loop:
        # the same crossbars one mca_solve call after another, same options
        plans = [Plan(c.geom, device=dev) for c in cbs]
        data = [(torch.from_numpy(c.g_dev).to(dev), torch.from_numpy(c.v_in).to(dev),
                 torch.zeros((c.geom.m, c.geom.n), dtype=torch.float64, device=dev),
                 torch.zeros((c.geom.m, c.geom.n), dtype=torch.float64, device=dev)) for c in cbs]
        wss = [p.workspace(opts) for p in plans]

        def loop_step():
            for p, (gg, vv, ot, ob), w in zip(plans, data, wss):
                B.mca_solve(p.handle, p.m, p.n, gg, vv, ot, ob, opts, w, stream)

        loop_step()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        reps = max(1, min(3, args.steps))
        for _ in range(reps):
            loop_step()
        torch.cuda.synchronize()
        loop_ms = 1e3 * (time.perf_counter() - t0) / reps
        loop = {"ms_per_batch": round(loop_ms, 3), "solves_per_s": round(count * 1e3 / loop_ms, 2),
                "speedup_of_batched": round(loop_ms / ms_per_step, 3)}
        print(f"# loop: {loop_ms:.2f} ms per batch", file=sys.stderr, flush=True)

    sizes = [c.geom.m * c.geom.n for c in cbs]
    out = {
        "metric": "MCA solves/s at 1024x1024, 1e-8 rel residual: plain FP64 vs batched+warm+mixed",
        "value": round(value, 3),
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": f"f64 (preconditioner {pname})",
        "data": "synthetic",
        "config": {"workload": f"{what} ({sum(sizes)} crosspoints), seed {args.seed}, "
                               f"Newton-FGMRES(30) with a {pname} per-mode preconditioner",
                   "newton_tol": opts.newton_tol, "gmres_tol": opts.gmres_tol,
                   "setup_ms": round(setup_ms, 1), "graph": bool(args.graph),
                   "newton_iters": [min(newton), max(newton)],
                   "krylov_iters": [min(krylov), max(krylov)]},
        "per_crossbar_loop": loop,
        "eager_launches": eager,
        # with the batch's host set-up (eigen-decompositions, upload) counted once
        "solves_per_s_with_setup": round(count * 1e3 / (ms_per_step + setup_ms), 2),
        "roofline": None,
    }
    print(json.dumps(out), flush=True)


def batched_products_roofline(B, bt, cbs, g, v, vt, vb, ws, stream, **base):
    """The batch's dominant kernels, the four grouped split-BF16 products of each
    preconditioner application: one more batched solve from V = 0 (outside any
    timed region) with every application's products bracketed by HIP events;
    their algorithmic flops over that time.  None unless the solve succeeds."""
    import torch

    o = B.options(flags=B.MCA_FLAG_TIMING, **base)
    status, stats = B.mca_solve_batched(bt.handle, bt.count, bt.total, int(bt.rows[-1]), g, v, vt,
                                        vb, o, ws, stream, check=False)
    torch.cuda.synchronize()
    pms = float(stats[0].kernel_ms[B.MCA_KCLASS_GEMM])
    apps = int(stats[0].kernel_launches[B.MCA_KCLASS_GEMM]) // 4
    # algorithmic flops of the per-mode form: 8 (m + n) per crosspoint and
    # application, every Arnoldi step applying P once per running crossbar
    flops = sum(8.0 * (c.geom.m + c.geom.n) * c.geom.m * c.geom.n * st.krylov_iters
                for c, st in zip(cbs, stats))
    if status != B.MCA_OK or pms <= 0 or apps <= 0:
        return None
    tf = flops / (pms * 1e-3) / 1e12
    return {
        "bound": "mfma", "kernel": "the four grouped split-BF16 products of one "
                                   "preconditioner application (k_gemm_nt_lp_grouped)",
        "achieved": round(tf, 1), "peak": 2500.0, "unit": "TFLOP/s",
        "frac": round(tf / 2500.0, 4),
        "flops_unit": "algorithmic: 8(m+n) per crosspoint per application (per-mode form), "
                      "counted once per split-BF16 product",
        "executed_note": "split-BF16 runs three BF16 MFMA products per product; the "
                         "persymmetric fold runs the two Q_m-side products at half depth",
        "ms_per_application": round(pms / apps, 4), "applications_timed": apps,
        "timing": "HIP events before the first and after the fourth product of every "
                  "application of one batched solve from V = 0; applications enqueued past "
                  "convergence (products that return at once) and the idle time an event "
                  "leaves are in the time, not in the flops"}


def compare_forms(args, dev):
    """The metric's other side at the same size and tolerance: batches of
    args.compare_batch crossbars (seeds seed .. seed + count - 1) solved by
    mca_solve_batched with the split-BF16 per-mode preconditioner, from V = 0,
    from the sweep start, and from the warm-start network's guess (prediction
    time included), each with the guess fallback."""
    import torch

    from paper_2109_07929_amd import Batch, synth, warmstart
    from paper_2109_07929_amd import binding as B

    count, m = args.compare_batch, args.size
    cbs = [synth.crossbar(m, m, seed=args.seed + i) for i in range(count)]
    bt = Batch([c.geom for c in cbs], device=dev)
    g = bt.concat([c.g_dev for c in cbs])
    v = bt.concat([c.v_in for c in cbs])
    vt = torch.zeros(bt.total, dtype=torch.float64, device=dev)
    vb = torch.zeros_like(vt)
    base = dict(precond=B.MCA_PRECOND_PERMODE, precision=B.MCA_PREC_BF16X3)
    ws = bt.workspace(B.options(**base))
    stream = torch.cuda.current_stream()
    rows = int(bt.rows[-1])
    params = None
    if os.path.exists(warmstart.DEFAULT_PARAMS):
        params = warmstart.load_params(device=dev)
        cws = torch.empty(B.mca_cnn_workspace_bytes(count, m, m), dtype=torch.uint8, device=dev)
        g3, v2 = g.view(count, m, m), v.view(count, m)
        pt = torch.empty((count, m, m), dtype=torch.float64, device=dev)
        pb = torch.empty_like(pt)

    def run(form):
        if form == "cnn":
            B.mca_cnn_predict(params, [c.geom for c in cbs], g3, v2, pt, pb, cws, stream)
            vt.copy_(pt.view(-1))
            vb.copy_(pb.view(-1))
            flags = B.MCA_FLAG_INITIAL_GUESS | B.MCA_FLAG_GUESS_FALLBACK
        else:
            flags = B.MCA_FLAG_SWEEP_START | B.MCA_FLAG_GUESS_FALLBACK if form == "sweep" else 0
        o = B.options(flags=flags, **base)
        return B.mca_solve_batched(bt.handle, count, bt.total, rows, g, v, vt, vb, o, ws,
                                   stream, check=False)

    out = {"batch": count, "precision": "bf16x3 (per-mode)", "forms": {},
           "form_notes": {
               "zero": "batched + mixed, Newton from V = 0",
               "sweep": "batched + mixed, Newton from one block Gauss-Seidel sweep on the "
                        "linearisation at V = 0 (a non-learned start)",
               "cnn": "batched + mixed + learned warm start: the network's guess (inference "
                      "timed), with the guess fallback"}}
    if params is not None:
        out["network"] = warmstart.describe_params(warmstart.DEFAULT_PARAMS)
    for form in ("zero", "sweep", "cnn"):
        if form == "cnn" and params is None:
            continue
        for _ in range(max(1, args.warmup)):
            run(form)
        torch.cuda.synchronize()
        ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        ev0.record(stream)
        for _ in range(args.steps):
            status, stats = run(form)
        ev1.record(stream)
        torch.cuda.synchronize()
        ms = ev0.elapsed_time(ev1) / args.steps
        out["forms"][form] = {
            "solves_per_s": round(count * 1e3 / ms, 2), "ms_per_batch": round(ms, 3),
            "status": B.status_string(status),
            "newton_iters": sum(s.newton_iters for s in stats) / count,
            "krylov_iters": sum(s.krylov_iters for s in stats) / count,
            "guess_used": sum(s.start for s in stats) / count,
            "max_rel_residual": max(s.rel_residual for s in stats)}
        print(f"# {form}: {ms:.2f} ms per batch of {count}", file=sys.stderr, flush=True)
    rf = batched_products_roofline(B, bt, cbs, g, v, vt, vb, ws, stream, **base)
    if rf is not None:
        out["products_roofline"] = rf
    return out


def leg_mixed_2048(args, dev, size=2048, reps=3):
    """The mixed-precision workload: one size x size standard crossbar (seed
    args.seed) solved with the FP64 literal preconditioner and with the
    split-BF16 and FP32 per-mode ones inside the same FP64 Newton-FGMRES; times
    (HIP events, `reps` solves after one warm-up each), iterations, and the
    largest relative voltage difference from the FP64 solve."""
    import torch

    from paper_2109_07929_amd import Plan, synth
    from paper_2109_07929_amd import binding as B

    cb = synth.crossbar(size, size, seed=args.seed)
    t0 = time.perf_counter()
    plan = Plan(cb.geom, device=dev)
    setup_ms = 1e3 * (time.perf_counter() - t0)
    g = torch.from_numpy(cb.g_dev).to(dev)
    v = torch.from_numpy(cb.v_in).to(dev)
    stream = torch.cuda.current_stream()
    out = {"workload": f"{size}x{size} crossbar ({2 * size * size} unknowns), seed {args.seed}",
           "setup_ms": round(setup_ms, 1), "forms": {}}
    ref = None
    for name, form, prec in (("fp64 literal", B.MCA_PRECOND_LITERAL, B.MCA_PREC_FP64),
                             ("bf16x3 per-mode", B.MCA_PRECOND_PERMODE, B.MCA_PREC_BF16X3),
                             ("fp32 per-mode", B.MCA_PRECOND_PERMODE, B.MCA_PREC_FP32)):
        o = B.options(precond=form, precision=prec)
        ws = plan.workspace(o)
        vt = torch.zeros((size, size), dtype=torch.float64, device=dev)
        vb = torch.zeros_like(vt)
        status, st = B.mca_solve(plan.handle, size, size, g, v, vt, vb, o, ws, stream, check=False)
        torch.cuda.synchronize()
        ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        ev0.record(stream)
        for _ in range(reps):
            status, st = B.mca_solve(plan.handle, size, size, g, v, vt, vb, o, ws, stream,
                                     check=False)
        ev1.record(stream)
        torch.cuda.synchronize()
        ms = ev0.elapsed_time(ev1) / reps
        rec = {"ms_per_solve": round(ms, 3), "solves_per_s": round(1e3 / ms, 2),
               "status": B.status_string(status), "newton_iters": st.newton_iters,
               "krylov_history": list(st.krylov_history[:st.newton_iters]),
               "rel_residual": st.rel_residual}
        if ref is None:
            ref = (vt.clone(), vb.clone(), ms)
        else:
            scale = float(torch.maximum(ref[0].abs().max(), ref[1].abs().max()))
            dv = float(torch.maximum((vt - ref[0]).abs().max(), (vb - ref[1]).abs().max()))
            rec["max_rel_dv_vs_fp64"] = dv / scale
            rec["speedup_vs_fp64"] = round(ref[2] / ms, 3)
        out["forms"][name] = rec
        print(f"# {size}^2 {name}: {ms:.2f} ms per solve", file=sys.stderr, flush=True)
        del ws
    return out


def leg_approx(args, dev, size=1024, reps=10):
    """The paper's own approximation of the preconditioner (M ~ Mhat, eq. (Mhat):
    tridiagonal line solves instead of the eigenbasis transforms) inside the
    same FP64 Newton-FGMRES on the metric's crossbar: time per solve (HIP events,
    `reps` solves after one warm-up), iterations, and the largest relative
    voltage difference from the exact-preconditioner (FP64 literal) solve."""
    import torch

    from paper_2109_07929_amd import Plan, synth
    from paper_2109_07929_amd import binding as B

    cb = synth.crossbar(size, size, seed=args.seed)
    plan = Plan(cb.geom, device=dev)
    g = torch.from_numpy(cb.g_dev).to(dev)
    v = torch.from_numpy(cb.v_in).to(dev)
    stream = torch.cuda.current_stream()
    out = {"workload": f"{size}x{size} crossbar ({2 * size * size} unknowns), seed {args.seed}",
           "forms": {}}
    ref = None
    for name, form in (("exact (literal)", B.MCA_PRECOND_LITERAL), ("approx (Mhat)", B.MCA_PRECOND_APPROX)):
        o = B.options(precond=form, precision=B.MCA_PREC_FP64)
        ws = plan.workspace(o)
        vt = torch.zeros((size, size), dtype=torch.float64, device=dev)
        vb = torch.zeros_like(vt)
        status, st = B.mca_solve(plan.handle, size, size, g, v, vt, vb, o, ws, stream, check=False)
        torch.cuda.synchronize()
        ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        ev0.record(stream)
        for _ in range(reps):
            status, st = B.mca_solve(plan.handle, size, size, g, v, vt, vb, o, ws, stream,
                                     check=False)
        ev1.record(stream)
        torch.cuda.synchronize()
        ms = ev0.elapsed_time(ev1) / reps
        rec = {"ms_per_solve": round(ms, 3), "solves_per_s": round(1e3 / ms, 2),
               "status": B.status_string(status), "newton_iters": st.newton_iters,
               "krylov_history": list(st.krylov_history[:st.newton_iters]),
               "rel_residual": st.rel_residual}
        if ref is None:
            ref = (vt.clone(), vb.clone(), ms)
        else:
            scale = float(torch.maximum(ref[0].abs().max(), ref[1].abs().max()))
            dv = float(torch.maximum((vt - ref[0]).abs().max(), (vb - ref[1]).abs().max()))
            rec["max_rel_dv_vs_exact"] = dv / scale
            rec["speedup_vs_exact"] = round(ref[2] / ms, 3)
        out["forms"][name] = rec
        print(f"# {size}^2 {name}: {ms:.2f} ms per solve", file=sys.stderr, flush=True)
        del ws
    return out


def leg_monte_carlo(args, dev, count=256):
    """The Monte-Carlo workload: `count` crossbars with m, n drawn from
    {64, ..., 512} (seed args.seed), split-BF16 per-mode preconditioner, solved
    by one mca_solve_batched per batch against a loop of mca_solve calls with
    the same options; with and without the host set-up (eigen-decompositions
    and uploads) counted."""
    import torch

    from paper_2109_07929_amd import Batch, Plan, synth
    from paper_2109_07929_amd import binding as B

    cbs = synth.mc_batch(count, seed=args.seed)
    opts = B.options(precond=B.MCA_PRECOND_PERMODE, precision=B.MCA_PREC_BF16X3)
    stream = torch.cuda.current_stream()
    t0 = time.perf_counter()
    bt = Batch([c.geom for c in cbs], device=dev)
    setup_ms = 1e3 * (time.perf_counter() - t0)
    g = bt.concat([c.g_dev for c in cbs])
    v = bt.concat([c.v_in for c in cbs])
    vt = torch.zeros(bt.total, dtype=torch.float64, device=dev)
    vb = torch.zeros_like(vt)
    ws = bt.workspace(opts)
    rows = int(bt.rows[-1])

    def step():
        return B.mca_solve_batched(bt.handle, bt.count, bt.total, rows, g, v, vt, vb, opts, ws,
                                   stream, check=False)

    step()
    torch.cuda.synchronize()
    reps = max(3, min(args.steps, 10))
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ev0.record(stream)
    for _ in range(reps):
        status, stats = step()
    ev1.record(stream)
    torch.cuda.synchronize()
    ms = ev0.elapsed_time(ev1) / reps
    print(f"# Monte-Carlo {count}: {ms:.2f} ms per batch", file=sys.stderr, flush=True)
    rf = batched_products_roofline(B, bt, cbs, g, v, vt, vb, ws, stream,
                                   precond=B.MCA_PRECOND_PERMODE, precision=B.MCA_PREC_BF16X3)
    del ws
    torch.cuda.empty_cache()
    # the loop: one plan and workspace per crossbar, one mca_solve after another
    t0 = time.perf_counter()
    plans = [Plan(c.geom, device=dev) for c in cbs]
    loop_setup_ms = 1e3 * (time.perf_counter() - t0)
    data = [(torch.from_numpy(c.g_dev).to(dev), torch.from_numpy(c.v_in).to(dev),
             torch.zeros((c.geom.m, c.geom.n), dtype=torch.float64, device=dev),
             torch.zeros((c.geom.m, c.geom.n), dtype=torch.float64, device=dev)) for c in cbs]
    ws_max = max(B.mca_workspace_bytes(p.handle, opts) for p in plans)
    wsl = torch.empty(ws_max, dtype=torch.uint8, device=dev)

    def loop_step():
        worst = B.MCA_OK
        for p, (gg, vv, ot, ob) in zip(plans, data):
            st, _ = B.mca_solve(p.handle, p.m, p.n, gg, vv, ot, ob, opts, wsl, stream,
                                check=False)
            worst = worst if st == B.MCA_OK else st
        return worst

    loop_step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    lreps = 2
    for _ in range(lreps):
        lstatus = loop_step()
    torch.cuda.synchronize()
    loop_ms = 1e3 * (time.perf_counter() - t0) / lreps
    print(f"# Monte-Carlo {count} loop: {loop_ms:.2f} ms", file=sys.stderr, flush=True)
    newton = [s.newton_iters for s in stats]
    return {"workload": f"{count} crossbars, m, n in {{64, ..., 512}}, seed {args.seed} "
                        f"({sum(c.geom.m * c.geom.n for c in cbs)} crosspoints), bf16x3 per-mode",
            "batched": {"ms_per_batch": round(ms, 3), "solves_per_s": round(count * 1e3 / ms, 1),
                        "status": B.status_string(status), "setup_ms": round(setup_ms, 1),
                        "solves_per_s_with_setup": round(count * 1e3 / (ms + setup_ms), 1),
                        "newton_iters": [min(newton), max(newton)],
                        "products_roofline": rf},
            "loop": {"ms_per_batch": round(loop_ms, 3),
                     "solves_per_s": round(count * 1e3 / loop_ms, 1),
                     "status": B.status_string(lstatus), "setup_ms": round(loop_setup_ms, 1),
                     "solves_per_s_with_setup": round(count * 1e3 / (loop_ms + loop_setup_ms), 1)},
            "speedup_of_batched": round(loop_ms / ms, 2),
            "speedup_of_batched_with_setup": round((loop_ms + loop_setup_ms) / (ms + setup_ms), 2)}


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}); this solver has no "
              "multi-GPU path", file=sys.stderr)
        sys.exit(2)
    if args.mc or args.batch:
        return bench_batched(args)
    import numpy as np
    import torch

    from paper_2109_07929_amd import Plan, synth
    from paper_2109_07929_amd import binding as B

    torch.cuda.init()
    dev = torch.device("cuda:0")
    m = n = args.size
    cb = synth.crossbar(m, n, seed=args.seed)
    g_dev = torch.from_numpy(cb.g_dev).to(dev)
    v_in = torch.from_numpy(cb.v_in).to(dev)

    t0 = time.perf_counter()
    plan = Plan(cb.geom, device=dev)
    setup_ms = 1e3 * (time.perf_counter() - t0)

    prec = {"fp64": B.MCA_PREC_FP64, "fp32": B.MCA_PREC_FP32, "bf16x3": B.MCA_PREC_BF16X3,
            "bf16": B.MCA_PREC_BF16}[args.precision]
    if args.precond is None:
        args.precond = "literal" if prec == B.MCA_PREC_FP64 else "permode"
    form = {"literal": B.MCA_PRECOND_LITERAL, "permode": B.MCA_PRECOND_PERMODE,
            "approx": B.MCA_PRECOND_APPROX, "jacobi": B.MCA_PRECOND_JACOBI,
            "none": B.MCA_PRECOND_NONE}[args.precond]
    # the timed solves carry only sampled events (every 4th preconditioner application);
    # the per-class breakdown comes from a separate pass with every group timed
    flags = 0 if args.no_timing else (B.MCA_FLAG_TIMING if args.full_timing
                                      else B.MCA_FLAG_TIMING_SAMPLED)
    if args.mgs_passes:
        flags |= B.MCA_FLAG_MGS_PASSES
    opts = B.options(precond=form, precision=prec, flags=flags)
    opts_full = B.options(precond=form, precision=prec,
                          flags=(flags & ~B.MCA_FLAG_TIMING_SAMPLED) | B.MCA_FLAG_TIMING)
    v_t = torch.zeros((m, n), dtype=torch.float64, device=dev)
    v_b = torch.zeros_like(v_t)
    ws = plan.workspace(opts)
    stream = torch.cuda.current_stream()

    def step(o=opts):
        return B.mca_solve(plan.handle, m, n, g_dev, v_in, v_t, v_b, o, ws, stream)[1]

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    print(f"# warmup done ({args.warmup} solves)", file=sys.stderr, flush=True)

    kms = np.zeros(B.MCA_NUM_KCLASS)
    klaunch = np.zeros(B.MCA_NUM_KCLASS, dtype=np.int64)
    newton, krylov = [], []
    torch.cuda.synchronize()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t_wall = time.perf_counter()
    ev0.record(stream)
    for _ in range(args.steps):
        st = step()
        st_last = st
        kms += np.array(st.kernel_ms[:])
        klaunch += np.array(st.kernel_launches[:])
        newton.append(st.newton_iters)
        krylov.append(st.krylov_iters)
    ev1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t_wall
    total_ms = ev0.elapsed_time(ev1)
    ms_per_step = total_ms / args.steps
    value = 1e3 / ms_per_step

    # per-class breakdown: a pass after the timed region with every group timed
    breakdown, kry_hbm = {}, None
    if not args.no_timing:
        nfull = 2
        fms = np.zeros(B.MCA_NUM_KCLASS)
        flaunch = np.zeros(B.MCA_NUM_KCLASS, dtype=np.int64)
        its_full = 0
        for _ in range(nfull):
            st_full = step(opts_full)
            its_full += st_full.krylov_iters
            fms += np.array(st_full.kernel_ms[:])
            flaunch += np.array(st_full.kernel_launches[:])
        torch.cuda.synchronize()
        names = ["gemm", "jacobian", "ortho", "residual"]
        breakdown["timed"] = f"{nfull} solves after the timed region, every kernel group timed"
        for c, nm in enumerate(names):
            breakdown[nm] = {"ms_per_solve": round(fms[c] / nfull, 4),
                             "launches_per_solve": int(flaunch[c] // nfull)}
        if fms[B.MCA_KCLASS_JACOBIAN] > 0:
            kry_hbm = krylov_hbm(st_full, m * n, opts_full, fms, nfull)
    # roofline of the dominant kernel: the FP64 eigenbasis GEMMs
    roofline = None
    if not args.no_timing and klaunch[B.MCA_KCLASS_GEMM] > 0 and form == B.MCA_PRECOND_APPROX:
        # two tridiagonal line-solve launches per application: columns read r_b and
        # write z_b (16 B per crosspoint), rows read r_t, z_b and write z_t (24 B)
        bytes_per_launch = 20.0 * m * n
        avg_ms = kms[B.MCA_KCLASS_GEMM] / klaunch[B.MCA_KCLASS_GEMM]
        achieved = bytes_per_launch / (avg_ms * 1e-3) / 1e9
        roofline = {"bound": "hbm", "kernel": "k_chunk_solve (tridiagonal line solves, chunked Thomas; "
                              "cyclic reduction past 2048 elements per line)",
                    "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                    "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None,
                    "avg_launch_us": round(avg_ms * 1e3, 2),
                    "bytes_per_launch": bytes_per_launch}
    elif not args.no_timing and klaunch[B.MCA_KCLASS_GEMM] > 0 and prec == B.MCA_PREC_FP64 and \
            form in (B.MCA_PRECOND_LITERAL, B.MCA_PRECOND_PERMODE):
        # unit: one preconditioner application = all its FP64 transform launches.
        # Literal form: Q_m side 2 n m^2 flops each way, Q_n side 2 m n^2 each way; with
        # a persymmetric G_bot (equal bottom terminations, m even) the Q_m side is two
        # half-size products (n m^2 each way) plus the unfold pass; the per-mode form
        # transforms both layers (twice the literal flops).
        g = cb.geom
        persym = (form == B.MCA_PRECOND_LITERAL and m % 2 == 0 and g.g_bot_end0 == g.g_bot_end1)
        # algorithmic flops (the method's unit): 4(m + n) per crosspoint for the literal
        # form (two transforms each way), 8(m + n) per mode for the per-mode form
        alg_app = (4.0 if form == B.MCA_PRECOND_LITERAL else 8.0) * (m + n) * m * n
        qm = (1.0 if persym else 2.0) * n * m * m
        flops_app = 2 * qm + 2 * (2.0 * m * n * n)
        # transform launches per application, from the pass with every group timed
        # (one application per GMRES iteration): 4 products, plus the unfold pass
        # when it is not fused into the last product
        launches_app = int(round(flaunch[B.MCA_KCLASS_GEMM] / max(its_full, 1)))
        if form == B.MCA_PRECOND_PERMODE:
            flops_app *= 2.0
        napps = klaunch[B.MCA_KCLASS_GEMM] / launches_app
        t_app_ms = kms[B.MCA_KCLASS_GEMM] / napps
        achieved = alg_app / (t_app_ms * 1e-3) / 1e12
        executed = flops_app / (t_app_ms * 1e-3) / 1e12
        traffic = gemm_traffic() if (m == 1024 and persym) else None
        roofline = {"bound": "mfma",
                    "kernel": "FP64 eigenbasis transforms of one preconditioner application "
                              "(k_gemm_tn_f64 launches" + (", the unfold fused or in k_unfold)" if persym else ")"),
                    "achieved": round(achieved, 3), "peak": FP64_MFMA_PEAK_TFLOPS,
                    "unit": "TFLOP/s", "frac": round(achieved / FP64_MFMA_PEAK_TFLOPS, 4),
                    "traffic": traffic,
                    "traffic_unit": "HBM bytes per application (rocprofv3 FETCH_SIZE x2 + "
                                    "WRITE_SIZE summed over its launches)",
                    "avg_application_us": round(t_app_ms * 1e3, 2),
                    "launches_per_application": launches_app,
                    "flops_per_application": alg_app,
                    "flops_unit": ("algorithmic: 4(m+n) per crosspoint for the literal form, "
                                   "8(m+n) for the per-mode form"),
                    "executed_flops_per_application": flops_app,
                    "executed_achieved": round(executed, 3),
                    "executed_frac": round(executed / FP64_MFMA_PEAK_TFLOPS, 4)}
    if roofline is not None:
        roofline["timed_groups"] = ("every 4th preconditioner application of the timed solves"
                                    if not args.full_timing else
                                    "every preconditioner application of the timed solves")

    kind = ("plain FP64 Newton-FGMRES(30)" if prec == B.MCA_PREC_FP64 else
            f"Newton-FGMRES(30) with a {args.precision} preconditioner")
    if form in (B.MCA_PRECOND_APPROX, B.MCA_PRECOND_JACOBI, B.MCA_PRECOND_NONE):
        kind = f"FP64 Newton-FGMRES(30), {args.precond} preconditioner"
    workload = f"{kind}, {m}x{n} crossbar ({2 * m * n} unknowns), seed {args.seed}"
    out = {
        "metric": "MCA solves/s at 1024x1024, 1e-8 rel residual: plain FP64 vs batched+warm+mixed",
        "value": round(value, 3),
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if prec == B.MCA_PREC_FP64 else f"f64 (preconditioner {args.precision})",
        "data": "synthetic",
        "config": {"workload": workload,
                   "precond": args.precond, "newton_tol": opts.newton_tol,
                   "gmres_tol": opts.gmres_tol, "setup_ms": round(setup_ms, 1),
                   "newton_iters": newton[-1], "krylov_iters": krylov[-1],
                   "wall_s": round(wall, 3)},
        "roofline": roofline,
        "krylov_hbm": kry_hbm,
        "kernel_breakdown": breakdown,
    }
    if not args.no_compare:
        cmp = compare_forms(args, dev)
        for f in cmp["forms"].values():
            f["speedup_vs_plain_fp64"] = (round(f["solves_per_s"] / value, 3)
                                          if f["status"] == "ok" else None)
        # the metric's "batched + warm + mixed" side is the learned warm start
        warm = cmp["forms"].get("cnn")
        cmp["warm_form"] = "cnn" if warm is not None else None
        cmp["speedup_vs_plain_fp64"] = warm["speedup_vs_plain_fp64"] if warm else None
        ok = {k: f for k, f in cmp["forms"].items() if f["status"] == "ok"}
        if ok:
            best = max(ok, key=lambda k: ok[k]["solves_per_s"])
            cmp["fastest_form"] = best
            cmp["fastest_speedup_vs_plain_fp64"] = ok[best]["speedup_vs_plain_fp64"]
        out["batched_warm_mixed"] = cmp
        del cmp
        torch.cuda.empty_cache()
    if not args.no_extra_configs and m == 1024:
        out["approx_preconditioner_1024"] = leg_approx(args, dev)
        torch.cuda.empty_cache()
        out["mixed_precision_2048"] = leg_mixed_2048(args, dev)
        torch.cuda.empty_cache()
        out["monte_carlo_256"] = leg_monte_carlo(args, dev)
        torch.cuda.empty_cache()
    # measured HBM ceiling: a 1 GiB device-to-device copy (read + write bytes / time);
    # not in counter runs, whose calibration copy is the only one
    if not args.copy_calib:
        hbm_copy(out, roofline, kry_hbm, ev0, ev1, stream, dev)
    if args.copy_calib:
        src = torch.rand(32 << 20, dtype=torch.float64, device=dev)   # 256 MiB
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        out["copy_calib_bytes"] = src.numel() * 8
    if not args.no_cpu_baseline:
        print("# cpu baseline (oracle) ...", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(cb)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
