"""Learned warm start: training data from the batched solver, training of the
network with the library's kernels, and the warm-started solve.

    python -m paper_2109_07929_amd.warmstart train --count 20000 --size 512 --out W.npy
    python -m paper_2109_07929_amd.warmstart eval --params W.npy --count 1000 --size 512

Training crossbars have one size, Monte-Carlo device and drive distributions
and one of synth.WIRE_LEVELS wire conductances each; their steady states
come from mca_solve_batched.  The network (mca_cnn_*) is trained with Adam on
the mean squared error of its outputs against the solved voltages.  A
warm-started solve predicts V with mca_cnn_predict and hands it to the solver
as its initial guess with MCA_FLAG_GUESS_FALLBACK, so a guess whose residual is
no better than that of V = 0 is dropped and the answer always meets the same
tolerance.
"""

from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

from . import Batch, binding as B, synth

HERE = os.path.dirname(os.path.abspath(__file__))
DEFAULT_PARAMS = os.path.join(HERE, "warmstart_512.npy")
CHUNK = 112


def _say(*a):
    print(*a, file=sys.stderr, flush=True)


def level_batches(per_level, m, n, device="cuda"):
    """One Batch of `per_level` crossbars for every wire level (their host set-up
    runs in parallel threads; every batch is reused for many input draws)."""
    from concurrent.futures import ThreadPoolExecutor
    with ThreadPoolExecutor(max_workers=16) as ex:
        return list(ex.map(lambda k: Batch([synth.level_geometry(m, n, k)] * per_level,
                                           device=device), range(synth.WIRE_LEVELS)))


def solve_batch(bt, g_dev, v_in, opts, ws, guess=None):
    """Batched solve of bt's crossbars; returns (v_t, v_b, status, stats, seconds)
    with v_t, v_b shaped like g_dev (count, m, n)."""
    import torch
    vt = torch.zeros(g_dev.numel(), dtype=torch.float64, device=g_dev.device)
    vb = torch.zeros_like(vt)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    out = bt.solve(g_dev.reshape(-1), v_in.reshape(-1), opts, ws=ws,
                   guess=None if guess is None else (guess[0].reshape(-1), guess[1].reshape(-1)),
                   out=(vt, vb), check=False)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    return vt.view(g_dev.shape), vb.view(g_dev.shape), out[2], out[3], dt


def _split(count, chunk_max):
    """per-level sample count and chunk size: count spread over the levels in
    equal chunks of at most chunk_max."""
    per_level = -(-count // synth.WIRE_LEVELS)
    chunks = -(-per_level // chunk_max)
    chunk = -(-per_level // chunks)
    return chunk, chunks


def generate(count, size, seed, device="cuda", precision=B.MCA_PREC_BF16X3):
    """Training set of about `count` solved size x size crossbars (rounded up to
    equal chunks per wire level), kept on the GPU in float32: dict of g (N, m, n),
    v_in (N, m), vt, vb (N, m, n), and level (N,) the wire level (host int64)."""
    import torch
    m = n = size
    chunk, chunks = _split(count, CHUNK)
    total = chunk * chunks * synth.WIRE_LEVELS
    ds = {"g": torch.empty((total, m, n), dtype=torch.float32, device=device),
          "v_in": torch.empty((total, m), dtype=torch.float32, device=device),
          "level": torch.empty(total, dtype=torch.int64),
          "vt": torch.empty((total, m, n), dtype=torch.float32, device=device),
          "vb": torch.empty((total, m, n), dtype=torch.float32, device=device)}
    opts = B.options(precond=B.MCA_PRECOND_PERMODE, precision=precision)
    t0 = time.perf_counter()
    batches = level_batches(chunk, m, n, device)
    ws = torch.empty(B.mca_batch_workspace_bytes(batches[0].handle, opts), dtype=torch.uint8,
                     device=device)
    _say(f"# {synth.WIRE_LEVELS} level batches of {chunk} ready ({time.perf_counter() - t0:.1f} s)")
    done = 0
    for c in range(chunks):
        for lv, bt in enumerate(batches):
            g, v = synth.mc_device_batch(chunk, m, n, (seed * 1000 + c) * 1000 + lv, device=device)
            vt, vb, status, _, _ = solve_batch(bt, g, v, opts, ws)
            if status != B.MCA_OK:
                raise RuntimeError(f"training solve failed: {B.status_string(status)}")
            sl = slice(done, done + chunk)
            ds["g"][sl] = g.float()
            ds["v_in"][sl] = v.float()
            ds["level"][sl] = lv
            ds["vt"][sl] = vt.float()
            ds["vb"][sl] = vb.float()
            done += chunk
        _say(f"# generated {done}/{total} ({time.perf_counter() - t0:.1f} s)")
    del ws, batches
    return ds


def train(ds, epochs=4, batch=16, lr=1e-3, seed=0, log_every=200):
    """Adam on the mean squared error; cosine learning-rate decay.  Returns
    (params as a float32 device tensor, list of (step, loss))."""
    import torch
    count, m, n = ds["g"].shape
    npar = B.mca_cnn_param_count()
    dev = ds["g"].device
    params = torch.from_numpy(synth.cnn_init(seed)).to(dev)
    grad = torch.zeros(npar, dtype=torch.float32, device=dev)
    am, av = torch.zeros_like(grad), torch.zeros_like(grad)
    loss = torch.zeros(1, dtype=torch.float32, device=dev)
    ws = torch.empty(B.mca_cnn_workspace_bytes(batch, m, n), dtype=torch.uint8, device=dev)
    gen = torch.Generator(device="cpu")
    gen.manual_seed(seed)
    geom_of = [B.geometry_from(synth.level_geometry(m, n, k)) for k in range(synth.WIRE_LEVELS)]
    steps_per_epoch = count // batch
    total = epochs * steps_per_epoch
    hist = []
    step = 0
    t0 = time.perf_counter()
    for ep in range(epochs):
        perm = torch.randperm(count, generator=gen).to(dev)
        for k in range(steps_per_epoch):
            idx = perm[k * batch:(k + 1) * batch]
            step += 1
            rate = 1e-5 + 0.5 * (lr - 1e-5) * (1 + math.cos(math.pi * (step - 1) / total))
            geoms = [geom_of[int(lv)] for lv in ds["level"][idx.cpu()].tolist()]
            B.mca_cnn_gradient(params, geoms, ds["g"][idx].double().contiguous(),
                               ds["v_in"][idx].double().contiguous(),
                               ds["vt"][idx].double().contiguous(),
                               ds["vb"][idx].double().contiguous(), grad, loss, ws)
            B.mca_cnn_adam(params, grad, am, av, step, rate)
            if step % log_every == 0 or step == total:
                hist.append((step, float(loss)))
                _say(f"# step {step}/{total} loss {hist[-1][1]:.4e} "
                     f"({time.perf_counter() - t0:.1f} s)")
    return params, hist


def predict(params, geoms, g_dev, v_in, ws=None):
    """(v_t, v_b) predicted for a batch of crossbars of one size (device tensors);
    geoms: one geometry per crossbar."""
    import torch
    count, m, n = g_dev.shape
    if ws is None:
        ws = torch.empty(B.mca_cnn_workspace_bytes(count, m, n), dtype=torch.uint8,
                         device=g_dev.device)
    vt = torch.empty((count, m, n), dtype=torch.float64, device=g_dev.device)
    vb = torch.empty_like(vt)
    B.mca_cnn_predict(params, geoms, g_dev.contiguous(), v_in.contiguous(), vt, vb, ws)
    return vt, vb


def describe_params(path=DEFAULT_PARAMS):
    """What a stored network was trained on: the JSON file beside its weights
    (same name, .json), written by `train`."""
    meta = os.path.splitext(path)[0] + ".json"
    try:
        with open(meta) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {"weights": os.path.basename(path), "trained_on": "unknown"}


def load_params(path=DEFAULT_PARAMS, device="cuda"):
    import torch
    flat = np.load(path, allow_pickle=False).astype(np.float32)
    if flat.size != B.mca_cnn_param_count():
        raise ValueError(f"{path}: {flat.size} parameters, the network has "
                         f"{B.mca_cnn_param_count()}")
    return torch.from_numpy(flat).to(device)


def evaluate(params, count, size, seed, device="cuda", precision=B.MCA_PREC_BF16X3,
             newton_tol=1e-10, keep=0):
    """Solve held-out crossbars from V = 0 and from the network's guess (with
    fallback) to the same Newton tolerance; returns per-crossbar Newton / GMRES
    counts, guess residuals and the wall time of both, prediction included.
    keep > 0 also returns the first `keep` crossbars (wire level after wire
    level) as host arrays (res["kept"]: geometry, g_dev, v_in, warm-started
    v_t, v_b)."""
    import torch
    m = n = size
    per_level = -(-count // synth.WIRE_LEVELS)
    batches = level_batches(per_level, m, n, device)
    cold = B.options(precond=B.MCA_PRECOND_PERMODE, precision=precision, newton_tol=newton_tol)
    warm = B.options(precond=B.MCA_PRECOND_PERMODE, precision=precision, newton_tol=newton_tol,
                     flags=B.MCA_FLAG_INITIAL_GUESS | B.MCA_FLAG_GUESS_FALLBACK)
    ws = torch.empty(B.mca_batch_workspace_bytes(batches[0].handle, cold), dtype=torch.uint8,
                     device=device)
    cws = torch.empty(B.mca_cnn_workspace_bytes(per_level, m, n), dtype=torch.uint8, device=device)
    res = {"newton_cold": [], "newton_warm": [], "krylov_cold": [], "krylov_warm": [],
           "guess_residual": [], "guess_used": [], "max_dv": [], "relres_warm": [],
           "t_cold": 0.0, "t_warm": 0.0, "t_predict": 0.0, "kept": []}
    for lv, bt in enumerate(batches):
        g, v = synth.mc_device_batch(per_level, m, n, seed * 1000 + lv, device=device)
        geoms = [synth.level_geometry(m, n, lv)] * per_level
        vt0, vb0, s0, st0, dt0 = solve_batch(bt, g, v, cold, ws)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        pt, pb = predict(params, geoms, g, v, cws)
        torch.cuda.synchronize()
        res["t_predict"] += time.perf_counter() - t0
        vt1, vb1, s1, st1, dt1 = solve_batch(bt, g, v, warm, ws, guess=(pt, pb))
        if s0 != B.MCA_OK or s1 != B.MCA_OK:
            raise RuntimeError("evaluation solve failed")
        res["t_cold"] += dt0
        res["t_warm"] += dt1
        for a, b in zip(st0, st1):
            res["newton_cold"].append(a.newton_iters)
            res["newton_warm"].append(b.newton_iters)
            res["krylov_cold"].append(a.krylov_iters)
            res["krylov_warm"].append(b.krylov_iters)
            res["guess_residual"].append(b.residual_history[0] if b.start else float("nan"))
            res["guess_used"].append(b.start)
            res["relres_warm"].append(b.rel_residual)
        for b in range(min(keep - len(res["kept"]), per_level)):
            res["kept"].append((geoms[b], g[b].cpu().numpy(), v[b].cpu().numpy(),
                                vt1[b].cpu().numpy(), vb1[b].cpu().numpy()))
        scale = torch.maximum(vt0.abs().amax(dim=(1, 2)), vb0.abs().amax(dim=(1, 2)))
        dv = torch.maximum((vt1 - vt0).abs().amax(dim=(1, 2)), (vb1 - vb0).abs().amax(dim=(1, 2)))
        res["max_dv"] += (dv / scale).tolist()
    res["t_warm_total"] = res["t_warm"] + res["t_predict"]
    return res


def summary(res):
    nc, nw = np.mean(res["newton_cold"]), np.mean(res["newton_warm"])
    kc, kw = np.mean(res["krylov_cold"]), np.mean(res["krylov_warm"])
    used = np.array(res["guess_used"], dtype=bool)
    gr = np.array(res["guess_residual"])[used]
    return {"crossbars": len(res["newton_cold"]),
            "newton_cold": round(float(nc), 3), "newton_warm": round(float(nw), 3),
            "krylov_cold": round(float(kc), 3), "krylov_warm": round(float(kw), 3),
            "guess_used_fraction": round(float(used.mean()), 4),
            "guess_residual_median": float(np.median(gr)) if gr.size else None,
            "max_rel_dv_warm_vs_cold": float(np.max(res["max_dv"])),
            "max_relres_warm": float(np.max(res["relres_warm"])),
            "t_cold_s": round(res["t_cold"], 4), "t_warm_s": round(res["t_warm_total"], 4),
            "t_predict_s": round(res["t_predict"], 4),
            "speedup": round(res["t_cold"] / res["t_warm_total"], 3)}


def main(argv=None):
    p = argparse.ArgumentParser()
    sub = p.add_subparsers(dest="cmd", required=True)
    t = sub.add_parser("train")
    t.add_argument("--count", type=int, default=20000)
    t.add_argument("--size", type=int, default=512)
    t.add_argument("--seed", type=int, default=1)
    t.add_argument("--epochs", type=int, default=4)
    t.add_argument("--batch", type=int, default=16)
    t.add_argument("--lr", type=float, default=1e-3)
    t.add_argument("--out", required=True)
    t.add_argument("--eval-count", type=int, default=1000)
    e = sub.add_parser("eval")
    e.add_argument("--params", default=DEFAULT_PARAMS)
    e.add_argument("--count", type=int, default=1000)
    e.add_argument("--size", type=int, default=512)
    e.add_argument("--seed", type=int, default=999)
    a = p.parse_args(argv)
    import torch
    torch.cuda.init()
    if a.cmd == "train":
        t0 = time.perf_counter()
        ds = generate(a.count, a.size, a.seed)
        t_gen = time.perf_counter() - t0
        params, hist = train(ds, epochs=a.epochs, batch=a.batch, lr=a.lr, seed=a.seed)
        torch.cuda.synchronize()
        t_train = time.perf_counter() - t0 - t_gen
        np.save(a.out, params.cpu().numpy())
        with open(os.path.splitext(a.out)[0] + ".json", "w") as f:
            json.dump({"weights": os.path.basename(a.out),
                       "trained_on": f"{a.count} solved {a.size} x {a.size} crossbars with the "
                                     "Monte-Carlo distributions (synth.mc_device_batch, wire "
                                     "conductance from synth.WIRE_LEVELS levels)",
                       "size": a.size, "count": a.count, "epochs": a.epochs, "batch": a.batch,
                       "lr": a.lr, "seed": a.seed}, f)
        del ds
        out = {"train": {"count": a.count, "size": a.size, "epochs": a.epochs, "batch": a.batch,
                         "lr": a.lr, "seed": a.seed, "generate_s": round(t_gen, 1),
                         "train_s": round(t_train, 1), "loss": hist}}
        if a.eval_count:
            # held-out crossbars: a seed the training chunks never use
            out["eval"] = summary(evaluate(params, a.eval_count, a.size, seed=10 ** 9 + a.seed))
        print(json.dumps(out), flush=True)
    else:
        params = load_params(a.params)
        print(json.dumps(summary(evaluate(params, a.count, a.size, a.seed))), flush=True)


if __name__ == "__main__":
    main()
