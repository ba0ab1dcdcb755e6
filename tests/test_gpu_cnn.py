"""Parity of the warm-start network's HIP kernels (mca_cnn_*) with the FP64
reference of oracle/cnn.py.

The GPU keeps weights and activations in bfloat16 (FP32 accumulation), so the
bar is relative: the reference runs with the same bf16-rounded weights, and
outputs / gradients must agree to a few bf16 roundings per layer, measured as
relative L2 error per tensor.
"""

import numpy as np
import pytest
import torch

from oracle import cnn
from paper_2109_07929_amd import binding as B
from paper_2109_07929_amd import synth

pytestmark = pytest.mark.gpu

SIZES = [(1, 1, 1), (1, 5, 3), (2, 13, 70), (2, 24, 130), (1, 9, 64)]


def say(*a):
    print(*a, flush=True)


def bf16(x):
    return torch.as_tensor(x, dtype=torch.float32).to(torch.bfloat16).to(torch.float64).numpy()


def case(batch, m, n, seed):
    rng = np.random.default_rng(seed)
    flat = synth.cnn_init(seed)
    # nonzero biases so that the bias paths are exercised
    params = cnn.unpack(flat.astype(np.float64))
    off = 0
    for (w, b) in params:
        off += w.size
        flat[off:off + b.size] = rng.standard_normal(b.size) * 0.05
        off += b.size
    g = 10 ** rng.uniform(-6, -4, (batch, m, n))
    v_in = rng.uniform(0, 0.3, (batch, m))
    geoms = []
    for w in rng.uniform(0.2, 0.8, batch):
        geoms.append(synth.Geometry(m, n, g_top=w, g_bot=w, g_src=w))
    vt = v_in[:, :, None] - 0.05 * rng.random((batch, m, n))
    vb = 0.02 * rng.random((batch, m, n))
    return flat, g, v_in, geoms, vt, vb


def ref_params(flat):
    """The reference network with the GPU's bf16 weights (biases stay FP32)."""
    return [(bf16(w), b.astype(np.float32).astype(np.float64)) for w, b in cnn.unpack(flat)]


def forward_stored_bf16(P, x):
    """The reference forward pass with every stored activation rounded to bfloat16,
    as the GPU stores them, so that both sides take each ReLU decision on the
    same values."""
    acts = [x]
    for (w, b), (_, _, relu) in zip(P, cnn.LAYERS):
        z = cnn.conv3x3(acts[-1], w, b)
        acts.append(bf16(np.maximum(z, 0.0)) if relu else z)
    return acts


def cuda(a, dtype=torch.float64):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=dtype).cuda()


def rel(a, b):
    return float(np.linalg.norm(np.ravel(a) - np.ravel(b)) / max(np.linalg.norm(np.ravel(b)), 1e-30))


@pytest.mark.parametrize("batch,m,n", SIZES)
def test_cnn_predict_parity(batch, m, n):
    say(f"cnn predict {batch}x{m}x{n}")
    flat, g, v_in, geoms, _, _ = case(batch, m, n, seed=m + n)
    ws = torch.empty(B.mca_cnn_workspace_bytes(batch, m, n), dtype=torch.uint8, device="cuda")
    vt = torch.zeros(batch * m * n, dtype=torch.float64, device="cuda")
    vb = torch.zeros_like(vt)
    B.mca_cnn_predict(cuda(flat, torch.float32), geoms, cuda(g), cuda(v_in), vt, vb, ws)
    torch.cuda.synchronize()
    gvt, gvb = vt.cpu().numpy().reshape(batch, m, n), vb.cpu().numpy().reshape(batch, m, n)
    P = ref_params(flat)
    for b in range(batch):
        y = cnn.forward(P, bf16(cnn.features(geoms[b], g[b], v_in[b])))[-1]
        # the network outputs y recovered from the GPU's voltages
        gy = cnn.targets(geoms[b], g[b], v_in[b], gvt[b], gvb[b])
        ey = rel(gy, y)
        say(f"  sample {b}: rel err of y {ey:.2e}")
        assert ey <= 2e-2


@pytest.mark.parametrize("batch,m,n", SIZES)
def test_cnn_gradient_parity(batch, m, n):
    say(f"cnn gradient {batch}x{m}x{n}")
    flat, g, v_in, geoms, vt, vb = case(batch, m, n, seed=3 * m + n)
    npar = B.mca_cnn_param_count()
    assert npar == cnn.param_count()
    ws = torch.empty(B.mca_cnn_workspace_bytes(batch, m, n), dtype=torch.uint8, device="cuda")
    grad = torch.zeros(npar, dtype=torch.float32, device="cuda")
    loss = torch.zeros(1, dtype=torch.float32, device="cuda")
    B.mca_cnn_gradient(cuda(flat, torch.float32), geoms, cuda(g), cuda(v_in), cuda(vt), cuda(vb),
                       grad, loss, ws)
    torch.cuda.synchronize()
    P = ref_params(flat)
    # the GPU's input channels are bfloat16 too
    acts = [forward_stored_bf16(P, bf16(cnn.features(geoms[b], g[b], v_in[b])))
            for b in range(batch)]
    ts = [cnn.targets(geoms[b], g[b], v_in[b], vt[b], vb[b]) for b in range(batch)]
    ref_loss = sum(((a[-1] - t) ** 2).sum() for a, t in zip(acts, ts)) / sum(t.size for t in ts)
    grads = cnn.backward(P, acts, ts)
    gg = cnn.unpack(grad.cpu().numpy().astype(np.float64))
    say(f"  loss gpu {float(loss):.6e} ref {ref_loss:.6e}")
    assert abs(float(loss) - ref_loss) <= 1e-2 * ref_loss
    errs = []
    for l, ((gw, gb), (rw, rb)) in enumerate(zip(gg, grads)):
        ew, eb = rel(gw, rw), rel(gb, rb)
        say(f"  layer {l}: rel err dW {ew:.2e} db {eb:.2e}")
        errs.append(max(ew, eb))
    assert max(errs) <= 5e-2


def test_cnn_adam_parity():
    npar = B.mca_cnn_param_count()
    rng = np.random.default_rng(0)
    p = synth.cnn_init(1)
    g = rng.standard_normal(npar).astype(np.float32) * 1e-3
    m = rng.standard_normal(npar).astype(np.float32) * 1e-3
    v = (rng.random(npar).astype(np.float32) * 1e-6)
    tp, tg, tm, tv = (cuda(x, torch.float32) for x in (p, g, m, v))
    B.mca_cnn_adam(tp, tg, tm, tv, 3, 1e-3)
    torch.cuda.synchronize()
    rp, rm, rv = cnn.adam_step(cnn.unpack(p.astype(np.float64)), cnn.unpack(g.astype(np.float64)),
                               cnn.unpack(m.astype(np.float64)), cnn.unpack(v.astype(np.float64)),
                               step=3, lr=1e-3)
    np.testing.assert_allclose(tp.cpu().numpy(), cnn.pack(rp), rtol=1e-5, atol=1e-7)
    np.testing.assert_allclose(tm.cpu().numpy(), cnn.pack(rm), rtol=1e-5, atol=1e-9)
    np.testing.assert_allclose(tv.cpu().numpy(), cnn.pack(rv), rtol=1e-5, atol=1e-12)


def test_cnn_training_steps_reduce_the_loss():
    batch, m, n = 2, 32, 32
    flat, g, v_in, geoms, vt, vb = case(batch, m, n, seed=5)
    npar = B.mca_cnn_param_count()
    ws = torch.empty(B.mca_cnn_workspace_bytes(batch, m, n), dtype=torch.uint8, device="cuda")
    params = cuda(flat, torch.float32)
    grad = torch.zeros(npar, dtype=torch.float32, device="cuda")
    am, av = torch.zeros_like(grad), torch.zeros_like(grad)
    loss = torch.zeros(1, dtype=torch.float32, device="cuda")
    args = (cuda(g), cuda(v_in), cuda(vt), cuda(vb))
    losses = []
    for step in range(1, 41):
        B.mca_cnn_gradient(params, geoms, *args, grad, loss, ws)
        losses.append(float(loss))
        B.mca_cnn_adam(params, grad, am, av, step, 3e-3)
    say(f"  loss {losses[0]:.3e} -> {losses[-1]:.3e}")
    assert losses[-1] < 0.5 * losses[0]


def test_cnn_errors():
    assert B.mca_cnn_workspace_bytes(0, 4, 4) == 0
    ws = torch.empty(256, dtype=torch.uint8, device="cuda")
    t = torch.zeros(16, dtype=torch.float64, device="cuda")
    params = torch.zeros(B.mca_cnn_param_count(), device="cuda")
    with pytest.raises(B.MCAError) as e:
        B.mca_cnn_predict(params, [synth.Geometry(4, 4)], t, t[:4].contiguous(), t.clone(),
                          t.clone(), ws)
    assert e.value.status == B.MCA_ERR_WORKSPACE
    with pytest.raises(B.MCAError) as e:       # sizes differ within the batch
        B.mca_cnn_predict(params, [synth.Geometry(4, 4), synth.Geometry(2, 8)], t.repeat(2),
                          t[:8].contiguous(), t.repeat(2), t.repeat(2), ws)
    assert e.value.status == B.MCA_ERR_INVALID_ARG
