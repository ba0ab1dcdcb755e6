"""Pins of the warm-start network's FP64 reference (oracle/cnn.py).

* the 3x3 convolution against scipy's 2-D cross-correlation with zero fill;
* every gradient against central finite differences of the loss;
* Adam's first step against its closed form (each weight moves by lr * sign(g));
* the voltage parameterisation round trip.
"""

import numpy as np
import pytest
from scipy.signal import correlate2d

from oracle import cnn
from paper_2109_07929_amd import synth


def test_conv_matches_scipy_correlate():
    rng = np.random.default_rng(0)
    x = rng.standard_normal((7, 5, 3))
    w = rng.standard_normal((3, 3, 3, 4))
    b = rng.standard_normal(4)
    out = cnn.conv3x3(x, w, b)
    for o in range(4):
        ref = b[o] + sum(correlate2d(x[..., c], w[..., c, o], mode="same", boundary="fill")
                         for c in range(3))
        np.testing.assert_allclose(out[..., o], ref, rtol=1e-13, atol=1e-13)


def test_conv_padding_and_orientation():
    """A delta input at (0, 0) with a single nonzero tap w[2, 2] (offset +1, +1)
    reaches out[-1, -1] only; the corner taps that leave the array contribute 0."""
    x = np.zeros((4, 4, 1))
    x[0, 0, 0] = 1.0
    w = np.zeros((3, 3, 1, 1))
    w[0, 0, 0, 0] = 2.0            # out[i, j] += 2 x[i - 1, j - 1]
    out = cnn.conv3x3(x, w, np.zeros(1))
    expect = np.zeros((4, 4))
    expect[1, 1] = 2.0
    np.testing.assert_array_equal(out[..., 0], expect)


def _small_net(seed):
    flat = synth.cnn_init(seed).astype(np.float64)
    params = cnn.unpack(flat)
    # biases nonzero so that every term of the gradient is exercised
    rng = np.random.default_rng(seed + 1)
    return [(w, rng.standard_normal(b.shape) * 0.05) for w, b in params]


def test_param_packing():
    assert cnn.param_count() == 4 * 9 * 32 + 32 + 4 * (32 * 9 * 32 + 32) + 32 * 9 * 2 + 2
    flat = synth.cnn_init(3)
    assert flat.size == cnn.param_count()
    np.testing.assert_array_equal(cnn.pack(cnn.unpack(flat)), flat.astype(np.float64))


def test_gradients_match_finite_differences():
    rng = np.random.default_rng(7)
    params = _small_net(0)
    xs, ts = [], []
    for shape in ((5, 4), (3, 6)):
        g = 10 ** rng.uniform(-6, -4, shape)
        w = rng.uniform(0.2, 0.8)
        geom = synth.Geometry(shape[0], shape[1], g_top=w, g_bot=w, g_src=w)
        xs.append(cnn.features(geom, g, rng.uniform(0, 0.3, shape[0])))
        ts.append(rng.standard_normal(shape + (2,)))

    def total_loss(ps):
        ys = [cnn.forward(ps, x)[-1] for x in xs]
        count = sum(t.size for t in ts)
        return sum(((y - t) ** 2).sum() for y, t in zip(ys, ts)) / count

    grads = cnn.backward(params, [cnn.forward(params, x) for x in xs], ts)
    h = 1e-6
    for layer in range(len(params)):
        for which in (0, 1):
            arr = params[layer][which]
            flat_idx = rng.choice(arr.size, size=min(6, arr.size), replace=False)
            for q in flat_idx:
                idx = np.unravel_index(q, arr.shape)
                saved = arr[idx]
                arr[idx] = saved + h
                lp = total_loss(params)
                arr[idx] = saved - h
                lm = total_loss(params)
                arr[idx] = saved
                fd = (lp - lm) / (2 * h)
                an = grads[layer][which][idx]
                assert abs(fd - an) <= 1e-6 * max(1.0, abs(fd)) + 1e-8, (layer, which, idx, fd, an)


def test_adam_first_step_is_lr_times_sign():
    params = _small_net(1)
    rng = np.random.default_rng(2)
    grads = [(rng.standard_normal(w.shape), rng.standard_normal(b.shape)) for w, b in params]
    zeros = [(np.zeros_like(w), np.zeros_like(b)) for w, b in params]
    new, m, v = cnn.adam_step(params, grads, zeros, zeros, step=1, lr=1e-3, eps=0.0)
    for (w, b), (nw, nb), (gw, gb) in zip(params, new, grads):
        np.testing.assert_allclose(w - nw, 1e-3 * np.sign(gw), rtol=1e-12)
        np.testing.assert_allclose(b - nb, 1e-3 * np.sign(gb), rtol=1e-12)
    # second step with the same gradient: the bias-corrected moments are still g, g^2
    new2, _, _ = cnn.adam_step(new, grads, m, v, step=2, lr=1e-3, eps=0.0)
    for (w, _), (nw, _), (gw, _) in zip(new, new2, grads):
        np.testing.assert_allclose(w - nw, 1e-3 * np.sign(gw), rtol=1e-9)


def test_voltage_parameterisation_round_trip():
    rng = np.random.default_rng(3)
    geom = synth.Geometry(4, 5)
    g = 10 ** rng.uniform(-6, -4, (4, 5))
    v_in = rng.uniform(0, 0.3, 4)
    vt, vb = rng.uniform(0, 0.3, (4, 5)), rng.uniform(0, 0.05, (4, 5))
    rt, rb = cnn.voltages(geom, g, v_in, cnn.targets(geom, g, v_in, vt, vb))
    np.testing.assert_allclose(rt, vt, atol=1e-15)
    np.testing.assert_allclose(rb, vb, atol=1e-15)


def test_features_definition():
    geom = synth.Geometry(1, 2, g_top=0.8, g_bot=0.8, g_src=0.8)
    f = cnn.features(geom, np.array([[1e-6, 1e-4]]), np.array([0.3]))
    np.testing.assert_allclose(f[0, :, 0], [-1.0, 1.0])
    np.testing.assert_allclose(f[0, :, 1], [1.0, 1.0])
    np.testing.assert_allclose(f[0, :, 2], [1.0, 1.0])


@pytest.mark.parametrize("m,n", [(3, 5), (6, 4), (1, 7)])
def test_mean_field_guess_is_the_approximate_preconditioner_applied_to_Y(m, n):
    """V0 = v_in[i] phi[j] equals the oracle's approximate preconditioner (eq.
    (block) with Mhat, the paper's order) applied to Y at a1 = a2 = mean(g_dev)."""
    import oracle
    rng = np.random.default_rng(m * n)
    geom = synth.Geometry(m, n, g_top=0.5, g_bot=0.5, g_src=0.5)
    g = 10 ** rng.uniform(-6, -4, (m, n))
    v_in = rng.uniform(0, 0.3, m)
    a = float(np.mean(g))
    yt = np.zeros((m, n))
    yt[:, 0] = geom.g_src * v_in
    zt, zb = oracle.precond_apply_approx(geom, a, a, yt, np.zeros((m, n)))
    bt, bb = cnn.base_guess(geom, g, v_in)
    # the literal order divides by a: its rounding sets the tolerance
    np.testing.assert_allclose(bt, zt, rtol=0, atol=1e-9 * np.abs(zt).max())
    np.testing.assert_allclose(bb, zb, rtol=0, atol=1e-9 * np.abs(zt).max())
