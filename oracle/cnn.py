"""Plain FP64 reference of the warm-start network (test infrastructure only).

TEST INFRASTRUCTURE: only the test suite, the smoke check and the benchmark's
CPU baseline may import this module; the HIP library never uses it and the two
share no code.

The network predicts the crossbar's steady state from its inputs, to start
Newton's method (eq. (Newton3)) closer to the solution than V = 0.  It
corrects a mean-field guess: the paper's approximate preconditioner (eq.
(block) with M ~ Mhat) applied to the drive vector Y at a1 = a2 = mean(g_dev).
With Y_b = 0 that guess is V0_t[i, j] = v_in[i] phi[j], V0_b = 0, where
phi = g_src (G_top + a I)^{-1} e_0 is the decay profile along one top wire.
  * input channels per crosspoint (i, j):
        f0 = log10(g_dev[i, j]) + 5             (device conductance, ~[-1, 1])
        f1 = v_in[i] / 0.15 - 1                 (the row's drive, ~[-1, 1])
        f2 = (g_top - 0.5) / 0.3                (the wire conductance, ~[-1, 1])
        f3 = v_in[i] (1 - phi[j]) / 0.1         (the mean-field IR drop)
  * six 3x3 convolutions (cross-correlation, zero "same" padding), 32
    channels, ReLU after the first five, a linear last layer with 2 outputs;
  * outputs (y_t, y_b) parameterise the voltages as
        V_t = v_in[i] phi[j] - 0.01 y_t,    V_b = 0.01 y_b;
  * training loss: the mean of (y - y_target)^2 over crosspoints and both
    outputs; optimiser Adam (Kingma & Ba) with bias correction.

Everything here is written from those definitions with numpy primitives
(a matrix product per filter tap), no blocking or fusion.
"""

from __future__ import annotations

import numpy as np

CH = 32
LAYERS = [(4, CH, True), (CH, CH, True), (CH, CH, True), (CH, CH, True), (CH, CH, True),
          (CH, 2, False)]
V_SCALE = 0.01


def wire_profile(geom, g_dev):
    """phi = g_src (G_top + a I)^{-1} e_0 with a = mean(g_dev): the top wire
    matrix with terminations (eq. (G)), shifted as G1 of eq. (G1)."""
    n = geom.n
    a = float(np.mean(g_dev))
    T = np.zeros((n, n))
    for k in range(n - 1):                  # one segment between k and k + 1
        T[k, k] += geom.g_top
        T[k + 1, k + 1] += geom.g_top
        T[k, k + 1] -= geom.g_top
        T[k + 1, k] -= geom.g_top
    T[0, 0] += geom.g_src
    T[-1, -1] += geom.g_top_end
    rhs = np.zeros(n)
    rhs[0] = geom.g_src
    return np.linalg.solve(T + a * np.eye(n), rhs)


def features(geom, g_dev, v_in):
    """(m, n, 4) input channels of one crossbar."""
    g_dev = np.asarray(g_dev, dtype=np.float64)
    v_in = np.asarray(v_in, dtype=np.float64)
    m, n = g_dev.shape
    phi = wire_profile(geom, g_dev)
    f = np.empty((m, n, 4))
    f[..., 0] = np.log10(g_dev) + 5.0
    f[..., 1] = (v_in / 0.15 - 1.0)[:, None]
    f[..., 2] = (float(geom.g_top) - 0.5) / 0.3
    f[..., 3] = v_in[:, None] * (1.0 - phi[None, :]) / 0.1
    return f


def base_guess(geom, g_dev, v_in):
    """The mean-field guess (V0_t, V0_b)."""
    phi = wire_profile(geom, g_dev)
    v_in = np.asarray(v_in, dtype=np.float64)
    return v_in[:, None] * phi[None, :], np.zeros((geom.m, geom.n))


def targets(geom, g_dev, v_in, v_t, v_b):
    """(m, n, 2) training targets of a solved crossbar."""
    b_t, _ = base_guess(geom, g_dev, v_in)
    return np.stack([(b_t - v_t) / V_SCALE, np.asarray(v_b) / V_SCALE], axis=-1)


def voltages(geom, g_dev, v_in, y):
    """(V_t, V_b) from the network's outputs y (m, n, 2)."""
    b_t, _ = base_guess(geom, g_dev, v_in)
    return b_t - V_SCALE * y[..., 0], V_SCALE * y[..., 1]


def conv3x3(x, w, b):
    """out[i, j, o] = b[o] + sum_{dy, dx, c} x[i + dy, j + dx, c] w[dy + 1, dx + 1, c, o],
    with x = 0 outside the array.  x (m, n, Ci), w (3, 3, Ci, Co)."""
    m, n, _ = x.shape
    xp = np.pad(x, ((1, 1), (1, 1), (0, 0)))
    out = np.broadcast_to(b, (m, n, w.shape[3])).astype(np.float64).copy()
    for dy in range(3):
        for dx in range(3):
            out += xp[dy:dy + m, dx:dx + n, :] @ w[dy, dx]
    return out


def forward(params, x):
    """Activations [x, a1, ..., a5, y] of one crossbar's features x (m, n, 4)."""
    acts = [np.asarray(x, dtype=np.float64)]
    for (w, b), (_, _, relu) in zip(params, LAYERS):
        z = conv3x3(acts[-1], w, b)
        acts.append(np.maximum(z, 0.0) if relu else z)
    return acts


def loss(y, t):
    return float(np.mean((y - t) ** 2))


def backward(params, acts_list, t_list):
    """Gradients of the mean loss over a batch (lists of per-crossbar activations
    and targets); the mean runs over every crosspoint and output of the batch."""
    count = sum(t.size for t in t_list)
    grads = [(np.zeros_like(w), np.zeros_like(b)) for w, b in params]
    for acts, t in zip(acts_list, t_list):
        d = 2.0 * (acts[-1] - t) / count               # dL/dy
        for layer in range(len(params) - 1, -1, -1):
            w, _ = params[layer]
            x = acts[layer]
            m, n, _ = x.shape
            gw, gb = grads[layer]
            gb += d.sum(axis=(0, 1))
            xp = np.pad(x, ((1, 1), (1, 1), (0, 0)))
            dp = np.zeros_like(xp)
            for dy in range(3):
                for dx in range(3):
                    # out[i, j] used x[i + dy - 1, j + dx - 1]
                    gw[dy, dx] += xp[dy:dy + m, dx:dx + n, :].reshape(-1, x.shape[2]).T @ \
                        d.reshape(-1, d.shape[2])
                    dp[dy:dy + m, dx:dx + n, :] += d @ w[dy, dx].T
            dxin = dp[1:m + 1, 1:n + 1, :]
            if layer > 0:
                # ReLU of the previous layer: a = max(z, 0), da/dz = [a > 0]
                d = dxin * (x > 0.0)
    return grads


def adam_step(params, grads, m_state, v_state, step, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update (step counts from 1); returns new (params, m, v)."""
    out_p, out_m, out_v = [], [], []
    for (w, b), (gw, gb), (mw, mb), (vw, vb) in zip(params, grads, m_state, v_state):
        new = []
        for p, g, mm, vv in ((w, gw, mw, vw), (b, gb, mb, vb)):
            mm = beta1 * mm + (1 - beta1) * g
            vv = beta2 * vv + (1 - beta2) * g * g
            mh = mm / (1 - beta1 ** step)
            vh = vv / (1 - beta2 ** step)
            new.append((p - lr * mh / (np.sqrt(vh) + eps), mm, vv))
        out_p.append((new[0][0], new[1][0]))
        out_m.append((new[0][1], new[1][1]))
        out_v.append((new[0][2], new[1][2]))
    return out_p, out_m, out_v


def unpack(flat):
    """Per-layer (w, b) from the packed parameter vector: per layer w[dy][dx][ci][co]
    (row-major) then b[co], layers in order."""
    flat = np.asarray(flat, dtype=np.float64)
    params, off = [], 0
    for ci, co, _ in LAYERS:
        w = flat[off:off + 9 * ci * co].reshape(3, 3, ci, co)
        off += 9 * ci * co
        b = flat[off:off + co]
        off += co
        params.append((w, b))
    assert off == flat.size
    return params


def pack(params):
    return np.concatenate([np.concatenate([w.ravel(), b.ravel()]) for w, b in params])


def param_count():
    return sum(9 * ci * co + co for ci, co, _ in LAYERS)
