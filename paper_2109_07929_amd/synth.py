"""Seeded synthetic crossbar inputs.

This module only draws numbers. It holds none of the solver's arithmetic, so
both the HIP path and the CPU oracle can take their inputs from it without
sharing any of the method.

The paper's own workload (RRAM devices with random internal state, wire
conductance normalised to 1; Section IV) is not available, so the crossbars
below stand in for it. One crossbar is described by

* a geometry: sizes m x n, the segment conductance of each uniform wire layer
  (Section II: both layers are uniform grids, one conductance per layer), the
  source conductance that ties each drive to node (i, 0) of the top layer,
  the terminations at the other wire ends, and the device voltage scale v0;
* ``g_dev``: one device conductance per crosspoint, m x n row-major float64;
* ``v_in``: one drive voltage per top-layer row, length m float64.

Draw order is fixed so that a seed names one input on every machine: numpy
PCG64 (``default_rng(seed)``), then ``g_dev`` row-major, then ``v_in``.
"""

from __future__ import annotations

import dataclasses
import math

import numpy as np

DEVICE_SINH = 0     # I = g * v0 * sinh(u / v0)
DEVICE_LINEAR = 1   # I = g * u


@dataclasses.dataclass(frozen=True)
class Geometry:
    m: int                      # rows: top-layer wires (one drive each)
    n: int                      # columns: bottom-layer wires
    g_top: float = 0.4          # top-layer segment conductance [S]
    g_bot: float = 0.4          # bottom-layer segment conductance [S]
    g_src: float = 0.4          # drive source -> node (i, 0) [S]
    g_top_end: float = 1e-3     # node (i, n-1) -> ground [S]   (1 kOhm)
    g_bot_end0: float = 0.1     # node (0, j)   -> ground [S]   (10 Ohm)
    g_bot_end1: float = 0.1     # node (m-1, j) -> ground [S]   (10 Ohm)
    v0: float = 0.25            # device voltage scale [V]
    device: int = DEVICE_SINH

    def with_(self, **kw) -> "Geometry":
        return dataclasses.replace(self, **kw)


@dataclasses.dataclass
class Crossbar:
    geom: Geometry
    g_dev: np.ndarray   # (m, n) float64
    v_in: np.ndarray    # (m,) float64
    seed: int


def crossbar(m: int, n: int, seed: int = 0, *, g_lo: float = 1e-6,
             g_hi: float = 1e-4, v_hi: float = 0.3, **geom_kw) -> Crossbar:
    """One crossbar with the standard distributions.

    Device conductances are log-uniform in [g_lo, g_hi] S, drives uniform in
    [0, v_hi] V; wires are 0.4 S per segment, the top rows end in 1 kOhm to
    ground and both ends of every bottom column go to ground through 10 Ohm.
    """
    rng = np.random.default_rng(seed)
    g_dev = np.exp(rng.uniform(math.log(g_lo), math.log(g_hi), size=(m, n)))
    v_in = rng.uniform(0.0, v_hi, size=m)
    return Crossbar(Geometry(m, n, **geom_kw), np.ascontiguousarray(g_dev),
                    np.ascontiguousarray(v_in), seed)


def uniform_crossbar(m: int, n: int, g: float, seed: int = 0, *,
                     v_hi: float = 0.3, **geom_kw) -> Crossbar:
    """All devices share one conductance ``g``; drives as in :func:`crossbar`."""
    rng = np.random.default_rng(seed)
    v_in = rng.uniform(0.0, v_hi, size=m)
    return Crossbar(Geometry(m, n, **geom_kw), np.full((m, n), float(g)),
                    np.ascontiguousarray(v_in), seed)


def vector(m: int, n: int, seed: int, scale: float = 1.0) -> tuple[np.ndarray, np.ndarray]:
    """A pair of m x n standard-normal arrays (top, bottom), e.g. a Krylov vector."""
    rng = np.random.default_rng(seed)
    return (scale * rng.standard_normal((m, n)),
            scale * rng.standard_normal((m, n)))


def voltages(m: int, n: int, seed: int, v_hi: float = 0.3) -> tuple[np.ndarray, np.ndarray]:
    """A pair of m x n node-voltage arrays uniform in [0, v_hi] V (a Newton iterate)."""
    rng = np.random.default_rng(seed)
    return (rng.uniform(0.0, v_hi, size=(m, n)),
            rng.uniform(0.0, 0.5 * v_hi, size=(m, n)))


# Monte-Carlo batch: sizes drawn from {64, 128, ..., 512}, 16-level programmed
# weights mapped log-linearly to [1e-6, 1e-4] S, lognormal device variation
# (sigma 0.3), one wire conductance per instance in [0.2, 0.8] S shared by both
# layers and by the drive source.
def mc_batch(count: int, seed: int = 0, sizes=tuple(range(64, 513, 64)),
             sigma: float = 0.3) -> list[Crossbar]:
    rng = np.random.default_rng(seed)
    out = []
    for k in range(count):
        m = int(rng.choice(sizes))
        n = int(rng.choice(sizes))
        gw = float(rng.uniform(0.2, 0.8))
        q = rng.integers(0, 16, size=(m, n))
        g_dev = 1e-6 * 100.0 ** (q / 15.0) * np.exp(sigma * rng.standard_normal((m, n)))
        v_in = rng.uniform(0.0, 0.3, size=m)
        geom = Geometry(m, n, g_top=gw, g_bot=gw, g_src=gw)
        out.append(Crossbar(geom, np.ascontiguousarray(g_dev), v_in, seed * 100003 + k))
    return out


# ------------------------------------------------------- warm-start network
CNN_LAYERS = [(4, 32), (32, 32), (32, 32), (32, 32), (32, 32), (32, 2)]


def cnn_init(seed: int = 0) -> np.ndarray:
    """Packed initial parameters of the warm-start network (float32): per layer
    w[dy][dx][ci][co] ~ N(0, 2 / (9 ci)) (He), then b[co] = 0; the last layer's
    weights are scaled by 0.1."""
    rng = np.random.default_rng(seed)
    out = []
    for k, (ci, co) in enumerate(CNN_LAYERS):
        std = np.sqrt(2.0 / (9 * ci)) * (0.1 if k == len(CNN_LAYERS) - 1 else 1.0)
        out.append(rng.standard_normal(9 * ci * co) * std)
        out.append(np.zeros(co))
    return np.concatenate(out).astype(np.float32)


# ------------------------------------------ warm-start training / evaluation
# Crossbars of one size with the Monte-Carlo distributions above (16-level
# weights with lognormal variation, drives U[0, 0.3]), drawn on the GPU with
# torch's seeded generator so that tens of thousands of 512 x 512 crossbars
# need no host work.  The wire conductance takes one of WIRE_LEVELS values
# spread evenly over [0.2, 0.8] S (equal shares), so that the crossbars of
# one level share a geometry and the solver's set-up for it.
WIRE_LEVELS = 64


def wire_level(k: int) -> float:
    return 0.2 + 0.6 * (k + 0.5) / WIRE_LEVELS


def level_geometry(m: int, n: int, k: int) -> Geometry:
    gw = wire_level(k)
    return Geometry(m, n, g_top=gw, g_bot=gw, g_src=gw)


def mc_device_batch(count: int, m: int, n: int, seed: int, device="cuda", sigma: float = 0.3):
    """(g_dev (count, m, n), v_in (count, m)) as float64 device tensors; draw
    order: weight levels, variation, drives."""
    import torch
    gen = torch.Generator(device=device)
    gen.manual_seed(int(seed))
    q = torch.randint(0, 16, (count, m, n), generator=gen, device=device).to(torch.float64)
    z = torch.randn((count, m, n), generator=gen, device=device, dtype=torch.float64)
    g_dev = 1e-6 * torch.pow(100.0, q / 15.0) * torch.exp(sigma * z)
    v_in = 0.3 * torch.rand((count, m), generator=gen, device=device, dtype=torch.float64)
    return g_dev.contiguous(), v_in.contiguous()
