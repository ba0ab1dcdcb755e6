"""Write tests/golden/oracle_32x32_seed0.json from the CPU oracle alone.

The paper prints no worked numerical example (its only table lists GMRES step
counts and CPU times, Section IV, Table I), so the stored values here are the
oracle's own steady state for the 32 x 32 standard crossbar with seed 0.  They
guard the oracle and the seeded input generator against silent changes; the
oracle itself is pinned by the independent checks in tests/test_oracle.py.

Run from the repository root:  python tests/golden/make_golden.py
"""

import json
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

import oracle  # noqa: E402
from paper_2109_07929_amd import synth  # noqa: E402


def main():
    cb = synth.crossbar(32, 32, seed=0)
    vt, vb, k, hist = oracle.solve(cb.geom, cb.g_dev, cb.v_in, method="band")
    rng = np.random.default_rng(12345)
    idx = [(int(i), int(j)) for i, j in zip(rng.integers(0, 32, 24), rng.integers(0, 32, 24))]
    out = {
        "what": "oracle steady state, 32x32 standard crossbar, seed 0 (band-Cholesky Newton)",
        "m": 32, "n": 32, "seed": 0,
        "newton_steps": int(k),
        "final_rel_residual": float(hist[-1]),
        "sum_vt": float(vt.sum()), "sum_vb": float(vb.sum()),
        "max_vt": float(vt.max()), "max_vb": float(vb.max()),
        "samples": [[i, j, float(vt[i, j]), float(vb[i, j])] for i, j in idx],
    }
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "oracle_32x32_seed0.json")
    with open(path, "w") as f:
        json.dump(out, f, indent=1)
    print("wrote", path)


if __name__ == "__main__":
    main()
