"""Host-side checks of bench.py that need no GPU: the one-GPU guard and the
byte accounting behind its Krylov roofline."""

import os
import subprocess
import sys
import types

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402
from paper_2109_07929_amd import binding as B  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""


def _stats(history):
    return types.SimpleNamespace(krylov_history=list(history), newton_iters=len(history))


@pytest.mark.parametrize("precond,extra", [(B.MCA_PRECOND_LITERAL, 8), (B.MCA_PRECOND_PERMODE, 0)])
def test_krylov_bytes_two_pass(precond, extra):
    """Per Arnoldi step j: the algorithm moves 40 + 16(j+1) + 32 bytes per crosspoint;
    the two passes read the basis twice, and the literal FP64 form's Jacobian pass
    also forms z_b (8 more bytes)."""
    mn = 1000
    opts = B.options(precond=precond)
    kms = [0.0] * B.MCA_NUM_KCLASS
    kms[B.MCA_KCLASS_JACOBIAN] = 1.0
    kms[B.MCA_KCLASS_ORTHO] = 1.0
    out = bench.krylov_hbm(_stats([2, 3]), mn, opts, kms, 1)
    steps = [0, 1, 0, 1, 2]
    alg = sum(40 + 16 * (j + 1) + 32 for j in steps) * mn
    kern = sum((40 + extra + 16 * (j + 1)) + (32 + 16 * (j + 1)) for j in steps) * mn
    assert out["algorithmic_bytes_per_solve"] == alg
    assert out["kernel_bytes_per_solve"] == kern
    assert out["ms_per_solve"] == 2.0
    assert out["form"].startswith("two-pass")


def test_krylov_bytes_restarts_and_one_pass_form():
    """Cycles restart after `restart` steps; the one-pass-per-vector form moves
    56 + 64 j + 48 + 32 bytes per crosspoint at step j."""
    mn = 10
    opts = B.options(restart=2, flags=B.MCA_FLAG_MGS_PASSES)
    kms = [0.0] * B.MCA_NUM_KCLASS
    kms[B.MCA_KCLASS_ORTHO] = 4.0
    out = bench.krylov_hbm(_stats([5]), mn, opts, kms, 2)
    steps = [0, 1, 0, 1, 0]
    assert out["kernel_bytes_per_solve"] == sum(56 + 64 * j + 48 + 32 for j in steps) * mn
    assert out["ms_per_solve"] == 2.0
    assert bench.krylov_hbm(_stats([5]), mn, opts, [0.0] * B.MCA_NUM_KCLASS, 1) is None
