"""mca_precond_apply_noalloc (the workspace-free preconditioner call, for
callers that cannot allocate) against mca_precond_apply on the same inputs.

Both run the same kernels, so the outputs must agree bit for bit.  Each case
makes two calls in a row on the library's per-GPU scratch array, the second
with a smaller crossbar (whatever the first call left in the array must not
leak into the second result).  Sizes past the array's limit are refused before
any launch.
"""

import numpy as np
import pytest
import torch

from paper_2109_07929_amd import Plan, synth
from paper_2109_07929_amd import binding as B

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)


def _call_both(plan, form, prec, seed):
    m, n = plan.m, plan.n
    gen = torch.Generator(device="cpu")
    gen.manual_seed(seed)
    r_t = torch.randn((m, n), generator=gen, dtype=torch.float64).cuda()
    r_b = torch.randn((m, n), generator=gen, dtype=torch.float64).cuda()
    a = 3.7e-5
    ref_t, ref_b = plan.precond_apply(a, a, r_t, r_b, form=form, precision=prec)
    z_t = torch.full((m, n), float("nan"), dtype=torch.float64, device="cuda")
    z_b = torch.full((m, n), float("nan"), dtype=torch.float64, device="cuda")
    B.mca_precond_apply_noalloc(plan.handle, m, n, form, prec, a, a, r_t, r_b, z_t, z_b)
    torch.cuda.synchronize()
    return ref_t, ref_b, z_t, z_b


@pytest.mark.parametrize("form,prec,big,small", [
    (B.MCA_PRECOND_LITERAL, B.MCA_PREC_FP64, (1024, 1024), (200, 300)),
    (B.MCA_PRECOND_LITERAL, B.MCA_PREC_FP64, (1023, 1024), (201, 77)),
    (B.MCA_PRECOND_PERMODE, B.MCA_PREC_FP64, (1024, 1024), (100, 70)),
    (B.MCA_PRECOND_PERMODE, B.MCA_PREC_BF16X3, (1024, 1024), (130, 257)),
    (B.MCA_PRECOND_PERMODE, B.MCA_PREC_FP32, (640, 512), (33, 65)),
    (B.MCA_PRECOND_APPROX, B.MCA_PREC_FP64, (512, 512), (64, 48)),
])
def test_noalloc_matches_precond_apply(form, prec, big, small):
    for k, (m, n) in enumerate((big, small)):
        say(f"noalloc form {form} prec {prec} call {k}: {m}x{n}")
        plan = Plan(synth.crossbar(m, n, seed=k).geom)
        assert B.mca_precond_workspace_bytes(plan.handle, form, prec) <= B.MCA_NOALLOC_SCRATCH_BYTES
        ref_t, ref_b, z_t, z_b = _call_both(plan, form, prec, seed=10 * k + form)
        assert torch.isfinite(z_t).all() and torch.isfinite(z_b).all()
        assert torch.equal(z_t, ref_t) and torch.equal(z_b, ref_b)


def test_noalloc_refuses_sizes_past_its_array():
    plan = Plan(synth.crossbar(1025, 1024, seed=0).geom)
    need = B.mca_precond_workspace_bytes(plan.handle, B.MCA_PRECOND_PERMODE, B.MCA_PREC_FP64)
    assert need > B.MCA_NOALLOC_SCRATCH_BYTES
    z = torch.zeros((1025, 1024), dtype=torch.float64, device="cuda")
    r = torch.ones_like(z)
    with pytest.raises(B.MCAError) as e:
        B.mca_precond_apply_noalloc(plan.handle, 1025, 1024, B.MCA_PRECOND_PERMODE,
                                    B.MCA_PREC_FP64, 1e-5, 1e-5, r, r, z, z)
    assert e.value.status == B.MCA_ERR_WORKSPACE
    assert torch.equal(z, torch.zeros_like(z))
