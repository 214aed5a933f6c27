"""The allocation-free entry point pat_reconstruct_noalloc against
pat_reconstruct (same kernels; the workspace is the library's static
per-device scratch instead of the caller's buffer)."""
import numpy as np
import pytest
import torch

from oracle import recon
from paper_0808_3510_amd import inputs, pat

pytestmark = pytest.mark.gpu
DEV = "cuda"


def plan_for(g, prec="f32"):
    return pat.Plan(g["n1"], g["n2"], g["nt"], g["nz"], g["dx"], g["dt"], g["dz"], g["vs"], precision=prec,
                    device=DEV)


def stream():
    return torch.cuda.current_stream().cuda_stream


def test_noalloc_two_calls_in_a_row_match_reconstruct():
    """128^2 x 256 -> 128^3 (the largest FP32 workload that fits the scratch),
    then a smaller 3D case, through the C ABI back to back; each against
    pat_reconstruct's output on the same input (bit for bit: same kernels)
    and the small one against the oracle."""
    big = dict(n1=128, n2=128, nt=256, nz=128, dx=1 / 128, dt=1 / 128, dz=1 / 128, vs=1.0)
    small = dict(n1=24, n2=20, nt=48, nz=24, dx=1.0, dt=0.8, dz=1.2, vs=1.1)
    cases = []
    for g, seed in ((big, 960), (small, 961)):
        print(f"noalloc reference {g}", flush=True)
        plan = plan_for(g)
        p = inputs.random_array((g["n1"], g["n2"], g["nt"]), seed)
        P = torch.from_numpy(p).to(DEV, torch.float32)
        ref = plan.reconstruct(P).clone()
        cases.append((g, plan, p, P, ref, torch.full_like(ref, float("nan"))))
    torch.cuda.synchronize()
    for g, plan, p, P, ref, out in cases:
        print(f"noalloc call {g}", flush=True)
        pat.pat_reconstruct_noalloc(plan.ptr, P.data_ptr(), P.numel() * 4, out.data_ptr(), out.numel() * 4,
                                    stream())
    torch.cuda.synchronize()
    for g, plan, p, P, ref, out in cases:
        assert torch.equal(out, ref), g
    g, plan, p, P, ref, out = cases[1]
    exp = recon.reconstruct(p, g)
    err = np.linalg.norm(out.cpu().double().numpy() - exp) / np.linalg.norm(exp)
    assert err < 1e-5


@pytest.mark.parametrize("prec", ["f64", "bf16grid"])
def test_noalloc_other_precisions(prec):
    """FP64 and the staged bf16-grid path (whose workspace includes the grid)."""
    g = dict(n1=16, n2=12, nt=40, nz=16, dx=1.0, dt=0.9, dz=1.1, vs=1.0)
    print(f"noalloc {prec} {g}", flush=True)
    plan = plan_for(g, prec)
    dt = torch.float64 if prec == "f64" else torch.float32
    P = torch.from_numpy(inputs.random_array((16, 12, 40), 962)).to(DEV, dt)
    ref = plan.reconstruct(P).clone()
    out = plan.reconstruct_noalloc(P)
    torch.cuda.synchronize()
    assert torch.equal(out, ref)


def test_noalloc_refuses_plans_beyond_the_scratch():
    """256^2 x 512 needs ~200 MB of workspace: refused on the host, before
    anything is enqueued, with the sizes in the message."""
    g = dict(n1=256, n2=256, nt=512, nz=256, dx=1 / 256, dt=1 / 256, dz=1 / 256, vs=1.0)
    plan = plan_for(g)
    P = torch.zeros((256, 256, 512), device=DEV)
    out = torch.full((256, 256, 256), 7.0, device=DEV)
    with pytest.raises(pat.PatError) as ei:
        pat.pat_reconstruct_noalloc(plan.ptr, P.data_ptr(), P.numel() * 4, out.data_ptr(), out.numel() * 4,
                                    stream())
    assert ei.value.status == 2 and "scratch" in str(ei.value)
    torch.cuda.synchronize()
    assert torch.all(out == 7.0)
