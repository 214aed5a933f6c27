"""Edge cases of the GPU operators against the oracle: the smallest
geometries the plan accepts (single-stage FFTs, a grid line of exactly 2cK
points), the longest grid lines (8192 points: fused kernels at 131 KB of LDS,
and the staged path where the fused lists do not fit), the widest detector
axis (transverse tiles one column wide), and all-zero data."""
import numpy as np
import pytest
import torch

from oracle import recon
from paper_0808_3510_amd import inputs, pat

pytestmark = pytest.mark.gpu

TOL = {"f32": 1e-5, "f64": 1e-9}
OPS = ["reconstruct", "reconstruct_adjoint", "forward", "forward_adjoint"]


def geo(n1, n2, nt, nz):
    return dict(n1=n1, n2=n2, nt=nt, nz=nz, dx=1.0, dt=0.9, dz=1.1, vs=1.0)


def shape(g, n):
    return (g["n1"], g["n2"], n) if g["n2"] > 1 else (g["n1"], n)


def relerr(a, b):
    return float(np.linalg.norm(np.ravel(a - b)) / np.linalg.norm(np.ravel(b)))


def run(op, g, prec, seed):
    print(f"edge {op} {prec} {g}", flush=True)
    n_in = g["nt"] if op in ("reconstruct", "forward_adjoint") else g["nz"]
    x = inputs.random_array(shape(g, n_in), seed)
    plan = pat.Plan(g["n1"], g["n2"], g["nt"], g["nz"], g["dx"], g["dt"], g["dz"], g["vs"], precision=prec,
                    device="cuda")
    dt = torch.float64 if prec == "f64" else torch.float32
    y = getattr(plan, op)(torch.from_numpy(x).to("cuda", dt))
    torch.cuda.synchronize()
    return relerr(y.cpu().double().numpy(), getattr(recon, op)(x, g))


@pytest.mark.parametrize("op", OPS)
@pytest.mark.parametrize("prec", ["f32", "f64"])
@pytest.mark.parametrize("g", [geo(2, 2, 6, 2), geo(2, 1, 8, 2)])
def test_smallest_geometries(op, prec, g):
    assert run(op, g, prec, 800) < TOL[prec]


@pytest.mark.parametrize("op", OPS)
def test_longest_grid_lines_fused(op):
    assert run(op, geo(4, 1, 4096, 1024), "f32", 801) < TOL["f32"]


def test_longest_grid_lines_staged():
    g = geo(4, 1, 4096, 2048)
    assert run("reconstruct", g, "f32", 802) < TOL["f32"]
    # the spreading lists of a 2048-sample depth line exceed one workgroup's LDS
    plan = pat.Plan(g["n1"], g["n2"], g["nt"], g["nz"], precision="f32", device="cuda")
    with pytest.raises(pat.PatError) as ei:
        plan.reconstruct_adjoint(torch.zeros(shape(g, g["nz"]), device="cuda"))
    assert ei.value.status == 2


@pytest.mark.parametrize("op", ["reconstruct", "reconstruct_adjoint"])
@pytest.mark.parametrize("prec", ["f32", "f64"])
def test_widest_detector_axis(op, prec):
    assert run(op, geo(4096, 1, 8, 8), prec, 803) < TOL[prec]


@pytest.mark.parametrize("op", OPS)
def test_zero_data_gives_zero(op):
    g = geo(16, 16, 32, 16)
    plan = pat.Plan(g["n1"], g["n2"], g["nt"], g["nz"], precision="f32", device="cuda")
    n_in = g["nt"] if op in ("reconstruct", "forward_adjoint") else g["nz"]
    y = getattr(plan, op)(torch.zeros(shape(g, n_in), device="cuda"))
    torch.cuda.synchronize()
    assert torch.count_nonzero(y).item() == 0
