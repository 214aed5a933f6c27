"""R with the other evaluations of the nonuniform sums that Section 4 compares
(truncated sinc, linear and nearest interpolation of the oversampled FFT),
against the oracle's own implementation of each method."""
import numpy as np
import pytest
import torch

from oracle import recon
from paper_0808_3510_amd import inputs, pat

pytestmark = pytest.mark.gpu

TOL = {"f32": 1e-5, "f64": 1e-9}
GEOS = [
    dict(n1=10, n2=6, nt=40, nz=12, dx=0.9, dt=0.7, dz=1.1, vs=1.3),
    dict(n1=16, n2=16, nt=32, nz=16, dx=1 / 16, dt=1 / 16, dz=1 / 16, vs=1.0),
    dict(n1=12, n2=1, nt=48, nz=24, dx=1.0, dt=0.8, dz=1.2, vs=1.0),
]
METHODS = [("sinc", 2.0), ("linear", 1.0), ("linear", 2.0), ("nearest", 1.0), ("nearest", 2.0), ("linear", 4.0)]


def relerr(a, b):
    return float(np.linalg.norm(np.ravel(a - b)) / np.linalg.norm(np.ravel(b)))


@pytest.mark.parametrize("prec", ["f32", "f64"])
@pytest.mark.parametrize("kind,c", METHODS)
@pytest.mark.parametrize("gi", range(len(GEOS)))
def test_reconstruct_with_method_matches_oracle(prec, kind, c, gi):
    g = GEOS[gi]
    print(f"R {kind} c={c} {prec} {g}", flush=True)
    shape = (g["n1"], g["n2"], g["nt"]) if g["n2"] > 1 else (g["n1"], g["nt"])
    p = inputs.random_array(shape, 400 + gi)
    expect = recon.reconstruct_with(p, g, kind, c)
    plan = pat.Plan(g["n1"], g["n2"], g["nt"], g["nz"], g["dx"], g["dt"], g["dz"], g["vs"], c=c, precision=prec,
                    device="cuda", interp=kind)
    dt = torch.float64 if prec == "f64" else torch.float32
    f = plan.reconstruct(torch.from_numpy(p).to("cuda", dt))
    torch.cuda.synchronize()
    assert relerr(f.cpu().double().numpy(), expect) < TOL[prec]


def test_methods_run_the_reconstruction_only():
    g = GEOS[0]
    plan = pat.Plan(g["n1"], g["n2"], g["nt"], g["nz"], g["dx"], g["dt"], g["dz"], g["vs"], c=2.0,
                    precision="f32", device="cuda", interp="linear")
    q = torch.zeros((g["n1"], g["n2"], g["nz"]), device="cuda")
    with pytest.raises(pat.PatError) as ei:
        plan.reconstruct_adjoint(q)
    assert ei.value.status == 2


# Kaiser-Bessel over the oversampling factors of Fig. 5 and one step past
# them (2cK taps capped at 64, so K = 2 at c = 16 and K = 1 at c = 32).  The
# last geometry has the paper's nt = 512: 8192-point grid lines at c = 16 (the
# fused kernel holds 131 KB of LDS; in FP64 the line alone is 128 KB, staged)
# and 16384-point lines at c = 32 (staged: one line per workgroup with its
# twiddles read from memory; in FP64 such a line exceeds LDS).
KB_SWEEP = [(4.0, 3.0), (8.0, 3.0), (16.0, 2.0), (32.0, 1.0)]
KB_GEOS = GEOS[:2] + [dict(n1=16, n2=1, nt=512, nz=64, dx=1 / 16, dt=1 / 512, dz=1 / 64, vs=1.0)]


@pytest.mark.parametrize("fused", [True, False])
@pytest.mark.parametrize("prec", ["f32", "f64"])
@pytest.mark.parametrize("c,K", KB_SWEEP)
@pytest.mark.parametrize("gi", range(len(KB_GEOS)))
def test_kaiser_bessel_oversampling_sweep(fused, prec, c, K, gi):
    g = KB_GEOS[gi]
    print(f"R kb c={c} K={K} {prec} fused={fused} {g}", flush=True)
    mk = lambda: pat.Plan(g["n1"], g["n2"], g["nt"], g["nz"], g["dx"], g["dt"], g["dz"], g["vs"], c=c, K=K,  # noqa: E731
                          precision=prec, device="cuda")
    m_bytes = c * g["nt"] * (16 if prec == "f64" else 8)
    if m_bytes + 64 * (16 if prec == "f64" else 8) > 160 * 1024:
        # one grid line beyond a workgroup's LDS: plan creation refuses it
        with pytest.raises(pat.PatError) as ei:
            mk()
        assert ei.value.status == 2
        return
    plan = mk()
    if fused and m_bytes > 64 * 1024:
        # the fused kernels hold a line twice (FFT order and natural order)
        with pytest.raises(pat.PatError) as ei:
            plan.set_fused(True)
        assert ei.value.status == 2
        return
    plan.set_fused(fused)
    shape = (g["n1"], g["n2"], g["nt"]) if g["n2"] > 1 else (g["n1"], g["nt"])
    p = inputs.random_array(shape, 500 + gi)
    expect = recon.reconstruct_with(p, g, "kb", c, K)
    dt = torch.float64 if prec == "f64" else torch.float32
    f = plan.reconstruct(torch.from_numpy(p).to("cuda", dt))
    torch.cuda.synchronize()
    assert relerr(f.cpu().double().numpy(), expect) < TOL[prec]


@pytest.mark.parametrize("kind", ["sinc", "linear", "nearest"])
def test_other_methods_at_c32_nt512(kind):
    """The oversampling c = 32 of Fig. 5 at the paper's nt = 512 (16384-point
    grid lines) for the methods other than Kaiser-Bessel, against the oracle."""
    g = KB_GEOS[2]
    print(f"R {kind} c=32 {g}", flush=True)
    p = inputs.random_array((g["n1"], g["nt"]), 510)
    K = 1.0
    expect = recon.reconstruct_with(p, g, kind, 32.0, K)
    plan = pat.Plan(g["n1"], g["n2"], g["nt"], g["nz"], g["dx"], g["dt"], g["dz"], g["vs"], c=32.0, K=K,
                    precision="f32", device="cuda", interp=kind)
    f = plan.reconstruct(torch.from_numpy(p).to("cuda", torch.float32))
    torch.cuda.synchronize()
    assert relerr(f.cpu().double().numpy(), expect) < TOL["f32"]
