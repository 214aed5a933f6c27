"""Element-wise parity of every compile-time instance of the fused line
kernels against the full FP64 oracle.

One FP32 instance with c = 2, K = 3 and power-of-two sizes runs the fused
kernels with their sizes fixed at compile time: the type-2 kernel (R, A^T)
and the type-1 kernel (R^T, A) exist for grid lines of m = 2^LM points,
LM = 8 .. 11, and depth lines of nz = m/4 or m/2.  Each (LM, nz) pair runs
here on thin geometries (8 x 1 and 8 x 4 detectors, nt = m/2), all four
operators against the oracle (the NUFFT of Section 3 against the direct sums
of Section 4), with relative L2 and largest-element bounds.  The planes whose
handling is special in the half-spectrum kernels, l = 0 (weight 0) and the
depth-Nyquist plane l = -nz/2 (mean of the nodes -+|nu|), are checked on
their own, since they hold a small share of a random volume's norm.
"""
import numpy as np
import pytest
import torch

from oracle import recon
from paper_0808_3510_amd import inputs, pat

pytestmark = pytest.mark.gpu
DEV = "cuda"
TOL = 1e-5
OPS = ["reconstruct", "reconstruct_adjoint", "forward", "forward_adjoint"]

INSTANCES = [(lm, lz) for lm in (8, 9, 10, 11) for lz in (lm - 2, lm - 1)]


def geo(lm, lz, n2):
    return dict(n1=8, n2=n2, nt=1 << (lm - 1), nz=1 << lz, dx=1.0, dt=0.9, dz=1.1, vs=1.0)


def shape(g, last):
    return (g["n1"], g["n2"], last) if g["n2"] > 1 else (g["n1"], last)


def plan_for(g):
    return pat.Plan(g["n1"], g["n2"], g["nt"], g["nz"], g["dx"], g["dt"], g["dz"], g["vs"], precision="f32",
                    device=DEV)


def run(plan, op, x):
    y = getattr(plan, op)(torch.from_numpy(np.ascontiguousarray(x)).to(DEV, torch.float32))
    torch.cuda.synchronize()
    return y.cpu().double().numpy()


def check(got, exp, what):
    rel = np.linalg.norm(got - exp) / np.linalg.norm(exp)
    mx = np.abs(got - exp).max() / np.abs(exp).max()
    print(f"  {what}: relL2 {rel:.2e}, max {mx:.2e}", flush=True)
    assert rel <= TOL and mx <= TOL, (what, rel, mx)


@pytest.mark.parametrize("op", OPS)
@pytest.mark.parametrize("n2", [1, 4])
@pytest.mark.parametrize("lm,lz", INSTANCES)
def test_instance_matches_oracle(lm, lz, n2, op):
    g = geo(lm, lz, n2)
    print(f"instance m=2^{lm} nz=2^{lz} {op} {g}", flush=True)
    n_in = g["nt"] if op in ("reconstruct", "forward_adjoint") else g["nz"]
    x = inputs.random_array(shape(g, n_in), 900 + lm * 10 + lz)
    got = run(plan_for(g), op, x)
    exp = getattr(recon, op)(x, g)
    check(got, exp, op)
    if op in ("reconstruct", "forward_adjoint"):
        # image-side outputs: the l = 0 and depth-Nyquist planes of their
        # depth spectra on their own
        Dg, De = np.fft.fft(got, axis=-1), np.fft.fft(exp, axis=-1)
        h = g["nz"] // 2
        check(Dg[..., h], De[..., h], "Nyquist plane")
        if op == "reconstruct":
            # weight 0 on l = 0: every output column has zero depth mean
            assert np.abs(Dg[..., 0]).max() <= TOL * np.abs(Dg).max()
        else:
            check(Dg[..., 0], De[..., 0], "l = 0 plane")


@pytest.mark.parametrize("op", ["reconstruct_adjoint", "forward"])
@pytest.mark.parametrize("lm,lz", INSTANCES)
def test_instance_single_planes(lm, lz, op):
    """Image-side inputs that live on one depth plane only: a depth-constant
    column (l = 0) and an alternating one (l = -nz/2)."""
    g = geo(lm, lz, 4)
    print(f"planes m=2^{lm} nz=2^{lz} {op}", flush=True)
    plan = plan_for(g)
    r = inputs.random_array((g["n1"], g["n2"], 1), 950 + lm)
    z = np.arange(g["nz"])
    full = run(plan, op, inputs.random_array(shape(g, g["nz"]), 951 + lm))
    for name, prof in (("l = 0", np.ones(g["nz"])), ("Nyquist", (-1.0) ** z)):
        x = r * prof[None, None, :]
        got = run(plan, op, x)
        exp = getattr(recon, op)(x, g)
        if op == "reconstruct_adjoint" and name == "l = 0":
            # weight 0: nothing reaches the data
            assert np.abs(exp).max() <= 1e-12 * np.abs(full).max()
            assert np.abs(got).max() <= TOL * np.abs(full).max()
        else:
            check(got, exp, name)


# The staged path (grid stored between stages; the bf16-grid option always
# runs it) has compile-time pipelines of its own for one FP32 instance with
# the c = 2 grid and m = 2^8 .. 2^11: the grid FFT of R and A^T
# (k_line_a2_pipe) and its transpose in R^T and A (k_line_a2t_pipe).  Every
# size against the oracle, FP32 and bf16 grid storage (8 mantissa bits).
STAGED_TOL = {"f32": TOL, "bf16grid": 1e-2}


@pytest.mark.parametrize("op", OPS)
@pytest.mark.parametrize("prec", ["f32", "bf16grid"])
@pytest.mark.parametrize("lm", [8, 9, 10, 11])
def test_staged_pipelines_match_oracle(lm, prec, op):
    g = geo(lm, lm - 2, 4)
    print(f"staged m=2^{lm} {prec} {op} {g}", flush=True)
    n_in = g["nt"] if op in ("reconstruct", "forward_adjoint") else g["nz"]
    x = inputs.random_array(shape(g, n_in), 970 + lm)
    plan = pat.Plan(g["n1"], g["n2"], g["nt"], g["nz"], g["dx"], g["dt"], g["dz"], g["vs"], precision=prec,
                    device=DEV)
    plan.set_fused(False)
    got = run(plan, op, x)
    exp = getattr(recon, op)(x, g)
    rel = np.linalg.norm(got - exp) / np.linalg.norm(exp)
    mx = np.abs(got - exp).max() / np.abs(exp).max()
    print(f"  relL2 {rel:.2e}, max {mx:.2e}", flush=True)
    assert rel <= STAGED_TOL[prec] and mx <= STAGED_TOL[prec], (rel, mx)


# FP64 runs the same compile-time kernels at two waves per SIMD: the type-2
# kernels (k_line_nufft2_mirror for R on 3D plans with nz = m/4,
# k_line_nufft2_pipe_c otherwise) for R and A^T, the wavefront-spreading
# kernel (k_line_nufft1_w, m up to 1024) for R^T and A: every size against
# the oracle at 1e-9.  (R^T and A in double at nz = 1024 pass the spreading
# lists' LDS limit of the ABI, about 900 in double: PAT_ERR_UNSUPPORTED.)
@pytest.mark.parametrize("op", ["reconstruct", "forward_adjoint", "reconstruct_adjoint", "forward"])
@pytest.mark.parametrize("n2", [1, 4])
@pytest.mark.parametrize("lm,lz", INSTANCES)
def test_instance_fp64_matches_oracle(lm, lz, n2, op):
    g = geo(lm, lz, n2)
    print(f"fp64 instance m=2^{lm} nz=2^{lz} {op} {g}", flush=True)
    spreads = op in ("reconstruct_adjoint", "forward")
    n_in = g["nz"] if spreads else g["nt"]
    x = inputs.random_array(shape(g, n_in), 990 + lm * 10 + lz)
    plan = pat.Plan(g["n1"], g["n2"], g["nt"], g["nz"], g["dx"], g["dt"], g["dz"], g["vs"], precision="f64",
                    device=DEV)
    xd = torch.from_numpy(np.ascontiguousarray(x)).to(DEV, torch.float64)
    if spreads and g["nz"] > 900:
        with pytest.raises(pat.PatError) as err:
            getattr(plan, op)(xd)
        assert err.value.status == 2  # PAT_ERR_UNSUPPORTED
        return
    y = getattr(plan, op)(xd)
    torch.cuda.synchronize()
    got = y.cpu().numpy()
    exp = getattr(recon, op)(x, g)
    rel = np.linalg.norm(got - exp) / np.linalg.norm(exp)
    mx = np.abs(got - exp).max() / np.abs(exp).max()
    print(f"  relL2 {rel:.2e}, max {mx:.2e}", flush=True)
    assert rel <= 1e-9 and mx <= 1e-9, (rel, mx)
