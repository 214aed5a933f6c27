"""The smooth cut-off of the partial-data model (eq. data-part) on the GPU: the
four operators with a cut-off against the oracle's cut-off weights composed
with its direct-sum operators (R(w p), w R^T(q), w A(f), A^T(w p))."""
import numpy as np
import pytest
import torch

from oracle import cutoff, recon
from paper_0808_3510_amd import inputs, pat

pytestmark = pytest.mark.gpu

TOL = {"f32": 1e-5, "f64": 1e-9}
CASES = [
    # 3D, powers of two, integer eps
    (dict(n1=16, n2=16, nt=32, nz=16, dx=1 / 16, dt=1 / 16, dz=1 / 16, vs=1.0), 2.0),
    # 2D line detectors, half-integer eps
    (dict(n1=24, n2=1, nt=48, nz=24, dx=1.0, dt=0.8, dz=1.2, vs=1.0), 2.5),
    # 3D, factors 3, 5, 7, rows of 70 samples (two-sample accesses), 4 eps = n1
    (dict(n1=12, n2=20, nt=70, nz=18, dx=1.0, dt=0.8, dz=1.2, vs=1.0), 3.0),
    # 3D, 128-point x1 columns: the passes over x1 take their compile-time
    # pipelines (FP32 and FP64), the weighted one included; 4 eps = n2
    (dict(n1=128, n2=4, nt=32, nz=16, dx=1 / 128, dt=1 / 32, dz=1 / 16, vs=1.0), 1.0),
]


def relerr(a, b):
    return float(np.linalg.norm(np.ravel(a - b)) / np.linalg.norm(np.ravel(b)))


def shape(g, n):
    return (g["n1"], g["n2"], n) if g["n2"] > 1 else (g["n1"], n)


def expected(op, x, g, eps):
    if op == "reconstruct":
        return recon.reconstruct(cutoff.apply(x, g, eps), g)
    if op == "reconstruct_adjoint":
        return cutoff.apply(recon.reconstruct_adjoint(x, g), g, eps)
    if op == "forward":
        return cutoff.apply(recon.forward(x, g), g, eps)
    return recon.forward_adjoint(cutoff.apply(x, g, eps), g)


@pytest.mark.parametrize("op", ["reconstruct", "reconstruct_adjoint", "forward", "forward_adjoint"])
@pytest.mark.parametrize("prec", ["f32", "f64"])
@pytest.mark.parametrize("ci", range(len(CASES)))
def test_operators_with_cutoff_match_oracle(op, prec, ci):
    g, eps = CASES[ci]
    print(f"cutoff {op} {prec} eps={eps} {g}", flush=True)
    n_in = g["nt"] if op in ("reconstruct", "forward_adjoint") else g["nz"]
    x = inputs.random_array(shape(g, n_in), 600 + ci)
    expect = expected(op, x, g, eps)
    plan = pat.Plan(g["n1"], g["n2"], g["nt"], g["nz"], g["dx"], g["dt"], g["dz"], g["vs"], precision=prec,
                    device="cuda", cutoff=eps)
    dt = torch.float64 if prec == "f64" else torch.float32
    y = getattr(plan, op)(torch.from_numpy(x).to("cuda", dt))
    torch.cuda.synchronize()
    assert relerr(y.cpu().double().numpy(), expect) < TOL[prec]


@pytest.mark.parametrize("ci", range(len(CASES)))
def test_cutoff_keeps_the_transpose_pairs_fp64(ci):
    g, eps = CASES[ci]
    print(f"cutoff dot products eps={eps} {g}", flush=True)
    rg = inputs.rng(9 + ci)
    p = rg.standard_normal(shape(g, g["nt"]))
    q = rg.standard_normal(shape(g, g["nz"]))
    plan = pat.Plan(g["n1"], g["n2"], g["nt"], g["nz"], g["dx"], g["dt"], g["dz"], g["vs"], precision="f64",
                    device="cuda", cutoff=eps)
    P, Q = torch.from_numpy(p).cuda(), torch.from_numpy(q).cuda()
    assert torch.sum(plan.reconstruct(P) * Q).item() == pytest.approx(
        torch.sum(P * plan.reconstruct_adjoint(Q)).item(), rel=1e-12)
    assert torch.sum(plan.forward(Q) * P).item() == pytest.approx(
        torch.sum(Q * plan.forward_adjoint(P)).item(), rel=1e-12)


def test_cutoff_on_samples_deep_inside_changes_nothing():
    # data that vanish within 2 eps of every face: the cut-off leaves them be
    g, eps = CASES[0]
    print("cutoff interior", flush=True)
    x = inputs.random_array(shape(g, g["nt"]), 610)
    e = int(np.ceil(2 * eps))
    x[:e] = 0
    x[-e + 1:] = 0
    x[:, :e] = 0
    x[:, -e + 1:] = 0
    x[..., :e] = 0
    x[..., -e + 1:] = 0
    kw = dict(precision="f64", device="cuda")
    a = pat.Plan(g["n1"], g["n2"], g["nt"], g["nz"], g["dx"], g["dt"], g["dz"], g["vs"], cutoff=eps, **kw)
    b = pat.Plan(g["n1"], g["n2"], g["nt"], g["nz"], g["dx"], g["dt"], g["dz"], g["vs"], **kw)
    X = torch.from_numpy(x).cuda()
    assert torch.equal(a.reconstruct(X), b.reconstruct(X))


def test_batched_instances_with_their_own_cutoffs():
    print("cutoff batched", flush=True)
    specs = [(16, 2.0), (24, 0.0), (20, 4.0)]
    plans, ps, expect = [], [], []
    for j, (n, eps) in enumerate(specs):
        g = dict(n1=n, n2=n, nt=2 * n, nz=n, dx=1.0, dt=1.0, dz=1.0, vs=1.0)
        p = inputs.random_array((n, n, 2 * n), 620 + j)
        plans.append(pat.Plan(n, n, 2 * n, n, precision="f32", device="cuda", cutoff=eps))
        ps.append(torch.from_numpy(p.astype(np.float32)).cuda())
        expect.append(recon.reconstruct(cutoff.apply(p, g, eps) if eps else p, g))
    outs, _ = pat.reconstruct_batched(plans, ps)
    torch.cuda.synchronize()
    for o, e in zip(outs, expect):
        assert relerr(o.cpu().double().numpy(), e) < TOL["f32"]
