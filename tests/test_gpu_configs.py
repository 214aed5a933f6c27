"""GPU parity at the five workload configurations, against the FP64 oracle.

1. 2D line detectors, 128 x 256 -> 128 x 128, three disks, data from the
   oracle's forward sums on a zero-padded grid; FP64 GPU <= 1e-9.
2. 3D 128^2 x 256 -> 128^3, eight balls + noise; FP32 <= 1e-5 against the
   full oracle reconstruction; FP64 <= 1e-9; bf16 grid <= 1e-2.
3. 3D 256^2 x 512 -> 256^3, 32 balls + noise, in the launch configuration the
   benchmark times; compared on sampled output lines (the oracle computes a
   line's spectrum directly), plus exact properties (shift equivariance,
   linearity) at full size.
4. Differentiable form: A / A^T against the oracle, gradient against central
   finite differences in FP64, 20 Landweber steps with decreasing loss.
5. Batched: 16 uneven instances (64^2 .. 184^2 planes) in one persistent
   launch per stage; per-instance parity and equality with single calls.
"""
import numpy as np
import pytest
import torch

from oracle import kb, recon
from paper_0808_3510_amd import inputs, pat

pytestmark = pytest.mark.gpu
DEV = "cuda"


def relerr(a, b):
    return float(np.linalg.norm(np.ravel(a - b)) / np.linalg.norm(np.ravel(b)))


def say(msg):
    print(msg, flush=True)


def dev(a, prec="f32"):
    dt = torch.float64 if prec == "f64" else torch.float32
    return torch.from_numpy(np.ascontiguousarray(a)).to(device=DEV, dtype=dt)


def plan_for(g, prec):
    return pat.Plan(g["n1"], g["n2"], g["nt"], g["nz"], g["dx"], g["dt"], g["dz"], g["vs"], precision=prec,
                    device=DEV)


def sampled_line_spectra(f_gpu, p, g, lines):
    """The spectrum of the GPU output on `lines` and the Hermitian part of the
    oracle's spectrum there, ``(len(lines), nz)`` each."""
    n1, n2, nz = g["n1"], g["n2"], g["nz"]
    D = np.fft.fftn(f_gpu.astype(np.float64).reshape(n1, n2, nz))
    ora = recon.spectrum_lines(p, g, lines)
    mir = recon.spectrum_lines(p, g, [(-a, -b) for a, b in lines])
    lneg = (-np.arange(nz)) % nz
    got = np.array([D[a % n1, b % n2] for a, b in lines])
    return got, 0.5 * (ora + np.conj(mir[:, lneg]))


def sampled_line_error(f_gpu, p, g, lines):
    """relL2 between the spectrum of the GPU output on `lines` and the
    Hermitian part of the oracle's spectrum there."""
    got, exp = sampled_line_spectra(f_gpu, p, g, lines)
    return relerr(got, exp)


# ---------------------------------------------------------------------------
# config 1

@pytest.fixture(scope="module")
def config1():
    n = 128
    disks = inputs.draw_disks(3, 1001, n)
    f_true = inputs.disk_image(disks, n, n)
    g = dict(n1=n, n2=1, nt=2 * n, nz=n, dx=1.0, dt=1.0, dz=1.0, vs=1.0)
    # zero padding so that no periodic image arrives within the 256 samples
    p = recon.forward_padded(f_true, g, pad_x=2 * n, nz_pad=3 * n + 8)
    return p, g, recon.reconstruct(p, g)


@pytest.mark.parametrize("prec,tol", [("f64", 1e-9), ("f32", 1e-5)])
def test_config1_2d(config1, prec, tol):
    p, g, expect = config1
    say(f"config1 {prec}")
    f = plan_for(g, prec).reconstruct(dev(p, prec))
    torch.cuda.synchronize()
    assert f.shape == (128, 128)
    assert relerr(f.cpu().double().numpy(), expect) < tol


# ---------------------------------------------------------------------------
# config 2

@pytest.fixture(scope="module")
def config2():
    p, g, balls = inputs.planar_case(128, 8, 1002, noise=1e-3)
    return p, g, recon.reconstruct(p, g)


@pytest.mark.parametrize("prec,tol", [("f32", 1e-5), ("f64", 1e-9), ("bf16grid", 1e-2)])
def test_config2_full_oracle(config2, prec, tol):
    p, g, expect = config2
    say(f"config2 {prec}")
    f = plan_for(g, prec).reconstruct(dev(p, prec))
    torch.cuda.synchronize()
    err = relerr(f.cpu().double().numpy(), expect)
    say(f"  relL2 = {err:.3e}")
    assert err < tol


# ---------------------------------------------------------------------------
# config 3 (the benchmark's workload and launch configuration)

@pytest.fixture(scope="module")
def config3():
    p, g, balls = inputs.planar_case(256, 32, 1003, noise=1e-3)
    rng = inputs.rng(303)
    lines = [(0, 0), (128, 128), (128, 0), (0, 128), (-128, 5), (1, -1)]
    lines += [(int(a), int(b)) for a, b in rng.integers(-128, 128, size=(506, 2))]
    return p, g, lines


@pytest.mark.parametrize("prec,tol", [("f32", 1e-5), ("f64", 1e-9), ("bf16grid", 1e-2)])
def test_config3_sampled_lines(config3, prec, tol):
    """R at full size on 512 sampled output lines, element by element, with
    the l = 0 plane (weight 0) and the depth-Nyquist plane on their own."""
    p, g, lines = config3
    say(f"config3 {prec}")
    f = plan_for(g, prec).reconstruct(dev(p, prec))
    torch.cuda.synchronize()
    got, exp = sampled_line_spectra(f.cpu().numpy(), p, g, lines)
    err = relerr(got, exp)
    mx = np.abs(got - exp).max() / np.abs(exp).max()
    h = g["nz"] // 2
    nyq = relerr(got[:, h], exp[:, h])
    say(f"  512 sampled lines: relL2 {err:.3e}, max {mx:.3e}, Nyquist plane {nyq:.3e}")
    assert err < tol and mx < tol and nyq < tol
    assert np.abs(got[:, 0]).max() <= tol * np.abs(exp).max()


@pytest.mark.parametrize("op", ["reconstruct_adjoint", "forward"])
def test_config3_type1_sampled_lines(config3, op):
    """The fused type-1 kernel at the benchmark's size (R^T, A) on 128 sampled
    lines of the output, element by element against the oracle's sums."""
    p, g, lines = config3
    say(f"config3 {op} sampled lines")
    n1, n2, nt = g["n1"], g["n2"], g["nt"]
    q = inputs.random_array((n1, n2, g["nz"]), 333)
    out = getattr(plan_for(g, "f32"), op)(dev(q)).cpu().double().numpy()
    sel = lines[:128]
    fn = recon.adjoint_lines if op == "reconstruct_adjoint" else recon.forward_lines
    X, Xm = fn(q, g, sel), fn(q, g, [(-a, -b) for a, b in sel])
    D = np.fft.fft2(out, axes=(0, 1))
    got = np.array([D[a % n1, b % n2] for a, b in sel])
    exp = 0.5 * (X + np.conj(Xm))
    err = relerr(got, exp)
    mx = np.abs(got - exp).max() / np.abs(exp).max()
    say(f"  relL2 {err:.3e}, max {mx:.3e}")
    assert got.shape == (128, nt) and err < 1e-5 and mx < 1e-5


def test_config3_properties(config3):
    """Shift equivariance along both detector axes (exact: the pipeline is
    diagonal in transverse frequency) and linearity."""
    p, g, _ = config3
    say("config3 properties")
    plan = plan_for(g, "f32")
    P = dev(p)
    f0 = plan.reconstruct(P).clone()
    fs = plan.reconstruct(torch.roll(P, shifts=(3, -5), dims=(0, 1)).contiguous())
    ref = torch.roll(f0, shifts=(3, -5), dims=(0, 1))
    assert (torch.linalg.vector_norm(fs - ref) / torch.linalg.vector_norm(ref)).item() < 1e-5
    Q = dev(inputs.random_array(p.shape, 9))
    lin = plan.reconstruct((2.0 * P - 0.5 * Q).contiguous())
    comb = 2.0 * f0 - 0.5 * plan.reconstruct(Q)
    assert (torch.linalg.vector_norm(lin - comb) / torch.linalg.vector_norm(comb)).item() < 1e-5
    assert torch.isfinite(f0).all()


@pytest.mark.parametrize("prec,tol", [("f32", 1e-6), ("f64", 1e-12)])
def test_config3_transpose_pairs(config3, prec, tol):
    """R^T and A at full size (the kernels of the benchmark's shape) against R
    and A^T through the transpose identities <R p, q> = <p, R^T q> and
    <A f, p'> = <f, A^T p'>.  The test vectors are q = R p + noise and
    p' = A q + noise, so each inner product is close to the product of the
    norms it is measured against (a random q would leave it sqrt(N) times
    smaller and the bound loose)."""
    p, g, _ = config3
    say(f"config3 transpose pairs {prec}")
    plan = plan_for(g, prec)
    gen = torch.Generator(device=DEV).manual_seed(31)

    def noisy(x):
        n = torch.randn(x.shape, device=DEV, dtype=x.dtype, generator=gen)
        return (x + 0.1 * x.std() * n).contiguous()

    def rel_gap(a, b, u, v):
        return abs(a - b) / (torch.linalg.vector_norm(u) * torch.linalg.vector_norm(v)).item()

    P = dev(p, prec)
    RP = plan.reconstruct(P).clone()
    Q = noisy(RP)
    lhs = torch.sum(RP.double() * Q.double()).item()
    rhs = torch.sum(P.double() * plan.reconstruct_adjoint(Q).double()).item()
    gap = rel_gap(lhs, rhs, RP.double(), Q.double())
    say(f"  <Rp,q> vs <p,R^T q>: {gap:.2e}")
    assert gap <= tol
    AQ = plan.forward(Q).clone()
    P2 = noisy(AQ)
    lhs = torch.sum(AQ.double() * P2.double()).item()
    rhs = torch.sum(Q.double() * plan.forward_adjoint(P2).double()).item()
    gap = rel_gap(lhs, rhs, AQ.double(), P2.double())
    say(f"  <Aq,p'> vs <q,A^T p'>: {gap:.2e}")
    assert gap <= tol


# ---------------------------------------------------------------------------
# config 4

@pytest.fixture(scope="module")
def config4():
    p, g, balls = inputs.planar_case(128, 16, 1004, noise=0.0)
    return p, g


def test_config4_adjoint_matches_oracle(config4):
    p, g = config4
    say("config4 A^T f32 vs oracle")
    expect = recon.forward_adjoint(p, g)
    got = plan_for(g, "f32").forward_adjoint(dev(p)).cpu().double().numpy()
    assert relerr(got, expect) < 1e-5


def test_config4_forward_matches_oracle_sampled(config4):
    """A at full size: its output lines equal the oracle's cosine sums."""
    p, g = config4
    say("config4 A f32 vs oracle (sampled)")
    f = inputs.random_array((128, 128, 128), 44)
    got = plan_for(g, "f32").forward(dev(f)).cpu().double().numpy()
    # the transverse spectrum of A f on a line k is (1/nz) sum_l F[k,l] cos(...)
    F = np.fft.fftn(f)
    D = np.fft.fft2(got, axes=(0, 1))
    l = recon.int_freqs(128)
    n = np.arange(256)
    errs = []
    for k1, k2 in [(0, 0), (3, 7), (-64, 64), (10, -2), (64, 0)]:
        nu = recon.node_plus(k1, k2, l, g)
        C = np.cos(2 * np.pi * np.mod(np.outer(nu, n), 256) / 256)
        expect = F[k1 % 128, k2 % 128] @ C / 128
        # Hermitian part: the output is real
        Fm = F[(-k1) % 128, (-k2) % 128]
        expect = 0.5 * (expect + np.conj(Fm @ C / 128))
        errs.append(relerr(D[k1 % 128, k2 % 128], expect))
    assert max(errs) < 1e-5


def _loss(plan, f, p):
    r = pat.ForwardFn.apply(f, plan) - p
    return torch.sum(r * r)


def test_config4_gradient_finite_differences(config4):
    p, g = config4
    say("config4 FD gradient f64")
    plan = plan_for(g, "f64")
    P = dev(p, "f64")
    f = (0.1 * dev(inputs.random_array((128, 128, 128), 45), "f64")).requires_grad_(True)
    L = _loss(plan, f, P)
    L.backward()
    grad = f.grad.detach()
    rng = inputs.rng(46)
    idx = [tuple(int(v) for v in rng.integers(0, 128, 3)) for _ in range(64)]
    h = 1e-3
    fd, an = [], []
    with torch.no_grad():
        base = f.detach().clone()
        for i in idx:
            fp = base.clone()
            fp[i] += h
            fm = base.clone()
            fm[i] -= h
            lp = torch.sum((plan.forward(fp) - P) ** 2).item()
            lm = torch.sum((plan.forward(fm) - P) ** 2).item()
            fd.append((lp - lm) / (2 * h))
            an.append(grad[i].item())
    fd, an = np.array(fd), np.array(an)
    assert np.abs(fd - an).max() <= 1e-6 * np.abs(an).max()
    # FP32 gradient against the FP64 one
    plan32 = plan_for(g, "f32")
    f32 = f.detach().float().clone().requires_grad_(True)
    _loss(plan32, f32, P.float()).backward()
    g32 = f32.grad.double()
    assert (torch.linalg.vector_norm(g32 - grad) / torch.linalg.vector_norm(grad)).item() < 1e-5


def test_config4_landweber(config4):
    """f <- f + mu A^T (p - A f) from zero, mu = 1 / ||A||^2 (power iteration),
    i.e. gradient steps of size mu/2 on ||A f - p||^2: the loss decreases."""
    p, g = config4
    say("config4 Landweber")
    plan = plan_for(g, "f32")
    P = dev(p)
    plan64 = plan_for(g, "f64")
    v = dev(inputs.random_array((128, 128, 128), 47), "f64")
    for _ in range(20):
        v = plan64.forward_adjoint(plan64.forward(v))
        lam = torch.linalg.vector_norm(v).item()
        v = v / lam
    mu = 1.0 / lam
    f = torch.zeros((128, 128, 128), device=DEV, dtype=torch.float32, requires_grad=True)
    losses = []
    for _ in range(20):
        L = _loss(plan, f, P)
        losses.append(L.item())
        f.grad = None
        L.backward()
        with torch.no_grad():
            f -= 0.5 * mu * f.grad
    losses.append(_loss(plan, f, P).item())
    say(f"  loss {losses[0]:.4e} -> {losses[-1]:.4e}")
    assert all(b < a for a, b in zip(losses, losses[1:]))


def test_gradcheck_tiny_fp64():
    g = dict(n1=6, n2=4, nt=10, nz=6, dx=1.0, dt=0.9, dz=1.1, vs=1.0)
    plan = plan_for(g, "f64")
    f = dev(inputs.random_array((6, 4, 6), 48), "f64").requires_grad_(True)
    assert torch.autograd.gradcheck(lambda x: pat.ForwardFn.apply(x, plan), (f,), eps=1e-6, atol=1e-8)
    p = dev(inputs.random_array((6, 4, 10), 49), "f64").requires_grad_(True)
    assert torch.autograd.gradcheck(lambda x: pat.ReconFn.apply(x, plan), (p,), eps=1e-6, atol=1e-8)


# ---------------------------------------------------------------------------
# config 5

@pytest.fixture(scope="module")
def config5():
    cases = inputs.batched_case(5000)
    plans = [plan_for(g, "f32") for _, g, _ in cases]
    ps = [dev(p) for p, _, _ in cases]
    say("config5 batched launch")
    outs, ws = pat.reconstruct_batched(plans, ps)
    torch.cuda.synchronize()
    return cases, plans, ps, [o.cpu().numpy() for o in outs]


def test_config5_batched_vs_oracle(config5):
    cases, plans, ps, outs = config5
    for (p, g, _), f in zip(cases, outs):
        e = g["n1"]
        if e <= 96:
            err = relerr(f.astype(np.float64), recon.reconstruct(p, g))
        else:
            rng = inputs.rng(e)
            lines = [(e // 2, e // 2), (0, 1)] + [(int(a), int(b)) for a, b in rng.integers(-e // 2, e // 2, (10, 2))]
            err = sampled_line_error(f, p, g, lines)
        say(f"  instance {e}: relL2 {err:.3e}")
        assert err < 1e-5, e


def test_config5_batched_equals_single_calls(config5):
    """The persistent batched launch against one call per instance.  A launch
    over mixed sizes runs the general-radix kernel build, a single call on a
    power-of-two instance the specialised one; the compiler may fuse multiply
    and add differently in the two, so the results agree to float rounding,
    not bit for bit."""
    cases, plans, ps, outs = config5
    for plan, p, f in zip(plans, ps, outs):
        single = plan.reconstruct(p).cpu().numpy()
        assert relerr(f.astype(np.float64), single.astype(np.float64)) < 1e-6
        sizes = (plan.n1, plan.n2, plan.m, plan.nz)
        if not all(s & (s - 1) == 0 for s in sizes):  # same kernel build: identical
            assert np.array_equal(single, f)


def test_batched_classes_join_the_callers_stream(config5):
    """The radix classes of a batch run on streams of their own, forked from
    the caller's stream and joined back into it.  Work that the caller
    enqueues on its stream after the call (copies of the outputs, on a side
    stream, with no device-wide wait in between) must see every class's
    complete output, bit for bit the outputs of the first launch."""
    cases, plans, ps, outs = config5
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        fo = [torch.full((pl.n1, pl.n2, pl.nz), float("nan"), device="cuda") for pl in plans]
        pat.reconstruct_batched(plans, ps, fo)
        copies = [o.clone() for o in fo]
        for o in fo:
            o.fill_(float("nan"))
    s.synchronize()
    for plan, c, f in zip(plans, copies, outs):
        assert np.array_equal(c.cpu().numpy(), f), plan.n1


# ---------------------------------------------------------------------------
# stage a3 alone

@pytest.mark.parametrize("prec,tol", [("f32", 1e-5), ("f64", 1e-9)])
def test_nufft2_lines_against_direct_sums(prec, tol):
    """The grid is built here from eq. (nufft-c) with the oracle's window; the
    interpolation output must equal W T[G](nu) / (n1 n2 nz) from direct sums."""
    g = dict(n1=12, n2=10, nt=40, nz=20, dx=1.0, dt=0.8, dz=1.1, vs=1.2)
    say(f"nufft2_lines {prec}")
    c, K = 2.0, 3.0
    alpha = 0.98 * np.pi * (2 * c - 1)
    nt, nz, m = g["nt"], g["nz"], int(c * g["nt"])
    p = inputs.random_array((12, 10, nt), 50)
    G = recon.transverse_dft(p, g)[: 12 // 2 + 1]                      # half spectrum (h1, n2, nt)
    n = np.arange(nt)
    u = G * (np.exp(alpha * K) / (np.i0(alpha * K) * kb.psi(2 * np.pi * n / nt - np.pi, K, alpha)))
    j = np.arange(m)
    E = np.exp(-2j * np.pi * np.outer(j, n - nt // 2) / m)
    grid = (u.reshape(-1, nt) @ E.T)
    cdt = torch.complex128 if prec == "f64" else torch.complex64
    plan = plan_for(g, prec)
    out = plan.nufft2_lines(torch.from_numpy(grid).to(DEV, cdt)).cpu().numpy()
    full = recon.spectrum(p, g)[: 12 // 2 + 1].reshape(-1, nz) / (12 * 10 * nz)
    # the depth-Nyquist plane holds the mean of the two nodes: compare it to
    # the Hermitian part there, everything else directly
    assert relerr(out[:, 1:nz // 2], full[:, 1:nz // 2]) < tol
    assert relerr(out[:, nz // 2 + 1:], full[:, nz // 2 + 1:]) < tol
    assert np.abs(out[:, 0]).max() == 0.0
