"""Benchmark: full NUFFT-based reconstruction R on one MI355X.

Default workload: 3D planar geometry at full size, 256 x 256 detectors x 512
time samples -> 256^3 volume, 32 seeded uniformly heated balls with
closed-form N-shaped traces plus Gaussian noise (sigma = 1e-3), FP32 compute
(FP64 nodes, phases, weights and deconvolution factors).  One step = one call
of R (all stages a1-a5) on inputs already resident in HBM.

Prints one JSON line: voxels/s, NUFFT points/s, the FP64-path comparison,
the roofline of the dominant kernel (per-kernel HIP events recorded by the
library on the stream its kernels run on), the error against the closed-form
phantom, the adjoint R^T, the stand-alone interpolation and spreading kernels,
the batched launch over sixteen uneven instances and the 128^3 workload (as
further line items), the accuracy-against-time study of the interpolation
methods Section 4 compares (on this workload and on Section 5's circle), and
the CPU oracle timed on a bounded sample of
the same workload.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_HBM_GBS = 8000.0
# Vector FP32 (and FP64) rate without packed FP32 instructions, which the
# build leaves out: 256 CUs x 4 SIMDs x 16 lanes x 2 flop per FMA x 2.4 GHz.
PEAK_VALU_TFLOPS = 78.6
WORKLOADS = {
    # name: (edge n, balls, seed)
    "planar-256x256x512-to-256^3": (256, 32, 1003),
    "planar-128x128x256-to-128^3": (128, 8, 1002),
}


def stage_bytes(name, n1, n2, nt, nz, m, prec):
    """Algorithmic HBM bytes of one launch of each R stage (read + write once)."""
    cs = 16 if prec == "f64" else 8
    rs = cs // 2
    gs = {"f64": 16, "f32": 8, "bf16grid": 4}[prec]
    h1 = n1 // 2 + 1
    lines = h1 * n2
    return {
        "dft_x1": n1 * n2 * nt * rs + lines * nt * cs,
        "dft_x2": 2 * lines * nt * cs,
        "deconv_pad_fft": lines * nt * cs + lines * m * gs,
        "interp": lines * m * gs + lines * nz * cs,
        "idft_z": 2 * lines * nz * cs,
        "idft_x2": 2 * lines * nz * cs,
        "idft_x1_c2r": lines * nz * cs + n1 * n2 * nz * rs,
        "nufft_fused": lines * nt * cs + lines * nz * cs,
    }.get(name)


def stage_flops(name, n1, n2, nt, nz, m, taps=12):
    """Algorithmic flops of one launch of the fused NUFFT stages, per line:
    deconvolution (2 nt), the oversampled FFT (5 m log2 m), per node the tap
    weights by the fitted even/odd polynomials (17 flops per tap pair plus
    one square, the cheapest evaluation of the window transform the
    library has), taps complex-by-real multiply-adds (4 each), phase and weight (8),
    and the depth FFT (5 nz log2 nz).  None for other stages."""
    if name not in ("nufft_fused", "nufft_adjoint_fused"):
        return None
    lines = (n1 // 2 + 1) * n2
    per_node = 17 * (taps // 2) + 1 + 4 * taps + 8
    per_line = 2 * nt + 5 * m * math.log2(m) + per_node * nz + 5 * nz * math.log2(nz)
    return lines * per_line


def roofline_of(name, nbytes, flops, ms):
    """The bound of a kernel is the larger of its HBM time (algorithmic bytes
    at 8 TB/s) and its vector-ALU time (algorithmic flops at the unpacked
    FP32 rate); achieved and peak are stated in that bound's unit."""
    t_hbm = nbytes / (PEAK_HBM_GBS * 1e9)
    t_alu = flops / (PEAK_VALU_TFLOPS * 1e12) if flops else 0.0
    sec = ms * 1e-3
    if t_alu > t_hbm:
        ach = flops / sec / 1e12
        return {"bound": "alu", "achieved": ach, "peak": PEAK_VALU_TFLOPS, "unit": "TFLOP/s",
                "frac": ach / PEAK_VALU_TFLOPS, "hbm_GBs": nbytes / sec / 1e9,
                "hbm_frac": nbytes / sec / 1e9 / PEAK_HBM_GBS}
    ach = nbytes / sec / 1e9
    return {"bound": "hbm", "achieved": ach, "peak": PEAK_HBM_GBS, "unit": "GB/s", "frac": ach / PEAK_HBM_GBS}


def code_of(text):
    """C++ source text without its comments, whitespace runs collapsed."""
    text = re.sub(r"/\*.*?\*/", " ", text, flags=re.S)
    text = re.sub(r"//[^\n]*", "", text)
    return " ".join(text.split())


def kernel_source_hash():
    """Hash of the kernel sources' code: comments and layout do not count, so
    that recorded counters stay valid across edits that change no kernel."""
    h = hashlib.sha256()
    for f in ("kernels.hip", "pat_internal.h"):
        with open(os.path.join(ROOT, "paper_0808_3510_amd", "csrc", f), encoding="utf-8") as fh:
            h.update(code_of(fh.read()).encode())
    return h.hexdigest()[:16]


def time_steps(plan, p, f, steps, torch):
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        plan.reconstruct(p, out=f)
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) / steps * 1e3


def per_stage(plan, p, f, steps, torch):
    """Average kernel time of every stage over `steps` instrumented steps."""
    plan.set_timing(True)
    plan.stage_times()  # drop stale records
    for _ in range(steps):
        plan.reconstruct(p, out=f)
    recs = plan.stage_times()
    plan.set_timing(False)
    acc = {}
    for name, ms in recs:
        acc.setdefault(name, []).append(ms)
    return {k: sum(v) / len(v) for k, v in acc.items()}, {k: len(v) for k, v in acc.items()}


def standalone_stages(n, g, steps, torch, dev, pat):
    """HBM roofline of the interpolation (a3) and spreading kernels run alone
    on full-size line sets: read grid + write node values, or the reverse."""
    res = {}
    for prec in ("f32", "bf16grid"):
        plan = pat.Plan(n, n, g["nt"], g["nz"], g["dx"], g["dt"], g["dz"], g["vs"], precision=prec, device=dev)
        gen = torch.Generator(device=dev).manual_seed(7)
        if prec == "bf16grid":
            grid = torch.randn((plan.lines, plan.m, 2), device=dev, generator=gen).to(torch.bfloat16)
            gbytes = 4
        else:
            grid = torch.randn((plan.lines, plan.m), device=dev, dtype=torch.complex64, generator=gen)
            gbytes = 8
        vals = torch.randn((plan.lines, plan.nz), device=dev, dtype=torch.complex64, generator=gen)
        out = plan.nufft2_lines(grid)
        gout = plan.nufft1_lines(vals)
        torch.cuda.synchronize()
        nbytes = plan.lines * plan.m * gbytes + plan.lines * plan.nz * 8
        plan.set_timing(True)
        plan.stage_times()
        for _ in range(steps):
            plan.nufft2_lines(grid, out=out)
        t_i = [ms for name, ms in plan.stage_times()]
        for _ in range(steps):
            plan.nufft1_lines(vals, out=gout)
        t_s = [ms for name, ms in plan.stage_times()]
        plan.set_timing(False)
        for key, ts in (("interp", t_i), ("spread", t_s)):
            avg = sum(ts) / len(ts)
            gbs = nbytes / (avg * 1e-3) / 1e9
            res[f"{key}_{prec}"] = {"avg_launch_ms": avg, "algorithmic_bytes_per_launch": nbytes,
                                    "achieved_GBs": gbs, "frac_of_hbm_peak": gbs / PEAK_HBM_GBS,
                                    "launches_timed": len(ts)}
        del plan
    return res


def batched_and_small(steps, torch, dev, pat, inputs, np, keep=None):
    """The other throughput configurations: sixteen uneven instances (plane
    edges 64 .. 184, time samples twice the edge, depth the edge) in one
    persistent launch per stage, against one R call per instance; and the
    128^2 x 256 -> 128^3 workload."""
    out = {}
    cases = inputs.batched_case(5000, dtype=np.float32)
    plans, ps = [], []
    for p_np, g, _ in cases:
        plans.append(pat.Plan(g["n1"], g["n2"], g["nt"], g["nz"], g["dx"], g["dt"], g["dz"], g["vs"],
                              precision="f32", device=dev))
        ps.append(torch.from_numpy(p_np).to(dev))
    vox = sum(pl.n1 * pl.n2 * pl.nz for pl in plans)
    outs, ws = pat.reconstruct_batched(plans, ps)
    singles = [pl.reconstruct(p) for pl, p in zip(plans, ps)]
    for _ in range(2):
        pat.reconstruct_batched(plans, ps, outs, ws)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        pat.reconstruct_batched(plans, ps, outs, ws)
    torch.cuda.synchronize()
    t_b = (time.perf_counter() - t0) / steps * 1e3
    t0 = time.perf_counter()
    for _ in range(steps):
        for pl, p, f in zip(plans, ps, singles):
            pl.reconstruct(p, out=f)
    torch.cuda.synchronize()
    t_s = (time.perf_counter() - t0) / steps * 1e3
    dev_rel = max(float((torch.linalg.vector_norm(o - s) / torch.linalg.vector_norm(s)).item())
                  for o, s in zip(outs, singles))
    if keep is not None:
        keep["batched"] = [(p_np, g, o.cpu().numpy()) for (p_np, g, _), o in zip(cases, outs)]
    out["batched_16_uneven"] = {
        "edges": [pl.n1 for pl in plans], "total_voxels": vox, "ms_per_launch_set": t_b,
        "voxels_per_s": vox / (t_b * 1e-3), "sequential_single_calls_ms": t_s,
        "speedup_over_single_calls": t_s / t_b, "max_relL2_batched_vs_single": dev_rel}
    del plans, ps, outs, ws, singles
    p_np, g, _ = inputs.planar_case(128, 8, 1002, noise=1e-3)
    plan = pat.Plan(128, 128, g["nt"], g["nz"], g["dx"], g["dt"], g["dz"], g["vs"], precision="f32", device=dev)
    p = torch.from_numpy(p_np).to(dev, torch.float32)
    f = plan.reconstruct(p)
    for _ in range(3):
        plan.reconstruct(p, out=f)
    ms = time_steps(plan, p, f, steps, torch)
    out["planar-128x128x256-to-128^3"] = {"ms_per_step": ms, "voxels_per_s": 128 ** 3 / (ms * 1e-3)}
    if keep is not None:
        keep["planar128"] = (p_np, g, f.cpu().numpy())
    return out


# Kaiser-Bessel over the oversampling factors of Fig. 5.  c = 1 is outside
# the window's range (deconvolving on [-pi, pi] needs alpha > pi, Section 3.2
# bounds alpha below pi (2c - 1)); past c = 8 the 2cK taps are capped at 64,
# so K shrinks.
# Fig. 5's oversampling factors and one step past them; 2cK <= 64 taps
KB_SWEEP = [("kb", 2.0, 3.0), ("kb", 4.0, 3.0), ("kb", 8.0, 3.0), ("kb", 16.0, 2.0), ("kb", 32.0, 1.0)]
C_SWEEP = (1, 2, 4, 8, 16, 32)


def interpolation_study(p_np, g, steps, torch, dev, pat, np):
    """Accuracy against time for the ways of evaluating the nonuniform sums
    that Section 4 compares (its Table 1 and Fig. 5), on this workload: each
    method's R time and its relative l2 distance to the FP64 Kaiser-Bessel
    reconstruction (c = 2, K = 3, which is within ~1e-11 of the direct sums)."""
    n, nt, nz = g["n1"], g["nt"], g["nz"]

    def plan_of(kind, c, prec, K=3.0):
        return pat.Plan(n, n, nt, nz, g["dx"], g["dt"], g["dz"], g["vs"], c=c, K=K, precision=prec, device=dev,
                        interp=kind)

    ref_plan = plan_of("kb", 2.0, "f64")
    ref = ref_plan.reconstruct(torch.from_numpy(p_np).to(dev, torch.float64))
    del ref_plan
    p32 = torch.from_numpy(p_np).to(dev, torch.float32)
    rows = []
    for kind, c, K, fused in [(k, c, K, True) for k, c, K in KB_SWEEP] + [("kb", 2.0, 3.0, False),
                                                                       ("sinc", 2.0, 3.0, False)] + \
            [(k, float(c), 3.0, False) for k in ("linear", "nearest") for c in C_SWEEP]:
        plan = plan_of(kind, c, "f32", K)
        if fused and not plan.fusable:
            fused = False  # (grid lines beyond the fused kernels' LDS share)
        plan.set_fused(fused)
        f = plan.reconstruct(p32)
        for _ in range(2):
            plan.reconstruct(p32, out=f)
        ms = time_steps(plan, p32, f, steps, torch)
        err = float((torch.linalg.vector_norm(f.double() - ref) / torch.linalg.vector_norm(ref)).item())
        row = {"method": kind, "c": c, "kernels": "fused" if fused else "staged", "ms": ms,
               "relL2_vs_reference": err}
        if kind == "kb":
            row["K"] = K
        rows.append(row)
        del plan, f
    return {"reference": "FP64 Kaiser-Bessel NUFFT, c = 2, K = 3", "rows": rows}


def circle_experiment(steps, torch, dev, pat, inputs, np):
    """Section 5's setting: the circular object, 512 line detectors on [0, 1),
    data on (0, 1)^2 (nt = nz = 512).  Per evaluation method (Table 1 and the
    c sweep of Fig. 5): R time and relative l2 distance to the direct Fourier
    reconstruction f-dagger, stood in for by the FP64 Kaiser-Bessel R (c = 2,
    K = 3: within 1e-11 of the direct sums).  Also the error with Gaussian
    noise of variance 20 % of the data maximum, and against the phantom."""
    p0, g, (x0, y0, a) = inputs.circle_case(512, 1006, 0.0)
    pn, _, _ = inputs.circle_case(512, 1006, 0.2)
    n = g["n1"]

    def plan_of(kind, c, prec, K=3.0):
        return pat.Plan(n, 1, g["nt"], g["nz"], g["dx"], g["dt"], g["dz"], g["vs"], c=c, K=K, precision=prec,
                        device=dev, interp=kind)

    ref = plan_of("kb", 2.0, "f64").reconstruct(torch.from_numpy(p0).to(dev, torch.float64))
    phantom = torch.from_numpy(inputs.circle_image(x0, y0, a, n, g["nz"], g["dx"], g["dz"])).to(dev)
    p32 = torch.from_numpy(p0).to(dev, torch.float32)
    rows = []
    for kind, c, K in KB_SWEEP + [("sinc", 2.0, 3.0)] + [(k, float(c), 3.0) for k in ("linear", "nearest")
                                                         for c in C_SWEEP]:
        plan = plan_of(kind, c, "f32", K)
        f = plan.reconstruct(p32)
        for _ in range(2):
            plan.reconstruct(p32, out=f)
        ms = time_steps(plan, p32, f, steps, torch)
        err = float((torch.linalg.vector_norm(f.double() - ref) / torch.linalg.vector_norm(ref)).item())
        row = {"method": kind, "c": c, "ms": ms, "relL2_vs_direct": err}
        if kind == "kb":
            row["K"] = K
        rows.append(row)
    kb = plan_of("kb", 2.0, "f32")
    fn = kb.reconstruct(torch.from_numpy(pn).to(dev, torch.float32)).double()
    f0 = kb.reconstruct(p32).double()
    rel = lambda u, v: float((torch.linalg.vector_norm(u - v) / torch.linalg.vector_norm(v)).item())
    return {"geometry": "2D, 512 line detectors, nt = nz = 512, dx = dt = dz = 1/512",
            "circle": {"x0": x0, "y0": y0, "a": a}, "rows": rows,
            "kb_noisy_relL2_vs_noiseless_direct": rel(fn, ref),
            "kb_relL2_vs_phantom": rel(f0, phantom)}


def cpu_baseline(p_np, g, f_gpu, budget_s, np):
    """The oracle (as it stands) on a bounded sample: its transverse DFT in
    full, plus its direct nonuniform DFT sums on a random sample of lines,
    extrapolated to all n1*n2 lines of its full-spectrum reconstruction."""
    from oracle import recon
    try:
        from threadpoolctl import threadpool_info
        blas_threads = max([d.get("num_threads", 1) for d in threadpool_info()] + [1])
    except Exception:  # pragma: no cover
        blas_threads = 1
    n1, n2, nz = g["n1"], g["n2"], g["nz"]
    rng = np.random.default_rng(12345)

    def draw(k):
        return [(int(rng.integers(-n1 // 2, n1 // 2)), int(rng.integers(-n2 // 2, n2 // 2))) for _ in range(k)]

    t0 = time.perf_counter()
    recon.transverse_dft(p_np, g)
    t_fft = time.perf_counter() - t0
    # calibrate the per-line cost, then spend the budget in one call
    probe = draw(16)
    t0 = time.perf_counter()
    recon.spectrum_lines(p_np, g, probe)
    per_line = max(time.perf_counter() - t0 - t_fft, 1e-6) / len(probe)
    lines = draw(max(16, min(n1 * n2, int(budget_s / per_line))))
    t0 = time.perf_counter()
    ora = recon.spectrum_lines(p_np, g, lines)
    t_lines = time.perf_counter() - t0 - t_fft
    per_line = t_lines / len(lines)
    t0 = time.perf_counter()
    np.fft.ifftn(np.zeros((n1, n2, nz), dtype=np.complex128))
    t_inv = time.perf_counter() - t0
    t_full = t_fft + per_line * n1 * n2 + t_inv
    # parity of the GPU output on sampled lines: the real output's spectrum is
    # the Hermitian part (F[k, l] + conj F[-k, -l]) / 2 of the oracle's
    k = min(64, len(lines))
    mir = recon.spectrum_lines(p_np, g, [(-a, -b) for a, b in lines[:k]])
    D = np.fft.fftn(f_gpu.astype(np.float64))
    lneg = (-np.arange(nz)) % nz
    got = np.array([D[a % n1, b % n2, :] for a, b in lines[:k]])
    exp = 0.5 * (ora[:k] + np.conj(mir[:, lneg]))
    rel = float(np.linalg.norm(got - exp) / np.linalg.norm(exp))
    return {
        "value": n1 * n2 * nz / t_full, "unit": "voxels/s", "cores": int(blas_threads), "kind": "oracle",
        "sample": (f"oracle transverse DFT in full ({t_fft:.2f} s) + its direct NDFT sums on {len(lines)} "
                   f"random lines of {n1 * n2} ({t_lines:.1f} s) + inverse FFT ({t_inv:.2f} s), "
                   f"extrapolated to all lines; exponentials single-threaded numpy, products on "
                   f"{blas_threads} BLAS threads"),
        "est_full_seconds": t_full,
        "sample_relL2_gpu_vs_oracle": rel,
        "host_cpus": len(os.sched_getaffinity(0)),
    }


def oracle_parity(p_np, g, outputs, keep, np):
    """Part of the oracle leg: the GPU outputs against the oracle.
    * each precision's R at full size on 64 sampled lines (and their mirrors),
      by the oracle's direct sums there;
    * every instance of the batched launch on 8 sampled lines;
    * one full oracle reconstruction of the 128^2 x 256 -> 128^3 workload,
      timed on the host cores, against the GPU's output in full."""
    from oracle import recon

    def sampled(f_gpu, p, gg, lines):
        n1, n2, nz = gg["n1"], gg["n2"], gg["nz"]
        ora = recon.spectrum_lines(p, gg, lines)
        mir = recon.spectrum_lines(p, gg, [(-a, -b) for a, b in lines])
        D = np.fft.fftn(f_gpu.astype(np.float64).reshape(n1, n2, nz))
        lneg = (-np.arange(nz)) % nz
        got = np.array([D[a % n1, b % n2, :] for a, b in lines])
        exp = 0.5 * (ora + np.conj(mir[:, lneg]))
        return float(np.linalg.norm(got - exp) / np.linalg.norm(exp))

    res = {}
    rng = np.random.default_rng(2024)
    n1, n2 = g["n1"], g["n2"]
    lines = [(int(rng.integers(-n1 // 2, n1 // 2)), int(rng.integers(-n2 // 2, n2 // 2))) for _ in range(64)]
    res["sampled_lines_relL2_vs_oracle"] = {k: sampled(v, p_np, g, lines) for k, v in outputs.items()}
    res["sampled_lines"] = len(lines)
    if "batched" in keep:
        per = []
        for p, gg, out in keep["batched"]:
            e = gg["n1"]
            ls = [(e // 2, e // 2), (0, 1)] + [(int(rng.integers(-e // 2, e // 2)), int(rng.integers(-e // 2, e // 2)))
                                               for _ in range(6)]
            per.append({"edge": e, "relL2_vs_oracle_8_lines": sampled(out, p, gg, ls)})
        res["batched_16_uneven_per_instance"] = per
    if "planar128" in keep:
        p, gg, f128 = keep["planar128"]
        t0 = time.perf_counter()
        ref = recon.reconstruct(p, gg)
        t = time.perf_counter() - t0
        res["full_oracle_planar-128x128x256-to-128^3"] = {
            "seconds": t, "voxels_per_s": 128 ** 3 / t,
            "gpu_f32_relL2_vs_oracle": float(np.linalg.norm(f128 - ref) / np.linalg.norm(ref))}
    return res


KERNEL_OF_STAGE = {
    # library stage name -> kernel symbol prefixes in the profiler's output
    "nufft_fused": ("void pat::k_line_nufft2<", "void pat::k_line_nufft2_pipe<", "void pat::k_line_nufft2_pipe_c<",
                    "void pat::k_line_nufft2_mirror<"),
    "nufft_adjoint_fused": ("void pat::k_line_nufft1<", "void pat::k_line_nufft1_c<", "void pat::k_line_nufft1_w<"),
    "dft_x1": ("void pat::k_tr_x1_r2c<", "void pat::k_tr_x1_pipe<"),
    "dft_x2": ("void pat::k_tr_x2<", "void pat::k_tr_x2_pipe<"),
    "idft_x1_c2r": ("void pat::k_tr_c2r_k1<", "void pat::k_tr_c2r_pipe<"),
    "interp": ("void pat::k_line_interp<", "void pat::k_line_interp_stream<"),
    "spread": ("void pat::k_line_spread<", "void pat::k_line_spread_w<"),
}


def traffic_of(stage, workload, precision):
    """HBM bytes per launch of a stage from profiles/traffic.json, or None
    when there is none or the kernel sources changed since it was taken."""
    tfile = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(tfile):
        return None
    with open(tfile) as fh:
        t = json.load(fh)
    key = f"{stage}:{workload}:{precision}"
    if t.get("kernel_source") != kernel_source_hash():
        return None
    return t.get("bytes_per_launch", {}).get(key)


def traffic_from_counters(fetch_csv, write_csv, copy_bytes, workload, precision, out_path=None):
    """HBM bytes per launch of each stage from two rocprofv3 --pmc runs of
    `bench.py --calibrate-copy copy_bytes` (FETCH_SIZE, then WRITE_SIZE; both
    in KiB per dispatch).  Each counter is scaled by what it reads for the
    plain copy of copy_bytes that the run starts with (fetch: the copy's
    source; write: the fill that creates it), and the result is stored in
    profiles/traffic.json with the hash of the kernel sources it belongs to."""
    import csv

    def per_dispatch(path, counter):
        # counter value of each dispatch (summed over the GPU's blocks)
        acc, name_grid = {}, {}
        with open(path) as fh:
            for r in csv.DictReader(fh):
                if r["Counter_Name"] != counter:
                    continue
                d = int(r.get("Dispatch_Id", r.get("Correlation_Id", "0")))
                acc[d] = acc.get(d, 0.0) + float(r["Counter_Value"])
                name_grid[d] = (r["Kernel_Name"], int(r["Grid_Size"]))
        return acc, name_grid

    fetch, fnames = per_dispatch(fetch_csv, "FETCH_SIZE")
    write, wnames = per_dispatch(write_csv, "WRITE_SIZE")

    def largest(vals, names, pred):
        # the largest copy/fill dispatch (the calibration one)
        best = None
        for d, v in vals.items():
            if pred(names[d][0]) and (best is None or v > best):
                best = v
        return best

    kib = copy_bytes / 1024.0
    f_copy = largest(fetch, fnames, lambda n: "copy" in n.lower() or "elementwise" in n.lower())
    w_fill = largest(write, wnames, lambda n: "fill" in n.lower() or "elementwise" in n.lower())
    f_scale, w_scale = kib / f_copy, kib / w_fill
    out = {"kernel_source": kernel_source_hash(), "copy_bytes": copy_bytes,
           "fetch_scale": f_scale, "write_scale": w_scale, "bytes_per_launch": {}, "raw_kib_per_launch": {}}
    # The two runs make the same dispatches, so FETCH and WRITE pair by
    # dispatch id.  A stage's dispatches are grouped by kernel, grid and size
    # class (the transverse kernels serve R and R^T on lines of nt and of nz
    # samples; their persistent forms launch the same grid for both), and the
    # key carries the group when a stage has several.
    for stage, prefixes in KERNEL_OF_STAGE.items():
        groups = {}
        for d, (name, grid) in fnames.items():
            if d not in write or not name.startswith(prefixes):
                continue
            size_class = int(round(math.log2(max(fetch[d], 1.0))))
            groups.setdefault((name, grid, size_class), []).append(d)
        for (name, grid, sc), ds in sorted(groups.items(), key=lambda kv: (kv[0][2], kv[0][1])):
            f_avg = sum(fetch[d] for d in ds) / len(ds)
            w_avg = sum(write[d] for d in ds) / len(ds)
            short = name.split("(")[0].replace("void ", "").replace("pat::", "")
            key = f"{stage}:{workload}:{precision}" + (f"[{short},grid={grid},class={sc}]" if len(groups) > 1
                                                       else "")
            out["raw_kib_per_launch"][key] = {"fetch": f_avg, "write": w_avg, "dispatches": len(ds),
                                              "grid_threads": grid, "kernel": name}
            out["bytes_per_launch"][key] = 1024.0 * (f_avg * f_scale + w_avg * w_scale)
    path = out_path or os.path.join(ROOT, "profiles", "traffic.json")
    with open(path, "w") as fh:
        json.dump(out, fh, indent=1, sort_keys=True)
    print(json.dumps(out, indent=1, sort_keys=True))
    return out


def counters_summary(counter_csvs, trace_csv, workload):
    """Markdown table of the SQ counters of each stage's kernels from
    rocprofv3 --pmc runs (one csv per pass) and the kernel durations from a
    --kernel-trace run of the same command.  Counters are summed over the
    GPU per dispatch and averaged over the dispatches of one kernel and grid.
    VALU busy is the share of SIMD cycles that issue VALU: 4 cycles per wave
    instruction (64 lanes on a 16-lane SIMD) over 1024 SIMDs at 2.4 GHz."""
    import csv

    def key_of(name):
        for stage, prefixes in KERNEL_OF_STAGE.items():
            if name.startswith(prefixes):
                return stage
        return None

    vals = {}  # (kernel, grid) -> counter -> [per-dispatch sums]
    for path in counter_csvs:
        acc, names = {}, {}
        with open(path) as fh:
            for r in csv.DictReader(fh):
                d = int(r.get("Dispatch_Id", r.get("Correlation_Id", "0")))
                acc[(d, r["Counter_Name"])] = acc.get((d, r["Counter_Name"]), 0.0) + float(r["Counter_Value"])
                names[d] = (r["Kernel_Name"], int(r["Grid_Size"]))
        for (d, c), v in acc.items():
            vals.setdefault(names[d], {}).setdefault(c, []).append(v)
    dur = {}
    with open(trace_csv) as fh:
        for r in csv.DictReader(fh):
            k = (r["Kernel_Name"], int(r.get("Grid_Size", r.get("Grid_Size_X", 0)) or 0))
            dur.setdefault(k, []).append((int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) * 1e-9)
    rows = []
    for (name, grid), cs in sorted(vals.items()):
        stage = key_of(name)
        if stage is None:
            continue
        avg = {c: sum(v) / len(v) for c, v in cs.items()}
        ds = dur.get((name, grid)) or [t for (n, _), ts in dur.items() if n == name for t in ts]
        sec = sum(ds) / len(ds) if ds else None
        waves = avg.get("SQ_WAVES")
        per_wave = lambda c: f"{avg[c] / waves:.0f}" if c in avg and waves else "-"  # noqa: E731
        busy = (4 * avg["SQ_INSTS_VALU"] / (1024 * 2.4e9 * sec)) if sec and "SQ_INSTS_VALU" in avg else None
        lds_conf = (avg["SQ_LDS_BANK_CONFLICT"] / avg["SQ_ACTIVE_INST_LDS"]
                    if avg.get("SQ_ACTIVE_INST_LDS") and "SQ_LDS_BANK_CONFLICT" in avg else None)
        rows.append((stage, name.split("(")[0].replace("void ", ""), grid, len(next(iter(cs.values()))),
                     sec * 1e6 if sec else None, waves, per_wave("SQ_INSTS_VALU"), per_wave("SQ_INSTS_LDS"),
                     per_wave("SQ_INSTS_SALU"), per_wave("SQ_INSTS_VMEM_RD"), per_wave("SQ_INSTS_VMEM_WR"), busy,
                     lds_conf))
    lines = [f"Counters per dispatch, workload {workload}:", "",
             "| stage | kernel | grid | dispatches | avg us | waves | VALU/wave | LDS/wave | SALU/wave | "
             "VMEM rd/wave | VMEM wr/wave | VALU busy | LDS conflict cycles per LDS cycle |",
             "|---|---|---:|---:|---:|---:|---:|---:|---:|---:|---:|---:|---:|"]
    for r in rows:
        lines.append("| " + " | ".join([r[0], f"`{r[1]}`", str(r[2]), str(r[3]),
                                        f"{r[4]:.1f}" if r[4] else "-", f"{r[5]:.0f}" if r[5] else "-",
                                        *r[6:11], f"{r[11]:.2f}" if r[11] is not None else "-",
                                        f"{r[12]:.2f}" if r[12] is not None else "-"]) + " |")
    text = "\n".join(lines)
    print(text)
    return text


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--workload", default="planar-256x256x512-to-256^3", choices=sorted(WORKLOADS))
    ap.add_argument("--precision", default="f32", choices=["f32", "f64", "bf16grid"])
    ap.add_argument("--no-fp64", action="store_true", help="skip the FP64-path comparison")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extra", action="store_true",
                    help="skip the batched and 128^3 workloads and the interpolation-method studies")
    ap.add_argument("--cpu-budget", type=float, default=15.0, help="seconds of oracle work in the sample")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="BYTES",
                    help="run one plain device-to-device copy of BYTES bytes first (scale for HBM counters)")
    ap.add_argument("--copy-ref", type=int, default=0, metavar="BYTES",
                    help="time a plain device copy and fill of BYTES (the HBM reference) and exit")
    ap.add_argument("--counters-from", nargs="+", metavar="CSV",
                    help="print the SQ counter table from rocprofv3 --pmc csvs; the last csv is the "
                         "--kernel-trace csv of the same command (no GPU work)")
    ap.add_argument("--traffic-from", nargs=3, metavar=("FETCH_CSV", "WRITE_CSV", "COPY_BYTES"),
                    help="write profiles/traffic.json from two rocprofv3 --pmc counter files (no GPU work)")
    args = ap.parse_args()
    if args.counters_from:
        counters_summary(args.counters_from[:-1], args.counters_from[-1], args.workload)
        return
    if args.traffic_from:
        traffic_from_counters(args.traffic_from[0], args.traffic_from[1], int(args.traffic_from[2]), args.workload,
                              args.precision)
        return
    if args.gpus != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path "
              f"(asked for --gpus {args.gpus}).", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_0808_3510_amd import inputs, pat

    n, nballs, seed = WORKLOADS[args.workload]
    print(f"[bench] generating {args.workload} (seed {seed})", file=sys.stderr, flush=True)
    p_np, g, balls = inputs.planar_case(n, nballs, seed, noise=1e-3)
    nt, nz = g["nt"], g["nz"]
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    if args.copy_ref > 0:
        # the practical HBM rate: torch's copy (read + write) and fill (write)
        a = torch.ones(args.copy_ref // 4, dtype=torch.float32, device=dev)
        b = torch.empty_like(a)
        res = {}
        for name, fn, nbytes in (("copy", lambda: b.copy_(a), 2 * args.copy_ref),
                                 ("fill", lambda: b.fill_(1.0), args.copy_ref)):
            for _ in range(3):
                fn()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            for _ in range(20):
                fn()
            e1.record()
            torch.cuda.synchronize()
            sec = e0.elapsed_time(e1) * 1e-3 / 20
            res[name] = {"bytes": nbytes, "us": sec * 1e6, "GBs": nbytes / sec / 1e9}
        print(json.dumps({"copy_reference": res}))
        return
    if args.calibrate_copy > 0:
        src = torch.ones(args.calibrate_copy // 4, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    def run_prec(prec, cutoff=0.0, repeats=1):
        """Plan, output, wall ms per step (the best of `repeats` timed loops of
        args.steps steps), per-stage kernel ms and launch counts."""
        plan = pat.Plan(n, n, nt, nz, g["dx"], g["dt"], g["dz"], g["vs"], precision=prec, device=dev,
                        cutoff=cutoff)
        dt = torch.float64 if prec == "f64" else torch.float32
        p = torch.from_numpy(p_np).to(device=dev, dtype=dt)
        f = torch.empty((n, n, nz), dtype=dt, device=dev)
        for _ in range(args.warmup):
            plan.reconstruct(p, out=f)
        ms = min(time_steps(plan, p, f, args.steps, torch) for _ in range(repeats))
        stages, counts = per_stage(plan, p, f, args.steps, torch)
        return plan, f, ms, stages, counts

    print(f"[bench] timing {args.precision}", file=sys.stderr, flush=True)
    plan, f, ms, stages, counts = run_prec(args.precision)
    vox = n * n * nz
    value = vox / (ms * 1e-3)
    m = plan.m
    dom = max(stages, key=stages.get)
    dom_ms = stages[dom]
    dom_bytes = stage_bytes(dom, n, n, nt, nz, m, args.precision)
    dom_flops = stage_flops(dom, n, n, nt, nz, m)
    roof = roofline_of(dom, dom_bytes, dom_flops, dom_ms)
    nufft_ms = sum(stages.get(k, 0.0) for k in ("deconv_pad_fft", "interp", "nufft_fused"))
    f_host = f.cpu().numpy()
    phantom = inputs.ball_volume(balls, n, n, nz, g["dx"], g["dz"])
    rel_phantom = float(np.linalg.norm(f_host - phantom) / np.linalg.norm(phantom))

    traffic = traffic_of(dom, args.workload, args.precision)

    out = {
        "metric": "voxels/s per full reconstruction; NUFFT pts/s; FP32 vs FP64 at relL2<=1e-5",
        "value": value,
        "unit": "voxels/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {"f32": "f32", "f64": "f64", "bf16grid": "f32 (bf16 grid storage)"}[args.precision],
        "data": "synthetic",
        "config": {"workload": args.workload, "detectors": [n, n], "nt": nt, "nz": nz, "volume": [n, n, nz],
                   "balls": nballs, "seed": seed, "noise_sigma": 1e-3, "c": 2.0, "K": 3.0, "taps": 12,
                   "precision": args.precision},
        "nufft_pts_per_s": vox / (nufft_ms * 1e-3) if nufft_ms > 0 else None,
        "stage_ms": stages,
        "relL2_vs_phantom": rel_phantom,
        "roofline": dict(roof, kernel=dom, traffic=traffic, algorithmic_bytes_per_launch=dom_bytes,
                         algorithmic_flops_per_launch=dom_flops, avg_launch_ms=dom_ms,
                         launches_timed=counts[dom]),
    }
    # adjoint R^T on the same plan (the gradient of R)
    q = f.detach().clone()
    pt = torch.empty((n, n, nt), dtype=f.dtype, device=dev)
    for _ in range(args.warmup):
        plan.reconstruct_adjoint(q, out=pt)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        plan.reconstruct_adjoint(q, out=pt)
    torch.cuda.synchronize()
    out["adjoint_ms_per_step"] = (time.perf_counter() - t0) / args.steps * 1e3
    plan.set_timing(True)
    plan.stage_times()
    for _ in range(args.steps):
        plan.reconstruct_adjoint(q, out=pt)
    acc = {}
    for name, ms_ in plan.stage_times():
        acc.setdefault(name, []).append(ms_)
    plan.set_timing(False)
    out["adjoint_stage_ms"] = {k: sum(v) / len(v) for k, v in acc.items()}
    if "nufft_adjoint_fused" in out["adjoint_stage_ms"]:
        adj_ms = out["adjoint_stage_ms"]["nufft_adjoint_fused"]
        out["adjoint_roofline"] = dict(
            roofline_of("nufft_adjoint_fused", stage_bytes("nufft_fused", n, n, nt, nz, m, args.precision),
                        stage_flops("nufft_adjoint_fused", n, n, nt, nz, m), adj_ms),
            kernel="nufft_adjoint_fused", avg_launch_ms=adj_ms,
            traffic=traffic_of("nufft_adjoint_fused", args.workload, args.precision))
    del plan, f, q, pt
    # R with the smooth cut-off of the partial-data model (eps = 4 steps):
    # the weights are applied inside the first transverse pass
    # (a secondary figure beside the headline: the best of three timed loops,
    # and the sum of its stages' kernel times)
    planc, fc, msc, stc, _ = run_prec(args.precision, cutoff=4.0, repeats=3)
    out["with_cutoff_eps4"] = {"ms_per_step": msc, "stage_sum_ms": sum(stc.values()), "dft_x1_ms": stc.get("dft_x1"),
                               "dft_x1_ms_without": stages.get("dft_x1")}
    del planc, fc
    out["standalone"] = standalone_stages(n, g, args.steps, torch, dev, pat)
    keep = {}
    outputs = {args.precision: f_host}
    if args.precision == "f32":
        # the bf16-grid option on the same workload (staged kernels: the option
        # concerns the stored grid)
        print("[bench] timing bf16grid", file=sys.stderr, flush=True)
        planb, fb, msb, stb, _ = run_prec("bf16grid")
        fbh = fb.cpu().numpy()
        outputs["bf16grid"] = fbh
        out["bf16grid_path"] = {"ms_per_step": msb, "value": vox / (msb * 1e-3), "stage_ms": stb,
                                "relL2_vs_f32": float(np.linalg.norm(fbh - f_host) / np.linalg.norm(f_host))}
        del planb, fb
    if not args.no_extra:
        print("[bench] batched and 128^3 workloads", file=sys.stderr, flush=True)
        out["other_workloads"] = batched_and_small(args.steps, torch, dev, pat, inputs, np, keep)
        print("[bench] interpolation methods", file=sys.stderr, flush=True)
        out["interpolation_study"] = interpolation_study(p_np, g, max(3, args.steps // 4), torch, dev, pat, np)
        print("[bench] circle experiment", file=sys.stderr, flush=True)
        out["circle_experiment"] = circle_experiment(args.steps, torch, dev, pat, inputs, np)
    if not args.no_fp64 and args.precision != "f64":
        print("[bench] timing f64", file=sys.stderr, flush=True)
        plan64, f64, ms64, st64, _ = run_prec("f64")
        f64h = f64.cpu().numpy()
        outputs["f64"] = f64h
        out["fp64_path"] = {"ms_per_step": ms64, "value": vox / (ms64 * 1e-3), "stage_ms": st64,
                            "speedup_fp32_over_fp64": ms64 / ms,
                            "relL2_fp32_vs_fp64_gpu": float(np.linalg.norm(f_host - f64h) / np.linalg.norm(f64h)),
                            "relL2_vs_phantom": float(np.linalg.norm(f64h - phantom) / np.linalg.norm(phantom))}
        del plan64, f64
    if not args.no_cpu_baseline:
        print("[bench] cpu baseline (oracle sample)", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(p_np, g, f_host, args.cpu_budget, np)
        print("[bench] oracle parity", file=sys.stderr, flush=True)
        out["oracle_parity"] = oracle_parity(p_np, g, outputs, keep, np)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
