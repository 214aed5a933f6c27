"""C ABI checks that need no GPU: the library loads, exports every declared
symbol, and the host-only plan creation validates its geometry."""
import ctypes

import numpy as np

import pytest

from paper_0808_3510_amd import pat


def test_library_exports_every_header_symbol():
    L = pat.lib()
    names = pat.header_functions()
    assert len(names) >= 15
    for n in names:
        assert hasattr(L, n), n
    # and the binding wraps each of them under the same name
    for n in names:
        assert callable(getattr(pat, n)), n


def _geom(**kw):
    base = dict(n1=16, n2=16, nt=32, nz=16, dx=1.0, dt=1.0, dz=1.0, vs=1.0, c=2.0, K=3.0, alpha=0.0,
                precision="f32")
    base.update(kw)
    return pat.make_geometry(**base)


def test_valid_plan_sizes():
    ptr = pat.pat_plan_create(_geom())
    try:
        tb, wb = pat.pat_plan_sizes(ptr)
        lines = 9 * 16
        # G (lines x nt) + grid (lines x 2nt) + F (lines x nz), complex64
        assert wb >= lines * (32 + 64 + 16) * 8
        assert tb > 0
    finally:
        pat.pat_plan_destroy(ptr)


@pytest.mark.parametrize("kw,status", [
    (dict(nt=31), 1), (dict(nz=0), 1), (dict(n1=15), 1), (dict(dx=0.0), 1), (dict(vs=-1.0), 1),
    (dict(c=1.0), 1), (dict(c=1.25, nt=30), 1), (dict(K=0.0), 1), (dict(K=1.3), 1),
    (dict(alpha=3.0), 1), (dict(alpha=20.0), 1), (dict(precision=7), 1),
    (dict(n1=58), 2),            # 29 is not a supported FFT radix
    (dict(n1=8192, n2=2), 2), (dict(nt=16384), 2), (dict(K=32.0, c=2.0), 1),
    (dict(nz=8192, precision="f64"), 2),   # a double depth line pair exceeds LDS
    (dict(c=32.0, K=1.0, nt=512, nz=64, precision="f64"), 2),  # a 16384-point double grid line exceeds LDS
    (dict(interp=7), 1), (dict(c=1.0, interp="kb"), 1), (dict(c=0.5, interp="linear"), 1),
    (dict(cutoff=-1.0), 1), (dict(cutoff=8.5, n1=64, n2=64, nt=64), 1), (dict(cutoff=float("nan")), 1),
    (dict(cutoff=4.5), 1),       # 4 eps exceeds the 16 detectors
    (dict(cutoff=3.0, n2=1, nt=8), 1),     # ... or the 8 time samples (2D)
])
def test_invalid_geometry_is_rejected(kw, status):
    with pytest.raises(pat.PatError) as ei:
        pat.pat_plan_create(_geom(**kw))
    assert ei.value.status == status
    assert pat.pat_last_error()


def test_2d_requires_unit_second_axis():
    g = _geom(n2=1)
    assert g.ndim == 2
    ptr = pat.pat_plan_create(g)
    pat.pat_plan_destroy(ptr)
    g.nx[1] = 4
    with pytest.raises(pat.PatError):
        pat.pat_plan_create(g)


def test_calls_before_upload_and_null_pointers_fail_cleanly():
    ptr = pat.pat_plan_create(_geom())
    try:
        with pytest.raises(pat.PatError) as ei:
            pat.pat_reconstruct(ptr, 16, 1 << 40, 16, 1 << 40, 16, 1 << 40, None)
        assert ei.value.status == 3  # tables not uploaded
        L = pat.lib()
        assert L.pat_reconstruct(None, None, 0, None, 0, None, 0, None) == 1
        assert L.pat_plan_sizes(None, None, None) == 1
        assert L.pat_plan_create(None, None) == 1
        assert pat.pat_status_string(2) == "PAT_ERR_UNSUPPORTED"
        assert L.pat_plan_upload(ptr, ctypes.c_void_p(8), 1 << 30, None) == 1  # misaligned
        tb = pat.pat_plan_sizes(ptr)[0]
        assert L.pat_plan_upload(ptr, ctypes.c_void_p(256), tb - 1, None) == 3  # short table buffer
    finally:
        pat.pat_plan_destroy(ptr)


def test_batched_size_validation():
    p1 = pat.pat_plan_create(_geom())
    p2 = pat.pat_plan_create(_geom(n1=24, n2=24, nt=48, nz=24))
    try:
        w = pat.pat_batched_workspace_size([p1, p2])
        w1 = pat.pat_plan_sizes(p1)[1]
        w2 = pat.pat_plan_sizes(p2)[1]
        assert w >= w1 + w2
        with pytest.raises(pat.PatError):
            pat.pat_batched_workspace_size([])
    finally:
        pat.pat_plan_destroy(p1)
        pat.pat_plan_destroy(p2)


@pytest.mark.parametrize("kw", [dict(c=1.0, interp="linear"), dict(c=1.0, interp="nearest"),
                                dict(c=2.0, interp="nearest"), dict(c=1.0, K=3.0, interp="sinc"),
                                dict(c=4.0, interp="linear")])
def test_interpolation_methods_make_plans(kw):
    """The methods Section 4 compares get plans (2 taps, 1 tap, or 2cK)."""
    ptr = pat.pat_plan_create(_geom(**kw))
    pat.pat_plan_destroy(ptr)


@pytest.mark.parametrize("eps,n2", [(0.5, 16), (2.0, 16), (2.5, 1), (4.0, 16)])
def test_cutoff_plans_carry_a_weight_table(eps, n2):
    """A cut-off adds its (E+1)^3 weight table, E = ceil(2 eps), to the plan's
    device tables."""
    base = pat.pat_plan_create(_geom(n2=n2))
    cut = pat.pat_plan_create(_geom(n2=n2, cutoff=eps))
    try:
        e = int(np.ceil(2 * eps))
        extra = pat.pat_plan_sizes(cut)[0] - pat.pat_plan_sizes(base)[0]
        assert (e + 1) ** 3 * 4 <= extra <= (e + 1) ** 3 * 4 + 256
        assert pat.pat_plan_sizes(cut)[1] == pat.pat_plan_sizes(base)[1]
    finally:
        pat.pat_plan_destroy(base)
        pat.pat_plan_destroy(cut)


@pytest.mark.parametrize("kw", [dict(c=32.0, K=1.0, nt=512, nz=64), dict(c=16.0, K=2.0, nt=512, nz=64, precision="f64"),
                                dict(nt=8192, nz=64, n1=2, n2=2)])
def test_long_grid_lines_plan_staged_only(kw):
    """Grid lines longer than the fused kernels' LDS share (16384 FP32 points:
    c = 32 at nt = 512; 8192 FP64 points) are planned for the staged kernels,
    and asking for the fused ones is refused."""
    ptr = pat.pat_plan_create(_geom(**kw))
    try:
        with pytest.raises(pat.PatError) as ei:
            pat.pat_plan_set_fused(ptr, True)
        assert ei.value.status == 2
        pat.pat_plan_set_fused(ptr, False)
    finally:
        pat.pat_plan_destroy(ptr)
