"""Python binding of ``libpatnufft.so`` (the C ABI in ``include/pat.h``).

Argument marshalling only: every stage of every operator runs in the HIP
library.  The functions ``pat_*`` mirror the C entry points one to one; the
:class:`Plan` class bundles a plan with its device table and workspace (torch
tensors on the caller's device) and checks dtype, device, contiguity and
shape before calling in.  There is no CPU fallback: without the built library
every call raises.
"""
from __future__ import annotations

import ctypes
import os
import re
from ctypes import POINTER, byref, c_char_p, c_double, c_float, c_int32, c_size_t, c_void_p

import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libpatnufft.so")
HEADER = os.path.join(os.path.dirname(HERE), "include", "pat.h")

PAT_OK = 0
STATUS = {0: "PAT_OK", 1: "PAT_ERR_INVALID_ARG", 2: "PAT_ERR_UNSUPPORTED", 3: "PAT_ERR_WORKSPACE",
          4: "PAT_ERR_HIP", 5: "PAT_ERR_INTERNAL"}
PRECISION = {"f64": 0, "f32": 1, "bf16grid": 2}


class PatError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status


class pat_geometry(ctypes.Structure):
    _fields_ = [("ndim", c_int32), ("nx", c_int32 * 2), ("nt", c_int32), ("nz", c_int32),
                ("dx", c_double), ("dt", c_double), ("dz", c_double), ("vs", c_double),
                ("c", c_double), ("K", c_double), ("alpha", c_double), ("precision", c_int32),
                ("interp", c_int32), ("cutoff", c_double)]


_lib = None


def lib():
    """The loaded library; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_0808_3510_amd.build`")
        L = ctypes.CDLL(LIB_PATH)
        vp = c_void_p
        sz = c_size_t
        sig = {
            "pat_plan_create": (c_int32, [POINTER(pat_geometry), POINTER(c_void_p)]),
            "pat_plan_sizes": (c_int32, [vp, POINTER(c_size_t), POINTER(c_size_t)]),
            "pat_plan_upload": (c_int32, [vp, vp, sz, vp]),
            "pat_reconstruct": (c_int32, [vp, vp, sz, vp, sz, vp, sz, vp]),
            "pat_reconstruct_noalloc": (c_int32, [vp, vp, sz, vp, sz, vp]),
            "pat_reconstruct_adjoint": (c_int32, [vp, vp, sz, vp, sz, vp, sz, vp]),
            "pat_forward": (c_int32, [vp, vp, sz, vp, sz, vp, sz, vp]),
            "pat_forward_adjoint": (c_int32, [vp, vp, sz, vp, sz, vp, sz, vp]),
            "pat_batched_workspace_size": (c_int32, [c_int32, POINTER(c_void_p), POINTER(c_size_t)]),
            "pat_reconstruct_batched": (c_int32, [c_int32, POINTER(c_void_p), POINTER(c_void_p), POINTER(c_size_t),
                                                  POINTER(c_void_p), POINTER(c_size_t), vp, sz, vp]),
            "pat_nufft2_lines": (c_int32, [vp, vp, sz, vp, sz, vp]),
            "pat_nufft1_lines": (c_int32, [vp, vp, sz, vp, sz, vp]),
            "pat_plan_set_fused": (c_int32, [vp, c_int32]),
            "pat_plan_set_timing": (c_int32, [vp, c_int32]),
            "pat_plan_stage_times": (c_int32, [vp, c_int32, POINTER(c_char_p), POINTER(c_float),
                                               POINTER(c_int32)]),
            "pat_plan_destroy": (None, [vp]),
            "pat_status_string": (c_char_p, [c_int32]),
            "pat_last_error": (c_char_p, []),
        }
        for name, (res, args) in sig.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def header_functions() -> list[str]:
    """Every function the public header declares."""
    with open(HEADER) as fh:
        text = fh.read()
    return sorted(set(re.findall(r"\b(pat_[a-z0-9_]+)\s*\(", text)))


def _check(status: int):
    if status != PAT_OK:
        raise PatError(status, lib().pat_last_error().decode())


# --------------------------------------------------------------------------
# one-to-one wrappers of the C entry points (pointers as Python ints)

def pat_plan_create(geom: pat_geometry) -> int:
    ptr = c_void_p()
    _check(lib().pat_plan_create(byref(geom), byref(ptr)))
    return ptr.value


def pat_plan_sizes(plan: int) -> tuple[int, int]:
    t, w = c_size_t(), c_size_t()
    _check(lib().pat_plan_sizes(plan, byref(t), byref(w)))
    return t.value, w.value


def pat_plan_upload(plan: int, table: int, table_bytes: int, stream: int):
    _check(lib().pat_plan_upload(plan, table, table_bytes, stream))


def pat_reconstruct(plan, p, p_bytes, f, f_bytes, ws, ws_bytes, stream):
    _check(lib().pat_reconstruct(plan, p, p_bytes, f, f_bytes, ws, ws_bytes, stream))


def pat_reconstruct_noalloc(plan, p, p_bytes, f, f_bytes, stream):
    _check(lib().pat_reconstruct_noalloc(plan, p, p_bytes, f, f_bytes, stream))


def pat_reconstruct_adjoint(plan, f, f_bytes, p, p_bytes, ws, ws_bytes, stream):
    _check(lib().pat_reconstruct_adjoint(plan, f, f_bytes, p, p_bytes, ws, ws_bytes, stream))


def pat_forward(plan, f, f_bytes, p, p_bytes, ws, ws_bytes, stream):
    _check(lib().pat_forward(plan, f, f_bytes, p, p_bytes, ws, ws_bytes, stream))


def pat_forward_adjoint(plan, p, p_bytes, f, f_bytes, ws, ws_bytes, stream):
    _check(lib().pat_forward_adjoint(plan, p, p_bytes, f, f_bytes, ws, ws_bytes, stream))


def _ptr_array(vals):
    return (c_void_p * len(vals))(*vals)


def _size_array(vals):
    return (c_size_t * len(vals))(*vals)


def pat_batched_workspace_size(plans) -> int:
    w = c_size_t()
    _check(lib().pat_batched_workspace_size(len(plans), _ptr_array(plans), byref(w)))
    return w.value


def pat_reconstruct_batched(plans, ps, p_bytes, fs, f_bytes, ws, ws_bytes, stream):
    _check(lib().pat_reconstruct_batched(len(plans), _ptr_array(plans), _ptr_array(ps), _size_array(p_bytes),
                                         _ptr_array(fs), _size_array(f_bytes), ws, ws_bytes, stream))


def pat_nufft2_lines(plan, grid, grid_bytes, out, out_bytes, stream):
    _check(lib().pat_nufft2_lines(plan, grid, grid_bytes, out, out_bytes, stream))


def pat_nufft1_lines(plan, values, values_bytes, grid, grid_bytes, stream):
    _check(lib().pat_nufft1_lines(plan, values, values_bytes, grid, grid_bytes, stream))


def pat_plan_set_fused(plan, fused: bool):
    _check(lib().pat_plan_set_fused(plan, 1 if fused else 0))


def pat_plan_set_timing(plan, on: bool):
    _check(lib().pat_plan_set_timing(plan, 1 if on else 0))


def pat_plan_stage_times(plan, cap: int = 64):
    names = (c_char_p * cap)()
    ms = (c_float * cap)()
    n = c_int32()
    _check(lib().pat_plan_stage_times(plan, cap, names, ms, byref(n)))
    return [(names[i].decode(), float(ms[i])) for i in range(min(n.value, cap))]


def pat_plan_destroy(plan):
    lib().pat_plan_destroy(plan)


def pat_status_string(s: int) -> str:
    return lib().pat_status_string(s).decode()


def pat_last_error() -> str:
    return lib().pat_last_error().decode()


# --------------------------------------------------------------------------

INTERP = {"kb": 0, "sinc": 1, "linear": 2, "nearest": 3}


def make_geometry(n1, n2, nt, nz, dx, dt, dz, vs=1.0, c=2.0, K=3.0, alpha=0.0, precision="f32",
                  interp="kb", cutoff=0.0) -> pat_geometry:
    g = pat_geometry()
    g.ndim = 2 if n2 == 1 else 3
    g.nx[0], g.nx[1] = int(n1), int(n2)
    g.nt, g.nz = int(nt), int(nz)
    g.dx, g.dt, g.dz, g.vs = float(dx), float(dt), float(dz), float(vs)
    g.c, g.K, g.alpha = float(c), float(K), float(alpha)
    g.precision = PRECISION[precision] if isinstance(precision, str) else int(precision)
    g.interp = INTERP[interp] if isinstance(interp, str) else int(interp)
    g.cutoff = float(cutoff)
    return g


def _nbytes(t: torch.Tensor) -> int:
    return t.numel() * t.element_size()


def _stream(device) -> int:
    return torch.cuda.current_stream(device).cuda_stream


class Plan:
    """A plan, its uploaded table and its workspace on one device.

    ``n2 = 1`` selects the 2D line geometry; ``cutoff`` > 0 applies the smooth
    cut-off of that radius (in sampling steps) on the data side (see
    ``pat_geometry.cutoff``).  Arrays are ``(n1, n2, nt)`` /
    ``(n1, n2, nz)`` (or ``(n1, nt)`` / ``(n1, nz)`` in 2D), contiguous, float64
    for ``precision="f64"`` and float32 otherwise.
    """

    def __init__(self, n1, n2, nt, nz, dx=1.0, dt=1.0, dz=1.0, vs=1.0, c=2.0, K=3.0, alpha=0.0,
                 precision="f32", device="cuda", interp="kb", cutoff=0.0):
        self.geom = make_geometry(n1, n2, nt, nz, dx, dt, dz, vs, c, K, alpha, precision, interp, cutoff)
        self.n1, self.n2, self.nt, self.nz = int(n1), int(n2), int(nt), int(nz)
        self.m = int(round(c * nt))
        self.lines = (self.n1 // 2 + 1) * self.n2
        self.precision = precision
        self.dtype = torch.float64 if precision == "f64" else torch.float32
        self.device = torch.device(device)
        self.ptr = pat_plan_create(self.geom)
        tb, wb = pat_plan_sizes(self.ptr)
        self.table = torch.empty(tb, dtype=torch.uint8, device=self.device)
        pat_plan_upload(self.ptr, self.table.data_ptr(), tb, _stream(self.device))
        self.ws = torch.empty(wb, dtype=torch.uint8, device=self.device)
        # a new plan runs the fused line kernels when it can; asking for them
        # again is a no-op there and refused elsewhere
        try:
            pat_plan_set_fused(self.ptr, True)
            self.fusable = True
        except PatError:
            self.fusable = False

    def __del__(self):
        ptr = getattr(self, "ptr", None)
        if ptr and _lib is not None:
            _lib.pat_plan_destroy(ptr)
            self.ptr = None

    # shape handling -------------------------------------------------------
    def _check(self, x: torch.Tensor, last: int, what: str) -> torch.Tensor:
        if not isinstance(x, torch.Tensor):
            raise TypeError(f"{what} must be a torch tensor")
        if not self._on_device(x):
            raise ValueError(f"{what} is on {x.device}, plan on {self.device}")
        if x.dtype != self.dtype:
            raise TypeError(f"{what} must be {self.dtype}, got {x.dtype}")
        if x.numel() != self.n1 * self.n2 * last or x.shape[-1] != last or x.shape[0] != self.n1:
            raise ValueError(f"{what} has shape {tuple(x.shape)}, expected ({self.n1}, {self.n2}, {last})")
        if not x.is_contiguous():
            raise ValueError(f"{what} must be contiguous")
        return x

    def _out(self, x: torch.Tensor, last: int) -> torch.Tensor:
        shape = (self.n1, last) if x.dim() == 2 else (self.n1, self.n2, last)
        return torch.empty(shape, dtype=self.dtype, device=self.device)

    def _call(self, fn, x, last_in, last_out, out=None):
        self._check(x, last_in, "input")
        y = self._out(x, last_out) if out is None else self._check(out, last_out, "output")
        fn(self.ptr, x.data_ptr(), _nbytes(x), y.data_ptr(), _nbytes(y), self.ws.data_ptr(), _nbytes(self.ws),
           _stream(self.device))
        return y

    # operators ------------------------------------------------------------
    def reconstruct(self, p, out=None):
        """R: detector data -> image."""
        return self._call(pat_reconstruct, p, self.nt, self.nz, out)

    def reconstruct_noalloc(self, p, out=None):
        """R through the allocation-free entry point (the library's static
        scratch instead of this plan's workspace; the output is still the
        caller's)."""
        self._check(p, self.nt, "input")
        y = self._out(p, self.nz) if out is None else self._check(out, self.nz, "output")
        pat_reconstruct_noalloc(self.ptr, p.data_ptr(), _nbytes(p), y.data_ptr(), _nbytes(y), _stream(self.device))
        return y

    def reconstruct_adjoint(self, q, out=None):
        """R^T: image-shaped -> data-shaped."""
        return self._call(pat_reconstruct_adjoint, q, self.nz, self.nt, out)

    def forward(self, f, out=None):
        """A: image -> detector data (spectral forward model)."""
        return self._call(pat_forward, f, self.nz, self.nt, out)

    def forward_adjoint(self, p, out=None):
        """A^T: data-shaped -> image-shaped."""
        return self._call(pat_forward_adjoint, p, self.nt, self.nz, out)

    def _on_device(self, x: torch.Tensor) -> bool:
        return x.device.type == self.device.type and (self.device.index is None or
                                                      x.device.index == self.device.index)

    def _check_lines(self, x, shape, dtype, what: str) -> torch.Tensor:
        """A line-stage array: exact dtype, shape, device and contiguity
        (the C ABI takes no sizes, so nothing short or misplaced may reach it)."""
        if not isinstance(x, torch.Tensor):
            raise TypeError(f"{what} must be a torch tensor")
        if x.dtype != dtype:
            raise ValueError(f"{what} must be {dtype}, got {x.dtype}")
        if tuple(x.shape) != tuple(shape):
            raise ValueError(f"{what} has shape {tuple(x.shape)}, expected {tuple(shape)}")
        if not self._on_device(x):
            raise ValueError(f"{what} is on {x.device}, plan on {self.device}")
        if not x.is_contiguous():
            raise ValueError(f"{what} must be contiguous")
        return x

    def _grid_spec(self):
        if self.precision == "bf16grid":
            return (self.lines, self.m, 2), torch.bfloat16
        cdt = torch.complex128 if self.precision == "f64" else torch.complex64
        return (self.lines, self.m), cdt

    def _values_spec(self):
        cdt = torch.complex128 if self.precision == "f64" else torch.complex64
        return (self.lines, self.nz), cdt

    def nufft2_lines(self, grid: torch.Tensor, out=None) -> torch.Tensor:
        """Stage a3 alone: grid ``(lines, m)`` complex (``(lines, m, 2)``
        bfloat16 for the bf16 grid) -> ``(lines, nz)`` complex."""
        gshape, gdt = self._grid_spec()
        vshape, vdt = self._values_spec()
        self._check_lines(grid, gshape, gdt, "grid")
        if out is None:
            out = torch.empty(vshape, dtype=vdt, device=self.device)
        else:
            self._check_lines(out, vshape, vdt, "out")
        pat_nufft2_lines(self.ptr, grid.data_ptr(), _nbytes(grid), out.data_ptr(), _nbytes(out), _stream(self.device))
        return out

    def nufft1_lines(self, values: torch.Tensor, out=None) -> torch.Tensor:
        """Spreading alone, the adjoint of :meth:`nufft2_lines`: values
        ``(lines, nz)`` complex -> grid ``(lines, m)`` complex (``(lines, m, 2)``
        bfloat16 for the bf16 grid)."""
        gshape, gdt = self._grid_spec()
        vshape, vdt = self._values_spec()
        self._check_lines(values, vshape, vdt, "values")
        if out is None:
            out = torch.empty(gshape, dtype=gdt, device=self.device)
        else:
            self._check_lines(out, gshape, gdt, "out")
        pat_nufft1_lines(self.ptr, values.data_ptr(), _nbytes(values), out.data_ptr(), _nbytes(out),
                         _stream(self.device))
        return out

    def set_fused(self, fused: bool = True):
        """Fused (default) or staged line kernels; see ``pat_plan_set_fused``."""
        pat_plan_set_fused(self.ptr, fused)

    def set_timing(self, on: bool = True):
        pat_plan_set_timing(self.ptr, on)

    def stage_times(self):
        return pat_plan_stage_times(self.ptr)


def reconstruct_batched(plans, ps, outs=None, ws=None):
    """R for several plans in one persistent launch per stage."""
    if len(plans) != len(ps):
        raise ValueError("one input per plan")
    for pl, p in zip(plans, ps):
        pl._check(p, pl.nt, "input")
    if outs is None:
        outs = [pl._out(p, pl.nz) for pl, p in zip(plans, ps)]
    elif len(outs) != len(plans):
        raise ValueError("one output per plan")
    else:
        for pl, o in zip(plans, outs):
            pl._check(o, pl.nz, "output")
    ptrs = [pl.ptr for pl in plans]
    need = pat_batched_workspace_size(ptrs)
    if ws is None or ws.numel() < need or not plans[0]._on_device(ws) or not ws.is_contiguous():
        ws = torch.empty(need, dtype=torch.uint8, device=plans[0].device)
    pat_reconstruct_batched(ptrs, [p.data_ptr() for p in ps], [_nbytes(p) for p in ps], [o.data_ptr() for o in outs],
                            [_nbytes(o) for o in outs], ws.data_ptr(), _nbytes(ws),
                            _stream(plans[0].device))
    return outs, ws


class ReconFn(torch.autograd.Function):
    """``f = R p`` with ``grad_p = R^T grad_f`` (type-1 spreading)."""

    @staticmethod
    def forward(ctx, p, plan):
        ctx.plan = plan
        return plan.reconstruct(p.contiguous())

    @staticmethod
    def backward(ctx, g):
        return ctx.plan.reconstruct_adjoint(g.contiguous()), None


class ForwardFn(torch.autograd.Function):
    """``p = A f`` (type-1 spreading) with ``grad_f = A^T grad_p`` (type-2)."""

    @staticmethod
    def forward(ctx, f, plan):
        ctx.plan = plan
        return plan.forward(f.contiguous())

    @staticmethod
    def backward(ctx, g):
        return ctx.plan.forward_adjoint(g.contiguous()), None
