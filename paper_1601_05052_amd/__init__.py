"""Brute-force incoherent dedispersion on AMD MI355X (gfx950).

Python view of libdedisp (``include/dedisp.h``).  Every step of the
computation runs in the library's HIP kernels; this module only passes
pointers, sizes and the current HIP stream.  PyTorch supplies device memory
and streams.  If the library is not built, importing the bindings raises --
there is no CPU fallback.

    plan = Plan(n_channels, f_min, df, t_samp, dm_first, dm_step, n_dm, n_samples)
    y = dedisperse(x, plan)                 # x: [C][>= plan.input_samples] f32/f16/u8 on GPU
    y = Dedisperse.apply(x, plan)           # differentiable (adjoint in backward)
    Batch([plan_a, plan_b, ...]).run([xa, xb, ...])
    rt = Realtime(plan, torch.uint8); y = rt.push(chunk)   # chunk: host [C][n_samples]
    snr, t, w = search_boxcar(y, n_widths=11)               # best boxcar per DM row
"""
from __future__ import annotations

import ctypes
from typing import Optional, Sequence

import numpy as np

from . import _lib
from ._lib import DD_ADJOINT, DD_F16, DD_F32, DD_FORWARD, DD_U8, DedispError, check  # noqa: F401

__all__ = ["Plan", "Batch", "Realtime", "search_boxcar", "Dedisperse", "dedisperse", "dedisperse_noalloc",
           "dedisperse_adjoint", "DedispError",
           "tile_variants", "DD_F32", "DD_F16", "DD_U8", "DD_FORWARD", "DD_ADJOINT"]


def _torch():
    import torch
    return torch


def _dtype_code(t) -> int:
    torch = _torch()
    if t == torch.float32:
        return DD_F32
    if t == torch.float16:
        return DD_F16
    if t == torch.uint8:
        return DD_U8
    raise TypeError("input dtype must be float32, float16 or uint8 (got %s)" % t)


def _stream_handle(device) -> ctypes.c_void_p:
    torch = _torch()
    return ctypes.c_void_p(torch.cuda.current_stream(device).cuda_stream)


def tile_variants():
    """[(id, items_t, items_acc, waves, kind)] of the compiled tile variants."""
    n = ctypes.c_int32()
    check(_lib.lib().dd_tile_count(ctypes.byref(n)))
    out = []
    for v in range(n.value):
        a, b, c, k = (ctypes.c_int32() for _ in range(4))
        check(_lib.lib().dd_tile_info(v, ctypes.byref(a), ctypes.byref(b), ctypes.byref(c), ctypes.byref(k)))
        out.append((v, a.value, b.value, c.value, k.value))
    return out


class Plan:
    """A dedispersion plan: setup + DM grid + the FP64 delay table."""

    def __init__(self, n_channels: int, f_min: float, df: float, t_samp: float, dm_first: float,
                 dm_step: float, n_dm: int, n_samples: int):
        L = _lib.lib()
        h = ctypes.c_void_p()
        check(L.dd_plan_create(ctypes.byref(h), int(n_channels), float(f_min), float(df), float(t_samp),
                               float(dm_first), float(dm_step), int(n_dm), int(n_samples)))
        self._h = h
        self.n_channels = int(n_channels)
        self.n_dm = int(n_dm)
        self.n_samples = int(n_samples)
        md = ctypes.c_int32()
        check(L.dd_plan_max_delay(h, ctypes.byref(md)))
        self.max_delay = md.value
        ti = ctypes.c_int64()
        check(L.dd_plan_input_samples(h, ctypes.byref(ti)))
        self.input_samples = ti.value

    @classmethod
    def from_setup(cls, setup) -> "Plan":
        return cls(*setup.plan_args())

    @property
    def handle(self) -> ctypes.c_void_p:
        return self._h

    def delays(self) -> np.ndarray:
        out = np.empty((self.n_dm, self.n_channels), dtype=np.int32)
        check(_lib.lib().dd_plan_delay_table(self._h, out.ctypes.data_as(ctypes.c_void_p)))
        return out

    @property
    def adds(self) -> int:
        return self.n_dm * self.n_samples * self.n_channels

    def prepare(self, direction: int = DD_FORWARD, dtype: int = DD_F32) -> None:
        check(_lib.lib().dd_plan_prepare(self._h, direction, dtype))

    def set_tile(self, variant: int, direction: int = DD_FORWARD, dtype: int = DD_F32) -> None:
        check(_lib.lib().dd_plan_set_tile(self._h, direction, dtype, int(variant)))

    def get_tile(self, direction: int = DD_FORWARD, dtype: int = DD_F32) -> int:
        v = ctypes.c_int32()
        check(_lib.lib().dd_plan_get_tile(self._h, direction, dtype, ctypes.byref(v)))
        return v.value

    def set_blocks(self, row_starts, variants, direction: int = DD_FORWARD, dtype: int = DD_F32) -> None:
        """Split the input rows into blocks (see dd_plan_set_blocks)."""
        n = len(row_starts)
        if len(variants) != n:
            raise ValueError("one variant per block")
        rs = (ctypes.c_int32 * n)(*[int(r) for r in row_starts])
        vs = (ctypes.c_int32 * n)(*[int(v) for v in variants])
        check(_lib.lib().dd_plan_set_blocks(self._h, direction, dtype, n, rs, vs))

    def get_blocks(self, direction: int = DD_FORWARD, dtype: int = DD_F32):
        """[(first row, variant)] of the launches the next call makes."""
        n = ctypes.c_int32()
        rs = (ctypes.c_int32 * _lib.DD_MAX_BLOCKS)()
        vs = (ctypes.c_int32 * _lib.DD_MAX_BLOCKS)()
        check(_lib.lib().dd_plan_get_blocks(self._h, direction, dtype, ctypes.byref(n), rs, vs))
        return [(rs[b], vs[b]) for b in range(n.value)]

    def autotune(self, direction: int = DD_FORWARD, dtype: int = DD_F32, reps: int = 3,
                 cache_path: Optional[str] = None, device=None):
        v, ms = ctypes.c_int32(), ctypes.c_float()
        cp = cache_path.encode() if cache_path else None
        check(_lib.lib().dd_autotune(self._h, direction, dtype, int(reps), cp, _stream_handle(device),
                                     ctypes.byref(v), ctypes.byref(ms)))
        return v.value, ms.value

    def close(self) -> None:
        if getattr(self, "_h", None) and self._h.value:
            _lib.lib().dd_plan_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _check_input(x, plan: Plan):
    torch = _torch()
    if not isinstance(x, torch.Tensor) or not x.is_cuda:
        raise TypeError("input must be a GPU tensor")
    if x.dim() != 2 or x.shape[0] != plan.n_channels:
        raise ValueError("input must be [n_channels][>= input_samples]")
    if x.stride(1) != 1 or x.stride(0) < plan.input_samples:
        raise ValueError("input rows must be contiguous and must not overlap")
    if x.shape[1] < plan.input_samples:
        raise ValueError("input rows hold %d samples, the plan needs %d" % (x.shape[1], plan.input_samples))


def _check_output(out, plan: Plan, device):
    """out must be float32 [n_dm][>= n_samples], unit column stride, on `device`."""
    torch = _torch()
    if not isinstance(out, torch.Tensor):
        raise TypeError("out must be a tensor")
    if (out.dtype != torch.float32 or out.device != device or out.dim() != 2
            or out.shape[0] != plan.n_dm or out.shape[1] < plan.n_samples or out.stride(1) != 1
            or out.stride(0) < plan.n_samples):
        raise ValueError("out must be float32 [n_dm][>= n_samples] with unit column stride on %s" % device)


def dedisperse(x, plan: Plan, out=None):
    """Forward dedispersion (Algorithm 1) of x [C][>= T_in] into out [D][S] float32."""
    torch = _torch()
    _check_input(x, plan)
    if out is None:
        out = torch.empty((plan.n_dm, plan.n_samples), dtype=torch.float32, device=x.device)
    else:
        _check_output(out, plan, x.device)
    with torch.cuda.device(x.device):
        check(_lib.lib().dd_dedisperse(plan.handle, ctypes.c_void_p(x.data_ptr()), _dtype_code(x.dtype),
                                       x.stride(0), ctypes.c_void_p(out.data_ptr()), out.stride(0),
                                       _stream_handle(x.device)))
    return out


def dedisperse_noalloc(x, plan: Plan, out):
    """``dedisperse`` through the allocation-free entry (dd_dedisperse_noalloc):
    ``out`` is required; the plan's forward tables must have been built
    (``plan.prepare(DD_FORWARD, dtype)`` or one ``dedisperse`` call)."""
    _check_input(x, plan)
    _check_output(out, plan, x.device)
    torch = _torch()
    with torch.cuda.device(x.device):
        check(_lib.lib().dd_dedisperse_noalloc(plan.handle, ctypes.c_void_p(x.data_ptr()), _dtype_code(x.dtype),
                                               x.stride(0), ctypes.c_void_p(out.data_ptr()), out.stride(0),
                                               _stream_handle(x.device)))
    return out


def dedisperse_adjoint(gy, plan: Plan, out=None):
    """Adjoint of ``dedisperse``: gy [D][>= S] float32 -> [C][T_in] float32."""
    torch = _torch()
    if not isinstance(gy, torch.Tensor) or not gy.is_cuda or gy.dtype != torch.float32:
        raise TypeError("gradient must be a float32 GPU tensor")
    if gy.dim() != 2 or gy.shape[0] != plan.n_dm or gy.shape[1] < plan.n_samples or gy.stride(1) != 1:
        raise ValueError("gradient must be [n_dm][>= n_samples] with contiguous rows")
    if out is None:
        out = torch.empty((plan.n_channels, plan.input_samples), dtype=torch.float32, device=gy.device)
    elif (out.dtype != torch.float32 or out.device != gy.device or out.dim() != 2
          or out.shape[0] != plan.n_channels or out.shape[1] < plan.input_samples or out.stride(1) != 1):
        raise ValueError("out must be float32 [n_channels][>= input_samples] on the gradient's device")
    with torch.cuda.device(gy.device):
        check(_lib.lib().dd_dedisperse_adjoint(plan.handle, ctypes.c_void_p(gy.data_ptr()), gy.stride(0),
                                               ctypes.c_void_p(out.data_ptr()), out.stride(0),
                                               _stream_handle(gy.device)))
    return out


def _make_autograd():
    torch = _torch()

    class Dedisperse(torch.autograd.Function):
        """y = A x (forward dedispersion); backward applies A^T with the
        library's adjoint kernel."""

        @staticmethod
        def forward(ctx, x, plan):
            ctx.plan = plan
            ctx.in_shape = tuple(x.shape)
            ctx.in_dtype = x.dtype
            return dedisperse(x, plan)

        @staticmethod
        def backward(ctx, gy):
            if not ctx.needs_input_grad[0]:
                return None, None
            gy = gy.contiguous()
            gx = dedisperse_adjoint(gy, ctx.plan)
            if ctx.in_shape[1] != gx.shape[1]:
                full = torch.zeros(ctx.in_shape, dtype=torch.float32, device=gx.device)
                full[:, :gx.shape[1]] = gx
                gx = full
            return gx.to(ctx.in_dtype), None

    return Dedisperse


class _LazyAutograd:
    _cls = None

    def __getattr__(self, name):
        if _LazyAutograd._cls is None:
            _LazyAutograd._cls = _make_autograd()
        return getattr(_LazyAutograd._cls, name)


Dedisperse = _LazyAutograd()


class Batch:
    """Many beams, one graph launch (see dd_batch_create)."""

    def __init__(self, plans: Sequence[Plan], dtype: int = DD_F32, tune: bool = False, reps: int = 2,
                 cache_path: Optional[str] = None, device=None):
        self.plans = list(plans)
        self.dtype = dtype
        arr = (ctypes.c_void_p * len(self.plans))(*[p.handle.value for p in self.plans])
        if tune:
            cp = cache_path.encode() if cache_path else None
            check(_lib.lib().dd_batch_autotune(arr, len(self.plans), dtype, int(reps), cp,
                                               _stream_handle(device)))
        h = ctypes.c_void_p()
        check(_lib.lib().dd_batch_create(ctypes.byref(h), arr, len(self.plans), dtype))
        self._h = h
        adds = ctypes.c_double()
        check(_lib.lib().dd_batch_adds(h, ctypes.byref(adds)))
        self.adds = adds.value

    def variants(self):
        """Tile variant of each beam."""
        v = (ctypes.c_int32 * len(self.plans))()
        check(_lib.lib().dd_batch_variants(self._h, v))
        return list(v)

    def run(self, xs, outs=None):
        torch = _torch()
        n = len(self.plans)
        if len(xs) != n:
            raise ValueError("one input per beam")
        code = {DD_F32: torch.float32, DD_F16: torch.float16, DD_U8: torch.uint8}[self.dtype]
        for x, p in zip(xs, self.plans):
            _check_input(x, p)
            if x.dtype != code:
                raise TypeError("batch inputs must all be %s" % code)
            if x.device != xs[0].device:
                raise ValueError("batch inputs must all be on one device")
        if outs is None:
            outs = [torch.empty((p.n_dm, p.n_samples), dtype=torch.float32, device=xs[0].device)
                    for p in self.plans]
        else:
            if len(outs) != n:
                raise ValueError("one output per beam")
            for o, p in zip(outs, self.plans):
                _check_output(o, p, xs[0].device)
        ins = (ctypes.c_void_p * n)(*[x.data_ptr() for x in xs])
        ins_s = (ctypes.c_int64 * n)(*[x.stride(0) for x in xs])
        os_ = (ctypes.c_void_p * n)(*[o.data_ptr() for o in outs])
        os_s = (ctypes.c_int64 * n)(*[o.stride(0) for o in outs])
        with torch.cuda.device(xs[0].device):
            check(_lib.lib().dd_batch_run(self._h, ins, ins_s, os_, os_s, _stream_handle(xs[0].device)))
        return outs

    def close(self):
        if getattr(self, "_h", None) and self._h.value:
            _lib.lib().dd_batch_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Realtime:
    """Streaming dedispersion of one beam (see dd_realtime_create).

    Each push appends one host chunk of ``plan.n_samples`` samples per channel
    and returns the dedispersed output for the ``n_samples`` output times that
    end ``plan.max_delay`` samples before the newest input; ``t0`` of push k is
    ``k * n_samples - max_delay`` in stream samples.  Work runs on the stream
    current at construction; chunks in pinned host memory overlap their copy
    with the previous chunk's kernels."""

    def __init__(self, plan: Plan, dtype=None, device=None):
        torch = _torch()
        self.plan = plan
        self.dtype = torch.float32 if dtype is None else dtype
        self.device = torch.device("cuda", torch.cuda.current_device()) if device is None else torch.device(device)
        self._stream = torch.cuda.current_stream(self.device)
        self._held = None
        h = ctypes.c_void_p()
        with torch.cuda.device(self.device):
            check(_lib.lib().dd_realtime_create(ctypes.byref(h), plan.handle, _dtype_code(self.dtype),
                                                ctypes.c_void_p(self._stream.cuda_stream)))
        self._h = h

    @property
    def pushed(self) -> int:
        n = ctypes.c_int64()
        check(_lib.lib().dd_realtime_pushed(self._h, ctypes.byref(n)))
        return n.value

    def push(self, chunk, out=None):
        """chunk: CPU tensor [n_channels][>= n_samples] (row stride >= n_samples,
        unit column stride) of the bound dtype.  Returns out [n_dm][n_samples]."""
        torch = _torch()
        p = self.plan
        if chunk.device.type != "cpu":
            raise ValueError("chunks are host tensors")
        if chunk.dtype != self.dtype:
            raise TypeError("chunk dtype %s, object bound to %s" % (chunk.dtype, self.dtype))
        if chunk.dim() != 2 or chunk.shape[0] != p.n_channels or chunk.shape[1] < p.n_samples or chunk.stride(1) != 1:
            raise ValueError("chunk must be [n_channels][>= n_samples] with unit column stride")
        if out is None:
            out = torch.empty((p.n_dm, p.n_samples), dtype=torch.float32, device=self.device)
        else:
            _check_output(out, p, self.device)
        with torch.cuda.device(self.device):
            check(_lib.lib().dd_realtime_push(self._h, ctypes.c_void_p(chunk.data_ptr()), chunk.stride(0),
                                              ctypes.c_void_p(out.data_ptr()), out.stride(0)))
        # The library reads the chunk asynchronously until the next push returns.
        self._held = chunk
        return out

    def close(self):
        if getattr(self, "_h", None) and self._h.value:
            _lib.lib().dd_realtime_destroy(self._h)
            self._h = ctypes.c_void_p()
            self._held = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def search_boxcar(rows, n_samples: Optional[int] = None, n_widths: int = 11):
    """Best boxcar S/N per row (see dd_search_boxcar): rows [n_rows][>= n_samples]
    float32 on the GPU -> (snr float32 [n_rows], t int32 [n_rows], width int32 [n_rows])."""
    torch = _torch()
    if not isinstance(rows, torch.Tensor) or not rows.is_cuda or rows.dtype != torch.float32:
        raise TypeError("rows must be a float32 GPU tensor")
    if rows.dim() != 2 or rows.stride(1) != 1:
        raise ValueError("rows must be 2-D with unit column stride")
    S = rows.shape[1] if n_samples is None else int(n_samples)
    if S > rows.shape[1]:
        raise ValueError("n_samples exceeds the row length")
    n = rows.shape[0]
    snr = torch.empty(n, dtype=torch.float32, device=rows.device)
    t = torch.empty(n, dtype=torch.int32, device=rows.device)
    w = torch.empty(n, dtype=torch.int32, device=rows.device)
    with torch.cuda.device(rows.device):
        check(_lib.lib().dd_search_boxcar(ctypes.c_void_p(rows.data_ptr()), rows.stride(0), n, S, int(n_widths),
                                          ctypes.c_void_p(snr.data_ptr()), ctypes.c_void_p(t.data_ptr()),
                                          ctypes.c_void_p(w.data_ptr()), _stream_handle(rows.device)))
    return snr, t, w
