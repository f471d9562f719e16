"""ctypes declarations for libdedisp.so (argument marshalling only)."""
from __future__ import annotations

import ctypes
import os

from .build import library_path

DD_OK, DD_EINVAL, DD_ESHAPE, DD_ENOMEM, DD_EHIP, DD_EUNSUPPORTED = 0, -1, -2, -3, -4, -5
DD_F32, DD_F16, DD_U8 = 0, 1, 2
DD_MAX_BLOCKS = 32
DD_FORWARD, DD_ADJOINT = 0, 1

STATUS_NAMES = {0: "DD_OK", -1: "DD_EINVAL", -2: "DD_ESHAPE", -3: "DD_ENOMEM", -4: "DD_EHIP",
                -5: "DD_EUNSUPPORTED"}


class DedispError(RuntimeError):
    """A libdedisp call returned a non-zero status."""

    def __init__(self, code: int, message: str):
        super().__init__("%s: %s" % (STATUS_NAMES.get(code, str(code)), message))
        self.code = code


_LIB = None

i32, i64, f32, dbl, vp = ctypes.c_int32, ctypes.c_int64, ctypes.c_float, ctypes.c_double, ctypes.c_void_p
P = ctypes.POINTER

SIGNATURES = {
    "dd_plan_create": [P(vp), i32, dbl, dbl, dbl, dbl, dbl, i32, i64],
    "dd_plan_destroy": [vp],
    "dd_plan_dims": [vp, P(i32), P(i32), P(i64)],
    "dd_plan_max_delay": [vp, P(i32)],
    "dd_plan_input_samples": [vp, P(i64)],
    "dd_plan_delay_table": [vp, vp],
    "dd_plan_prepare": [vp, ctypes.c_int, ctypes.c_int],
    "dd_dedisperse": [vp, vp, ctypes.c_int, i64, vp, i64, vp],
    "dd_dedisperse_noalloc": [vp, vp, ctypes.c_int, i64, vp, i64, vp],
    "dd_dedisperse_adjoint": [vp, vp, i64, vp, i64, vp],
    "dd_tile_count": [P(i32)],
    "dd_tile_info": [i32, P(i32), P(i32), P(i32), P(i32)],
    "dd_plan_set_tile": [vp, ctypes.c_int, ctypes.c_int, i32],
    "dd_plan_get_tile": [vp, ctypes.c_int, ctypes.c_int, P(i32)],
    "dd_plan_set_blocks": [vp, ctypes.c_int, ctypes.c_int, i32, P(i32), P(i32)],
    "dd_plan_get_blocks": [vp, ctypes.c_int, ctypes.c_int, P(i32), P(i32), P(i32)],
    "dd_autotune": [vp, ctypes.c_int, ctypes.c_int, i32, ctypes.c_char_p, vp, P(i32), P(f32)],
    "dd_batch_create": [P(vp), P(vp), i32, ctypes.c_int],
    "dd_batch_autotune": [P(vp), i32, ctypes.c_int, i32, ctypes.c_char_p, vp],
    "dd_batch_run": [vp, P(vp), P(i64), P(vp), P(i64), vp],
    "dd_batch_adds": [vp, P(dbl)],
    "dd_batch_variants": [vp, P(i32)],
    "dd_batch_destroy": [vp],
    "dd_realtime_create": [P(vp), vp, ctypes.c_int, vp],
    "dd_realtime_push": [vp, vp, i64, vp, i64],
    "dd_realtime_pushed": [vp, P(i64)],
    "dd_realtime_destroy": [vp],
    "dd_search_boxcar": [vp, i64, i32, i64, i32, vp, vp, vp, vp],
    "dd_last_error": [],
    "dd_version": [],
}


def _load_torch_runtime() -> None:
    """Load PyTorch (and with it PyTorch's HIP runtime) before libdedisp.

    Both runtimes carry the soname libamdhip64.so.7: if PyTorch's copy is
    already in the process, libdedisp binds to it, so the process has one HIP
    runtime and PyTorch's streams and allocations are valid handles for the
    library.  Loaded the other way round, the process would hold two HIP/HSA
    runtimes, and the one initialised second finds no device."""
    try:
        import torch  # noqa: F401
    except ImportError:
        pass


def lib():
    """Load the in-tree libdedisp.so (or the library DEDISP_LIBRARY names, e.g.
    the auto-tuning study's build).  Raises ImportError if it is not built:
    there is no fallback implementation."""
    global _LIB
    if _LIB is None:
        _load_torch_runtime()
        path = os.environ.get("DEDISP_LIBRARY") or library_path()
        if not os.path.exists(path):
            raise ImportError("libdedisp.so is not built (%s); run: python -m paper_1601_05052_amd.build"
                              % path)
        handle = ctypes.CDLL(path)
        for name, args in SIGNATURES.items():
            fn = getattr(handle, name)
            fn.argtypes = args
            fn.restype = ctypes.c_char_p if name in ("dd_last_error", "dd_version") else ctypes.c_int
        _LIB = handle
    return _LIB


def check(code: int) -> None:
    if code != DD_OK:
        msg = lib().dd_last_error()
        raise DedispError(code, msg.decode() if msg else "")
