"""FP64 CPU oracle for brute-force dedispersion.

TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
benchmark's CPU-baseline leg may import this package.  It shares no code with
the GPU library (``paper_1601_05052_amd``) and never imports it.

Two implementations of what the method computes (Sclocco et al., Sec. III-A,
Algorithm 1, with delays from Sec. II, Eq. (1)):

* ``alg1`` -- pure Python loops, Algorithm 1 written out, for tiny inputs;
* the C functions in ``dd_oracle.c`` (OpenMP, FP64 accumulators) for
  realistic sizes, called through ctypes below.

All arrays handed to the C side are float64 / int32 / int64, C-contiguous.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

from . import alg1  # noqa: F401  (re-exported)
from .build import build_oracle, library_path


class COracle:
    """ctypes view of one compiled copy of ``dd_oracle.c``."""

    def __init__(self, path: str):
        lib = ctypes.CDLL(path)
        i32, i64, dbl, ptr = ctypes.c_int32, ctypes.c_int64, ctypes.c_double, ctypes.c_void_p
        lib.oracle_delay_table.argtypes = [i32, dbl, dbl, dbl, dbl, dbl, i32, ptr]
        lib.oracle_delay_table.restype = ctypes.c_int
        lib.oracle_dedisperse_points.argtypes = [i32, ptr, ptr, i64, i64, ptr, ptr, ptr]
        lib.oracle_dedisperse_points.restype = None
        lib.oracle_dedisperse.argtypes = [i32, i32, i64, ptr, ptr, i64, ptr]
        lib.oracle_dedisperse.restype = None
        lib.oracle_adjoint.argtypes = [i32, i32, i64, ptr, ptr, i64, ptr]
        lib.oracle_adjoint.restype = None
        lib.oracle_num_threads.argtypes = []
        lib.oracle_num_threads.restype = ctypes.c_int
        self.lib = lib
        self.path = path

    def delay_table(self, n_channels, f_min, df, t_samp, dm_first, dm_step, n_dm) -> np.ndarray:
        """Eq. (1) sampled: int32 [n_dm][n_channels] delays in samples."""
        out = np.empty((int(n_dm), int(n_channels)), dtype=np.int32)
        rc = self.lib.oracle_delay_table(int(n_channels), float(f_min), float(df), float(t_samp),
                                         float(dm_first), float(dm_step), int(n_dm), _p(out))
        if rc != 0:
            raise ValueError("invalid plan parameters or delay outside int32")
        return out

    def dedisperse(self, x: np.ndarray, delay: np.ndarray, n_samples: int) -> np.ndarray:
        """Algorithm 1: y[i][t] = sum_ch x[ch][t + delay[i][ch]], FP64, [D][S]."""
        delay = np.ascontiguousarray(delay, dtype=np.int32)
        D, C = delay.shape
        x64 = _as_f64_rows(x)
        if x64.shape[0] != C:
            raise ValueError("channel count mismatch")
        S = int(n_samples)
        if S + int(delay.max(initial=0)) > x64.shape[1] or int(delay.min(initial=0)) < 0:
            raise ValueError("input rows too short for the delays")
        y = np.empty((D, S), dtype=np.float64)
        self.lib.oracle_dedisperse(C, D, S, _p(delay), _p(x64), x64.shape[1], _p(y))
        return y

    def dedisperse_points(self, x: np.ndarray, delay: np.ndarray, dm_idx, t_idx) -> np.ndarray:
        """Algorithm 1 evaluated only at the given (dm, t) pairs."""
        delay = np.ascontiguousarray(delay, dtype=np.int32)
        D, C = delay.shape
        x64 = _as_f64_rows(x)
        dm_idx = np.ascontiguousarray(dm_idx, dtype=np.int32)
        t_idx = np.ascontiguousarray(t_idx, dtype=np.int64)
        if dm_idx.shape != t_idx.shape:
            raise ValueError("index arrays differ in shape")
        if dm_idx.size and (dm_idx.min() < 0 or dm_idx.max() >= D or t_idx.min() < 0):
            raise ValueError("index out of range")
        if dm_idx.size and int(t_idx.max()) + int(delay.max()) >= x64.shape[1]:
            raise ValueError("input rows too short for the requested points")
        out = np.empty(dm_idx.shape, dtype=np.float64)
        self.lib.oracle_dedisperse_points(C, _p(delay), _p(x64), x64.shape[1], dm_idx.size,
                                          _p(dm_idx), _p(t_idx), _p(out))
        return out

    def adjoint(self, gy: np.ndarray, delay: np.ndarray, n_input_samples: int) -> np.ndarray:
        """Transpose of Algorithm 1: gx[ch][tau] for tau < n_input_samples, FP64."""
        delay = np.ascontiguousarray(delay, dtype=np.int32)
        D, C = delay.shape
        gy64 = np.ascontiguousarray(gy, dtype=np.float64)
        if gy64.ndim != 2 or gy64.shape[0] != D:
            raise ValueError("gradient must be [n_dm][n_samples]")
        S = gy64.shape[1]
        T = int(n_input_samples)
        gx = np.empty((C, T), dtype=np.float64)
        self.lib.oracle_adjoint(C, D, S, _p(delay), _p(gy64), T, _p(gx))
        return gx

    def num_threads(self) -> int:
        return int(self.lib.oracle_num_threads())


def _p(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def _as_f64_rows(x: np.ndarray) -> np.ndarray:
    x = np.asarray(x)
    if x.ndim != 2:
        raise ValueError("input must be 2-D [channels][samples]")
    return np.ascontiguousarray(x, dtype=np.float64)


_DEFAULT = None


def default() -> COracle:
    """The oracle built from this directory's source (compiled on first use)."""
    global _DEFAULT
    if _DEFAULT is None:
        path = library_path()
        if not os.path.exists(path):
            build_oracle()
        _DEFAULT = COracle(path)
    return _DEFAULT


def delay_table(*args) -> np.ndarray:
    return default().delay_table(*args)


def dedisperse(x, delay, n_samples) -> np.ndarray:
    return default().dedisperse(x, delay, n_samples)


def dedisperse_points(x, delay, dm_idx, t_idx) -> np.ndarray:
    return default().dedisperse_points(x, delay, dm_idx, t_idx)


def adjoint(gy, delay, n_input_samples) -> np.ndarray:
    return default().adjoint(gy, delay, n_input_samples)


def num_threads() -> int:
    return default().num_threads()
