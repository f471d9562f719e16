"""Helpers shared by the GPU tests: device transfer and oracle references."""
from __future__ import annotations

import numpy as np

import oracle
import synth


def torch_mod():
    import torch
    if not torch.cuda.is_available():
        raise RuntimeError("GPU tests need a HIP device")
    return torch


def to_dev(a: np.ndarray):
    torch = torch_mod()
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


def to_host(t) -> np.ndarray:
    torch_mod().cuda.synchronize()
    return t.detach().cpu().numpy()


def oracle_delays(setup: synth.Setup) -> np.ndarray:
    return oracle.delay_table(*setup.plan_args()[:7])


def workload_input(setup: synth.Setup, dtype: str = "f32", stride_pad: int = 0):
    """Seeded noise + the workload's pulses, with pulse arrivals from the
    oracle's delay table.  Returns (x [C][T_in + pad], delays, T_in)."""
    table = oracle_delays(setup)
    T = setup.n_samples + int(table.max())
    arrivals = {dm_i: table[dm_i] for dm_i, _ in synth.pulse_sites(setup)}
    x = synth.make_input(setup, T + stride_pad, dtype, arrivals=arrivals)
    return x, table, T


def ref_and_abs(x: np.ndarray, table: np.ndarray, S: int):
    x64 = x.astype(np.float64)
    return oracle.dedisperse(x64, table, S), oracle.dedisperse(np.abs(x64), table, S)


def sample_points(D: int, S: int, n: int, seed: int):
    rng = np.random.default_rng(seed)
    i = rng.integers(0, D, size=n)
    t = rng.integers(0, S, size=n)
    # always include the corners and ragged tails
    i = np.concatenate([i, [0, 0, D - 1, D - 1]])
    t = np.concatenate([t, [0, S - 1, 0, S - 1]])
    return i.astype(np.int32), t.astype(np.int64)
