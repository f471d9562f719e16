"""Seeded synthetic inputs for dedispersion runs.

Shared by the GPU tests, the benchmark and the oracle tests.  This module
holds NO dedispersion arithmetic: no delay law, no sums.  Where a dispersed
pulse is injected, the caller passes the per-channel arrival offsets (in
samples) that it computed itself.

Workloads (``WORKLOADS``) follow the observational setups of Sclocco et al.,
Sec. IV (Apertif-like: 1,024 channels over 1,420-1,720 MHz at 20,000
samples/s; LOFAR-like: 32 channels over 138-144 MHz at 200,000 samples/s),
plus a tiny case, a batch of uneven Apertif-band beams and an 8-beam
training-style case.  All data is synthetic: Gaussian noise from NumPy's
PCG64 generator with a fixed seed, plus boxcar pulses.
"""
from __future__ import annotations

from dataclasses import dataclass, replace
from typing import List, Optional, Sequence

import numpy as np


@dataclass(frozen=True)
class Setup:
    """One beam's observational setup and DM grid (all inputs to a plan)."""
    name: str
    n_channels: int
    f_min: float          # MHz, frequency of channel 0 (the lowest)
    df: float             # MHz, channel width (> 0)
    t_samp: float         # s, sampling time
    dm_first: float       # pc/cm^3
    dm_step: float        # pc/cm^3
    n_dm: int
    n_samples: int        # output samples per DM
    seed: int = 0

    def plan_args(self):
        return (self.n_channels, self.f_min, self.df, self.t_samp,
                self.dm_first, self.dm_step, self.n_dm, self.n_samples)

    @property
    def adds(self) -> int:
        """Additions of the brute-force sum: one per (DM, sample, channel)."""
        return self.n_dm * self.n_samples * self.n_channels


TINY = Setup("tiny", 64, 1400.0, 1.5625, 5e-5, 0.0, 0.5, 128, 4096, seed=1)
APERTIF = Setup("apertif", 1024, 1420.0, 300.0 / 1024, 1.0 / 20000, 0.0, 0.25, 2048, 20000, seed=2)
LOFAR = Setup("lofar", 32, 138.0, 6.0 / 32, 1.0 / 200000, 0.0, 0.01, 2048, 200000, seed=3)
# Training-style slice: every 64th Apertif channel, the first 32 DMs, 256 samples.
FD_SLICE = Setup("fd_slice", 16, 1420.0, 64 * 300.0 / 1024, 1.0 / 20000, 0.0, 0.25, 32, 256, seed=5)

WORKLOADS = {s.name: s for s in (TINY, APERTIF, LOFAR, FD_SLICE)}

TINY_PULSE_DM_INDEX = 50       # DM 25.0 on the tiny grid (0.5 step)
PULSE_AMPLITUDE = 5.0
PULSE_WIDTH = 3


def batched_beams(n_beams: int = 64, seed: int = 4) -> List[Setup]:
    """Uneven Apertif-band beams: channels in {256, 512, 1024} over
    1,420-1,720 MHz, DM counts uniform in [512, 4096] at step 0.25, output
    samples uniform in [10,000, 40,000] at 20,000 samples/s."""
    rng = np.random.default_rng(seed)
    beams = []
    for b in range(n_beams):
        c = int(rng.choice([256, 512, 1024]))
        d = int(rng.integers(512, 4096, endpoint=True))
        s = int(rng.integers(10000, 40000, endpoint=True))
        beams.append(Setup("beam%02d" % b, c, 1420.0, 300.0 / c, 1.0 / 20000, 0.0, 0.25, d, s,
                           seed=4000 + b))
    return beams


def fwd_bwd_beams(n_beams: int = 8) -> List[Setup]:
    """Eight Apertif-shaped beams for the differentiable case."""
    return [replace(APERTIF, name="fb%d" % b, seed=500 + b) for b in range(n_beams)]


# ---------------------------------------------------------------- generators

def rng_for(seed: int) -> np.random.Generator:
    return np.random.default_rng(seed)


def noise_f32(n_rows: int, n_cols: int, seed: int) -> np.ndarray:
    """i.i.d. N(0, 1) float32, [n_rows][n_cols]."""
    return rng_for(seed).standard_normal((n_rows, n_cols), dtype=np.float32)


def noise_u8(n_rows: int, n_cols: int, seed: int, mean: float = 128.0, sigma: float = 16.0) -> np.ndarray:
    """round(N(mean, sigma)) clipped to [0, 255], uint8."""
    z = rng_for(seed).standard_normal((n_rows, n_cols), dtype=np.float32)
    return np.clip(np.rint(z * np.float32(sigma) + np.float32(mean)), 0, 255).astype(np.uint8)


def noise_f16(n_rows: int, n_cols: int, seed: int) -> np.ndarray:
    """N(0, 1) rounded to float16."""
    return noise_f32(n_rows, n_cols, seed).astype(np.float16)


def integers_f32(n_rows: int, n_cols: int, seed: int, lo: int = -8, hi: int = 8) -> np.ndarray:
    """Integer-valued float32 (uniform in [lo, hi]); any-order float sums of
    these are exact while partial sums stay below 2**24."""
    return rng_for(seed).integers(lo, hi, size=(n_rows, n_cols), endpoint=True).astype(np.float32)


def uniform_f32(n_rows: int, n_cols: int, seed: int) -> np.ndarray:
    """U(0, 1) float32."""
    return rng_for(seed).random((n_rows, n_cols), dtype=np.float32)


def inject_pulse(x: np.ndarray, arrival: Sequence[int], t0: int, amplitude: float, width: int) -> None:
    """Add a boxcar of ``width`` samples and height ``amplitude`` to every
    channel ch starting at sample t0 + arrival[ch], in place.  Samples past the
    row end are dropped.  ``arrival`` comes from the caller."""
    n_rows, n_cols = x.shape
    arrival = np.asarray(arrival)
    if arrival.shape != (n_rows,):
        raise ValueError("one arrival offset per channel")
    for ch in range(n_rows):
        start = int(t0) + int(arrival[ch])
        lo, hi = max(start, 0), min(start + int(width), n_cols)
        if lo < hi:
            if x.dtype == np.uint8:
                x[ch, lo:hi] = np.clip(x[ch, lo:hi].astype(np.int32) + int(amplitude), 0, 255).astype(np.uint8)
            else:
                x[ch, lo:hi] += x.dtype.type(amplitude)


def pulse_positions(n_pulses: int, n_dm: int, n_samples: int, seed: int):
    """Seeded (dm_index, t0) pairs for injected pulses, t0 in the first 3/4
    of the output span."""
    rng = rng_for(seed + 7919)
    dms = rng.integers(0, n_dm, size=n_pulses)
    ts = rng.integers(0, max(1, (3 * n_samples) // 4), size=n_pulses)
    return [(int(d), int(t)) for d, t in zip(dms, ts)]


def n_pulses_for(name: str) -> int:
    return {"tiny": 1, "apertif": 4, "lofar": 2}.get(name, 0)


def make_input(setup: Setup, n_in_samples: int, dtype: str, arrivals: Optional[dict] = None,
               stride: Optional[int] = None) -> np.ndarray:
    """Noise input [channels][stride] of ``dtype`` ('f32', 'f16', 'u8') with
    the workload's pulses.  ``arrivals`` maps dm_index -> per-channel arrival
    offsets for each pulse (supplied by the caller); pulses whose DM is
    missing from it are skipped."""
    stride = int(stride or n_in_samples)
    c = setup.n_channels
    if dtype == "f32":
        x = noise_f32(c, stride, setup.seed)
    elif dtype == "f16":
        x = noise_f16(c, stride, setup.seed)
    elif dtype == "u8":
        x = noise_u8(c, stride, setup.seed)
    else:
        raise ValueError("dtype must be f32, f16 or u8")
    if arrivals:
        amp = PULSE_AMPLITUDE if dtype != "u8" else 3 * 16.0
        for dm_i, t0 in pulse_sites(setup):
            if dm_i in arrivals:
                inject_pulse(x, arrivals[dm_i], t0, amp, PULSE_WIDTH)
    return x


def pulse_sites(setup: Setup):
    """The (dm_index, t0) pulse sites of a workload."""
    if setup.name == "tiny":
        return [(TINY_PULSE_DM_INDEX, 1000)]
    n = n_pulses_for(setup.name) if setup.name in ("apertif", "lofar") else 1
    return pulse_positions(n, setup.n_dm, setup.n_samples, setup.seed)
