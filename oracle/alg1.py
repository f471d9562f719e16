"""Pure-Python dedispersion for tiny inputs (test infrastructure only).

Written from Sclocco et al., Sec. III-A, Algorithm 1 (loops over DM, then
sample, then channel, one running sum per output) and Sec. II, Eq. (1) for
the delays.  Python floats are IEEE binary64, so every sum is FP64.
"""
from __future__ import annotations


def delays(n_channels, f_min, df, t_samp, dm_first, dm_step, n_dm):
    """Eq. (1) per (DM, channel), in samples, rounded half-to-even.

    Channel ch is at f_min + ch*df; the reference frequency is the highest
    channel's.  Python's round() on a float is round-half-to-even.
    """
    f_h = f_min + (n_channels - 1) * df
    table = []
    for i in range(n_dm):
        dm = dm_first + i * dm_step
        row = []
        for ch in range(n_channels):
            f = f_min + ch * df
            seconds = (4150.0 * dm) * (1.0 / (f * f) - 1.0 / (f_h * f_h))
            row.append(int(round(seconds / t_samp)))
        table.append(row)
    return table


def dedisperse(x, delay, n_samples):
    """Algorithm 1: out[dm][sample] = sum over channels of x[ch][sample + delay]."""
    n_dm = len(delay)
    n_ch = len(delay[0]) if n_dm else 0
    out = []
    for dm in range(n_dm):
        row = []
        for sample in range(n_samples):
            d_sample = 0.0
            for ch in range(n_ch):
                d_sample += float(x[ch][sample + delay[dm][ch]])
            row.append(d_sample)
        out.append(row)
    return out


def adjoint(gy, delay, n_input_samples):
    """Transpose of Algorithm 1 by its definition: each input sample collects
    every output that read it."""
    n_dm = len(delay)
    n_ch = len(delay[0]) if n_dm else 0
    n_samples = len(gy[0]) if n_dm else 0
    gx = [[0.0] * n_input_samples for _ in range(n_ch)]
    for ch in range(n_ch):
        for tau in range(n_input_samples):
            acc = 0.0
            for dm in range(n_dm):
                t = tau - delay[dm][ch]
                if 0 <= t < n_samples:
                    acc += float(gy[dm][t])
            gx[ch][tau] = acc
    return gx
