"""Streaming dedispersion (dd_realtime_*) on the GPU against the FP64 oracle.

The stream x (zero before time 0) is pushed in chunks of n_samples; push k
must equal the oracle's dedispersion of the window of stream times
[k*S - max_delay, (k+1)*S), i.e. the slice [k*S - max_delay, k*S - max_delay + S)
of the oracle's output over the whole zero-padded stream."""
import numpy as np
import pytest

import oracle
import synth
from paper_1601_05052_amd import Plan, Realtime, dedisperse
from tests import gates
from tests.gpu_util import sample_points, to_dev, to_host, torch_mod

pytestmark = pytest.mark.gpu


def stream_windows(x_full: np.ndarray, max_delay: int, S: int, k: int) -> np.ndarray:
    """Window of push k: stream times [k*S - max_delay, (k+1)*S), zeros before 0."""
    C = x_full.shape[0]
    padded = np.concatenate([np.zeros((C, max_delay), dtype=x_full.dtype), x_full], axis=1)
    return padded[:, k * S:k * S + S + max_delay]


def host_chunk(torch, a: np.ndarray, pinned: bool):
    t = torch.from_numpy(np.ascontiguousarray(a))
    return t.pin_memory() if pinned else t


def make_stream(dtype: str, C: int, n: int, seed: int) -> np.ndarray:
    if dtype == "u8":
        return synth.noise_u8(C, n, seed)
    if dtype == "f16":
        return synth.noise_f16(C, n, seed)
    return synth.noise_f32(C, n, seed)


@pytest.mark.parametrize("dtype", ["f32", "u8", "f16"])
def test_tiny_stream_against_oracle(dtype):
    torch = torch_mod()
    s = synth.TINY
    plan = Plan.from_setup(s)
    table = oracle.delay_table(*s.plan_args()[:7])
    S, M, K = s.n_samples, plan.max_delay, 4
    x = make_stream(dtype, s.n_channels, K * S, seed=11)
    tdt = {"f32": torch.float32, "u8": torch.uint8, "f16": torch.float16}[dtype]
    rt = Realtime(plan, tdt)
    full = oracle.dedisperse(np.concatenate([np.zeros((s.n_channels, M)), x.astype(np.float64)], axis=1), table,
                             K * S)
    for k in range(K):
        y = to_host(rt.push(host_chunk(torch, x[:, k * S:(k + 1) * S], pinned=(k % 2 == 0))))
        w = stream_windows(x, M, S, k).astype(np.float64)
        ref = oracle.dedisperse(w, table, S)
        assert np.array_equal(ref, full[:, k * S:(k + 1) * S])  # windows tile the stream
        if dtype == "u8":
            gates.exact(y, ref, what="u8 push %d" % k)
        else:
            gates.gate(y, ref, oracle.dedisperse(np.abs(w), table, S), what="%s push %d" % (dtype, k))
    assert rt.pushed == K
    rt.close()


@pytest.mark.parametrize("dtype,S", [("f32", 100), ("u8", 100), ("u8", 101), ("f16", 102), ("f16", 103)])
def test_chunks_shorter_than_max_delay_exact(dtype, S):
    """S < max_delay: a window spans several earlier chunks.  Chunk lengths
    whose byte size is and is not a multiple of 4 (the window tail is then
    moved by words or by samples).  Integer-valued samples: exact."""
    torch = torch_mod()
    args = (64, 1400.0, 1.5625, 5e-5, 0.0, 0.5, 128, S)
    plan = Plan(*args)
    table = oracle.delay_table(*args[:7])
    M, K = plan.max_delay, 9
    assert M > 3 * S
    if dtype == "u8":
        x = synth.noise_u8(64, K * S, seed=21)
    else:
        x = synth.integers_f32(64, K * S, seed=21)
        if dtype == "f16":
            x = x.astype(np.float16)
    tdt = {"f32": torch.float32, "u8": torch.uint8, "f16": torch.float16}[dtype]
    rt = Realtime(plan, tdt)
    for k in range(K):
        y = to_host(rt.push(host_chunk(torch, x[:, k * S:(k + 1) * S], pinned=True)))
        w = stream_windows(x, M, S, k).astype(np.float64)
        gates.exact(y, oracle.dedisperse(w, table, S), what="%s push %d" % (dtype, k))
    rt.close()


def test_strided_chunk_and_output_canaries():
    torch = torch_mod()
    s = synth.TINY
    plan = Plan.from_setup(s)
    table = oracle.delay_table(*s.plan_args()[:7])
    S, M = s.n_samples, plan.max_delay
    x = synth.integers_f32(s.n_channels, 3 * S, seed=31)
    rt = Realtime(plan, torch.float32)
    for k in range(3):
        wide = np.full((s.n_channels, S + 13), 99.0, dtype=np.float32)
        wide[:, :S] = x[:, k * S:(k + 1) * S]
        chunk = torch.from_numpy(wide).pin_memory()[:, :S]   # row stride S + 13
        out = torch.full((s.n_dm, S + 5), float("nan"), device="cuda")
        rt.push(chunk, out=out)
        o = to_host(out)
        assert np.all(np.isnan(o[:, S:]))
        gates.exact(o[:, :S], oracle.dedisperse(stream_windows(x, M, S, k), table, S), what="push %d" % k)
    rt.close()


def test_non_default_stream():
    torch = torch_mod()
    s = synth.TINY
    plan = Plan.from_setup(s)
    table = oracle.delay_table(*s.plan_args()[:7])
    S, M = s.n_samples, plan.max_delay
    x = synth.integers_f32(s.n_channels, 2 * S, seed=41)
    st = torch.cuda.Stream()
    with torch.cuda.stream(st):
        rt = Realtime(plan, torch.float32)
        outs = [rt.push(host_chunk(torch, x[:, k * S:(k + 1) * S], pinned=True)) for k in range(2)]
    st.synchronize()
    for k in range(2):
        gates.exact(to_host(outs[k]), oracle.dedisperse(stream_windows(x, M, S, k), table, S), what="push %d" % k)
    rt.close()


def test_apertif_stream_u8():
    """Full-size Apertif beam, u8 chunks: each push equals the one-shot forward
    on the same window bit for bit, and the oracle on sampled outputs."""
    torch = torch_mod()
    s = synth.APERTIF
    plan = Plan.from_setup(s)
    table = oracle.delay_table(*s.plan_args()[:7])
    S, M, K = s.n_samples, plan.max_delay, 3
    x = synth.noise_u8(s.n_channels, K * S, seed=51)
    rt = Realtime(plan, torch.uint8)
    for k in range(K):
        y = to_host(rt.push(host_chunk(torch, x[:, k * S:(k + 1) * S], pinned=True)))
        w = np.ascontiguousarray(stream_windows(x, M, S, k))
        one = to_host(dedisperse(to_dev(w), plan))
        gates.exact(y, one, what="push %d vs one-shot" % k)
        i, t = sample_points(s.n_dm, S, 5000, 60 + k)
        gates.exact(y[i, t], oracle.dedisperse_points(w, table, i, t), what="push %d sampled" % k)
    rt.close()
