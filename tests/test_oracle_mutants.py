"""Planted mistakes in copies of the oracle must trip at least one pin.

Each case rewrites one expression of ``oracle/dd_oracle.c`` in a temporary
copy, compiles it on the CPU and runs the full pin set against it.  All
mutants keep every memory access in bounds.
"""
import os

import pytest

import oracle
from oracle.build import SRC, build_oracle
from tests import pins

MUTANTS = {
    "floor_instead_of_rint": ("const double r = rint(samples);", "const double r = floor(samples);"),
    "band_edge_reference": ("f_min + (double)(C - 1) * df;", "f_min + (double)C * df;"),
    "dm_grid_off_by_one": ("dm_first + (double)i * dm_step;", "dm_first + (double)(i + 1) * dm_step;"),
    "constant_4148": ("(4150.0 * dm) * k;", "(4148.808 * dm) * k;"),
    "forward_drops_channel_0": ("            for (int32_t ch = 0; ch < C; ++ch) {\n                const double *row",
                                "            for (int32_t ch = 1; ch < C; ++ch) {\n                const double *row"),
    "forward_half_delay": ("x + (int64_t)ch * x_stride + delay[(int64_t)i * C + ch];",
                           "x + (int64_t)ch * x_stride + delay[(int64_t)i * C + ch] / 2;"),
    "forward_reversed_dm_rows": ("x + (int64_t)ch * x_stride + delay[(int64_t)i * C + ch];",
                                 "x + (int64_t)ch * x_stride + delay[(int64_t)(D - 1 - i) * C + ch];"),
    "forward_reversed_channels": ("x + (int64_t)ch * x_stride + delay[(int64_t)i * C + ch];",
                                  "x + (int64_t)ch * x_stride + delay[(int64_t)i * C + (C - 1 - ch)];"),
    "adjoint_half_delay": ("const int64_t tau = t + d;", "const int64_t tau = t + d / 2;"),
    "adjoint_drops_dm_0": ("        for (int32_t i = 0; i < D; ++i) {\n            const int64_t d",
                           "        for (int32_t i = 1; i < D; ++i) {\n            const int64_t d"),
    "adjoint_shift_by_one": ("if (tau >= 0 && tau < T_in)\n                    row[tau] += g[t];",
                             "if (tau >= 1 && tau < T_in)\n                    row[tau - 1] += g[t];"),
}


def test_unmutated_oracle_passes():
    pins.run_all(oracle.default())


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_mutant_is_caught(name, tmp_path):
    old, new = MUTANTS[name]
    src = open(SRC).read()
    assert src.count(old) == 1, "mutation site not found exactly once"
    mutated = tmp_path / "mutant.c"
    mutated.write_text(src.replace(old, new))
    lib = build_oracle(src=str(mutated), out=str(tmp_path / "libmutant.so"))
    mutant = oracle.COracle(lib)
    with pytest.raises(AssertionError):
        pins.run_all(mutant)


# Planted mistakes in copies of the pure-Python delay law (oracle/alg1.py).
ALG1_MUTANTS = {
    "truncate_instead_of_round": ("row.append(int(round(seconds / t_samp)))", "row.append(int(seconds / t_samp))"),
    "band_edge_reference": ("f_h = f_min + (n_channels - 1) * df", "f_h = f_min + n_channels * df"),
    "dm_grid_off_by_one": ("        dm = dm_first + i * dm_step\n", "        dm = dm_first + (i + 1) * dm_step\n"),
    "reversed_channels": ("            f = f_min + ch * df\n", "            f = f_min + (n_channels - 1 - ch) * df\n"),
}


def _mutated_module(path, old, new, name):
    import types
    src = open(path).read()
    assert src.count(old) == 1, "mutation site not found exactly once"
    mod = types.ModuleType(name)
    exec(compile(src.replace(old, new), name + ".py", "exec"), mod.__dict__)
    return mod


def test_unmutated_alg1_delays_pass():
    from oracle import alg1
    pins.check_alg1_delays(alg1.delays)


@pytest.mark.parametrize("name", sorted(ALG1_MUTANTS))
def test_alg1_mutant_is_caught(name):
    from oracle import alg1
    mod = _mutated_module(alg1.__file__, *ALG1_MUTANTS[name], "alg1_mutant")
    with pytest.raises(AssertionError):
        pins.check_alg1_delays(mod.delays)


# Planted mistakes in copies of the search oracle (oracle/search.py).
SEARCH_MUTANTS = {
    "sample_std": ("return mu, np.sqrt(np.mean((y - mu) ** 2))",
                   "return mu, np.sqrt(np.sum((y - mu) ** 2) / (len(y) - 1))"),
    "no_mean_subtraction": ("c = np.concatenate([[0.0], np.cumsum(y - mu)])",
                            "c = np.concatenate([[0.0], np.cumsum(y)])"),
    "width_not_sqrt": ("s = (c[w:] - c[:-w]) / (sigma * np.sqrt(w))", "s = (c[w:] - c[:-w]) / (sigma * w)"),
    "window_off_by_one": ("s = (c[w:] - c[:-w]) / (sigma * np.sqrt(w))",
                          "s = (c[w:] - c[:-w]) / (sigma * np.sqrt(w)); s = np.roll(s, 1)"),
    "widths_skip_one": ("return [1 << k for k in range(n_widths) if (1 << k) <= n_samples]",
                        "return [1 << k for k in range(1, n_widths) if (1 << k) <= n_samples]"),
    "ties_to_larger_width": ("if s[t] > best[0]:", "if s[t] >= best[0]:"),
    "ties_to_later_start": ("t = int(np.argmax(s))", "t = len(s) - 1 - int(np.argmax(s[::-1]))"),
}


def test_unmutated_search_oracle_passes():
    from oracle import search
    pins.run_search(search.search_row)


@pytest.mark.parametrize("name", sorted(SEARCH_MUTANTS))
def test_search_mutant_is_caught(name):
    from oracle import search
    mod = _mutated_module(search.__file__, *SEARCH_MUTANTS[name], "search_mutant")
    with pytest.raises(AssertionError):
        pins.run_search(mod.search_row)
