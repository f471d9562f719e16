"""Code-generation checks on the built device assembly (no GPU needed).

The register-window kernels pin accumulators and windows to fixed VGPRs via
inline assembly; their speed depends on keeping four waves per SIMD (at most
128 VGPRs) and on never touching scratch memory.  The build keeps the device
assembly of the kernel units (-save-temps); these tests read it."""
import os
import re

import pytest

from paper_1601_05052_amd import build


def _listing():
    texts = []
    for path, name in zip(build.listing_paths(), build.LISTED):
        src = os.path.join(build.CSRC, name)
        if not os.path.exists(path) or os.path.getmtime(path) < os.path.getmtime(src):
            pytest.skip("device assembly listing not built (python -m paper_1601_05052_amd.build)")
        with open(path) as f:
            texts.append(f.read())
    return "\n".join(texts)


def _kernels(text):
    """(name, vgpr_count, scratch bytes) of every kernel in the listing."""
    out = []
    for m in re.finditer(r"\.name:\s+(\S+)\n(.*?)\.vgpr_count:\s+(\d+)", text, re.S):
        scratch = re.search(r"\.private_segment_fixed_size:\s+(\d+)", m.group(2))
        out.append((m.group(1), int(m.group(3)), int(scratch.group(1)) if scratch else 0))
    return out


def test_register_window_kernels_have_no_scratch():
    ks = [k for k in _kernels(_listing()) if "regwin" in k[0]]
    assert ks
    for name, _, scratch in ks:
        assert scratch == 0, name


def test_occupancy_targets_met():
    """Variants compiled with an occupancy target of four waves per SIMD
    (template argument OCC = 4, the last one) fit in 128 VGPRs."""
    ks = [k for k in _kernels(_listing()) if "regwin" in k[0] and re.search(r"ELi4EEEv", k[0])]
    assert len(ks) >= 12  # variants 17, 18, 31 in three input types, single- and multi-beam
    for name, vgprs, _ in ks:
        assert vgprs <= 128, (name, vgprs)


def test_index_mode_regions_balanced():
    """Every VGPR-index-mode region opened in the kernels is closed."""
    text = _listing()
    for blk in re.findall(r";;#ASMSTART\n(.*?);;#ASMEND", text, re.S):
        assert blk.count("s_set_gpr_idx_on") == blk.count("s_set_gpr_idx_off"), blk[:120]


def test_no_packed_fp32_instructions():
    """Every kernel unit is built without packed FP32 arithmetic (v_pk_add_f32,
    v_pk_mul_f32, v_pk_fma_f32): ordinary float code only."""
    text = _listing()
    found = sorted(set(re.findall(r"\bv_pk_(?:add|mul|fma)_f32\b", text)))
    assert not found, found


def test_direct_kernels_have_no_scratch():
    ks = [k for k in _kernels(_listing()) if "direct" in k[0]]
    assert ks
    for name, _, scratch in ks:
        assert scratch == 0, name
