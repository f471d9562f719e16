"""Generate regwin_asm.h: the inline-assembly row step of the register-window
dedispersion kernel (gfx950).

Each lane keeps IT consecutive output samples of TDW accumulator rows in
VGPRs.  For one input row it copies a window of up to NWR consecutive input
samples from LDS into VGPRs, then every accumulator row a adds
window[off_a + j] (j < IT) at its own wave-uniform offset off_a.  CDNA's VGPR
index mode (s_set_gpr_idx_on with SRC0) adds an SGPR index to the first
source operand of every VALU instruction until s_set_gpr_idx_off, so one index
switch serves IT additions:

    s_set_gpr_idx_on s_off_a, gpr_idx(SRC0)
    v_add_f32 acc[a][0], win[0], acc[a][0]      ; reads win[off_a + 0]
    ...
    v_add_f32 acc[a][IT-1], win[IT-1], acc[a][IT-1]
    s_set_gpr_idx_off

LDS layout of a staged row: 16-byte quads with one padding quad after every
S = IT/4 quads (none when S = 1), so the lanes' windows, S quads apart, start
in distinct bank groups and ds_read_b128 is conflict-free.  Logical quad Q
lives at physical quad Q + floor(Q/S); a window starting at logical quad
S*l + c (c a multiple of S) has its q-th quad at physical
(S+1)*l + (c + c/S) + q + floor(q/S): a per-lane base plus compile-time
offsets.

Only the quads a row needs are loaded (rounded up to a pair past the first
S): the first S unconditionally, the rest two at a time behind a
compare-and-branch on the row's quad count.  Accumulators and the
window are pinned with explicit-register constraints; the window is the
output of load() and an input of add(), so scalar work can be placed between
the LDS wait and the additions.

    python gen_regwin_asm.py      # rewrites regwin_asm.h next to this file
"""
from __future__ import annotations

import os

# (IT, TDW, NWR, ACC0): samples per lane, accumulator rows per wave, window
# registers, first accumulator VGPR.  The window registers follow the
# accumulators.
CONFIGS = [
    (8, 8, 40, 24),
    (8, 4, 32, 24),
    (16, 4, 48, 24),
    (4, 8, 32, 24),
    (8, 16, 48, 24),
    (8, 4, 44, 24),   # wider windows for the adjoint (delays spread more across channels)
    (8, 8, 76, 24),
    (8, 12, 56, 24),  # more accumulator rows per window: fewer LDS bytes per addition
    (16, 8, 60, 24),
]

# Register-tuple widths LLVM's AMDGPU backend can bind to one constraint.
TUPLES = (32, 16, 12, 11, 10, 9, 8, 7, 6, 5, 4, 3, 2, 1)


def split(n):
    out = []
    while n:
        t = next(t for t in TUPLES if t <= n)
        out.append(t)
        n -= t
    return out


def vec_type(n):
    return "float" if n == 1 else "v%df" % n


def quad_offset(q, s):
    """Physical quad offset of the window's q-th quad from its first."""
    return q if s == 1 else q + q // s


def gen_config(it, tdw, nwr, acc0):
    s = it // 4
    n_acc = it * tdw
    w0 = acc0 + n_acc
    nq_max = nwr // 4
    acc_parts = split(n_acc)
    name = "RegWin<%d, %d, %d>" % (it, tdw, nwr)
    L = []
    L.append("template <>")
    L.append("struct %s {" % name)
    L.append("    static constexpr int IT = %d, TDW = %d, NWR = %d, S = %d, NQ_MIN = %d, NQ_MAX = %d;"
             % (it, tdw, nwr, s, s, nq_max))
    L.append("    static constexpr int ACC0 = %d, WIN0 = %d;" % (acc0, w0))
    L.append("    struct Acc {")
    for k, n in enumerate(acc_parts):
        L.append("        %s p%d;" % (vec_type(n), k))
    L.append("    };")
    L.append("    __device__ static __forceinline__ float get_acc(const Acc &x, int i) {")
    start = 0
    for k, n in enumerate(acc_parts):
        L.append("        if (i < %d) return x.p%d[i - %d];" % (start + n, k, start) if n > 1
                 else "        if (i == %d) return x.p%d;" % (start, k))
        start += n
    L.append("        __builtin_unreachable();")
    L.append("    }")
    L.append("    __device__ static __forceinline__ void set_acc(Acc &x, int i, float v) {")
    start = 0
    for k, n in enumerate(acc_parts):
        L.append("        if (i < %d) { x.p%d[i - %d] = v; return; }" % (start + n, k, start) if n > 1
                 else "        if (i == %d) { x.p%d = v; return; }" % (start, k))
        start += n
    L.append("    }")
    outs = []
    reg = acc0
    for k, n in enumerate(acc_parts):
        outs.append('"+{v[%d:%d]}"(a.p%d)' % (reg, reg + n - 1, k) if n > 1 else '"+{v%d}"(a.p%d)' % (reg, k))
        reg += n

    def loads(win0, addr, nq):
        # Quads past the first S come in pairs behind one compare-and-branch:
        # at most one quad more than the row needs is read (the layout keeps
        # it inside the staged row), for half the scalar instructions.
        out = []
        for q in range(nq_max):
            if q >= s and (q - s) % 2 == 0:
                out.append('            "s_cmp_lt_u32 %%[%s], %d\\n\\t"' % (nq, q + 1))
                out.append('            "s_cbranch_scc1 L_rw_ld_%=\\n\\t"')
            out.append('            "ds_read_b128 v[%d:%d], %%[%s] offset:%d\\n\\t"'
                       % (win0 + 4 * q, win0 + 4 * q + 3, addr, 16 * quad_offset(q, s)))
        out.append('            "L_rw_ld_%=:\\n\\t"')
        return out

    def adds(win0):
        # One index-mode region: s_set_gpr_idx_idx moves the index between
        # accumulator rows without leaving the mode.
        out = ['            "s_set_gpr_idx_on %[o0], gpr_idx(SRC0)\\n\\t"']
        for a in range(tdw):
            if a:
                out.append('            "s_set_gpr_idx_idx %%[o%d]\\n\\t"' % a)
            for j in range(it):
                r = acc0 + a * it + j
                out.append('            "v_add_f32 v%d, v%d, v%d\\n\\t"' % (r, win0 + j, r))
        out.append('            "s_set_gpr_idx_off\\n\\t"')
        return out

    def clobbers(regs):
        clob = ['"v%d"' % r for r in regs] + ['"scc"', '"m0"', '"memory"']
        cl, line = [], "            : "
        for i, c in enumerate(clob):
            piece = c + (", " if i + 1 < len(clob) else ");")
            if len(line) + len(piece) > 110:
                cl.append(line.rstrip())
                line = "              "
            line += piece
        cl.append(line)
        return cl

    o_ins = ['[o%d] "s"(o[%d])' % (a, a) for a in range(tdw)]
    win_parts = split(nwr)

    # Window registers as values: load() defines them, add() reads them, so
    # scalar work can sit between the two (e.g. the next chunk's records).
    L.append("    struct Win {")
    for k, n in enumerate(win_parts):
        L.append("        %s p%d;" % (vec_type(n), k))
    L.append("    };")
    w_outs, w_ins = [], []
    reg = w0
    for k, n in enumerate(win_parts):
        rng = "v[%d:%d]" % (reg, reg + n - 1) if n > 1 else "v%d" % reg
        w_outs.append('"=&{%s}"(w.p%d)' % (rng, k))
        w_ins.append('"{%s}"(w.p%d)' % (rng, k))
        reg += n

    # Load nq window quads from LDS byte address `addr` and wait for them; dep
    # is an SGPR set to 0 after the wait (a data dependence that keeps later
    # scalar loads from being scheduled above it).  The row's packed offsets
    # pk (four bytes per dword) are unpacked into o[] between issuing the LDS
    # reads and waiting for them, so that scalar work overlaps their latency.
    L.append("    // addr: LDS byte address of this lane's first window quad; nq: quads to")
    L.append("    // load (NQ_MIN <= nq <= NQ_MAX).  Quads past nq are left undefined.")
    L.append("    // pk: the row's window offsets, four bytes per dword; o: unpacked.")
    L.append("    __device__ static __forceinline__ void load(Win &w, uint32_t addr, int nq, const uint32_t (&pk)[%d],"
             % (tdw // 4))
    L.append("                                                int (&o)[%d], int &dep) {" % tdw)
    L.append("        asm volatile(")
    L.extend(loads(w0, "addr", "nq"))
    for a in range(tdw):
        if a % 4 == 0:
            L.append('            "s_and_b32 %%[o%d], %%[pk%d], 0xff\\n\\t"' % (a, a // 4))
        elif a % 4 == 3:
            L.append('            "s_lshr_b32 %%[o%d], %%[pk%d], 24\\n\\t"' % (a, a // 4))
        else:
            L.append('            "s_bfe_u32 %%[o%d], %%[pk%d], 0x%x\\n\\t"' % (a, a // 4, 0x80000 | (8 * (a % 4))))
    L.append('            "s_waitcnt lgkmcnt(0)\\n\\t"')
    L.append('            "s_mov_b32 %[dep], 0\\n\\t"')
    L.append("            : " + ", ".join(w_outs + ['[o%d] "=&s"(o[%d])' % (a, a) for a in range(tdw)] + ['[dep] "=&s"(dep)']))
    L.append("            : " + ", ".join(['[addr] "v"(addr)', '[nq] "s"(nq)'] +
                                 ['[pk%d] "s"(pk[%d])' % (k, k) for k in range(tdw // 4)]))
    L.append('            : "scc", "memory");')
    L.append("    }")
    # Add the window at every accumulator row's offset o[a].
    L.append("    // o: per-accumulator-row window offsets, 0 <= o[a] <= NWR - IT.")
    L.append("    __device__ static __forceinline__ void add(Acc &a, const Win &w, const int (&o)[%d]) {" % tdw)
    L.append("        asm volatile(")
    L.extend(adds(w0))
    L.append("            : " + ", ".join(outs))
    L.append("            : " + ", ".join(w_ins + o_ins))
    L.append('            : "scc", "m0");')
    L.append("    }")
    L.append("};")
    return "\n".join(L)


def render(configs=None) -> str:
    """The full text of regwin_asm.h (for CONFIGS, or the given configs)."""
    out = [
        "// GENERATED by gen_regwin_asm.py -- do not edit by hand.",
        "// Inline-assembly row step of the register-window kernel (gfx950).",
        "#pragma once",
        "",
        "#include <cstdint>",
        "",
        "namespace dd {",
        "namespace dev {",
        "",
        "typedef float v2f __attribute__((ext_vector_type(2)));",
    ]
    for n in sorted({t for t in TUPLES if t > 2}):
        out.append("typedef float v%df __attribute__((ext_vector_type(%d)));" % (n, n))
    out += ["", "template <int IT, int TDW, int NWR>", "struct RegWin;", ""]
    for cfg in (CONFIGS if configs is None else configs):
        out.append(gen_config(*cfg))
        out.append("")
    out += ["}  // namespace dev", "}  // namespace dd", ""]
    return "\n".join(out)


def main(path=None):
    path = path or os.path.join(os.path.dirname(os.path.abspath(__file__)), "regwin_asm.h")
    with open(path, "w") as f:
        f.write(render())
    return path


if __name__ == "__main__":
    print(main())
