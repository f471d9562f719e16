// Plans: argument checks, the FP64 delay table and the per-tile offset tables.
//
// The delay law is Sec. II, Eq. (1) of Sclocco et al.: a channel at f MHz lags
// the highest frequency f_h by 4150 * DM * (1/f^2 - 1/f_h^2) seconds.  Sampled
// at t_samp and rounded to the nearest sample (ties to even), this is the
// delay table that Sec. III-A says is computed ahead of the sums.  This file is
// compiled with -ffp-contract=off: every binary64 operation below is one IEEE
// operation in the order written.
#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <limits>
#include <new>

#include "internal.h"

namespace dd {

static thread_local std::string g_last_error;

void set_error(const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    g_last_error = buf;
}

void clear_error() { g_last_error.clear(); }

int fail(int code, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    g_last_error = buf;
    return code;
}

const char *last_error() { return g_last_error.c_str(); }

static bool fault_inject_alloc() {
    const char *e = std::getenv("DD_FAULT_INJECT");
    return e && std::strcmp(e, "alloc") == 0;
}

// Delay of channel ch at trial DM i, in samples, before the integer cast.
static double delay_samples(double f_min, double df, double t_samp, double dm_first,
                            double dm_step, int32_t C, int32_t i, int32_t ch) {
    const double f_top = f_min + static_cast<double>(C - 1) * df;  // highest channel
    const double f = f_min + static_cast<double>(ch) * df;
    const double dm = dm_first + static_cast<double>(i) * dm_step;
    const double k = 1.0 / (f * f) - 1.0 / (f_top * f_top);       // MHz^-2
    return std::rint(((4150.0 * dm) * k) / t_samp);
}

static inline int32_t offset_of(const dd_plan *p, int direction, int32_t r, int32_t a) {
    // Forward: O[ch][i] = delay[i][ch]; adjoint: O[i][ch] = -delay[i][ch].
    return direction == DD_FORWARD ? p->delay[(int64_t)a * p->C + r] : -p->delay[(int64_t)r * p->C + a];
}

// Register-window records: dwords per (row, wave) and rows per table (padded
// to whole chunks of waves * rpw rows).
static int32_t regwin_rd(const Variant &v) { return 1 + v.items_acc / 4; }
static int64_t regwin_rows(const Variant &v, int32_t rows) {
    const int64_t cr = (int64_t)v.waves * v.rpw;
    return (rows + cr - 1) / cr * cr;
}

void compute_layout(const dd_plan *p, int direction, const Variant &v, bool build, Layout *L, int32_t r0,
                    int32_t r1) {
    const int32_t R = direction == DD_FORWARD ? p->C : p->D;
    const int32_t A = direction == DD_FORWARD ? p->D : p->C;
    const int32_t TA = v.ta(), TT = v.tt();
    const int32_t n_tiles = (A + TA - 1) / TA;
    if (r1 < 0)
        r1 = R;
    const int32_t Rb = r1 - r0;  // rows of the block the tables hold (index r - r0)
    *L = Layout();
    L->n_tiles = n_tiles;
    // A block must be non-empty and, for the staged kinds, start on a whole
    // chunk of rows; the direct kind splits rows its own way (whole plans only).
    const int32_t cr = v.kind == KIND_LDS && v.kmax == 0 ? 1 : v.waves * std::max(1, v.rpw);
    if (r0 < 0 || r1 > R || r0 >= r1 || r0 % cr != 0 || (v.kind == KIND_DIRECT && (r0 != 0 || r1 != R)))
        return;
    // Skewed tiles (staged kinds): within an accumulator tile, row a's tiles
    // start skew[a] samples later, skew[a] being the offset of row a from the
    // tile's first row averaged over the block's first and last input rows
    // (the delays are a product of a DM and a channel term, monotone in both,
    // so these rows bound the offset differences), rounded down to a multiple
    // of 4 samples.  The tables then hold O[r][a] - skew[a]: their spread
    // across a tile shrinks from the widest row's to half the change over
    // the block, and the kernels store tile sample tau at tau - skew[a].
    std::vector<int32_t> sk;
    int32_t max_skew = 0;
    if (block_capable(v)) {
        sk.assign(A, 0);
        for (int32_t k = 0; k < n_tiles; ++k) {
            const int32_t a0 = k * TA, a1 = std::min(A, a0 + TA);
            int64_t lo = std::numeric_limits<int64_t>::max();
            std::vector<int64_t> raw(a1 - a0);
            for (int32_t a = a0; a < a1; ++a) {
                const int64_t d0 = (int64_t)offset_of(p, direction, r0, a) - offset_of(p, direction, r0, a0);
                const int64_t d1 = (int64_t)offset_of(p, direction, r1 - 1, a) - offset_of(p, direction, r1 - 1, a0);
                const int64_t sum = d0 + d1;
                raw[a - a0] = sum >= 0 ? sum / 2 : -((-sum + 1) / 2);  // floor((d0 + d1) / 2)
                lo = std::min(lo, raw[a - a0]);
            }
            for (int32_t a = a0; a < a1; ++a) {
                sk[a] = static_cast<int32_t>((raw[a - a0] - lo) / 4 * 4);
                max_skew = std::max(max_skew, sk[a]);
            }
        }
        if (max_skew == 0)
            sk.clear();
    }
    // Offsets as the tables hold them.
    auto off = [&](int32_t r, int32_t a) { return offset_of(p, direction, r, a) - (sk.empty() ? 0 : sk[a]); };
    if (build) {
        L->base.resize((size_t)n_tiles * Rb);
        if (v.kind != KIND_REGWIN)
            L->rel.resize((size_t)n_tiles * Rb * TA);
        else  // rows padded to whole chunks; padding records stay zero
            L->recs.assign((size_t)n_tiles * v.waves * regwin_rows(v, Rb) * regwin_rd(v), 0);
    }
    int32_t max_spread = 0;
    int32_t max_reach = 0;  // largest (offset - staged-row start) + 1 over rows and tiles
    int64_t need = 0;  // regwin: largest staged-row index a lane window touches, + 1
    bool ok = true;
    // Row spans: per (accumulator tile, time tile), the rows [lo, hi) with at
    // least one operand index t + O[r][a] inside [0, in_valid); the others add
    // only zeros there.  Rows are kept when the hull of their operand indices
    // meets the input, so the span is conservative.
    const bool want_span =
        build && (v.kind == KIND_REGWIN || v.kind == KIND_DIRECT || (v.kind == KIND_LDS && v.kmax > 0));
    const int64_t n_t = direction == DD_FORWARD ? p->S : p->T_in;
    const int64_t in_valid = direction == DD_FORWARD ? p->T_in : p->S;
    const int32_t n_t_tiles = static_cast<int32_t>((n_t + max_skew + TT - 1) / TT);
    L->n_t_tiles = n_t_tiles;
    std::vector<int32_t> row_lo, row_hi;
    if (want_span) {
        L->span.assign(static_cast<size_t>(n_tiles) * n_t_tiles * 2, 0);
        row_lo.resize(R);
        row_hi.resize(R);
    }
    for (int32_t k = 0; k < n_tiles && ok; ++k) {
        for (int32_t r = 0; r < R && ok; ++r) {
            int32_t lo = std::numeric_limits<int32_t>::max(), hi = std::numeric_limits<int32_t>::min();
            for (int32_t j = 0; j < TA; ++j) {
                const int32_t o = off(r, std::min(A - 1, k * TA + j));  // ragged tile repeats its last row
                lo = std::min(lo, o);
                hi = std::max(hi, o);
            }
            if (want_span) {  // spans cover every row; the rest only the block's
                row_lo[r] = lo;
                row_hi[r] = hi;
            }
            if (r < r0 || r >= r1)
                continue;
            const int32_t rb = r - r0;
            max_spread = std::max(max_spread, hi - lo);
            // Register-window rows start on a multiple of 4 samples, so the
            // staging's 16-byte loads are aligned for every input type
            // (floor, also for the adjoint's negative offsets).
            const int32_t b = v.kind == KIND_REGWIN ? lo - (((lo % 4) + 4) % 4) : lo;
            max_reach = std::max(max_reach, hi - b + 1);
            if (build)
                L->base[(size_t)k * Rb + rb] = b;
            if (v.kind != KIND_REGWIN) {
                if (build)
                    for (int32_t j = 0; j < TA; ++j)
                        L->rel[((size_t)k * Rb + rb) * TA + j] = off(r, std::min(A - 1, k * TA + j)) - lo;
                continue;
            }
            const int32_t TDW = v.items_acc;
            const int32_t S = v.items_t / 4;  // window quads per lane step (see regwin_asm.h)
            const int32_t align = 4 * S;      // window starts on multiples of S quads
            for (int32_t w = 0; w < v.waves; ++w) {
                int32_t wmin = std::numeric_limits<int32_t>::max(), wmax = 0;
                for (int32_t j = 0; j < TDW; ++j) {
                    const int32_t o = off(r, std::min(A - 1, k * TA + w * TDW + j)) - b;
                    wmin = std::min(wmin, o);
                    wmax = std::max(wmax, o);
                }
                const int32_t ws = wmin - wmin % align;
                const int32_t nq = (wmax - ws + v.items_t + 3) / 4;
                if (4 * nq > v.nwr) {
                    ok = false;  // this wave's delays spread wider than its register window
                    break;
                }
                // Quads past the first S are loaded in pairs (regwin_asm.h): the
                // staged row must hold the rounded-up count, capped at the window.
                const int32_t nq_loaded = std::min(v.nwr / 4, S + (nq - S + 1) / 2 * 2);
                need = std::max<int64_t>(need, (int64_t)63 * v.items_t + ws + 4 * std::max(nq, nq_loaded));
                if (build) {
                    const int32_t c = ws / 4;
                    const int32_t u_bytes = 16 * (S == 1 ? c : c + c / S);  // padded LDS layout
                    const int32_t RD = regwin_rd(v);
                    int32_t *rec = &L->recs[(((size_t)k * v.waves + w) * regwin_rows(v, Rb) + rb) * RD];
                    rec[0] = u_bytes | (nq << 20);
                    for (int32_t j = 0; j < TDW; ++j) {
                        const uint32_t o = (uint32_t)(off(r, std::min(A - 1, k * TA + w * TDW + j)) -
                                                      b - ws);  // 0 <= o <= nwr - items_t < 256
                        rec[1 + j / 4] = (int32_t)((uint32_t)rec[1 + j / 4] | (o << (8 * (j % 4))));
                    }
                }
            }
        }
        if (want_span && ok) {
            for (int32_t j = 0; j < n_t_tiles; ++j) {
                const int64_t t_first = static_cast<int64_t>(j) * TT;
                const int64_t t_last = std::min<int64_t>(n_t + max_skew, t_first + TT) - 1;
                int32_t first = R, last = -1;
                for (int32_t r = 0; r < R; ++r) {
                    if (t_first + row_lo[r] <= in_valid - 1 && t_last + row_hi[r] >= 0) {
                        first = std::min(first, r);
                        last = r;
                    }
                }
                int32_t *sp = &L->span[((size_t)k * n_t_tiles + j) * 2];
                sp[0] = last < 0 ? 0 : first;
                sp[1] = last < 0 ? 0 : last + 1;
            }
        }
    }
    L->max_spread = max_spread;
    if (!ok)
        return;
    if (build)
        L->skew = sk;
    // Spans that skip nothing (every forward plan: the input covers every
    // operand) are dropped; the kernels then take all rows.
    bool skips = false;
    for (size_t i = 0; i < L->span.size() && !skips; i += 2)
        skips = L->span[i] != 0 || L->span[i + 1] != R;
    if (!skips)
        L->span.clear();
    const int64_t lds_limit = 160 * 1024;
    if (v.kind == KIND_DIRECT) {
        L->wcap = 0;
        L->rows_per_chunk = 0;
        L->lds_bytes = 0;
    } else if (v.kind == KIND_LDS && v.kmax > 0) {
        // Prefetched staging: rows padded to whole 64-sample pieces, two buffers.
        const int64_t w64 = ((int64_t)TT + max_spread + 63) & ~int64_t(63);
        const int64_t rows = (int64_t)v.waves * v.rpw;
        if (w64 > (int64_t)64 * v.kmax || 2 * rows * w64 * 4 > lds_limit)
            return;
        L->wcap = (int32_t)w64;
        L->rows_per_chunk = (int32_t)rows;
        L->lds_bytes = (int32_t)(2 * rows * w64 * 4);
    } else if (v.kind == KIND_LDS) {
        const int64_t w4 = ((int64_t)TT + max_spread + 3) & ~int64_t(3);
        const int64_t row_bytes = w4 * 4;
        if (row_bytes > lds_limit)
            return;
        int64_t rpc = (64 * 1024) / row_bytes;  // leave room for two or more work-groups per CU
        rpc = std::max<int64_t>(1, std::min<int64_t>(rpc, 32));
        L->wcap = (int32_t)w4;
        L->rows_per_chunk = (int32_t)rpc;
        L->lds_bytes = (int32_t)(rpc * row_bytes);
    } else {
        const int64_t w64 = (std::max<int64_t>(need, (int64_t)TT + max_reach - 1) + 63) & ~int64_t(63);
        if (w64 > (int64_t)64 * v.kmax)
            return;
        const int64_t rows = (int64_t)v.waves * v.rpw;
        const int64_t S = v.items_t / 4;
        const int64_t row_dw = S == 1 ? w64 : w64 / S * (S + 1);  // padded layout
        if (2 * rows * row_dw * 4 > lds_limit || (need >> 20) != 0)  // two chunk buffers
            return;
        L->wcap = (int32_t)w64;
        L->rows_per_chunk = (int32_t)rows;
        L->lds_bytes = (int32_t)(2 * rows * row_dw * 4);
    }
    L->feasible = true;
}

int32_t plan_rows(const dd_plan *p, int direction) { return direction == DD_FORWARD ? p->C : p->D; }

bool block_capable(const Variant &v) { return v.kind == KIND_REGWIN || v.kind == KIND_LDS; }

bool variant_fits(const dd_plan *p, int direction, const Variant &v, int32_t r0, int32_t r1) {
    if (r1 < 0)
        r1 = plan_rows(p, direction);
    const auto key = std::make_tuple(direction, (int)v.id, (int)r0, (int)r1);
    {
        std::lock_guard<std::mutex> lock(p->mu);
        auto it = p->fit.find(key);
        if (it != p->fit.end())
            return std::get<0>(it->second);
    }
    Layout L;
    compute_layout(p, direction, v, false, &L, r0, r1);
    std::lock_guard<std::mutex> lock(p->mu);
    p->fit[key] = std::make_tuple(L.feasible, L.wcap, L.rows_per_chunk);
    return L.feasible;
}

static int upload(const std::vector<int32_t> &h, int32_t **d) {
    *d = nullptr;
    if (h.empty())
        return DD_OK;
    if (hipMalloc(d, h.size() * sizeof(int32_t)) != hipSuccess) {
        (void)hipGetLastError();
        *d = nullptr;
        return fail(DD_ENOMEM, "device allocation of %zu table entries failed", h.size());
    }
    hipError_t e = hipMemcpy(*d, h.data(), h.size() * sizeof(int32_t), hipMemcpyHostToDevice);
    if (e != hipSuccess)
        return fail(DD_EHIP, "upload of tile tables failed: %s", hipGetErrorString(e));
    return DD_OK;
}

static void free_tables(TileTables &t) {
    (void)hipFree(t.d_base);
    (void)hipFree(t.d_rel);
    (void)hipFree(t.d_recs);
    (void)hipFree(t.d_span);
    (void)hipFree(t.d_skew);
    t = TileTables();
}

int plan_tables(const dd_plan *p, int direction, const Variant &v, const TileTables **out, int32_t r0, int32_t r1) {
    if (r1 < 0)
        r1 = plan_rows(p, direction);
    int dev = 0;
    DD_HIP_TRY(hipGetDevice(&dev));
    const auto key = std::make_tuple(dev, direction, (int)v.id, (int)r0, (int)r1);
    {
        std::lock_guard<std::mutex> lock(p->mu);
        auto it = p->tables.find(key);
        if (it != p->tables.end()) {
            *out = &it->second;
            return DD_OK;
        }
    }
    Layout L;
    try {
        compute_layout(p, direction, v, true, &L, r0, r1);
    } catch (const std::bad_alloc &) {
        return fail(DD_ENOMEM, "host allocation of tile tables failed");
    }
    if (!L.feasible)
        return fail(DD_EUNSUPPORTED, "tile variant %d cannot serve this plan (delay spread too wide)", v.id);
    if (fault_inject_alloc())
        return fail(DD_ENOMEM, "device allocation of tile tables failed (DD_FAULT_INJECT=alloc)");
    TileTables t;
    t.n_tiles = L.n_tiles;
    t.wcap = L.wcap;
    t.rows_per_chunk = L.rows_per_chunk;
    t.lds_bytes = L.lds_bytes;
    t.n_t_tiles = L.n_t_tiles;
    int rc = upload(L.base, &t.d_base);
    if (rc == DD_OK)
        rc = upload(L.rel, &t.d_rel);
    if (rc == DD_OK)
        rc = upload(L.recs, &t.d_recs);
    if (rc == DD_OK)
        rc = upload(L.span, &t.d_span);
    if (rc == DD_OK)
        rc = upload(L.skew, &t.d_skew);
    if (rc != DD_OK) {
        free_tables(t);
        return rc;
    }
    std::lock_guard<std::mutex> lock(p->mu);
    auto ins = p->tables.emplace(key, t);
    if (!ins.second)
        free_tables(t);  // another thread built it first
    *out = &ins.first->second;
    p->host_tables.emplace(std::make_tuple(direction, (int)v.id, (int)r0, (int)r1), std::move(L));
    return DD_OK;
}

void release_block_tables(const dd_plan *p, int direction, const std::vector<Block> &keep) {
    const int32_t R = plan_rows(p, direction);
    int cur = 0;
    const bool have_dev = hipGetDevice(&cur) == hipSuccess;
    std::lock_guard<std::mutex> lock(p->mu);
    for (auto it = p->tables.begin(); it != p->tables.end();) {
        const int dev = std::get<0>(it->first), dir = std::get<1>(it->first), id = std::get<2>(it->first);
        const int r0 = std::get<3>(it->first), r1 = std::get<4>(it->first);
        bool kept = dir != direction || (r0 == 0 && r1 == R);
        for (const Block &b : keep)
            kept = kept || (b.variant == id && b.r0 == r0 && b.r1 == r1);
        if (kept) {
            ++it;
            continue;
        }
        if (have_dev)
            (void)hipSetDevice(dev);
        free_tables(it->second);
        p->host_tables.erase(std::make_tuple(dir, id, r0, r1));
        it = p->tables.erase(it);
    }
    if (have_dev)
        (void)hipSetDevice(cur);
}

const Layout *plan_host_layout(const dd_plan *p, int direction, int32_t variant, int32_t r0, int32_t r1) {
    if (r1 < 0)
        r1 = plan_rows(p, direction);
    std::lock_guard<std::mutex> lock(p->mu);
    auto it = p->host_tables.find(std::make_tuple(direction, (int)variant, (int)r0, (int)r1));
    return it == p->host_tables.end() ? nullptr : &it->second;
}

void args_dims(const dd_plan *p, int direction, const void *in, int64_t in_stride, float *out, int64_t out_stride,
               SrsArgs *a) {
    a->in = in;
    a->in_stride = in_stride;
    a->out = out;
    a->out_stride = out_stride;
    if (direction == DD_FORWARD) {
        a->in_valid = p->T_in;
        a->n_t = p->S;
        a->n_acc = p->D;
        a->n_rows = p->C;
    } else {
        a->in_valid = p->S;
        a->n_t = p->T_in;
        a->n_acc = p->C;
        a->n_rows = p->D;
    }
    a->r_begin = 0;
    a->r_end = a->n_rows;
    a->carry = 0;
}

int make_args(const dd_plan *p, int direction, const Variant &v, const void *in, int64_t in_stride,
              float *out, int64_t out_stride, SrsArgs *a, int32_t r0, int32_t r1) {
    if (r1 < 0)
        r1 = plan_rows(p, direction);
    const TileTables *t = nullptr;
    int rc = plan_tables(p, direction, v, &t, r0, r1);
    if (rc != DD_OK)
        return rc;
    args_dims(p, direction, in, in_stride, out, out_stride, a);
    a->r_begin = r0;
    a->r_end = r1;
    a->carry = r0 > 0 ? 1 : 0;  // blocks run in row order
    a->rel = t->d_rel;
    a->base = t->d_base;
    a->recs = t->d_recs;
    a->span = t->d_span;
    a->skew = t->d_skew;
    a->n_t_tiles = t->n_t_tiles;
    a->wcap = t->wcap;
    a->rows_per_chunk = t->rows_per_chunk;
    a->lds_bytes = t->lds_bytes;
    return DD_OK;
}

}  // namespace dd

using namespace dd;

extern "C" {

int dd_plan_create(dd_plan **out, int32_t n_channels, double f_min_mhz, double df_mhz,
                   double t_samp_s, double dm_first, double dm_step, int32_t n_dm,
                   int64_t n_samples) {
    clear_error();
    if (!out)
        return fail(DD_EINVAL, "out is NULL");
    *out = nullptr;
    if (n_channels < 1)
        return fail(DD_EINVAL, "n_channels must be >= 1 (got %d)", n_channels);
    if (n_dm < 1)
        return fail(DD_EINVAL, "n_dm must be >= 1 (got %d)", n_dm);
    if (n_samples < 1)
        return fail(DD_EINVAL, "n_samples must be >= 1 (got %lld)", (long long)n_samples);
    const double vals[] = {f_min_mhz, df_mhz, t_samp_s, dm_first, dm_step};
    for (double v : vals)
        if (!std::isfinite(v))
            return fail(DD_EINVAL, "plan parameters must be finite");
    if (!(f_min_mhz > 0.0))
        return fail(DD_EINVAL, "f_min_mhz must be > 0 (got %g)", f_min_mhz);
    if (!(df_mhz > 0.0))
        return fail(DD_EINVAL, "df_mhz must be > 0 (got %g)", df_mhz);
    if (!(t_samp_s > 0.0))
        return fail(DD_EINVAL, "t_samp_s must be > 0 (got %g)", t_samp_s);
    if (dm_first < 0.0)
        return fail(DD_EINVAL, "dm_first must be >= 0 (got %g)", dm_first);
    if (dm_step < 0.0)
        return fail(DD_EINVAL, "dm_step must be >= 0 (got %g)", dm_step);
    if (!std::isfinite(f_min_mhz + static_cast<double>(n_channels - 1) * df_mhz) ||
        !std::isfinite(dm_first + static_cast<double>(n_dm - 1) * dm_step))
        return fail(DD_EINVAL, "frequency or DM range overflows");

    dd_plan *p = nullptr;
    try {
        p = new dd_plan();
        p->delay.resize((size_t)n_dm * n_channels);
    } catch (const std::bad_alloc &) {
        delete p;
        return fail(DD_ENOMEM, "host allocation of the delay table failed");
    }
    p->C = n_channels;
    p->D = n_dm;
    p->S = n_samples;
    p->f_min = f_min_mhz;
    p->df = df_mhz;
    p->t_samp = t_samp_s;
    p->dm_first = dm_first;
    p->dm_step = dm_step;
    int32_t maxd = 0;
    for (int32_t i = 0; i < n_dm; ++i) {
        for (int32_t ch = 0; ch < n_channels; ++ch) {
            const double r = delay_samples(f_min_mhz, df_mhz, t_samp_s, dm_first, dm_step, n_channels, i, ch);
            if (!(r >= 0.0 && r <= 2147483647.0)) {
                delete p;
                return fail(DD_EINVAL, "delay of DM index %d, channel %d (%g samples) does not fit int32", i,
                            ch, r);
            }
            const int32_t d = static_cast<int32_t>(r);
            p->delay[(size_t)i * n_channels + ch] = d;
            maxd = std::max(maxd, d);
        }
    }
    p->max_delay = maxd;
    p->T_in = n_samples + maxd;
    if (p->T_in >= (int64_t(1) << 29)) {
        delete p;
        return fail(DD_EINVAL, "n_samples + max delay must be below 2^29 samples");
    }
    *out = p;
    return DD_OK;
}

int dd_plan_destroy(dd_plan *p) {
    clear_error();
    if (!p)
        return DD_OK;
    int cur = 0;
    bool have_dev = hipGetDevice(&cur) == hipSuccess;
    for (auto &kv : p->tables) {
        const int dev = std::get<0>(kv.first);
        if (have_dev)
            (void)hipSetDevice(dev);
        free_tables(kv.second);
    }
    if (have_dev)
        (void)hipSetDevice(cur);
    delete p;
    return DD_OK;
}

int dd_plan_dims(const dd_plan *p, int32_t *n_channels, int32_t *n_dm, int64_t *n_samples) {
    clear_error();
    if (!p)
        return fail(DD_EINVAL, "plan is NULL");
    if (n_channels)
        *n_channels = p->C;
    if (n_dm)
        *n_dm = p->D;
    if (n_samples)
        *n_samples = p->S;
    return DD_OK;
}

int dd_plan_max_delay(const dd_plan *p, int32_t *out) {
    clear_error();
    if (!p || !out)
        return fail(DD_EINVAL, "NULL argument");
    *out = p->max_delay;
    return DD_OK;
}

int dd_plan_input_samples(const dd_plan *p, int64_t *out) {
    clear_error();
    if (!p || !out)
        return fail(DD_EINVAL, "NULL argument");
    *out = p->T_in;
    return DD_OK;
}

int dd_plan_delay_table(const dd_plan *p, int32_t *host_dst) {
    clear_error();
    if (!p || !host_dst)
        return fail(DD_EINVAL, "NULL argument");
    std::memcpy(host_dst, p->delay.data(), p->delay.size() * sizeof(int32_t));
    return DD_OK;
}

const char *dd_last_error(void) { return dd::last_error(); }

const char *dd_version(void) { return "libdedisp 0.1 (gfx950)"; }

}  // extern "C"
