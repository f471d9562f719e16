// Internal declarations of libdedisp (not part of the C ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <map>
#include <mutex>
#include <string>
#include <tuple>
#include <vector>

#include "dedisp.h"

namespace dd {

// ------------------------------------------------------------------ errors
void set_error(const char *fmt, ...) __attribute__((format(printf, 1, 2)));
void clear_error();
int fail(int code, const char *fmt, ...) __attribute__((format(printf, 2, 3)));

#define DD_HIP_TRY(expr)                                                                   \
    do {                                                                                   \
        hipError_t e_ = (expr);                                                            \
        if (e_ != hipSuccess)                                                              \
            return ::dd::fail(DD_EHIP, "%s failed: %s", #expr, hipGetErrorString(e_));     \
    } while (0)

// ------------------------------------------------------------------ tiles
//
// Both directions are one computation, a "shifted-row sum":
//     out[a][t] = sum_r in[r][t + O[r][a]]    (in[r][g] = 0 outside [0, in_valid))
// Forward: rows r = channels, accumulator rows a = DMs, O[ch][i] = delay[i][ch].
// Adjoint: rows r = DMs, accumulator rows a = channels, O[i][ch] = -delay[i][ch].
// A work-group owns a tile of TA accumulator rows x TT samples.  For each input
// row it stages the window in[r][t0 + base .. t0 + base + TT + spread) in LDS,
// where base/spread are the min/range of O[r][.] over the tile.

enum Kind : int32_t {
    KIND_LDS = 0,     // one LDS read per addition, lanes strided by 64 samples
    KIND_REGWIN = 1,  // per-lane register window, offsets applied by VGPR index mode
    KIND_DIRECT = 2,  // operands read straight from memory (no reuse between accumulator rows)
};

struct Variant {
    int32_t id;
    int32_t items_t;    // samples per lane
    int32_t items_acc;  // accumulator rows per wave
    int32_t waves;      // wavefronts per work-group
    int32_t kind;
    int32_t rpw;        // input rows per wave per staged chunk (direct: rows in flight)
    int32_t nwr;        // regwin: window registers per lane
    int32_t kmax;       // max 64-sample pieces per staged row (wcap <= 64*kmax); 0: direct staging
    float rate;         // sustained additions per second (1e12) on an Apertif-shaped forward, MI355X
    int32_t tt() const { return 64 * items_t; }
    int32_t ta() const { return items_acc * waves; }
};

const Variant *variants(int32_t *count);
const Variant *find_variant(int32_t id);

struct SrsArgs {
    const void *in;
    int64_t in_stride;
    int64_t in_valid;
    float *out;
    int64_t out_stride;
    int64_t n_t;
    int32_t n_acc;
    int32_t n_rows;
    const int32_t *rel;    // LDS kind: [n_tiles][n_rows][TA] offsets relative to base
    const int32_t *base;   // [n_tiles][n_rows] staged-row start relative to the tile's first sample
    const int32_t *recs;   // regwin: [n_tiles][waves][n_chunks * rows per chunk][1 + items_acc/4] window records
    const int32_t *span;   // regwin, direct, LDS prefetched: [n_tiles][n_t_tiles][2] rows [lo, hi) with an operand in range
    int32_t wcap;          // samples per staged row
    int32_t rows_per_chunk;
    int32_t lds_bytes;     // dynamic LDS per work-group
    int32_t r_begin = 0;   // input rows [r_begin, r_end) summed by this launch
    int32_t r_end = 0;
    int32_t carry = 0;     // 1: continue the partial sums already in out
    const int32_t *skew = nullptr;  // LDS kinds, regwin: [n_acc] tile skew per accumulator row (null: none)
    int32_t n_t_tiles = 0;          // time tiles (0: ceil(n_t / tt), the count without skew)
};

// Element types the kernels read.
enum InType : int32_t { IN_F32 = DD_F32, IN_F16 = DD_F16, IN_U8 = DD_U8 };

namespace dev {
struct SrsDims;
}
// Launcher of one variant for one input type (srs_launch.h).
using LaunchFn = hipError_t (*)(const SrsArgs &, const dev::SrsDims &, uint32_t, size_t, hipStream_t);

// One variant's launcher in a slice of the auto-tuning study's list (the
// study library compiles its float32 kernels in slices, see gen_study.py).
struct StudyEntry {
    int32_t id;
    LaunchFn fn;
};

// Whether this library holds the variant's single-beam kernel for in_type
// (every variant and type in the product library; float32 only in the study
// library).
bool has_kernel(const Variant &v, int32_t in_type);
// Launch one shifted-row-sum problem with the given variant.
hipError_t launch_srs(const Variant &v, int32_t in_type, const SrsArgs &a, hipStream_t stream);
// The variant's multi-beam kernel (arguments: BatchPtrs by value, const
// BeamDesc *, const uint32_t *items; 64 * waves threads per work-group), or
// null where the library has none (the study library).
const void *multi_kernel(const Variant &v, int32_t in_type);

// One block of a row split: input rows [r0, r1) summed by `variant`.
struct Block {
    int32_t r0, r1, variant;
};

// Host-side layout of one (direction, variant) on one plan.
struct Layout {
    bool feasible = false;
    int32_t n_tiles = 0;
    int32_t wcap = 0;
    int32_t rows_per_chunk = 0;
    int32_t lds_bytes = 0;
    int32_t max_spread = 0;
    int32_t n_t_tiles = 0;  // time tiles: ceil((n_t + max skew) / tt)
    std::vector<int32_t> base, rel, recs, span;
    std::vector<int32_t> skew;  // per accumulator row, multiples of 4 samples; empty when all zero
};

// Device copy of a Layout's tables.
struct TileTables {
    int32_t n_tiles = 0;
    int32_t wcap = 0;
    int32_t rows_per_chunk = 0;
    int32_t lds_bytes = 0;
    int32_t *d_base = nullptr;
    int32_t *d_rel = nullptr;
    int32_t *d_recs = nullptr;
    int32_t *d_span = nullptr;
    int32_t *d_skew = nullptr;
    int32_t n_t_tiles = 0;
};

int32_t max_lds_bytes();

}  // namespace dd

struct dd_plan {
    int32_t C = 0, D = 0;
    int64_t S = 0;
    double f_min = 0, df = 0, t_samp = 0, dm_first = 0, dm_step = 0;
    int32_t max_delay = 0;
    int64_t T_in = 0;
    std::vector<int32_t> delay;  // [D][C]

    mutable std::mutex mu;
    // (device, direction, variant id, first row, end row) -> device tables of
    // that block of input rows (the whole plan: rows [0, R))
    mutable std::map<std::tuple<int, int, int, int, int>, dd::TileTables> tables;
    // (direction, variant id, first row, end row) -> the same tables in host
    // memory, kept once built (the allocation-free entry stages them into its
    // own device array)
    mutable std::map<std::tuple<int, int, int, int>, dd::Layout> host_tables;
    // (direction, variant id, first row, end row) -> (feasible, wcap, rows per
    // chunk), host only
    mutable std::map<std::tuple<int, int, int, int>, std::tuple<bool, int32_t, int32_t>> fit;
    // forced tile per (direction, dtype); -1 = automatic
    int32_t forced[2][3] = {{-1, -1, -1}, {-1, -1, -1}};
    int32_t tuned[2][3] = {{-1, -1, -1}, {-1, -1, -1}};
    // Row blocks per (direction, dtype), forced or tuned: the input rows split
    // into consecutive blocks, each summed by its own variant in its own launch
    // (later blocks continue the partial sums).  Empty: one variant for all.
    // Used unless a single variant is forced; never by batches.
    std::vector<dd::Block> blocks[2][3];
};

namespace dd {
// Compute the layout of (direction, variant); arrays only if build_arrays.
// Tables for input rows [r0, r1) only (r1 < 0: every row); spans always cover
// every row.
void compute_layout(const dd_plan *p, int direction, const Variant &v, bool build_arrays, Layout *L,
                    int32_t r0 = 0, int32_t r1 = -1);
// Build (once) and return the device tables for (direction, variant) on the
// current device.  Returns DD_OK or an error code.
int plan_tables(const dd_plan *p, int direction, const Variant &v, const TileTables **out, int32_t r0 = 0,
                int32_t r1 = -1);
// Variant the plan uses for (direction, dtype) when nothing is forced.
int32_t default_variant(const dd_plan *p, int direction, int32_t in_type);
// Whether variant v can serve (direction) of this plan (cached, host only).
bool variant_fits(const dd_plan *p, int direction, const Variant &v, int32_t r0 = 0, int32_t r1 = -1);
int32_t choose_variant(const dd_plan *p, int direction, int32_t in_type);
// The variant a call uses: forced, else tuned, else the cost model's default.
int32_t resolved_variant(const dd_plan *p, int direction, int32_t in_type);
// Cost-model choice among `cand` (ids) that fit; -1 if none fits.
int32_t best_by_model(const dd_plan *p, int direction, int32_t in_type, const int32_t *cand, int32_t n_cand);
// The cost model's time for a variant over rows [r0, r1) of the plan (r1 < 0:
// all rows), in seconds, after variant_fits has accepted it for those rows.
double model_seconds(const dd_plan *p, int direction, const Variant &v, int32_t r0 = 0, int32_t r1 = -1);
// Time the candidates on the plan's own sizes (scratch buffers allocated
// here); best id and mean ms.  Synchronises the stream.
// With split_out, row splits are timed too; *split_out receives the best
// split if it beats the best single variant (else stays empty) and *best_ms
// the time of what won.  With times_out, the mean ms of every single variant
// timed.
int tune_candidates(const dd_plan *p, int direction, int32_t in_type, int32_t reps, const int32_t *cand,
                    int32_t n_cand, hipStream_t stream, int32_t *best, float *best_ms,
                    std::vector<Block> *split_out = nullptr, std::map<int32_t, float> *times_out = nullptr);
// Free the device tables of row blocks of `direction` that `keep` does not
// use (the tuner builds one per block and candidate).
void release_block_tables(const dd_plan *p, int direction, const std::vector<Block> &keep);
// Fill SrsArgs for one call (tables built on demand).
int make_args(const dd_plan *p, int direction, const Variant &v, const void *in, int64_t in_stride,
              float *out, int64_t out_stride, SrsArgs *a, int32_t r0 = 0, int32_t r1 = -1);
// The sizes and data pointers of SrsArgs for one call (no tables).
void args_dims(const dd_plan *p, int direction, const void *in, int64_t in_stride, float *out, int64_t out_stride,
               SrsArgs *a);
// Host copy of the tables of (direction, variant), or null if no call has
// built them yet (dd_plan_prepare or a first compute call does).
const Layout *plan_host_layout(const dd_plan *p, int direction, int32_t variant, int32_t r0 = 0, int32_t r1 = -1);
// Input rows of a direction (channels forward, DMs adjoint).
int32_t plan_rows(const dd_plan *p, int direction);
// Whether the variant's kind can run as one block of a row split (the
// register-window and LDS kinds; the direct kind splits rows on its own).
bool block_capable(const Variant &v);
// The launches one call makes: the row blocks in use, else one block of
// every row with the resolved variant.  Empty if no variant fits.
std::vector<Block> launch_list(const dd_plan *p, int direction, int32_t in_type);
// Run one call as the launch list: block b sums its rows with its variant,
// continuing the partial sums of the blocks before it.
int run_blocks(const dd_plan *p, int direction, int32_t in_type, const std::vector<Block> &blocks, const void *in,
               int64_t in_stride, float *out, int64_t out_stride, hipStream_t stream);
// Argument checks of the forward (api.cpp).
int check_forward_args(const dd_plan *p, const void *d_in, int32_t in_type, int64_t in_stride, const float *d_out,
                       int64_t out_stride);
}  // namespace dd
