// Auto-tuning of the tile shape (Sclocco et al., Sec. IV-A): run every tile
// variant that can serve the plan, on the plan's own sizes, and keep the
// fastest.  Results can be cached in a text file keyed by device, direction,
// input type and plan shape (the best configuration differs between setups and
// instances, Sec. V-A, so the key includes the whole setup).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <fstream>
#include <functional>
#include <map>
#include <sstream>
#include <string>
#include <vector>

#include "internal.h"

using namespace dd;

namespace {

// Tuning input: samples of magnitude 0.5..1 with random signs (float32,
// float16) or random bytes (u8) from a counter hash, so the variants are timed
// on data that toggles the adders as real data does (all-zero input draws
// less power, lets the clock run higher and flatters some variants more than
// others).
__global__ __launch_bounds__(256) void fill_tuning_input(void *buf, int64_t n, int32_t elem_size) {
    for (int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < n;
         i += static_cast<int64_t>(gridDim.x) * blockDim.x) {
        uint32_t x = static_cast<uint32_t>(i) * 0x9E3779B1u ^ static_cast<uint32_t>(i >> 32) * 0x85EBCA77u;
        x ^= x >> 15;
        x *= 0x2C1B3C6Du;
        x ^= x >> 12;
        if (elem_size == 4)
            static_cast<uint32_t *>(buf)[i] = (x & 0x807FFFFFu) | 0x3F000000u;
        else if (elem_size == 2)
            static_cast<uint16_t *>(buf)[i] = static_cast<uint16_t>((x & 0x83FFu) | 0x3800u);
        else
            static_cast<uint8_t *>(buf)[i] = static_cast<uint8_t>(x >> 24);
    }
}

std::string cache_key(const dd_plan *p, int direction, int32_t in_type) {
    int dev = 0;
    hipDeviceProp_t prop;
    std::memset(&prop, 0, sizeof(prop));
    if (hipGetDevice(&dev) == hipSuccess)
        (void)hipGetDeviceProperties(&prop, dev);
    char buf[512];
    std::snprintf(buf, sizeof(buf), "%s|cu%d|dir%d|dt%d|C%d|D%d|S%lld|%.17g|%.17g|%.17g|%.17g|%.17g|v1",
                  prop.gcnArchName, prop.multiProcessorCount, direction, in_type, p->C, p->D,
                  (long long)p->S, p->f_min, p->df, p->t_samp, p->dm_first, p->dm_step);
    for (char *c = buf; *c; ++c)
        if (*c == ' ')
            *c = '_';
    return buf;
}

// Cache lines: "key variant ms" or "key variant ms r0:v,r0:v,..." (a row split).
bool cache_lookup(const char *path, const std::string &key, int32_t *variant, float *ms,
                  std::vector<std::pair<int32_t, int32_t>> *split) {
    std::ifstream f(path);
    if (!f)
        return false;
    std::string line;
    bool found = false;
    while (std::getline(f, line)) {
        std::istringstream ss(line);
        std::string k, blocks;
        int32_t v;
        float t;
        if (ss >> k >> v >> t && k == key && find_variant(v)) {
            *variant = v;
            *ms = t;
            split->clear();
            if (ss >> blocks) {
                std::istringstream bs(blocks);
                std::string item;
                while (std::getline(bs, item, ',')) {
                    int32_t r0 = -1, bv = -1;
                    if (std::sscanf(item.c_str(), "%d:%d", &r0, &bv) == 2 && find_variant(bv))
                        split->emplace_back(r0, bv);
                }
            }
            found = true;  // last entry wins
        }
    }
    return found;
}

void cache_store(const char *path, const std::string &key, int32_t variant, float ms, const std::vector<Block> &split) {
    std::ofstream f(path, std::ios::app);
    if (!f)
        return;
    f << key << ' ' << variant << ' ' << ms;
    for (size_t b = 0; b < split.size(); ++b)
        f << (b ? ',' : ' ') << split[b].r0 << ':' << split[b].variant;
    f << '\n';
}

}  // namespace

namespace dd {

// Mean milliseconds of `reps` runs of one launch list, after one warm-up run.
// The tables are built first, so the warm-up run times the kernels alone; if
// it takes longer than cap_ms (> 0), its time is returned without the
// repeated runs (a variant that slow cannot win, and some are very slow:
// staged windows far wider than their tiles).
static int time_blocks(const dd_plan *p, int direction, int32_t in_t, const std::vector<Block> &blocks, int32_t reps,
                       const void *d_in, int64_t in_cols, float *d_out, int64_t out_cols, hipStream_t stream,
                       hipEvent_t e0, hipEvent_t e1, float *ms, float cap_ms = 0.f) {
    for (const Block &b : blocks) {
        const Variant *v = find_variant(b.variant);
        const TileTables *t = nullptr;
        const int rc = v ? plan_tables(p, direction, *v, &t, b.r0, b.r1) : fail(DD_EINVAL, "unknown tile variant");
        if (rc != DD_OK)
            return rc;
    }
    (void)hipEventRecord(e0, stream);
    int rc = run_blocks(p, direction, in_t, blocks, d_in, in_cols, d_out, out_cols, stream);
    (void)hipEventRecord(e1, stream);
    if (rc != DD_OK)
        return rc;
    if (hipEventSynchronize(e1) != hipSuccess)
        return fail(DD_EHIP, "tuning run failed");
    float warm = 0.f;
    (void)hipEventElapsedTime(&warm, e0, e1);
    if (cap_ms > 0.f && warm > cap_ms) {
        *ms = warm;
        return DD_OK;
    }
    (void)hipEventRecord(e0, stream);
    for (int32_t r = 0; r < reps && rc == DD_OK; ++r)
        rc = run_blocks(p, direction, in_t, blocks, d_in, in_cols, d_out, out_cols, stream);
    (void)hipEventRecord(e1, stream);
    if (rc != DD_OK)
        return rc;
    if (hipEventSynchronize(e1) != hipSuccess)
        return fail(DD_EHIP, "tuning run failed");
    (void)hipEventElapsedTime(ms, e0, e1);
    *ms /= reps;
    return rc;
}

// A variant whose first run takes longer than this many times the fastest
// mean so far is not run again.
constexpr float kPruneFactor = 3.f;
// A split is timed as a whole when its blocks, each timed alone, add up to
// less than this many times the time to beat.
constexpr float kSplitSlack = 1.05f;

// Row splits tried by the tuner: the rows cut into 2, 3 or 4 blocks of about
// equal size at multiples of 64 rows (a multiple of every variant's rows per
// chunk), at least 64 rows each; every block is timed alone with every
// variant that can serve it.  With `fine` also 8, 16 and 32 blocks: where only
// the direct kind serves all rows at once (no staged window fits), short
// blocks can bring the skewed tiles' window within a staged kind's reach.
static std::vector<std::vector<int32_t>> split_candidates(int32_t R, bool fine) {
    std::vector<std::vector<int32_t>> out;
    if (R < 256)
        return out;
    for (int32_t nb : {2, 3, 4, 8, 16, 32}) {
        if (R / nb < 64 || (nb > 4 && !fine))
            break;
        std::vector<int32_t> starts{0};
        for (int32_t k = 1; k < nb; ++k) {
            const int32_t r = static_cast<int32_t>(static_cast<int64_t>(R) * k / nb) / 64 * 64;
            if (r > starts.back() && r < R)
                starts.push_back(r);
        }
        if (starts.size() == static_cast<size_t>(nb))
            out.push_back(starts);
    }
    return out;
}

int tune_candidates(const dd_plan *p, int direction, int32_t in_type, int32_t reps, const int32_t *cand,
                    int32_t n_cand, hipStream_t stream, int32_t *best_out, float *best_ms_out,
                    std::vector<Block> *split_out, std::map<int32_t, float> *times_out) {
    const size_t esz = direction == DD_ADJOINT ? 4 : (in_type == DD_F32 ? 4 : in_type == DD_F16 ? 2 : 1);
    const int64_t in_rows = direction == DD_FORWARD ? p->C : p->D;
    const int64_t in_cols = direction == DD_FORWARD ? p->T_in : p->S;
    const int64_t out_rows = direction == DD_FORWARD ? p->D : p->C;
    const int64_t out_cols = direction == DD_FORWARD ? p->S : p->T_in;
    void *d_in = nullptr;
    float *d_out = nullptr;
    if (hipMalloc(&d_in, (size_t)in_rows * in_cols * esz) != hipSuccess ||
        hipMalloc(reinterpret_cast<void **>(&d_out), (size_t)out_rows * out_cols * 4) != hipSuccess) {
        (void)hipGetLastError();
        (void)hipFree(d_in);
        return fail(DD_ENOMEM, "tuning scratch allocation failed");
    }
    int rc = DD_OK;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    int32_t best = -1;
    float best_t = 0.f;
    do {
        const int64_t n_in = in_rows * in_cols;
        hipLaunchKernelGGL(fill_tuning_input, dim3(static_cast<uint32_t>(std::min<int64_t>((n_in + 255) / 256, 8192))),
                           dim3(256), 0, stream, d_in, n_in, static_cast<int32_t>(esz));
        if (hipGetLastError() != hipSuccess || hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
            rc = fail(DD_EHIP, "tuning setup failed");
            break;
        }
        const int32_t in_t = direction == DD_FORWARD ? in_type : (int32_t)DD_F32;
        const int32_t R = plan_rows(p, direction);
        // Candidates that fit, in the cost model's order (fastest expected
        // first), so the slow ones meet a low pruning bound.
        std::vector<std::pair<double, int32_t>> order;
        for (int32_t i = 0; i < n_cand; ++i) {
            const Variant *v = find_variant(cand[i]);
            if (v && has_kernel(*v, in_t) && variant_fits(p, direction, *v))
                order.emplace_back(model_seconds(p, direction, *v), v->id);
        }
        std::stable_sort(order.begin(), order.end(),
                         [](const std::pair<double, int32_t> &a, const std::pair<double, int32_t> &b) {
                             return a.first < b.first;
                         });
        // The clock ramps up under load: the first variant timed (the model's
        // favourite) would be timed slow, so it runs untimed first.
        if (!order.empty()) {
            for (int32_t r = 0; r < reps && rc == DD_OK; ++r)
                rc = run_blocks(p, direction, in_t, {Block{0, R, order[0].second}}, d_in, in_cols, d_out, out_cols,
                                stream);
        }
        std::vector<std::pair<float, int32_t>> full;  // variants timed over all reps
        for (size_t k = 0; k < order.size() && rc == DD_OK; ++k) {
            const int32_t id = order[k].second;
            const float cap = best < 0 ? 0.f : kPruneFactor * best_t;
            float ms = 0.f;
            rc = time_blocks(p, direction, in_t, {Block{0, R, id}}, reps, d_in, in_cols, d_out, out_cols, stream, e0,
                             e1, &ms, cap);
            if (rc != DD_OK)
                break;
            if (times_out)
                (*times_out)[id] = ms;
            if (cap <= 0.f || ms <= cap)
                full.emplace_back(ms, id);
            if (best < 0 || ms < best_t) {
                best = id;
                best_t = ms;
            }
        }
        // The three fastest are timed once more and ranked by their two
        // means, so one noisy measurement does not decide.
        if (rc == DD_OK && full.size() > 1) {
            std::sort(full.begin(), full.end());
            full.resize(std::min<size_t>(full.size(), 3));
            best = -1;
            for (auto it = full.rbegin(); it != full.rend() && rc == DD_OK; ++it) {
                float ms = 0.f;
                rc = time_blocks(p, direction, in_t, {Block{0, R, it->second}}, reps, d_in, in_cols, d_out, out_cols,
                                 stream, e0, e1, &ms);
                const float mean = 0.5f * (ms + it->first);
                if (rc == DD_OK) {
                    if (times_out)
                        (*times_out)[it->second] = mean;
                    if (best < 0 || mean < best_t) {
                        best = it->second;
                        best_t = mean;
                    }
                }
            }
        }
        if (rc != DD_OK || best < 0 || !split_out)
            break;
        // Row splits: each block's fastest variant, timed alone; the split
        // replaces the single variant only if it is faster by more than 2%.
        float split_t = 0.98f * best_t;
        const bool fine = find_variant(best)->kind == KIND_DIRECT;
        for (const std::vector<int32_t> &starts : split_candidates(R, fine)) {
            std::vector<Block> blocks;
            float total = 0.f;
            for (size_t b = 0; b < starts.size() && rc == DD_OK; ++b) {
                const int32_t r0 = starts[b], r1 = b + 1 < starts.size() ? starts[b + 1] : R;
                Block bb{r0, r1, -1};
                float bb_t = 0.f;
                std::vector<std::pair<double, int32_t>> border;  // this block's candidates, model order
                for (int32_t i = 0; i < n_cand; ++i) {
                    const Variant *v = find_variant(cand[i]);
                    if (v && block_capable(*v) && has_kernel(*v, in_t) && variant_fits(p, direction, *v, r0, r1))
                        border.emplace_back(model_seconds(p, direction, *v, r0, r1), v->id);
                }
                std::stable_sort(border.begin(), border.end(),
                                 [](const std::pair<double, int32_t> &a, const std::pair<double, int32_t> &b) {
                                     return a.first < b.first;
                                 });
                for (const auto &o : border) {
                    float ms = 0.f;
                    rc = time_blocks(p, direction, in_t, {Block{r0, r1, o.second}}, reps, d_in, in_cols, d_out,
                                     out_cols, stream, e0, e1, &ms, bb.variant < 0 ? 0.f : kPruneFactor * bb_t);
                    if (rc != DD_OK)
                        break;
                    if (bb.variant < 0 || ms < bb_t) {
                        bb.variant = o.second;
                        bb_t = ms;
                    }
                }
                if (bb.variant < 0)
                    break;
                blocks.push_back(bb);
                total += bb_t;
                if (total >= kSplitSlack * split_t)
                    break;  // already slower than the best so far: the other blocks need no timing
            }
            if (rc != DD_OK)
                break;
            if (blocks.size() == starts.size() && total < kSplitSlack * split_t) {
                // Confirm the split as one call (the blocks back to back; a
                // block timed alone can take a few per cent longer than
                // after the previous one, whose partial sums are still in
                // the caches).
                float ms = 0.f;
                rc = time_blocks(p, direction, in_t, blocks, reps, d_in, in_cols, d_out, out_cols, stream, e0, e1, &ms);
                if (rc == DD_OK && ms < split_t) {
                    *split_out = blocks;
                    split_t = ms;
                }
            }
        }
        if (rc == DD_OK && !split_out->empty())
            best_t = split_t;
        release_block_tables(p, direction, *split_out);
    } while (false);
    if (e0)
        (void)hipEventDestroy(e0);
    if (e1)
        (void)hipEventDestroy(e1);
    (void)hipStreamSynchronize(stream);
    (void)hipFree(d_in);
    (void)hipFree(d_out);
    if (rc != DD_OK)
        return rc;
    if (best < 0)
        return fail(DD_EUNSUPPORTED, "no tile variant can serve this plan");
    *best_out = best;
    *best_ms_out = best_t;
    return DD_OK;
}

}  // namespace dd

static int check_tune_args(const dd_plan *p, int direction, int in_type, int32_t reps) {
    if (!p)
        return fail(DD_EINVAL, "plan is NULL");
    if (direction != DD_FORWARD && direction != DD_ADJOINT)
        return fail(DD_EINVAL, "unknown direction %d", direction);
    if (in_type != DD_F32 && in_type != DD_F16 && in_type != DD_U8)
        return fail(DD_EINVAL, "unknown input dtype %d", in_type);
    if (direction == DD_ADJOINT && in_type != DD_F32)
        return fail(DD_EINVAL, "the adjoint works on float32 only");
    if (reps < 1 || reps > 1000)
        return fail(DD_EINVAL, "reps must be in [1, 1000]");
    return DD_OK;
}

namespace {

// Tune one (plan, direction, dtype): the cache file first, then `memo` (plans
// of the same shape tuned earlier in this call), else time every variant and,
// if `splits`, row splits (batches use one variant per beam: no splits).
struct MemoEntry {
    int32_t best;
    float ms;
    std::map<int32_t, float> times;  // every variant timed (empty when the result came from the cache file)
};

int tune_one(dd_plan *p, int direction, int32_t in_type, int32_t reps, const char *cache_path, hipStream_t stream,
             std::map<std::string, MemoEntry> *memo, bool splits, int32_t *best_out, float *ms_out,
             std::map<int32_t, float> *times_out = nullptr) {
    const std::string key = cache_key(p, direction, in_type) + (splits ? "_split" : "");
    int32_t best = -1;
    float best_t = 0.f;
    std::vector<Block> split;
    bool have = false;
    if (memo) {
        auto it = memo->find(key);
        if (it != memo->end()) {
            best = it->second.best;
            best_t = it->second.ms;
            if (times_out)
                *times_out = it->second.times;
            have = true;
        }
    }
    std::vector<std::pair<int32_t, int32_t>> cached;
    if (!have && cache_path && cache_lookup(cache_path, key, &best, &best_t, &cached) &&
        variant_fits(p, direction, *find_variant(best))) {
        have = true;
        const int32_t R = plan_rows(p, direction);
        for (size_t b = 0; b < cached.size() && have; ++b) {
            const int32_t r0 = cached[b].first, r1 = b + 1 < cached.size() ? cached[b + 1].first : R;
            const Variant *v = find_variant(cached[b].second);
            if (!block_capable(*v) || !variant_fits(p, direction, *v, r0, r1))
                have = false;
            split.push_back(Block{r0, r1, v->id});
        }
        if (!have)
            split.clear();
    }
    if (!have) {
        int32_t n = 0;
        variants(&n);
        std::vector<int32_t> all(n);
        for (int32_t i = 0; i < n; ++i)
            all[i] = i;
        int rc = tune_candidates(p, direction, in_type, reps, all.data(), n, stream, &best, &best_t,
                                 splits ? &split : nullptr, times_out);
        if (rc != DD_OK)
            return rc;
        if (cache_path)
            cache_store(cache_path, key, best, best_t, split);
    }
    if (memo)
        (*memo)[key] = MemoEntry{best, best_t, times_out ? *times_out : std::map<int32_t, float>()};
    {
        std::lock_guard<std::mutex> lock(p->mu);
        p->tuned[direction][in_type] = best;
        p->blocks[direction][in_type] = split;
    }
    // Report what a call now uses: with a split, its largest block's variant.
    if (!split.empty()) {
        const Block *big = &split[0];
        for (const Block &b : split)
            if (b.r1 - b.r0 > big->r1 - big->r0)
                big = &b;
        best = big->variant;
    }
    *best_out = best;
    *ms_out = best_t;
    return DD_OK;
}

}  // namespace

extern "C" int dd_autotune(dd_plan *p, dd_direction direction, dd_dtype in_type, int32_t reps,
                           const char *cache_path, void *stream_v, int32_t *best_variant, float *best_ms) {
    clear_error();
    int rc = check_tune_args(p, direction, in_type, reps);
    if (rc != DD_OK)
        return rc;
    int32_t best = -1;
    float best_t = 0.f;
    rc = tune_one(p, direction, in_type, reps, cache_path, static_cast<hipStream_t>(stream_v), nullptr, true, &best,
                  &best_t);
    if (rc != DD_OK)
        return rc;
    if (best_variant)
        *best_variant = best;
    if (best_ms)
        *best_ms = best_t;
    return DD_OK;
}

extern "C" int dd_batch_autotune(dd_plan *const *plans, int32_t n_beams, dd_dtype in_type, int32_t reps,
                                 const char *cache_path, void *stream_v) {
    clear_error();
    if (!plans || n_beams < 1)
        return fail(DD_EINVAL, "plans is NULL or n_beams < 1");
    for (int32_t b = 0; b < n_beams; ++b) {
        int rc = check_tune_args(plans[b], DD_FORWARD, in_type, reps);
        if (rc != DD_OK)
            return rc;
    }
    hipStream_t stream = static_cast<hipStream_t>(stream_v);
    std::map<std::string, MemoEntry> memo;
    std::vector<std::map<int32_t, float>> times(n_beams);
    bool complete = true;  // every beam's variants were timed in this call
    std::string beams_key;
    for (int32_t b = 0; b < n_beams; ++b) {
        int32_t best = -1;
        float best_t = 0.f;
        int rc = tune_one(plans[b], DD_FORWARD, in_type, reps, cache_path, stream, &memo, false, &best, &best_t,
                          &times[b]);
        if (rc != DD_OK)
            return rc;
        complete = complete && !times[b].empty();
        beams_key += cache_key(plans[b], DD_FORWARD, in_type) + ";";
    }
    // One variant for every beam, when it costs at most 1% more than each
    // beam's own best (summed over the beams, each timed alone): the batch is
    // then a single multi-beam launch.  The choice is cached under a key of
    // all beams' shapes.
    char hash[32];
    std::snprintf(hash, sizeof(hash), "%016llx",
                  static_cast<unsigned long long>(std::hash<std::string>()(beams_key)));
    const std::string bkey = std::string("batch|") + hash + "|n" + std::to_string(n_beams) + "|dt" +
                             std::to_string(static_cast<int>(in_type)) + "|v1";
    int32_t common = -1;
    float common_ms = 0.f;
    std::vector<std::pair<int32_t, int32_t>> unused;
    bool cached = cache_path && cache_lookup(cache_path, bkey, &common, &common_ms, &unused);
    if (!cached && complete) {
        double own = 0.0;
        for (const auto &t : times) {
            float m = 0.f;
            bool first = true;
            for (const auto &kv : t)
                if (first || kv.second < m) {
                    m = kv.second;
                    first = false;
                }
            own += m;
        }
        double best_sum = 0.0;
        for (const auto &kv : times[0]) {
            double sum = 0.0;
            bool all = true;
            for (const auto &t : times) {
                auto it = t.find(kv.first);
                if (it == t.end()) {
                    all = false;
                    break;
                }
                sum += it->second;
            }
            if (all && (common < 0 || sum < best_sum)) {
                common = kv.first;
                best_sum = sum;
            }
        }
        if (common >= 0 && best_sum > 1.01 * own)
            common = -1;
        if (common >= 0) {
            common_ms = static_cast<float>(best_sum);
            if (cache_path)
                cache_store(cache_path, bkey, common, common_ms, {});
        }
    }
    if (common >= 0) {
        for (int32_t b = 0; b < n_beams; ++b)
            if (!variant_fits(plans[b], DD_FORWARD, *find_variant(common)))
                common = -1;
    }
    if (common >= 0) {
        for (int32_t b = 0; b < n_beams; ++b) {
            std::lock_guard<std::mutex> lock(plans[b]->mu);
            plans[b]->tuned[DD_FORWARD][in_type] = common;
            plans[b]->blocks[DD_FORWARD][in_type].clear();
        }
    }
    return DD_OK;
}
