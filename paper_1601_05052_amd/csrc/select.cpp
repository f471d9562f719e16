// Tile-variant selection: the forced or tuned choice of a plan, else a cost
// model's choice among the variants that fit (Sec. IV-A replaces the model
// with measurement; see tune.cpp).
#include <algorithm>
#include <cstdint>
#include <mutex>
#include <vector>

#include "internal.h"

namespace dd {

// Rough time model for choosing a variant without measuring it (the
// auto-tuner replaces it with timings, Sec. IV-A): the additions of whole
// tiles (ragged tiles do full work) at the variant's sustained rate, scaled
// down when the grid has fewer waves than half the chip holds, plus the
// staged input samples at an L2-to-LDS rate (the direct kind stages none).  Rates and both constants were
// fitted to every variant's measured time on Apertif- and LOFAR-shaped beams
// of 2 to 4,096 trial DMs on MI355X.
static double estimate_seconds(const dd_plan *p, int direction, const Variant &v, int32_t wcap, int32_t R) {
    const int32_t A = direction == DD_FORWARD ? p->D : p->C;
    const int64_t n_t = direction == DD_FORWARD ? p->S : p->T_in;
    const double n_t_tiles = static_cast<double>((n_t + v.tt() - 1) / v.tt());
    const double tiles = n_t_tiles * ((A + v.ta() - 1) / v.ta());
    const double work = tiles * v.tt() * v.ta() * static_cast<double>(R);
    const double fill = std::min(1.0, tiles * v.waves / 4096.0);  // 256 CUs x 4 SIMDs x 4 waves
    if (v.kind == KIND_DIRECT)  // one 4-byte read per addition from L2 / HBM, no staging
        return work / (static_cast<double>(v.rate) * 1e12 * fill);
    const double staged = tiles * R * static_cast<double>(wcap);
    return work / (static_cast<double>(v.rate) * 1e12 * fill) + staged / 8e12;
}

double model_seconds(const dd_plan *p, int direction, const Variant &v, int32_t r0, int32_t r1) {
    if (r1 < 0)
        r1 = plan_rows(p, direction);
    int32_t wcap = 0;
    {
        std::lock_guard<std::mutex> lock(p->mu);
        auto it = p->fit.find(std::make_tuple(direction, (int)v.id, (int)r0, (int)r1));
        if (it != p->fit.end())
            wcap = std::get<1>(it->second);
    }
    return estimate_seconds(p, direction, v, wcap, r1 - r0);
}

int32_t best_by_model(const dd_plan *p, int direction, int32_t in_type, const int32_t *cand, int32_t n_cand) {
    int32_t best = -1;
    double best_t = 0.0;
    const int32_t kt = direction == DD_FORWARD ? in_type : (int32_t)DD_F32;
    for (int32_t i = 0; i < n_cand; ++i) {
        const Variant *v = find_variant(cand[i]);
        if (!v || !has_kernel(*v, kt) || !variant_fits(p, direction, *v))
            continue;
        const double t = model_seconds(p, direction, *v);
        if (best < 0 || t < best_t) {
            best = v->id;
            best_t = t;
        }
    }
    return best;
}

int32_t default_variant(const dd_plan *p, int direction, int32_t in_type) {
    int32_t n = 0;
    variants(&n);
    std::vector<int32_t> all(n);
    for (int32_t i = 0; i < n; ++i)
        all[i] = i;
    return best_by_model(p, direction, in_type, all.data(), n);
}

int32_t choose_variant(const dd_plan *p, int direction, int32_t in_type) {
    std::lock_guard<std::mutex> lock(p->mu);
    if (p->forced[direction][in_type] >= 0)
        return p->forced[direction][in_type];
    if (p->tuned[direction][in_type] >= 0)
        return p->tuned[direction][in_type];
    return -2;  // caller computes the default outside the lock
}

int32_t resolved_variant(const dd_plan *p, int direction, int32_t in_type) {
    const int32_t id = choose_variant(p, direction, in_type);
    return id == -2 ? default_variant(p, direction, in_type) : id;
}

std::vector<Block> launch_list(const dd_plan *p, int direction, int32_t in_type) {
    {
        std::lock_guard<std::mutex> lock(p->mu);
        if (p->forced[direction][in_type] < 0 && !p->blocks[direction][in_type].empty())
            return p->blocks[direction][in_type];
    }
    const int32_t id = resolved_variant(p, direction, in_type);
    if (id < 0)
        return {};
    return {Block{0, plan_rows(p, direction), id}};
}

}  // namespace dd
