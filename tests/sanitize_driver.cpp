// Host-side checks of libdedisp's plan, layout and argument code and of the C
// oracle, built with AddressSanitizer and UndefinedBehaviorSanitizer on the
// CPU (tests/test_sanitizers.py).  Nothing here touches a GPU: device calls
// fail on a machine without one and the library reports DD_EHIP.
//
// Exercised: plan creation over the workloads and random setups, every
// argument error path of the C ABI, the tile tables of every variant in both
// directions (built in host memory), and the oracle's delay table, forward,
// point evaluation and adjoint on small inputs.
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <random>
#include <vector>

#include "dedisp.h"
#include "internal.h"

// The per-input-type kernel tables live in the HIP units, which this build
// leaves out: every entry is a stand-in that launches nothing (no call here
// gets as far as a launch: the device is missing).
namespace dd {
static hipError_t no_launch(const SrsArgs &, const dev::SrsDims &, uint32_t, size_t, hipStream_t) {
    return hipErrorInvalidDeviceFunction;
}
static const LaunchFn *stand_in_table() {
    static LaunchFn t[1024];
    for (LaunchFn &f : t)
        f = no_launch;
    return t;
}
const LaunchFn *launchers_f32 = stand_in_table(), *launchers_f16 = launchers_f32, *launchers_u8 = launchers_f32;
const void *const *multis_f32 = nullptr, *const *multis_f16 = nullptr, *const *multis_u8 = nullptr;
}  // namespace dd

extern "C" {
int oracle_delay_table(int32_t C, double f_min, double df, double t_samp, double dm_first, double dm_step,
                       int32_t D, int32_t *out);
void oracle_dedisperse(int32_t C, int32_t D, int64_t S, const int32_t *delay, const double *x, int64_t in_stride,
                       double *y);
void oracle_dedisperse_points(int32_t C, const int32_t *delay, const double *x, int64_t in_stride, int64_t n,
                              const int32_t *dm_idx, const int64_t *t_idx, double *out);
void oracle_adjoint(int32_t C, int32_t D, int64_t S, const int32_t *delay, const double *gy, int64_t T,
                    double *gx);
}

static int failures = 0;
#define CHECK(cond)                                                        \
    do {                                                                   \
        if (!(cond)) {                                                     \
            std::fprintf(stderr, "CHECK failed %s:%d: %s\n", __FILE__, __LINE__, #cond); \
            ++failures;                                                    \
        }                                                                  \
    } while (0)

struct Setup {
    int32_t C;
    double f_min, df, t_samp, dm_first, dm_step;
    int32_t D;
    int64_t S;
};

static void plan_and_layouts(const Setup &s, bool full_tables) {
    dd_plan *p = nullptr;
    CHECK(dd_plan_create(&p, s.C, s.f_min, s.df, s.t_samp, s.dm_first, s.dm_step, s.D, s.S) == DD_OK);
    if (!p)
        return;
    int32_t c = 0, d = 0, md = -1;
    int64_t n = 0, T = 0;
    CHECK(dd_plan_dims(p, &c, &d, &n) == DD_OK && c == s.C && d == s.D && n == s.S);
    CHECK(dd_plan_max_delay(p, &md) == DD_OK && md >= 0);
    CHECK(dd_plan_input_samples(p, &T) == DD_OK && T == s.S + md);
    std::vector<int32_t> table(static_cast<size_t>(s.C) * s.D);
    CHECK(dd_plan_delay_table(p, table.data()) == DD_OK);
    std::vector<int32_t> ref(table.size());
    CHECK(oracle_delay_table(s.C, s.f_min, s.df, s.t_samp, s.dm_first, s.dm_step, s.D, ref.data()) == 0);
    CHECK(table == ref);
    int32_t nv = 0;
    CHECK(dd_tile_count(&nv) == DD_OK && nv > 0);
    for (int dir = 0; dir < 2; ++dir) {
        for (int32_t v = 0; v < nv; ++v) {
            const int rc = dd_plan_set_tile(p, static_cast<dd_direction>(dir), DD_F32, v);
            CHECK(rc == DD_OK || rc == DD_EUNSUPPORTED);
            if (full_tables && rc == DD_OK) {
                const dd::Variant &var = *dd::find_variant(v);
                dd::Layout L;
                dd::compute_layout(p, dir, var, true, &L);
                CHECK(L.feasible);
                // the cost model the tuner orders its candidates by
                const double est = dd::model_seconds(p, dir, var);
                CHECK(est > 0.0 && est < 1e6);
                CHECK(L.base.size() == static_cast<size_t>(L.n_tiles) * (dir == 0 ? s.C : s.D));
                // Skewed tiles: one non-negative multiple of 4 per accumulator
                // row (or none), and enough time tiles for the largest skew.
                const int32_t A = dir == 0 ? s.D : s.C;
                const int64_t n_t = dir == 0 ? s.S : T;
                int32_t kmax = 0;
                CHECK(L.skew.empty() || L.skew.size() == static_cast<size_t>(A));
                for (int32_t k : L.skew) {
                    CHECK(k >= 0 && k % 4 == 0);
                    kmax = k > kmax ? k : kmax;
                }
                CHECK(static_cast<int64_t>(L.n_t_tiles) * var.tt() >= n_t + kmax);
                // The second half of the rows as a block of its own (tables
                // relative to the block; its own skews).
                const int32_t R = dir == 0 ? s.C : s.D;
                const int32_t cr = var.kind == dd::KIND_LDS && var.kmax == 0 ? 1 : var.waves * (var.rpw > 0 ? var.rpw : 1);
                const int32_t r0 = R / 2 / cr * cr;
                if (dd::block_capable(var) && r0 > 0) {
                    dd::Layout B;
                    dd::compute_layout(p, dir, var, true, &B, r0, R);
                    if (B.feasible) {
                        CHECK(B.base.size() == static_cast<size_t>(B.n_tiles) * (R - r0));
                        CHECK(dd::variant_fits(p, dir, var, r0, R));
                        const double eb = dd::model_seconds(p, dir, var, r0, R);
                        CHECK(eb > 0.0 && eb < 1e6);
                    }
                }
            }
        }
        CHECK(dd_plan_set_tile(p, static_cast<dd_direction>(dir), DD_F32, -1) == DD_OK);
        int32_t got = -7;
        CHECK(dd_plan_get_tile(p, static_cast<dd_direction>(dir), DD_U8, &got) == DD_OK && got >= 0);
    }
    // A compute call with valid arguments reaches the device and fails there
    // (no GPU); every shape error is caught before that.
    std::vector<float> in(static_cast<size_t>(s.C) * T + 16), out(static_cast<size_t>(s.D) * s.S + 16);
    CHECK(dd_dedisperse(p, in.data(), DD_F32, T - 1, out.data(), s.S, nullptr) == DD_ESHAPE);
    CHECK(dd_dedisperse(p, in.data(), DD_F32, T, out.data(), s.S - 1, nullptr) == DD_ESHAPE);
    CHECK(dd_dedisperse(p, in.data(), static_cast<dd_dtype>(7), T, out.data(), s.S, nullptr) == DD_EINVAL);
    CHECK(dd_dedisperse(p, nullptr, DD_F32, T, out.data(), s.S, nullptr) == DD_EINVAL);
    CHECK(dd_dedisperse(p, reinterpret_cast<const char *>(in.data()) + 1, DD_F32, T, out.data(), s.S, nullptr) ==
          DD_ESHAPE);
    CHECK(dd_dedisperse(p, in.data(), DD_F32, T, reinterpret_cast<float *>(in.data()), s.S, nullptr) == DD_ESHAPE);
    CHECK(dd_dedisperse_adjoint(p, out.data(), s.S, in.data(), T - 1, nullptr) == DD_ESHAPE);
    CHECK(dd_dedisperse_adjoint(p, out.data(), s.S - 1, in.data(), T, nullptr) == DD_ESHAPE);
    const int rc = dd_dedisperse(p, in.data(), DD_F32, T, out.data(), s.S, nullptr);
    CHECK(rc == DD_EHIP || rc == DD_OK);
    CHECK(dd_plan_destroy(p) == DD_OK);
}

static void api_errors() {
    dd_plan *p = nullptr;
    CHECK(dd_plan_create(nullptr, 4, 1400, 1, 1e-4, 0, 1, 3, 10) == DD_EINVAL);
    CHECK(dd_plan_create(&p, 0, 1400, 1, 1e-4, 0, 1, 3, 10) == DD_EINVAL && !p);
    CHECK(dd_plan_create(&p, 4, -1, 1, 1e-4, 0, 1, 3, 10) == DD_EINVAL);
    CHECK(dd_plan_create(&p, 4, 1400, 0, 1e-4, 0, 1, 3, 10) == DD_EINVAL);
    CHECK(dd_plan_create(&p, 4, 1400, 1, 0, 0, 1, 3, 10) == DD_EINVAL);
    CHECK(dd_plan_create(&p, 4, 1400, 1, 1e-4, -1, 1, 3, 10) == DD_EINVAL);
    CHECK(dd_plan_create(&p, 4, 1400, 1, 1e-4, 0, NAN, 3, 10) == DD_EINVAL);
    CHECK(dd_plan_create(&p, 4, 1400, 1, 1e-4, 0, 1, 0, 10) == DD_EINVAL);
    CHECK(dd_plan_create(&p, 4, 1400, 1, 1e-4, 0, 1, 3, 0) == DD_EINVAL);
    CHECK(dd_plan_create(&p, 4, 1, 1, 1e-9, 0, 1e9, 3, 10) == DD_EINVAL);  // delay beyond int32
    CHECK(dd_plan_destroy(nullptr) == DD_OK);
    CHECK(dd_tile_info(-1, nullptr, nullptr, nullptr, nullptr) == DD_EINVAL);
    CHECK(dd_tile_info(1 << 20, nullptr, nullptr, nullptr, nullptr) == DD_EINVAL);
    CHECK(dd_plan_create(&p, 4, 1400, 1, 1e-4, 0, 1, 3, 10) == DD_OK);
    CHECK(dd_plan_set_tile(p, DD_FORWARD, DD_F32, 1 << 20) == DD_EINVAL);
    CHECK(dd_plan_set_tile(p, static_cast<dd_direction>(3), DD_F32, 0) == DD_EINVAL);
    CHECK(dd_plan_get_tile(p, DD_FORWARD, static_cast<dd_dtype>(9), nullptr) == DD_EINVAL);
    CHECK(dd_plan_prepare(p, static_cast<dd_direction>(2), DD_F32) == DD_EINVAL);
    CHECK(dd_plan_destroy(p) == DD_OK);
    CHECK(dd_last_error() != nullptr);
}

static void oracle_small() {
    const Setup s{7, 1400.0, 2.5, 5e-5, 0.0, 0.75, 5, 61};
    std::vector<int32_t> delay(static_cast<size_t>(s.C) * s.D);
    CHECK(oracle_delay_table(s.C, s.f_min, s.df, s.t_samp, s.dm_first, s.dm_step, s.D, delay.data()) == 0);
    int32_t md = 0;
    for (int32_t v : delay)
        md = v > md ? v : md;
    const int64_t T = s.S + md;
    std::mt19937 g(5);
    std::uniform_int_distribution<int> u(-3, 3);
    std::vector<double> x(static_cast<size_t>(s.C) * T), y(static_cast<size_t>(s.D) * s.S);
    for (double &v : x)
        v = u(g);
    oracle_dedisperse(s.C, s.D, s.S, delay.data(), x.data(), T, y.data());
    std::vector<int32_t> di{0, 4, 2};
    std::vector<int64_t> ti{0, s.S - 1, 17};
    std::vector<double> pts(3);
    oracle_dedisperse_points(s.C, delay.data(), x.data(), T, 3, di.data(), ti.data(), pts.data());
    for (int k = 0; k < 3; ++k)
        CHECK(pts[k] == y[static_cast<size_t>(di[k]) * s.S + ti[k]]);
    std::vector<double> gy(y.size()), gx(static_cast<size_t>(s.C) * T);
    for (double &v : gy)
        v = u(g);
    oracle_adjoint(s.C, s.D, s.S, delay.data(), gy.data(), T, gx.data());
    double lhs = 0, rhs = 0;  // <A x, gy> = <x, A^T gy>, exact on integers
    for (size_t i = 0; i < y.size(); ++i)
        lhs += y[i] * gy[i];
    for (size_t i = 0; i < x.size(); ++i)
        rhs += x[i] * gx[i];
    CHECK(lhs == rhs);
}

int main() {
    api_errors();
    oracle_small();
    const Setup fixed[] = {
        {64, 1400.0, 1.5625, 5e-5, 0.0, 0.5, 128, 4096},          // tiny workload
        {16, 1420.0, 64 * 300.0 / 1024, 1.0 / 20000, 0.0, 0.25, 32, 256},
        {37, 1400.0, 2.5, 5e-5, 0.0, 0.75, 77, 1001},
        {5, 140.0, 0.2, 5e-6, 0.0, 0.02, 9, 3333},
        {1, 1400.0, 1.0, 5e-5, 0.0, 1.0, 1, 1},
        {3, 1400.0, 1.0, 5e-5, 2.0, 0.0, 5, 65},
        {130, 1420.0, 300.0 / 130, 5e-5, 10.0, 0.25, 33, 515},
        {32, 138.0, 0.1875, 5e-6, 0.0, 0.01, 200, 3000},           // LOFAR band, wide delays
    };
    for (const Setup &s : fixed)
        plan_and_layouts(s, true);
    std::mt19937 g(11);
    for (int k = 0; k < 12; ++k) {
        std::uniform_int_distribution<int> c(1, 200), d(1, 150), n(1, 3000);
        std::uniform_real_distribution<double> step(0.0, 1.0);
        const Setup s{c(g), 1300.0, 300.0 / 256, 5e-5, 0.0, step(g), d(g), n(g)};
        plan_and_layouts(s, k < 6);
    }
    if (failures) {
        std::fprintf(stderr, "%d checks failed\n", failures);
        return 1;
    }
    std::printf("sanitized host checks ok\n");
    return 0;
}
