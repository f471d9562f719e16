/*
 * Dedispersion oracle: plain, slow, FP64 CPU implementation.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing on the product path may link, load or
 * call this file: only the test suite, the smoke check and the CPU-baseline
 * leg of the benchmark use it.  It shares no code, header or table with the
 * GPU library; the two meet only on seeded inputs.
 *
 * What it computes (Sclocco et al., "Auto-Tuning Dedispersion for Many-Core
 * Accelerators"):
 *   - the per-(DM, channel) delay in samples, from the cold-plasma law of
 *     Sec. II, Eq. (1): k = 4150 * DM * (1/f_ch^2 - 1/f_h^2) seconds, with f in
 *     MHz and f_h the highest frequency, divided by the sampling time and
 *     rounded to the nearest sample;
 *   - brute-force dedispersion, Sec. III-A, Algorithm 1: every output sample
 *     of every trial DM is the sum over channels of the input sample shifted
 *     by that channel's delay;
 *   - the transpose (adjoint) of that linear map.
 *
 * Readings of points the paper leaves open (each is stated where used):
 *   channel ch sits at f_min + ch*df (channel 0 lowest); f_h is the top
 *   channel's frequency f_min + (C-1)*df; the constant is exactly 4150;
 *   DM_i = dm_first + i*dm_step (a product, not a running sum); rounding is
 *   round-half-to-even (rint in the default rounding mode).
 *
 * Precision: every floating-point operation is one IEEE-754 binary64 op in
 * the order written; the build disables contraction (-ffp-contract=off) and
 * fast-math.  Accumulators are double.
 *
 * Parity status: delay table pinned to exact rational arithmetic; forward
 * pinned to brute force, the zero-DM channel sum, impulse responses and
 * linearity; adjoint pinned to the explicit matrix transpose and the
 * dot-product identity (tests/test_oracle.py).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#ifdef _OPENMP
#include <omp.h>
#endif

/* Delay table, Eq. (1), sampled: delay[i*C + ch] for DM index i and channel ch.
 * Returns 0 on success, -1 on invalid arguments or a delay outside int32. */
int oracle_delay_table(int32_t C, double f_min, double df, double t_samp,
                       double dm_first, double dm_step, int32_t D,
                       int32_t *delay)
{
    if (C < 1 || D < 1 || !(f_min > 0.0) || !(df > 0.0) || !(t_samp > 0.0))
        return -1;
    const double f_h = f_min + (double)(C - 1) * df;   /* highest channel */
    const double inv_fh2 = 1.0 / (f_h * f_h);
    for (int32_t i = 0; i < D; ++i) {
        const double dm = dm_first + (double)i * dm_step;
        for (int32_t ch = 0; ch < C; ++ch) {
            const double f = f_min + (double)ch * df;
            const double k = 1.0 / (f * f) - inv_fh2;      /* MHz^-2 */
            const double seconds = (4150.0 * dm) * k;      /* Eq. (1) */
            const double samples = seconds / t_samp;
            const double r = rint(samples);
            if (!(r >= -2147483648.0 && r <= 2147483647.0))
                return -1;
            delay[(int64_t)i * C + ch] = (int32_t)r;
        }
    }
    return 0;
}

/* Algorithm 1, literally: one output at a time, channels in ascending order.
 * Evaluates only the n_points outputs (dm_idx[p], t_idx[p]); used to check
 * sampled outputs of full-size runs. */
void oracle_dedisperse_points(int32_t C, const int32_t *delay,
                              const double *x, int64_t x_stride,
                              int64_t n_points, const int32_t *dm_idx,
                              const int64_t *t_idx, double *out)
{
#pragma omp parallel for schedule(static)
    for (int64_t p = 0; p < n_points; ++p) {
        const int64_t i = dm_idx[p];
        const int64_t t = t_idx[p];
        double acc = 0.0;
        for (int32_t ch = 0; ch < C; ++ch)
            acc += x[(int64_t)ch * x_stride + t + delay[i * C + ch]];
        out[p] = acc;
    }
}

/* Algorithm 1 over the whole output y[D][S].  For each DM the channel loop is
 * taken outermost over a row of S double accumulators; every output still
 * receives its channels in ascending order, so each y[i][t] is the same
 * double as the one-at-a-time loop gives.  Threads split the DM rows. */
void oracle_dedisperse(int32_t C, int32_t D, int64_t S, const int32_t *delay,
                       const double *x, int64_t x_stride, double *y)
{
#pragma omp parallel
    {
        double *acc = (double *)malloc(sizeof(double) * (size_t)S);
#pragma omp for schedule(dynamic, 1)
        for (int32_t i = 0; i < D; ++i) {
            for (int64_t t = 0; t < S; ++t)
                acc[t] = 0.0;
            for (int32_t ch = 0; ch < C; ++ch) {
                const double *row = x + (int64_t)ch * x_stride + delay[(int64_t)i * C + ch];
                for (int64_t t = 0; t < S; ++t)
                    acc[t] += row[t];
            }
            memcpy(y + (int64_t)i * S, acc, sizeof(double) * (size_t)S);
        }
        free(acc);
    }
}

/* Transpose of Algorithm 1: gx[ch][tau] = sum over DMs i with
 * 0 <= tau - delay[i][ch] < S of gy[i][tau - delay[i][ch]], for tau < T_in.
 * Written as the scatter that the forward's definition transposes: each
 * output sample y[i][t] sends its weight back to x[ch][t + delay].  DMs are
 * visited in ascending order.  Threads split the channels. */
void oracle_adjoint(int32_t C, int32_t D, int64_t S, const int32_t *delay,
                    const double *gy, int64_t T_in, double *gx)
{
#pragma omp parallel for schedule(dynamic, 1)
    for (int32_t ch = 0; ch < C; ++ch) {
        double *row = gx + (int64_t)ch * T_in;
        for (int64_t tau = 0; tau < T_in; ++tau)
            row[tau] = 0.0;
        for (int32_t i = 0; i < D; ++i) {
            const int64_t d = delay[(int64_t)i * C + ch];
            const double *g = gy + (int64_t)i * S;
            for (int64_t t = 0; t < S; ++t) {
                const int64_t tau = t + d;
                if (tau >= 0 && tau < T_in)
                    row[tau] += g[t];
            }
        }
    }
}

int oracle_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
