// Boxcar candidate search over dedispersed rows.
//
// The dedispersed time-series are analysed further to find pulses (Sec. I);
// the paper does not define that step.  This is the plain single-pulse
// search: per row y[0:S], with mu and sigma the row's mean and population
// standard deviation,
//     snr_w(t) = sum_{i < w} (y[t + i] - mu) / (sigma * sqrt(w)),
// for widths w = 1, 2, 4, ..., 2^(n_widths - 1) (those <= S) and
// 0 <= t <= S - w; the result is the largest snr with one (t, w) reaching it
// (0 at (0, 1) when sigma is 0).
//
// One work-group per row.  Mean and standard deviation are accumulated in
// binary64 (one pass over the row); the centred samples are formed in
// binary64 and rounded to binary32, so the row's offset never enters the
// binary32 boxcar sums.  Boxcars are built by doubling in LDS,
// B_2w(t) = B_w(t) + B_w(t + w), over chunks of the row with a halo of the
// widest boxcar: pairwise sums, one addition per sample and width.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>

#include "internal.h"

namespace dd {
namespace {

constexpr int kSearchThreads = 256;
constexpr int kChunk = 4096;         // boxcar starts owned per chunk
constexpr int kMaxWidthsLog = 12;    // widths up to 2^11 = 2048 samples
constexpr int kHalo = 1 << (kMaxWidthsLog - 1);
constexpr int kExt = kChunk + kHalo;  // samples staged per chunk

__device__ __forceinline__ double block_sum(double v, double *red) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1)
        v += __shfl_down(v, o, 64);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    __syncthreads();  // red is reused between calls
    if (lane == 0)
        red[wave] = v;
    __syncthreads();
    double s = 0.0;
#pragma unroll
    for (int w = 0; w < kSearchThreads / 64; ++w)
        s += red[w];
    return s;
}

typedef float v4f __attribute__((ext_vector_type(4)));

struct Cand {
    float snr;
    int32_t t;
    int32_t w;
};

// a before b: larger snr, then smaller width, then earlier start.
__device__ __forceinline__ bool better(const Cand &a, const Cand &b) {
    if (a.snr != b.snr)
        return a.snr > b.snr;
    if (a.w != b.w)
        return a.w < b.w;
    return a.t < b.t;
}

__global__ __launch_bounds__(kSearchThreads) void boxcar_search_kernel(const float *__restrict__ rows,
                                                                     int64_t row_stride, int64_t S, int32_t n_widths,
                                                                     float *__restrict__ snr_out,
                                                                     int32_t *__restrict__ t_out,
                                                                     int32_t *__restrict__ w_out) {
    __shared__ __attribute__((aligned(16))) float box[kExt];
    __shared__ double red[kSearchThreads / 64];
    __shared__ Cand cred[kSearchThreads];
    const int tid = threadIdx.x;
    const float *y = rows + static_cast<int64_t>(blockIdx.x) * row_stride;

    // One pass: sums of d = y - y[0] and d^2 in binary64 (the shift keeps the
    // terms near the row's spread), 16-byte loads when the row allows.
    const double k0 = static_cast<double>(y[0]);
    double s = 0.0, q = 0.0;
    auto acc = [&](float v) {
        const double d = static_cast<double>(v) - k0;
        s += d;
        q += d * d;
    };
    int64_t done = 0;
    if ((reinterpret_cast<uintptr_t>(y) & 15) == 0) {
        const float4 *y4 = reinterpret_cast<const float4 *>(y);
        const int64_t n4 = S / 4;
        for (int64_t i = tid; i < n4; i += kSearchThreads) {
            const float4 v = y4[i];
            acc(v.x);
            acc(v.y);
            acc(v.z);
            acc(v.w);
        }
        done = 4 * n4;
    }
    for (int64_t i = done + tid; i < S; i += kSearchThreads)
        acc(y[i]);
    const double sd = block_sum(s, red) / static_cast<double>(S);
    const double qd = block_sum(q, red) / static_cast<double>(S);
    const double mu = k0 + sd;
    const double sigma = sqrt(fmax(qd - sd * sd, 0.0));

    Cand best{-INFINITY, 0, 1};
    if (sigma > 0.0) {
        const float inv_sigma = static_cast<float>(1.0 / sigma);
        int32_t wmax = 1;
        while (2 * wmax <= S && (31 - __builtin_clz(2 * wmax)) < n_widths)
            wmax *= 2;
        for (int64_t c0 = 0; c0 < S; c0 += kChunk) {
            __syncthreads();  // the previous chunk's boxcars are consumed
            if ((reinterpret_cast<uintptr_t>(y) & 15) == 0) {  // c0 is a multiple of 4
                for (int i = 4 * tid; i < kExt; i += 4 * kSearchThreads) {
                    const int64_t g = c0 + i;
                    float v[4];
                    if (g + 3 < S) {
                        const float4 u = *reinterpret_cast<const float4 *>(y + g);
                        v[0] = u.x;
                        v[1] = u.y;
                        v[2] = u.z;
                        v[3] = u.w;
                    } else {
#pragma unroll
                        for (int k = 0; k < 4; ++k)
                            v[k] = g + k < S ? y[g + k] : 0.f;
                    }
#pragma unroll
                    for (int k = 0; k < 4; ++k)
                        box[i + k] = g + k < S ? static_cast<float>(static_cast<double>(v[k]) - mu) : 0.f;
                }
            } else {
                for (int i = tid; i < kExt; i += kSearchThreads) {
                    const int64_t g = c0 + i;
                    box[i] = g < S ? static_cast<float>(static_cast<double>(y[g]) - mu) : 0.f;
                }
            }
            __syncthreads();
            // box holds B_w(c0 + i) for i + w <= kExt; widths double per level.
            // Each level scores the boxcars starting in this chunk and, in the
            // same pass, forms B_2w(i) = B_w(i) + B_w(i + w) for i + 2w <= kExt:
            // all reads, then a barrier, then the writes, so no thread reads a
            // value already doubled.
            // Thread tid holds the quads j = tid + q * kSearchThreads (samples
            // 4j .. 4j + 3): 16-byte LDS reads and writes throughout.
            constexpr int kQ = kExt / (4 * kSearchThreads);       // quads per thread
            constexpr int kQOwn = kChunk / (4 * kSearchThreads);  // of which hold starts of this chunk
            constexpr int kOwn = 4 * kQOwn;                       // starts this thread scores per chunk
            static_assert(kExt % (4 * kSearchThreads) == 0 && kChunk % (4 * kSearchThreads) == 0,
                          "chunk and halo split evenly into quads over the threads");
            static_assert((kOwn & (kOwn - 1)) == 0, "pairwise argmax over a power of two");
            v4f *box4 = reinterpret_cast<v4f *>(box);
            for (int32_t w = 1;; w *= 2) {
                // 1/sqrt(w) correctly rounded (exact for even powers of two),
                // so boxcars whose binary64 S/N tie also tie here.
                const float scale = inv_sigma * static_cast<float>(1.0 / sqrt(static_cast<double>(w)));
                const bool last = w >= wmax;
                // starts c0 + i with i <= lim end inside the row (i < kExt here)
                const int32_t lim = static_cast<int32_t>(min(S - c0 - w, static_cast<int64_t>(kExt)));
                v4f nv[kQ];
                float sv[kOwn];
                int32_t sk[kOwn];
#pragma unroll
                for (int q = 0; q < kQ; ++q) {
                    const int j = tid + q * kSearchThreads;
                    const v4f b = box4[j];
                    if (q < kQOwn) {
#pragma unroll
                        for (int e = 0; e < 4; ++e) {
                            // starts past S - w score -inf, which no valid start loses to
                            sv[4 * q + e] = 4 * j + e <= lim ? b[e] * scale : -INFINITY;
                            sk[4 * q + e] = 4 * q + e;
                        }
                    }
                    if (!last) {
                        // B_w at samples 4j + e + w: a whole quad w/4 quads on for
                        // w >= 4, else the tail of this quad and the head of the next.
                        v4f u;
                        if (w >= 4) {
                            const int jw = j + (w >> 2);
                            u = jw < kExt / 4 ? box4[jw] : v4f{0.f, 0.f, 0.f, 0.f};
                        } else {
                            const v4f n = j + 1 < kExt / 4 ? box4[j + 1] : v4f{0.f, 0.f, 0.f, 0.f};
                            u = w == 1 ? v4f{b.y, b.z, b.w, n.x} : v4f{b.z, b.w, n.x, n.y};
                        }
#pragma unroll
                        for (int e = 0; e < 4; ++e)
                            nv[q][e] = 4 * j + e + 2 * w <= kExt ? b[e] + u[e] : 0.f;
                    }
                }
                // This width's best start among this thread's (index 4q + e
                // grows with the start), pairwise over neighbouring runs: the
                // earlier run's pick is kept unless the later one scores
                // higher (a NaN never wins, as in better()).
#pragma unroll
                for (int h = 1; h < kOwn; h *= 2)
#pragma unroll
                    for (int k = 0; k < kOwn; k += 2 * h)
                        if (sv[k + h] == sv[k + h] && !(sv[k + h] <= sv[k])) {
                            sv[k] = sv[k + h];
                            sk[k] = sk[k + h];
                        }
                if (sv[0] > -INFINITY) {
                    const int32_t k = sk[0];
                    const Cand c{sv[0], static_cast<int32_t>(c0 + 4 * (tid + (k >> 2) * kSearchThreads) + (k & 3)), w};
                    if (better(c, best))
                        best = c;
                }
                if (last)
                    break;
                __syncthreads();
#pragma unroll
                for (int q = 0; q < kQ; ++q)
                    box4[tid + q * kSearchThreads] = nv[q];
                __syncthreads();
            }
        }
    } else {
        best = Cand{0.f, 0, 1};
    }
    cred[tid] = best;
    __syncthreads();
    for (int o = kSearchThreads / 2; o > 0; o >>= 1) {
        if (tid < o && better(cred[tid + o], cred[tid]))
            cred[tid] = cred[tid + o];
        __syncthreads();
    }
    if (tid == 0) {
        snr_out[blockIdx.x] = cred[0].snr;
        t_out[blockIdx.x] = cred[0].t;
        w_out[blockIdx.x] = cred[0].w;
    }
}

}  // namespace
}  // namespace dd

using namespace dd;

extern "C" int dd_search_boxcar(const float *d_rows, int64_t row_stride, int32_t n_rows, int64_t n_samples,
                                int32_t n_widths, float *d_snr, int32_t *d_t, int32_t *d_width, void *stream) {
    clear_error();
    if (!d_rows || !d_snr || !d_t || !d_width)
        return fail(DD_EINVAL, "NULL argument");
    if (n_rows < 1 || n_samples < 1 || n_samples > 0x7fffffffLL)
        return fail(DD_EINVAL, "need n_rows >= 1 and 1 <= n_samples < 2^31");
    if (n_widths < 1 || n_widths > kMaxWidthsLog)
        return fail(DD_EINVAL, "n_widths must be in [1, %d] (got %d)", kMaxWidthsLog, n_widths);
    if (row_stride < n_samples)
        return fail(DD_ESHAPE, "row_stride %lld < n_samples %lld", (long long)row_stride, (long long)n_samples);
    if (reinterpret_cast<uintptr_t>(d_rows) % 4 || reinterpret_cast<uintptr_t>(d_snr) % 4 ||
        reinterpret_cast<uintptr_t>(d_t) % 4 || reinterpret_cast<uintptr_t>(d_width) % 4)
        return fail(DD_ESHAPE, "pointers must be 4-byte aligned");
    hipLaunchKernelGGL(boxcar_search_kernel, dim3(static_cast<uint32_t>(n_rows)), dim3(kSearchThreads), 0,
                       static_cast<hipStream_t>(stream), d_rows, row_stride, n_samples, n_widths, d_snr, d_t,
                       d_width);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess)
        return fail(DD_EHIP, "search launch failed: %s", hipGetErrorString(e));
    return DD_OK;
}
