// In-core ceilings of the kernels' inner loops on gfx950, without HBM traffic:
// the rates the roofline discussion compares the kernels with.
//
//   add_plain   v_add_f32 on independent chains (no index mode)
//   add_index   the register-window additions alone: VGPR index mode, 8
//               accumulator rows x 8 samples per window (RegWin<8, 8, 40>)
//   rowstep_nq  the register-window row step: nq window quads from LDS
//               (ds_read_b128, padded layout) and the index-mode additions
//   lds_b32     the LDS form's reads: 16 samples per lane 64 apart at a
//               wave-uniform offset, one 4-byte read per addition
//   lds_b128    the same with each lane owning 4 consecutive samples at a
//               16-byte aligned offset, one 16-byte read per 4 additions
//
// Every LDS address stays inside the work-group's static LDS array.  Rates
// count additions per second over the whole chip (best of 3 launches after a
// warm-up); LDS rates are bytes per clock per CU at 2.4 GHz.
//
//     paper_1601_05052_amd/ceilings        (built by build.py --ceilings)
#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>
#include <vector>

#include "regwin_asm.h"

namespace {

using dd::dev::RegWin;
using RW = RegWin<8, 8, 40>;
typedef float v4f __attribute__((ext_vector_type(4)));

constexpr int kThreads = 512;  // 8 waves per work-group
constexpr int kLds = 16384;    // floats of LDS per work-group (64 KiB)

__global__ void __launch_bounds__(256) add_plain(float *out, int iters) {
    float a0 = threadIdx.x, a1 = a0 + 1, a2 = a0 + 2, a3 = a0 + 3, a4 = a0 + 4, a5 = a0 + 5, a6 = a0 + 6, a7 = a0 + 7;
    const float b = 1e-7f;
    for (int i = 0; i < iters; ++i) {
        asm volatile(
            "v_add_f32 %0, %0, %8\n\tv_add_f32 %1, %1, %8\n\tv_add_f32 %2, %2, %8\n\tv_add_f32 %3, %3, %8\n\t"
            "v_add_f32 %4, %4, %8\n\tv_add_f32 %5, %5, %8\n\tv_add_f32 %6, %6, %8\n\tv_add_f32 %7, %7, %8\n\t"
            "v_add_f32 %0, %0, %8\n\tv_add_f32 %1, %1, %8\n\tv_add_f32 %2, %2, %8\n\tv_add_f32 %3, %3, %8\n\t"
            "v_add_f32 %4, %4, %8\n\tv_add_f32 %5, %5, %8\n\tv_add_f32 %6, %6, %8\n\tv_add_f32 %7, %7, %8\n\t"
            : "+v"(a0), "+v"(a1), "+v"(a2), "+v"(a3), "+v"(a4), "+v"(a5), "+v"(a6), "+v"(a7)
            : "v"(b));
    }
    out[blockIdx.x * blockDim.x + threadIdx.x] = a0 + a1 + a2 + a3 + a4 + a5 + a6 + a7;
}

// MODE 0: index-mode additions only; 1: window loads and additions (row step).
template <int MODE>
__global__ void __launch_bounds__(kThreads) regwin_step(float *out, int iters, int nq) {
    __shared__ __attribute__((aligned(16))) float lds[kLds];
    for (int i = threadIdx.x; i < kLds; i += kThreads)
        lds[i] = 0.001f * i;
    __syncthreads();
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    // Lane windows 3 quads apart (padded layout for 8 samples per lane); the
    // furthest quad read is 63 * 48 + 208 bytes past the wave's 4 KiB region.
    const uint32_t addr = static_cast<uint32_t>(wave * 4096 + 48 * lane);
    RW::Acc a;
#pragma unroll
    for (int k = 0; k < 64; ++k)
        RW::set_acc(a, k, 0.f);
    union {
        RW::Win w;
        float f[40];
    } u;
#pragma unroll
    for (int k = 0; k < 40; ++k)
        u.f[k] = lane + k;
    int o[8];
#pragma unroll
    for (int k = 0; k < 8; ++k)
        o[k] = (3 * k) & 31;
    float s = 0.f;
    for (int i = 0; i < iters; ++i) {
        // window offsets, four bytes per dword, each at most 31 (<= NWR - 8)
        const uint32_t m = static_cast<uint32_t>(i & 3) * 0x01010101u;
        const uint32_t pk[2] = {static_cast<uint32_t>(__builtin_amdgcn_readfirstlane(0x1c100400u + m)),
                                static_cast<uint32_t>(__builtin_amdgcn_readfirstlane(0x14080c18u + m))};
        if (MODE == 1) {
            int dep;
            RW::load(u.w, addr, nq, pk, o, dep);  // waits for its reads inside the asm block
            s += u.f[0];
        } else {
#pragma unroll
            for (int k = 0; k < 8; ++k)
                o[k] = __builtin_amdgcn_readfirstlane((i + 3 * k) & 31);
        }
        RW::add(a, u.w, o);
    }
    float t = s;
#pragma unroll
    for (int k = 0; k < 64; ++k)
        t += RW::get_acc(a, k);
    out[blockIdx.x * blockDim.x + threadIdx.x] = t;
}

// MODE 0: 4-byte reads (lane l: samples o + l + 64 j); 1: 16-byte reads (lane
// l: samples o + 4 l + 256 k .. + 3, o a multiple of 4).  Offsets o < 4096.
template <int MODE>
__global__ void __launch_bounds__(256) lds_read(float *out, int iters, const int *offs) {
    __shared__ __attribute__((aligned(16))) float lds[kLds];
    for (int i = threadIdx.x; i < kLds; i += 256)
        lds[i] = float(i);
    __syncthreads();
    const int lane = threadIdx.x & 63;
    float acc[4][16];
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int j = 0; j < 16; ++j)
            acc[a][j] = 0.f;
    for (int i = 0; i < iters; ++i) {
#pragma unroll
        for (int a = 0; a < 4; ++a) {
            const int o = __builtin_amdgcn_readfirstlane(offs[(i * 4 + a) & 1023]);
            if (MODE == 0) {
                const float *p = lds + o + lane;  // furthest: 4095 + 63 + 960
#pragma unroll
                for (int j = 0; j < 16; ++j)
                    acc[a][j] += p[64 * j];
            } else {
                const v4f *p = reinterpret_cast<const v4f *>(lds + (o & ~3)) + lane;  // furthest: 4092 + 252 + 768 + 3
#pragma unroll
                for (int k = 0; k < 4; ++k) {
                    const v4f v = p[64 * k];
                    acc[a][4 * k] += v.x;
                    acc[a][4 * k + 1] += v.y;
                    acc[a][4 * k + 2] += v.z;
                    acc[a][4 * k + 3] += v.w;
                }
            }
        }
    }
    float t = 0.f;
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int j = 0; j < 16; ++j)
            t += acc[a][j] * (1 + a + j);
    out[blockIdx.x * blockDim.x + threadIdx.x] = t;
}

template <typename F>
float best_ms(F launch) {
    hipEvent_t e0, e1;
    (void)hipEventCreate(&e0);
    (void)hipEventCreate(&e1);
    launch();
    (void)hipDeviceSynchronize();
    float best = 1e30f;
    for (int rep = 0; rep < 3; ++rep) {
        (void)hipEventRecord(e0, 0);
        launch();
        (void)hipEventRecord(e1, 0);
        (void)hipEventSynchronize(e1);
        float ms = 0.f;
        (void)hipEventElapsedTime(&ms, e0, e1);
        best = ms < best ? ms : best;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    return best;
}

void report(const char *name, double adds, float ms, double lds_bytes) {
    const double per_clk_cu = lds_bytes / (ms * 1e-3) / (256 * 2.4e9);
    printf("{\"name\": \"%s\", \"ms\": %.4f, \"T_adds_per_s\": %.2f", name, ms, adds / (ms * 1e-3) / 1e12);
    if (lds_bytes > 0)
        printf(", \"lds_B_per_clk_per_CU\": %.1f", per_clk_cu);
    printf("}\n");
    fflush(stdout);
}

}  // namespace

int main() {
    const int blocks = 256 * 8;
    float *out = nullptr;
    int *offs = nullptr;
    if (hipMalloc(&out, sizeof(float) * blocks * kThreads) != hipSuccess ||
        hipMalloc(&offs, sizeof(int) * 1024) != hipSuccess) {
        fprintf(stderr, "allocation failed\n");
        return 1;
    }
    std::vector<int> h(1024);
    uint32_t s = 12345u;
    for (int &x : h) {
        s = s * 1103515245u + 12345u;
        x = static_cast<int>((s >> 8) % 4096u);
    }
    if (hipMemcpy(offs, h.data(), sizeof(int) * 1024, hipMemcpyHostToDevice) != hipSuccess)
        return 1;

    {
        const int b = 256 * 16, it = 20000;
        const float ms = best_ms([&] { hipLaunchKernelGGL(add_plain, dim3(b), dim3(256), 0, 0, out, it); });
        report("add_plain", double(b) * 256 * it * 16, ms, 0);
    }
    {
        const int it = 4000;
        const double adds = double(blocks) * kThreads * it * 64;
        float ms = best_ms([&] { hipLaunchKernelGGL(regwin_step<0>, dim3(blocks), dim3(kThreads), 0, 0, out, it, 6); });
        report("add_index", adds, ms, 0);
        for (int nq : {6, 10}) {
            ms = best_ms([&] { hipLaunchKernelGGL(regwin_step<1>, dim3(blocks), dim3(kThreads), 0, 0, out, it, nq); });
            char name[32];
            snprintf(name, sizeof(name), "rowstep_nq%d", nq);
            report(name, adds, ms, double(blocks) * kThreads * it * nq * 16);
        }
    }
    {
        const int it = 2000;
        const double adds = double(blocks) * 256 * it * 4 * 16;
        float ms = best_ms([&] { hipLaunchKernelGGL(lds_read<0>, dim3(blocks), dim3(256), 0, 0, out, it, offs); });
        report("lds_b32", adds, ms, adds * 4);
        ms = best_ms([&] { hipLaunchKernelGGL(lds_read<1>, dim3(blocks), dim3(256), 0, 0, out, it, offs); });
        report("lds_b128", adds, ms, adds * 4);
    }
    (void)hipFree(out);
    (void)hipFree(offs);
    return 0;
}
