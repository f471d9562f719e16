// Shifted-row-sum kernels for gfx950 (CDNA4), used by both directions:
//     out[a][t] = sum_r in[r][t + O[r][a]]
// (forward dedispersion, Sec. III-A Algorithm 1, with rows = channels and
// accumulator rows = trial DMs; the adjoint with rows = DMs, accumulator rows =
// channels and O = -delay).
//
// Decomposition follows Sec. III-B: DM (accumulator) and time are the
// independent axes; a work-group owns TA accumulator rows x TT consecutive
// samples, lanes run along time so stores are coalesced and aligned, each
// lane keeps its outputs in registers, and the work-group stages each input
// row's window in LDS once so every accumulator row of the tile reuses it
// (the data reuse of Sec. III-A, Eq. (3)).  Only binary32 additions; no MFMA.
#include <hip/hip_runtime.h>

#include "batch_desc.h"
#include "internal.h"
#include "srs_regwin.h"
#include "srs_tile.h"

namespace dd {

namespace {

using dev::SrsDims;

template <typename TIn, int IT, int TDW, int NW>
__global__ void __launch_bounds__(64 * NW)
    srs_lds_kernel(const TIn *__restrict__ in, float *__restrict__ out, const int32_t *__restrict__ rel,
                   const int32_t *__restrict__ base, SrsDims d) {
    extern __shared__ float lds[];
    int32_t tile_t, tile_a;
    dev::tile_of_block(d, tile_t, tile_a);
    dev::srs_tile_lds<TIn, IT, TDW, NW>(in, out, dev::as_ctab(rel), dev::as_ctab(base), d, tile_t, tile_a, lds);
}

template <typename TIn, int IT, int TDW, int NWR, int NW, int RPW, int KMAX>
__global__ void __launch_bounds__(64 * NW)
    srs_regwin_kernel(const TIn *__restrict__ in, float *__restrict__ out, const int32_t *__restrict__ base,
                      const int32_t *__restrict__ recs, SrsDims d) {
    extern __shared__ __attribute__((aligned(16))) float lds_rw[];
    int32_t tile_t, tile_a;
    dev::tile_of_block(d, tile_t, tile_a);
    dev::srs_tile_regwin<TIn, IT, TDW, NWR, NW, RPW, KMAX>(in, out, dev::as_ctab(base), dev::as_ctab(recs), d,
                                                           tile_t, tile_a, lds_rw);
}

template <typename TIn, int IT, int TDW, int NW, int RPW, int KMAX>
__global__ void __launch_bounds__(64 * NW)
    srs_ldsp_kernel(const TIn *__restrict__ in, float *__restrict__ out, const int32_t *__restrict__ rel,
                    const int32_t *__restrict__ base, SrsDims d) {
    extern __shared__ __attribute__((aligned(16))) float lds_p[];
    int32_t tile_t, tile_a;
    dev::tile_of_block(d, tile_t, tile_a);
    dev::srs_tile_ldsp<TIn, IT, TDW, NW, RPW, KMAX>(in, out, dev::as_ctab(rel), dev::as_ctab(base), d, tile_t, tile_a,
                                                    lds_p);
}

template <typename TIn, int IT, int NW, int U>
__global__ void __launch_bounds__(64 * NW)
    srs_direct_kernel(const TIn *__restrict__ in, float *__restrict__ out, const int32_t *__restrict__ rel,
                      const int32_t *__restrict__ base, SrsDims d) {
    int32_t tile_t, tile_a;
    dev::tile_of_block(d, tile_t, tile_a);
    dev::srs_tile_direct<TIn, IT, NW, U>(in, out, dev::as_ctab(rel), dev::as_ctab(base), d, tile_t, tile_a);
}

// Multi-beam forms: work-group g takes items[g] = (beam << 24) | logical tile
// (the host lays the list out so each XCD walks contiguous runs of every
// beam's tiles) and runs the same tile routine as the single-beam kernel.
struct BeamTile {
    const void *in;
    float *out;
    const BeamDesc *desc;
    dev::ctab *rel, *base, *recs;
    SrsDims d;
    int32_t tile_t, tile_a;
};

// Wave-uniform copies (the compiler cannot see that values read through a
// dynamically indexed kernel argument are uniform; without this it wraps every
// buffer load in a per-lane loop over the resource descriptor).
__device__ __forceinline__ uint64_t uniform64(uint64_t v) {
    const uint32_t lo = __builtin_amdgcn_readfirstlane(static_cast<uint32_t>(v));
    const uint32_t hi = __builtin_amdgcn_readfirstlane(static_cast<uint32_t>(v >> 32));
    return (static_cast<uint64_t>(hi) << 32) | lo;
}
// Uniform pointer into global memory.  The round trip through a global
// (address space 1) pointer lets the compiler treat loads through it as global
// -- pointers read from memory are otherwise generic, and generic loads count
// as divergent (they could address per-lane private memory).
template <typename T>
__device__ __forceinline__ T *uniform_ptr(T *p) {
    typedef __attribute__((address_space(1))) T GT;
    GT *g = (GT *)uniform64(reinterpret_cast<uintptr_t>(p));  // integer straight to a global pointer
    return (T *)g;
}

__device__ __forceinline__ bool beam_tile(const BatchPtrs &ptrs, const BeamDesc *__restrict__ descs,
                                          const uint32_t *__restrict__ items, BeamTile &bt) {
    const uint32_t w = __builtin_amdgcn_readfirstlane(items[blockIdx.x]);
    if (w == kNoItem)
        return false;
    const uint32_t beam = w >> 24, tile = w & 0xffffffu;
    const BeamPtrs &bp = ptrs.b[beam];
    bt.in = uniform_ptr(bp.in);
    bt.out = uniform_ptr(bp.out);
    bt.desc = uniform_ptr(&descs[beam]);
    bt.d = bt.desc->d;
    bt.rel = dev::as_ctab(bt.desc->rel);
    bt.base = dev::as_ctab(bt.desc->base);
    bt.recs = dev::as_ctab(bt.desc->recs);
    bt.d.in_stride = static_cast<int64_t>(uniform64(static_cast<uint64_t>(bp.in_stride)));
    bt.d.out_stride = static_cast<int64_t>(uniform64(static_cast<uint64_t>(bp.out_stride)));
    bt.tile_a = static_cast<int32_t>(tile % static_cast<uint32_t>(bt.d.n_acc_tiles));
    bt.tile_t = static_cast<int32_t>(tile / static_cast<uint32_t>(bt.d.n_acc_tiles));
    return true;
}

template <typename TIn, int IT, int TDW, int NW>
__global__ void __launch_bounds__(64 * NW)
    multi_lds_kernel(BatchPtrs ptrs, const BeamDesc *__restrict__ descs, const uint32_t *__restrict__ items) {
    extern __shared__ float lds_ml[];
    BeamTile bt;
    if (!beam_tile(ptrs, descs, items, bt))
        return;
    dev::srs_tile_lds<TIn, IT, TDW, NW>(static_cast<const TIn *>(bt.in), bt.out, bt.rel, bt.base, bt.d,
                                        bt.tile_t, bt.tile_a, lds_ml);
}

// OCC: waves per SIMD the multi-beam form must keep (1: no constraint); set
// where the single-beam kernel sits exactly at a VGPR occupancy step.
template <typename TIn, int IT, int TDW, int NWR, int NW, int RPW, int KMAX, int OCC>
__global__ void __launch_bounds__(64 * NW) __attribute__((amdgpu_waves_per_eu(OCC)))
    multi_regwin_kernel(BatchPtrs ptrs, const BeamDesc *__restrict__ descs, const uint32_t *__restrict__ items) {
    extern __shared__ __attribute__((aligned(16))) float lds_mr[];
    BeamTile bt;
    if (!beam_tile(ptrs, descs, items, bt))
        return;
    dev::srs_tile_regwin<TIn, IT, TDW, NWR, NW, RPW, KMAX>(static_cast<const TIn *>(bt.in), bt.out, bt.base, bt.recs, bt.d,
                                                           bt.tile_t, bt.tile_a, lds_mr);
}

template <typename TIn, int IT, int TDW, int NW, int RPW, int KMAX>
__global__ void __launch_bounds__(64 * NW)
    multi_ldsp_kernel(BatchPtrs ptrs, const BeamDesc *__restrict__ descs, const uint32_t *__restrict__ items) {
    extern __shared__ __attribute__((aligned(16))) float lds_mp[];
    BeamTile bt;
    if (!beam_tile(ptrs, descs, items, bt))
        return;
    dev::srs_tile_ldsp<TIn, IT, TDW, NW, RPW, KMAX>(static_cast<const TIn *>(bt.in), bt.out, bt.rel,
                                                    bt.base, bt.d, bt.tile_t, bt.tile_a, lds_mp);
}

template <typename TIn, int IT, int NW, int U>
__global__ void __launch_bounds__(64 * NW)
    multi_direct_kernel(BatchPtrs ptrs, const BeamDesc *__restrict__ descs, const uint32_t *__restrict__ items) {
    BeamTile bt;
    if (!beam_tile(ptrs, descs, items, bt))
        return;
    dev::srs_tile_direct<TIn, IT, NW, U>(static_cast<const TIn *>(bt.in), bt.out, bt.rel, bt.base,
                                         bt.d, bt.tile_t, bt.tile_a);
}

using LaunchFn = hipError_t (*)(const SrsArgs &, const SrsDims &, uint32_t, size_t, hipStream_t);

hipError_t set_lds_limit(const void *fn, size_t lds) {
    if (lds <= 65536)
        return hipSuccess;
    return hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(lds));
}

template <typename TIn, int IT, int TDW, int NW>
hipError_t launch_lds(const SrsArgs &a, const SrsDims &d, uint32_t blocks, size_t lds, hipStream_t s) {
    auto fn = srs_lds_kernel<TIn, IT, TDW, NW>;
    hipError_t e = set_lds_limit(reinterpret_cast<const void *>(fn), lds);
    if (e != hipSuccess)
        return e;
    hipLaunchKernelGGL(fn, dim3(blocks), dim3(64 * NW), lds, s, static_cast<const TIn *>(a.in), a.out, a.rel,
                       a.base, d);
    return hipGetLastError();
}

template <typename TIn, int IT, int TDW, int NWR, int NW, int RPW, int KMAX>
hipError_t launch_regwin(const SrsArgs &a, const SrsDims &d, uint32_t blocks, size_t lds, hipStream_t s) {
    auto fn = srs_regwin_kernel<TIn, IT, TDW, NWR, NW, RPW, KMAX>;
    hipError_t e = set_lds_limit(reinterpret_cast<const void *>(fn), lds);
    if (e != hipSuccess)
        return e;
    hipLaunchKernelGGL(fn, dim3(blocks), dim3(64 * NW), lds, s, static_cast<const TIn *>(a.in), a.out, a.base,
                       a.recs, d);
    return hipGetLastError();
}

template <typename TIn, int IT, int TDW, int NW, int RPW, int KMAX>
hipError_t launch_ldsp(const SrsArgs &a, const SrsDims &d, uint32_t blocks, size_t lds, hipStream_t s) {
    auto fn = srs_ldsp_kernel<TIn, IT, TDW, NW, RPW, KMAX>;
    hipError_t e = set_lds_limit(reinterpret_cast<const void *>(fn), lds);
    if (e != hipSuccess)
        return e;
    hipLaunchKernelGGL(fn, dim3(blocks), dim3(64 * NW), lds, s, static_cast<const TIn *>(a.in), a.out, a.rel,
                       a.base, d);
    return hipGetLastError();
}

template <typename TIn, int IT, int NW, int U>
hipError_t launch_direct(const SrsArgs &a, const SrsDims &d, uint32_t blocks, size_t, hipStream_t s) {
    hipLaunchKernelGGL((srs_direct_kernel<TIn, IT, NW, U>), dim3(blocks), dim3(64 * NW), 0, s,
                       static_cast<const TIn *>(a.in), a.out, a.rel, a.base, d);
    return hipGetLastError();
}

struct VariantImpl {
    Variant v;
    LaunchFn fn[3];       // by input type: f32, f16, u8
    const void *multi[3]; // multi-beam kernel, by input type
};

#define DD_FN(f) reinterpret_cast<const void *>(f)

#define DD_LDS_VARIANT(ID, IT, TDW, NW, RATE)                                             \
    {{ID, IT, TDW, NW, KIND_LDS, 0, 0, 0, RATE},                                                \
     {launch_lds<float, IT, TDW, NW>, launch_lds<_Float16, IT, TDW, NW>, launch_lds<uint8_t, IT, TDW, NW>},    \
     {DD_FN((multi_lds_kernel<float, IT, TDW, NW>)), DD_FN((multi_lds_kernel<_Float16, IT, TDW, NW>)),       \
      DD_FN((multi_lds_kernel<uint8_t, IT, TDW, NW>))}}

#define DD_LDSP_VARIANT(ID, IT, TDW, NW, RPW, KMAX, RATE)                                        \
    {{ID, IT, TDW, NW, KIND_LDS, RPW, 0, KMAX, RATE},                                                   \
     {launch_ldsp<float, IT, TDW, NW, RPW, KMAX>, launch_ldsp<_Float16, IT, TDW, NW, RPW, KMAX>, \
      launch_ldsp<uint8_t, IT, TDW, NW, RPW, KMAX>},                                                    \
     {DD_FN((multi_ldsp_kernel<float, IT, TDW, NW, RPW, KMAX>)),                                          \
      DD_FN((multi_ldsp_kernel<_Float16, IT, TDW, NW, RPW, KMAX>)),                                       \
      DD_FN((multi_ldsp_kernel<uint8_t, IT, TDW, NW, RPW, KMAX>))}}

#define DD_DIRECT_VARIANT(ID, IT, NW, U, RATE)                                                            \
    {{ID, IT, 1, NW, KIND_DIRECT, U, 0, 0, RATE},                                                              \
     {launch_direct<float, IT, NW, U>, launch_direct<_Float16, IT, NW, U>, launch_direct<uint8_t, IT, NW, U>}, \
     {DD_FN((multi_direct_kernel<float, IT, NW, U>)), DD_FN((multi_direct_kernel<_Float16, IT, NW, U>)),      \
      DD_FN((multi_direct_kernel<uint8_t, IT, NW, U>))}}

#define DD_RW_VARIANT(ID, IT, TDW, NWR, NW, RPW, KMAX, RATE) DD_RW_VARIANT_OCC(ID, IT, TDW, NWR, NW, RPW, KMAX, 1, RATE)
#define DD_RW_VARIANT_OCC(ID, IT, TDW, NWR, NW, RPW, KMAX, OCC, RATE)                                    \
    {{ID, IT, TDW, NW, KIND_REGWIN, RPW, NWR, KMAX, RATE},                                               \
     {launch_regwin<float, IT, TDW, NWR, NW, RPW, KMAX>,                                           \
      launch_regwin<_Float16, IT, TDW, NWR, NW, RPW, KMAX>,                                        \
      launch_regwin<uint8_t, IT, TDW, NWR, NW, RPW, KMAX>},                                        \
     {DD_FN((multi_regwin_kernel<float, IT, TDW, NWR, NW, RPW, KMAX, OCC>)),                       \
      DD_FN((multi_regwin_kernel<_Float16, IT, TDW, NWR, NW, RPW, KMAX, OCC>)),                    \
      DD_FN((multi_regwin_kernel<uint8_t, IT, TDW, NWR, NW, RPW, KMAX, OCC>))}}

const VariantImpl kImpls[] = {
    DD_LDS_VARIANT(0, 4, 8, 4, 5.4f),   // 256 samples x 32 rows
    DD_LDS_VARIANT(1, 4, 4, 4, 6.3f),   // 256 x 16
    DD_LDS_VARIANT(2, 2, 8, 4, 7.1f),   // 128 x 32
    DD_LDS_VARIANT(3, 8, 4, 4, 3.2f),   // 512 x 16
    DD_LDS_VARIANT(4, 4, 16, 4, 4.7f),  // 256 x 64
    DD_LDS_VARIANT(5, 2, 16, 4, 5.3f),  // 128 x 64
    DD_LDS_VARIANT(6, 4, 2, 4, 3.9f),   // 256 x 8
    DD_LDS_VARIANT(7, 4, 1, 4, 2.3f),   // 256 x 4
    DD_LDS_VARIANT(8, 2, 1, 4, 2.9f),   // 128 x 4
    DD_LDS_VARIANT(9, 1, 1, 1, 0.8f),   // 64 x 1: no cross-row window, always fits
    DD_RW_VARIANT(10, 8, 8, 40, 4, 1, 16, 20.1f),   // 512 x 32, register window; rates: measured T adds/s
    DD_RW_VARIANT(11, 8, 8, 40, 4, 2, 16, 15.1f),   // 512 x 32, two rows per wave per chunk
    DD_RW_VARIANT(12, 8, 4, 32, 4, 2, 16, 10.7f),   // 512 x 16
    DD_RW_VARIANT(13, 16, 4, 48, 4, 1, 24, 18.9f),  // 1024 x 16
    DD_RW_VARIANT(14, 4, 8, 32, 4, 2, 12, 15.7f),   // 256 x 32
    DD_RW_VARIANT(15, 8, 8, 40, 8, 1, 16, 16.2f),   // 512 x 64, eight waves
    DD_RW_VARIANT(16, 8, 16, 48, 4, 1, 16, 15.0f),  // 512 x 64, sixteen rows per wave
    DD_RW_VARIANT(17, 8, 8, 40, 4, 1, 12, 23.0f),   // 512 x 32, shorter staging (fewer VGPRs)
    DD_RW_VARIANT(18, 8, 8, 40, 2, 1, 12, 22.0f),    // 512 x 16, two waves per group
    DD_RW_VARIANT(19, 8, 4, 32, 4, 1, 12, 19.3f),   // 512 x 16, short staging
    DD_LDSP_VARIANT(20, 4, 8, 4, 1, 24, 10.9f),        // 256 x 32, LDS form with prefetched staging
    DD_LDSP_VARIANT(21, 4, 4, 4, 1, 16, 11.4f),        // 256 x 16
    DD_LDSP_VARIANT(22, 8, 4, 4, 1, 24, 11.0f),        // 512 x 16
    DD_LDSP_VARIANT(23, 2, 8, 4, 2, 12, 9.6f),        // 128 x 32
    DD_LDSP_VARIANT(24, 4, 2, 4, 2, 12, 10.3f),        // 256 x 8
    DD_LDSP_VARIANT(25, 4, 1, 4, 2, 8, 7.2f),         // 256 x 4
    DD_LDSP_VARIANT(26, 8, 8, 4, 1, 32, 9.6f),        // 512 x 32
    DD_DIRECT_VARIANT(27, 4, 4, 4, 4.8f),             // 256 x 4, operands read straight from memory
    DD_DIRECT_VARIANT(28, 8, 4, 2, 7.3f),             // 512 x 4
    DD_RW_VARIANT(29, 8, 4, 44, 4, 1, 12, 17.5f),   // 512 x 16, wide window (adjoint)
    DD_RW_VARIANT(30, 8, 8, 76, 4, 1, 12, 20.8f),   // 512 x 32, wide window (adjoint)
    DD_RW_VARIANT_OCC(31, 8, 8, 40, 8, 1, 12, 4, 20.0f),  // 512 x 64, eight waves, short staging
    DD_RW_VARIANT(32, 16, 4, 48, 4, 1, 20, 18.0f),  // 1024 x 16, short staging
};
constexpr int32_t kNumImpls = sizeof(kImpls) / sizeof(kImpls[0]);

Variant g_variants[kNumImpls];
bool g_variants_init = false;

}  // namespace

const Variant *variants(int32_t *count) {
    if (!g_variants_init) {
        for (int32_t i = 0; i < kNumImpls; ++i)
            g_variants[i] = kImpls[i].v;
        g_variants_init = true;
    }
    *count = kNumImpls;
    return g_variants;
}

const Variant *find_variant(int32_t id) {
    int32_t n = 0;
    const Variant *vs = variants(&n);
    return (id >= 0 && id < n) ? &vs[id] : nullptr;
}

int32_t max_lds_bytes() {
    static int32_t cached = 0;
    if (!cached) {
        int dev = 0, v = 0;
        if (hipGetDevice(&dev) == hipSuccess &&
            hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) == hipSuccess && v > 0)
            cached = v;
        else
            cached = 160 * 1024;  // gfx950
    }
    return cached;
}

const void *multi_kernel(const Variant &v, int32_t in_type) { return kImpls[v.id].multi[in_type]; }

hipError_t launch_srs(const Variant &v, int32_t in_type, const SrsArgs &a, hipStream_t stream) {
    const VariantImpl &impl = kImpls[v.id];
    SrsDims d;
    d.in_stride = a.in_stride;
    d.in_valid = a.in_valid;
    d.out_stride = a.out_stride;
    d.n_t = a.n_t;
    d.n_acc = a.n_acc;
    d.n_rows = a.n_rows;
    d.wcap = a.wcap;
    d.rows_per_chunk = a.rows_per_chunk;
    d.n_t_tiles = static_cast<int32_t>((a.n_t + v.tt() - 1) / v.tt());
    d.n_acc_tiles = (a.n_acc + v.ta() - 1) / v.ta();
    const uint64_t blocks = static_cast<uint64_t>(d.n_t_tiles) * d.n_acc_tiles;
    if (blocks == 0)
        return hipSuccess;
    if (blocks > 0x7fffffffull)
        return hipErrorInvalidConfiguration;
    return impl.fn[in_type](a, d, static_cast<uint32_t>(blocks), static_cast<size_t>(a.lds_bytes), stream);
}

}  // namespace dd
