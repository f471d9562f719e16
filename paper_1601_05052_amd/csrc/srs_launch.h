// Kernels and launch helpers of the shifted-row sum for gfx950 (CDNA4),
// used by both directions:
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
//
// Included by the per-input-type instantiation units only.
#pragma once

#include <hip/hip_runtime.h>

#include "batch_desc.h"
#include "internal.h"
#include "srs_regwin.h"
#include "srs_tile.h"

namespace dd {
namespace kern {

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

// OCC: waves per SIMD the register-window kernels must keep (1: no
// constraint); set where the kernel sits at a VGPR occupancy step.
template <typename TIn, int IT, int TDW, int NWR, int NW, int RPW, int KMAX, int OCC>
__global__ void __launch_bounds__(64 * NW) __attribute__((amdgpu_waves_per_eu(OCC)))
    srs_regwin_kernel(const TIn *__restrict__ in, float *__restrict__ out, const int32_t *__restrict__ base,
                      const int32_t *__restrict__ recs, const int32_t *__restrict__ span, SrsDims d) {
    extern __shared__ __attribute__((aligned(16))) float lds_rw[];
    int32_t tile_t, tile_a;
    dev::tile_of_block(d, tile_t, tile_a);
    dev::srs_tile_regwin<TIn, IT, TDW, NWR, NW, RPW, KMAX>(in, out, dev::as_ctab(base), dev::as_ctab(recs),
                                                           dev::as_ctab(span), d, tile_t, tile_a, lds_rw);
}

template <typename TIn, int IT, int TDW, int NW, int RPW, int KMAX>
__global__ void __launch_bounds__(64 * NW)
    srs_ldsp_kernel(const TIn *__restrict__ in, float *__restrict__ out, const int32_t *__restrict__ rel,
                    const int32_t *__restrict__ base, const int32_t *__restrict__ span, SrsDims d) {
    extern __shared__ __attribute__((aligned(16))) float lds_p[];
    int32_t tile_t, tile_a;
    dev::tile_of_block(d, tile_t, tile_a);
    dev::srs_tile_ldsp<TIn, IT, TDW, NW, RPW, KMAX>(in, out, dev::as_ctab(rel), dev::as_ctab(base), dev::as_ctab(span),
                                                    d, tile_t, tile_a, lds_p);
}

// VEC: consecutive ownership with 16-byte loads (float32 input only; other
// input types take the strided form).
template <typename TIn, int IT, int NW, int U, bool CARRY, bool VEC>
__global__ void __launch_bounds__(64 * NW)
    srs_direct_kernel(const TIn *__restrict__ in, float *__restrict__ out, const int32_t *__restrict__ rel,
                      const int32_t *__restrict__ base, const int32_t *__restrict__ span, SrsDims d, int32_t r_begin,
                      int32_t r_end) {
    int32_t tile_t, tile_a;
    dev::tile_of_block(d, tile_t, tile_a);
    if constexpr (VEC && sizeof(TIn) == 4)
        dev::srs_tile_direct_vec<IT, NW, U, CARRY>(reinterpret_cast<const float *>(in), out, dev::as_ctab(rel),
                                                   dev::as_ctab(base), dev::as_ctab(span), d, tile_t, tile_a, r_begin,
                                                   r_end);
    else
        dev::srs_tile_direct<TIn, IT, NW, U, CARRY>(in, out, dev::as_ctab(rel), dev::as_ctab(base), dev::as_ctab(span),
                                                    d, tile_t, tile_a, r_begin, r_end);
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

template <typename TIn, int IT, int TDW, int NWR, int NW, int RPW, int KMAX, int OCC>
__global__ void __launch_bounds__(64 * NW) __attribute__((amdgpu_waves_per_eu(OCC)))
    multi_regwin_kernel(BatchPtrs ptrs, const BeamDesc *__restrict__ descs, const uint32_t *__restrict__ items) {
    extern __shared__ __attribute__((aligned(16))) float lds_mr[];
    BeamTile bt;
    if (!beam_tile(ptrs, descs, items, bt))
        return;
    dev::srs_tile_regwin<TIn, IT, TDW, NWR, NW, RPW, KMAX>(static_cast<const TIn *>(bt.in), bt.out, bt.base, bt.recs,
                                                           nullptr, bt.d, bt.tile_t, bt.tile_a, lds_mr);
}

template <typename TIn, int IT, int TDW, int NW, int RPW, int KMAX>
__global__ void __launch_bounds__(64 * NW)
    multi_ldsp_kernel(BatchPtrs ptrs, const BeamDesc *__restrict__ descs, const uint32_t *__restrict__ items) {
    extern __shared__ __attribute__((aligned(16))) float lds_mp[];
    BeamTile bt;
    if (!beam_tile(ptrs, descs, items, bt))
        return;
    dev::srs_tile_ldsp<TIn, IT, TDW, NW, RPW, KMAX>(static_cast<const TIn *>(bt.in), bt.out, bt.rel,
                                                    bt.base, nullptr, bt.d, bt.tile_t, bt.tile_a, lds_mp);
}

template <typename TIn, int IT, int NW, int U>
__global__ void __launch_bounds__(64 * NW)
    multi_direct_kernel(BatchPtrs ptrs, const BeamDesc *__restrict__ descs, const uint32_t *__restrict__ items) {
    BeamTile bt;
    if (!beam_tile(ptrs, descs, items, bt))
        return;
    dev::srs_tile_direct<TIn, IT, NW, U, false>(static_cast<const TIn *>(bt.in), bt.out, bt.rel, bt.base, nullptr,
                                                bt.d, bt.tile_t, bt.tile_a, 0, bt.d.n_rows);
}

inline hipError_t set_lds_limit(const void *fn, size_t lds) {
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

template <typename TIn, int IT, int TDW, int NWR, int NW, int RPW, int KMAX, int OCC>
hipError_t launch_regwin(const SrsArgs &a, const SrsDims &d, uint32_t blocks, size_t lds, hipStream_t s) {
    auto fn = srs_regwin_kernel<TIn, IT, TDW, NWR, NW, RPW, KMAX, OCC>;
    hipError_t e = set_lds_limit(reinterpret_cast<const void *>(fn), lds);
    if (e != hipSuccess)
        return e;
    hipLaunchKernelGGL(fn, dim3(blocks), dim3(64 * NW), lds, s, static_cast<const TIn *>(a.in), a.out, a.base,
                       a.recs, a.span, d);
    return hipGetLastError();
}

template <typename TIn, int IT, int TDW, int NW, int RPW, int KMAX>
hipError_t launch_ldsp(const SrsArgs &a, const SrsDims &d, uint32_t blocks, size_t lds, hipStream_t s) {
    auto fn = srs_ldsp_kernel<TIn, IT, TDW, NW, RPW, KMAX>;
    hipError_t e = set_lds_limit(reinterpret_cast<const void *>(fn), lds);
    if (e != hipSuccess)
        return e;
    hipLaunchKernelGGL(fn, dim3(blocks), dim3(64 * NW), lds, s, static_cast<const TIn *>(a.in), a.out, a.rel,
                       a.base, a.span, d);
    return hipGetLastError();
}

// RB > 0: the rows are summed in blocks of RB by successive launches, each
// continuing the partial sums the previous one left in the output (the
// kernel boundary keeps every work-group within one block of rows).
template <typename TIn, int IT, int NW, int U, int RB, bool VEC>
hipError_t launch_direct(const SrsArgs &a, const SrsDims &d, uint32_t blocks, size_t, hipStream_t s) {
    const int32_t step = RB > 0 ? RB : d.n_rows;
    for (int32_t r0 = 0; r0 < d.n_rows; r0 += step) {
        const int32_t r1 = d.n_rows - r0 > step ? r0 + step : d.n_rows;
        hipLaunchKernelGGL((srs_direct_kernel<TIn, IT, NW, U, (RB > 0), VEC>), dim3(blocks), dim3(64 * NW), 0, s,
                           static_cast<const TIn *>(a.in), a.out, a.rel, a.base, a.span, d, r0, r1);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess)
            return e;
    }
    return hipSuccess;
}

}  // namespace kern
}  // namespace dd
