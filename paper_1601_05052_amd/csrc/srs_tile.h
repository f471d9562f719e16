// Device-side tile routines shared by the single-beam and batched kernels.
//
// Shifted-row sum: out[a][t] = sum_r in[r][t + O[r][a]] (forward dedispersion,
// Sec. III-A Algorithm 1, with rows = channels and accumulator rows = trial
// DMs; the adjoint with rows = DMs, accumulator rows = channels, O = -delay).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "srs_dims.h"

namespace dd {
namespace dev {

template <typename T>
__device__ __forceinline__ float to_f32(T v);
template <>
__device__ __forceinline__ float to_f32<float>(float v) { return v; }
template <>
__device__ __forceinline__ float to_f32<_Float16>(_Float16 v) { return static_cast<float>(v); }
template <>
__device__ __forceinline__ float to_f32<uint8_t>(uint8_t v) { return static_cast<float>(v); }

// Tile tables are read-only for the whole launch: reading them through the
// constant address space lets the compiler use scalar loads for wave-uniform
// indices, also when the table pointer itself was read from memory.
typedef const __attribute__((address_space(4))) int32_t ctab;
__device__ __forceinline__ ctab *as_ctab(const int32_t *p) { return (ctab *)reinterpret_cast<uintptr_t>(p); }

// Tile skew of accumulator row ag: its tile sample tau is output sample
// tau - skew (0 without skew tables or past the last row).
__device__ __forceinline__ int32_t skew_of(const SrsDims &d, int32_t ag) {
    return d.skew && ag < d.n_acc ? __builtin_amdgcn_readfirstlane(as_ctab(d.skew)[ag]) : 0;
}


// Map the hardware work-group id to (time tile, accumulator tile).  Work-groups
// are dealt round-robin to the 8 XCDs; renumber so that each XCD receives a
// contiguous run of logical tiles, ordered accumulator-tile fastest, so the
// work-groups resident on one XCD share input windows in its L2.
__device__ __forceinline__ void tile_of_block(const SrsDims &d, int32_t &tile_t, int32_t &tile_a) {
    const uint32_t n = static_cast<uint32_t>(d.n_t_tiles) * static_cast<uint32_t>(d.n_acc_tiles);
    const uint32_t b = blockIdx.x;
    const uint32_t per = n / 8u, extra = n % 8u;
    const uint32_t xcd = b % 8u, k = b / 8u;
    // XCDs 0..extra-1 hold per+1 tiles, the rest hold per tiles.
    const uint32_t start = xcd * per + (xcd < extra ? xcd : extra);
    const uint32_t logical = start + k;
    tile_a = static_cast<int32_t>(logical % static_cast<uint32_t>(d.n_acc_tiles));
    tile_t = static_cast<int32_t>(logical / static_cast<uint32_t>(d.n_acc_tiles));
}

// One tile, LDS-read-per-addition form.  Lane l of a wave owns samples
// t0 + l + 64*j (j < IT) of that wave's TDW accumulator rows; every addition
// reads its operand from the staged window at a wave-uniform offset, so the
// 64 lanes read 64 consecutive LDS words (conflict-free).
template <typename TIn, int IT, int TDW, int NW>
__device__ __forceinline__ void srs_tile_lds(const TIn *__restrict__ in, float *__restrict__ out,
                                             ctab *__restrict__ rel, ctab *__restrict__ base, const SrsDims &d,
                                             int32_t tile_t, int32_t tile_a, float *lds) {
    constexpr int TT = 64 * IT;
    constexpr int TA = TDW * NW;
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int64_t t0 = static_cast<int64_t>(tile_t) * TT;
    // The tables hold this launch's block of rows, [r_begin, r_end).
    const int32_t nb = d.r_end - d.r_begin;
    ctab *rel_tile = rel + static_cast<int64_t>(tile_a) * nb * TA + wave * TDW;
    ctab *base_tile = base + static_cast<int64_t>(tile_a) * nb;

    float acc[TDW][IT];
#pragma unroll
    for (int k = 0; k < TDW; ++k) {
        const int32_t ag = tile_a * TA + wave * TDW + k;
        const int64_t ts = t0 - skew_of(d, ag);  // output sample of this row's tile sample t0
#pragma unroll
        for (int j = 0; j < IT; ++j) {
            const int64_t t = ts + lane + 64 * j;
            // carry: continue the partial sums of the previous blocks of rows
            acc[k][j] = d.carry && ag < d.n_acc && t >= 0 && t < d.n_t ? out[static_cast<int64_t>(ag) * d.out_stride + t]
                                                                       : 0.f;
        }
    }

    for (int32_t r0 = d.r_begin; r0 < d.r_end; r0 += d.rows_per_chunk) {  // this launch's block of rows
        const int32_t nr = min(d.rows_per_chunk, d.r_end - r0);
        __syncthreads();  // previous chunk fully consumed
        for (int32_t rr = wave; rr < nr; rr += NW) {
            const int32_t r = r0 + rr;
            const int64_t g0 = t0 + base_tile[r - d.r_begin];
            const TIn *src = in + static_cast<int64_t>(r) * d.in_stride;
            float *dst = lds + rr * d.wcap;
#pragma unroll 4
            for (int32_t w = lane; w < d.wcap; w += 64) {
                const int64_t g = g0 + w;
                float v = 0.f;
                if (g >= 0 && g < d.in_valid)
                    v = to_f32<TIn>(src[g]);
                dst[w] = v;
            }
        }
        __syncthreads();  // window staged
        for (int32_t rr = 0; rr < nr; ++rr) {
            ctab *o = rel_tile + static_cast<int64_t>(r0 - d.r_begin + rr) * TA;
            const float *row = lds + rr * d.wcap + lane;
#pragma unroll
            for (int k = 0; k < TDW; ++k) {
                const float *p = row + o[k];
#pragma unroll
                for (int j = 0; j < IT; ++j)
                    acc[k][j] += p[64 * j];
            }
        }
    }

#pragma unroll
    for (int k = 0; k < TDW; ++k) {
        const int32_t ag = tile_a * TA + wave * TDW + k;
        if (ag < d.n_acc) {
            float *dst = out + static_cast<int64_t>(ag) * d.out_stride;
            const int64_t ts = t0 - skew_of(d, ag);
#pragma unroll
            for (int j = 0; j < IT; ++j) {
                const int64_t t = ts + lane + 64 * j;
                if (t >= 0 && t < d.n_t)
                    __builtin_nontemporal_store(acc[k][j], dst + t);
            }
        }
    }
}

}  // namespace dev
}  // namespace dd
