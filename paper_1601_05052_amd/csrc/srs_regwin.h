// Register-window tile routine (gfx950) for the shifted-row sum
//     out[a][t] = sum_r in[r][t + O[r][a]].
//
// Same decomposition as the LDS form (Sec. III-B: DM x time work-groups,
// several outputs per work-item kept in registers, input rows staged once per
// work-group in LDS), but each lane owns IT *consecutive* samples and copies
// the part of the staged row it needs -- IT + (spread of its wave's
// accumulator rows) samples -- into VGPRs once per input row.  Every
// accumulator row then adds that register window at its own wave-uniform
// offset through VGPR index mode (see regwin_asm.h): one VALU addition per
// output element and one LDS word per ~IT*TDW/(IT+spread) additions, instead
// of one LDS word per addition.  This is the data reuse of Sec. III-A, Eq. (3)
// moved from local memory into registers.
//
// Staging: every wave owns RPW rows of each chunk of NW*RPW input rows.  Its
// lanes fetch them with bounds-checked buffer loads of four samples each
// (samples outside [0, in_valid) read as zero) into registers two chunks
// ahead, widen them to binary32 and write them to the other of two LDS chunk
// buffers; one barrier per chunk.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#ifdef DD_STUDY
#include "study_regwin_asm.h"  // every window shape of the study's grid
#else
#include "regwin_asm.h"
#endif
#include "srs_tile.h"

namespace dd {
namespace dev {

typedef int v4i __attribute__((ext_vector_type(4)));
typedef int v3i __attribute__((ext_vector_type(3)));
typedef int v2i __attribute__((ext_vector_type(2)));

constexpr uint32_t kBufferFlags = 0x00020000u;  // raw buffer, 32-bit data format (gfx9 V# word 3)
constexpr uint32_t kOutOfRange = 0x80000000u;   // any offset >= num_records reads 0

template <typename TIn>
__device__ __forceinline__ float buffer_ld(__amdgpu_buffer_rsrc_t rs, uint32_t byte_off);
template <>
__device__ __forceinline__ float buffer_ld<float>(__amdgpu_buffer_rsrc_t rs, uint32_t off) {
    return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(rs, off, 0, 0));
}
template <>
__device__ __forceinline__ float buffer_ld<_Float16>(__amdgpu_buffer_rsrc_t rs, uint32_t off) {
    return static_cast<float>(__builtin_bit_cast(_Float16, __builtin_amdgcn_raw_buffer_load_b16(rs, off, 0, 0)));
}
template <>
__device__ __forceinline__ float buffer_ld<uint8_t>(__amdgpu_buffer_rsrc_t rs, uint32_t off) {
    return static_cast<float>(__builtin_amdgcn_raw_buffer_load_b8(rs, off, 0, 0));
}

// Fetch samples [g0, g0 + 64*nk) of input row `row` into pre[]: lane l gets
// samples g0 + l + 64k for k < KMAX.  The buffer's range is clipped to
// min(in_valid, g0 + 64*nk), so every sample outside the row or past the
// window reads zero and the loads need no per-lane conditions (which would
// otherwise force a wait on each load).
template <typename TIn, int KMAX>
__device__ __forceinline__ void fetch_row(const TIn *__restrict__ in, int64_t in_stride, int64_t in_valid,
                                          int32_t row, int64_t g0, int32_t nk, int lane, float (&pre)[KMAX]) {
    const TIn *rp = in + static_cast<int64_t>(row) * in_stride;
    const int64_t end = min(in_valid, g0 + 64 * static_cast<int64_t>(nk));
    const int32_t n_bytes = end > 0 ? static_cast<int32_t>(end * static_cast<int64_t>(sizeof(TIn))) : 0;
    const __amdgpu_buffer_rsrc_t rs =
        __builtin_amdgcn_make_buffer_rsrc(const_cast<TIn *>(rp), 0, n_bytes, kBufferFlags);
    if (g0 >= 0) {
        // g0 < 2^29 keeps every offset below 2^31.
        const uint32_t voff = static_cast<uint32_t>(g0 + lane) * sizeof(TIn);
#pragma unroll
        for (int k = 0; k < KMAX; ++k)
            pre[k] = buffer_ld<TIn>(rs, voff + k * 64 * sizeof(TIn));
    } else {
        // Window starts before sample 0 (adjoint near t = 0): lanes whose sample
        // index is negative read out of range, i.e. zero.
#pragma unroll
        for (int k = 0; k < KMAX; ++k) {
            const int64_t g = g0 + lane + 64 * k;
            const uint32_t off = g >= 0 ? static_cast<uint32_t>(g) * sizeof(TIn) : kOutOfRange;
            pre[k] = buffer_ld<TIn>(rs, off);
        }
    }
}

// 32-bit LDS address of a pointer into __shared__ memory.
__device__ __forceinline__ uint32_t lds_address(const float *p) {
    return static_cast<uint32_t>(reinterpret_cast<uintptr_t>((const __attribute__((address_space(3))) float *)p));
}

// Raw dwords of one staged quad (four consecutive samples) as loaded: float32
// exactly the quad; float16 and u8 one dword more, so that a quad starting
// inside a dword can be realigned.
template <typename TIn>
struct QuadRaw;
template <>
struct QuadRaw<float> {
    typedef v4i T;
};
template <>
struct QuadRaw<_Float16> {
    typedef v3i T;
};
template <>
struct QuadRaw<uint8_t> {
    typedef v2i T;
};

// Staging loads of one row: lane l fetches quad k (k < KL), samples
// g0 + 4l + 256k .. +3, with one bounds-checked buffer load.  g0 is a
// multiple of 4 (register-window rows start there), so a quad lies wholly
// before sample 0 -- it reads zero (adjoint windows near t = 0) -- or wholly
// at or after it.  The data is only used when the row is stored to LDS (two
// chunks later), so the loads' latency stays hidden.
//   float32: the buffer's range is clipped to min(in_valid, g0 + wcap)
//     samples; samples past it read zero (the adjoint relies on zeros past
//     its input).
//   float16 / u8 (forward only): rows may start at any byte, so the loads are
//     made from the dword boundary at or below the quad, one dword longer than
//     the quad; *delta (the quad's byte offset in its first dword, the same for
//     every quad of the row) realigns them when they are stored.  The range is
//     clipped to the dword holding the last valid sample: every dword read
//     holds at least one byte of the caller's buffer, and bytes past the valid
//     samples only reach samples that no stored output reads.
template <typename TIn, int KL>
__device__ __forceinline__ void fetch_quads(const TIn *__restrict__ in, int64_t in_stride, int64_t in_valid,
                                            int32_t row, int64_t g0, int32_t wcap, int lane,
                                            typename QuadRaw<TIn>::T (&raw)[KL], uint32_t *delta) {
    constexpr uint32_t ES = sizeof(TIn);
    const TIn *rp = in + static_cast<int64_t>(row) * in_stride;
    const int64_t end = min(in_valid, g0 + wcap);
    const int64_t q0 = g0 + 4 * lane;  // first sample of quad 0 (multiple of 4)
    if constexpr (ES == 4) {
        const int32_t end_b = end > 0 ? static_cast<int32_t>(end * 4) : 0;
        const __amdgpu_buffer_rsrc_t rs =
            __builtin_amdgcn_make_buffer_rsrc(const_cast<TIn *>(rp), 0, end_b, kBufferFlags);
#pragma unroll
        for (int k = 0; k < KL; ++k) {
            const int64_t s = q0 + 256 * k;  // |s| < 2^29
            const uint32_t off = s >= 0 ? static_cast<uint32_t>(s) * 4u : kOutOfRange;
            raw[k] = __builtin_bit_cast(v4i, __builtin_amdgcn_raw_buffer_load_b128(rs, off, 0, 0));
        }
        *delta = 0;
    } else {
        const uintptr_t ra = reinterpret_cast<uintptr_t>(rp);
        const uint32_t a_r = static_cast<uint32_t>(ra & 3u);  // row start within its dword
        const uint32_t end_b = end > 0 ? static_cast<uint32_t>(end) * ES + a_r : 0;
        const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc(
            reinterpret_cast<void *>(ra - a_r), 0, static_cast<int32_t>((end_b + 3u) & ~3u), kBufferFlags);
        // Every quad starts at the same byte within a dword (4 * ES bytes apart).
        const uint32_t dl = (static_cast<uint32_t>(g0) * ES + a_r) & 3u;  // wave-uniform
#pragma unroll
        for (int k = 0; k < KL; ++k) {
            const int64_t s = q0 + 256 * k;
            const uint32_t off = s >= 0 ? static_cast<uint32_t>(s) * ES + a_r - dl : kOutOfRange;
            if constexpr (ES == 1)
                raw[k] = __builtin_bit_cast(v2i, __builtin_amdgcn_raw_buffer_load_b64(rs, off, 0, 0));
            else
                raw[k] = __builtin_bit_cast(v3i, __builtin_amdgcn_raw_buffer_load_b96(rs, off, 0, 0));
        }
        *delta = dl;
    }
}

// One staged quad, realigned by delta bytes (float16 / u8) and widened to
// binary32.  alignbyte(hi, lo, d) is bytes d .. d + 3 of hi:lo.
__device__ __forceinline__ v4f widen_quad(const v4i &r, uint32_t) { return __builtin_bit_cast(v4f, r); }
__device__ __forceinline__ v4f widen_quad(const v3i &r, uint32_t delta) {
    const uint32_t lo = __builtin_amdgcn_alignbyte(static_cast<uint32_t>(r.y), static_cast<uint32_t>(r.x), delta);
    const uint32_t hi = __builtin_amdgcn_alignbyte(static_cast<uint32_t>(r.z), static_cast<uint32_t>(r.y), delta);
    return v4f{static_cast<float>(__builtin_bit_cast(_Float16, static_cast<uint16_t>(lo & 0xffffu))),
               static_cast<float>(__builtin_bit_cast(_Float16, static_cast<uint16_t>(lo >> 16))),
               static_cast<float>(__builtin_bit_cast(_Float16, static_cast<uint16_t>(hi & 0xffffu))),
               static_cast<float>(__builtin_bit_cast(_Float16, static_cast<uint16_t>(hi >> 16)))};
}
__device__ __forceinline__ v4f widen_quad(const v2i &r, uint32_t delta) {
    const uint32_t w = __builtin_amdgcn_alignbyte(static_cast<uint32_t>(r.y), static_cast<uint32_t>(r.x), delta);
    return v4f{static_cast<float>(w & 0xffu), static_cast<float>((w >> 8) & 0xffu),
               static_cast<float>((w >> 16) & 0xffu), static_cast<float>(w >> 24)};
}

// Staging of input rows into padded LDS rows for the register-window forms.
// Every wave owns RPW rows of each chunk of NW*RPW rows; fetch() loads them
// into registers a quad (four samples) per lane and load, store() widens
// them to binary32 and writes each quad with one 16-byte LDS write.  Padded
// layout: logical quad Q at physical quad Q + floor(Q/S) (no padding when
// S == 1).
template <typename TIn, int S, int NW, int RPW, int KMAX>
struct ChunkStager {
    static constexpr int KL = (KMAX + 3) / 4;  // quads per lane per row (256 samples each over the wave)
    static constexpr int CR = NW * RPW;
    typedef typename QuadRaw<TIn>::T Raw;
    const TIn *in;
    ctab *base_tile;  // staged-row starts of this tile, for rows [r_begin, r_end)
    const SrsDims &d;
    int64_t t0;
    int wave, lane;
    int32_t row_dw;
    Raw raw[RPW][KL];
    uint32_t delta[RPW];  // realignment of each fetched row (wave-uniform)

    __device__ ChunkStager(const TIn *in_, ctab *base_tile_, const SrsDims &d_, int64_t t0_, int wave_, int lane_)
        : in(in_), base_tile(base_tile_), d(d_), t0(t0_), wave(wave_), lane(lane_) {
        row_dw = S == 1 ? d.wcap : d.wcap / S * (S + 1);
    }

    // Physical dword offset of logical quad Q in a padded row.
    __device__ static __forceinline__ int32_t quad_dw(int32_t Q) { return 4 * (S == 1 ? Q : Q + Q / S); }

    __device__ __forceinline__ void fetch(int32_t c) {
#pragma unroll
        for (int q = 0; q < RPW; ++q) {
            const int32_t row = c * CR + wave * RPW + q;
            if (row < d.r_end)
                fetch_quads<TIn, KL>(in, d.in_stride, d.in_valid, row, t0 + base_tile[row - d.r_begin], d.wcap, lane,
                                     raw[q], &delta[q]);
        }
    }

    // Write the fetched rows of chunk c into the chunk buffer at buf.
    __device__ __forceinline__ void store(int32_t c, float *buf) const {
#pragma unroll
        for (int q = 0; q < RPW; ++q) {
            const int32_t rr = wave * RPW + q;
            if (c * CR + rr < d.r_end) {
                float *rowp = buf + rr * row_dw;
#pragma unroll
                for (int k = 0; k < KL; ++k) {
                    const int32_t Q = 64 * k + lane;  // logical quad
                    if (4 * Q < d.wcap)
                        *reinterpret_cast<v4f *>(rowp + quad_dw(Q)) = widen_quad(raw[q][k], delta[q]);
                }
            }
        }
    }
};

// Store a wave's accumulators: lane l holds samples t0 + IT*l .. +IT-1 of
// accumulator rows tile_a*TA + wave*TDW + a.
template <typename RW, int IT, int TDW, int TA>
__device__ __forceinline__ void store_acc(const typename RW::Acc &acc, float *__restrict__ out, const SrsDims &d,
                                          int64_t t0, int32_t tile_a, int wave, int lane) {
#pragma unroll
    for (int a = 0; a < TDW; ++a) {
        const int32_t ag = tile_a * TA + wave * TDW + a;
        if (ag >= d.n_acc)
            break;
        const int64_t tl = t0 - skew_of(d, ag) + static_cast<int64_t>(lane) * IT;
        float *dst = out + static_cast<int64_t>(ag) * d.out_stride + tl;
        const bool vec = (reinterpret_cast<uintptr_t>(dst) & 15) == 0;
        if (tl >= 0 && tl + IT <= d.n_t && vec) {
#pragma unroll
            for (int j = 0; j < IT; j += 4) {
                v4f v;
                v.x = RW::get_acc(acc, a * IT + j + 0);
                v.y = RW::get_acc(acc, a * IT + j + 1);
                v.z = RW::get_acc(acc, a * IT + j + 2);
                v.w = RW::get_acc(acc, a * IT + j + 3);
                __builtin_nontemporal_store(v, reinterpret_cast<v4f *>(dst + j));
            }
        } else {
#pragma unroll
            for (int j = 0; j < IT; ++j)
                if (tl + j >= 0 && tl + j < d.n_t)
                    dst[j] = RW::get_acc(acc, a * IT + j);
        }
    }
}

// Register-window tile.  Per (accumulator tile, wave, input row) a record of
// RD = 1 + TDW/4 dwords: the lane window's LDS byte offset in the staged row
// (bits 0..19) and its quad count (bits 20..), then the TDW window offsets as
// bytes.  Records are laid out [tile][wave][row][RD] with rows padded to whole
// chunks, so one wave's records for a group of rows are contiguous and come in
// with a few scalar loads.  The next group's records are requested right after
// the LDS wait of the current group's first row, so they arrive while that
// row's additions run.
template <typename TIn, int IT, int TDW, int NWR, int NW, int RPW, int KMAX>
__device__ __forceinline__ void srs_tile_regwin(const TIn *__restrict__ in, float *__restrict__ out,
                                                ctab *__restrict__ base, ctab *__restrict__ recs, ctab *span,
                                                const SrsDims &d, int32_t tile_t, int32_t tile_a, float *lds) {
    using RW = RegWin<IT, TDW, NWR>;
    constexpr int TT = 64 * IT;
    constexpr int TA = TDW * NW;
    constexpr int CR = NW * RPW;     // input rows per chunk
    constexpr int RD = 1 + TDW / 4;  // record dwords per (row, wave)
    constexpr int S = RW::S;
    static_assert(TDW % 4 == 0, "offsets are packed four to a dword");
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int64_t t0 = static_cast<int64_t>(tile_t) * TT;
    // The tables hold this launch's block of rows, [r_begin, r_end) (r_begin a
    // multiple of CR): records for chunks c_first .. c_first + n_chunks - 1.
    const int32_t c_first = d.r_begin / CR;
    const int32_t n_chunks = (d.r_end - d.r_begin + CR - 1) / CR;
    ctab *rec_tile = recs + (static_cast<int64_t>(tile_a) * NW + wave) * n_chunks * (CR * RD);
    // Chunks [c_lo, c_hi) hold the launch's block of rows; with a span, only
    // those with an operand inside the input for this tile (the rest would add
    // only zeros; span: null = all rows).
    int32_t c_lo = c_first, c_hi = c_first + n_chunks;
    if (span) {
        const int64_t k = 2 * (static_cast<int64_t>(tile_a) * d.n_t_tiles + tile_t);
        c_lo = max(c_lo, __builtin_amdgcn_readfirstlane(span[k]) / CR);
        c_hi = min(c_hi, (__builtin_amdgcn_readfirstlane(span[k + 1]) + CR - 1) / CR);
    }

    typename RW::Acc acc;
#pragma unroll
    for (int i = 0; i < IT * TDW; ++i)
        RW::set_acc(acc, i, 0.f);
    if (d.carry) {  // continue the partial sums of the previous blocks
#pragma unroll
        for (int a = 0; a < TDW; ++a) {
            const int32_t ag = tile_a * TA + wave * TDW + a;
            if (ag < d.n_acc) {
                const int64_t tl = t0 - skew_of(d, ag) + static_cast<int64_t>(lane) * IT;
                const float *src = out + static_cast<int64_t>(ag) * d.out_stride + tl;
#pragma unroll
                for (int j = 0; j < IT; ++j)
                    if (tl + j >= 0 && tl + j < d.n_t)
                        RW::set_acc(acc, a * IT + j, src[j]);
            }
        }
    }

    ChunkStager<TIn, S, NW, RPW, KMAX> st(in, base + static_cast<int64_t>(tile_a) * (d.r_end - d.r_begin), d, t0,
                                          wave, lane);
    const int32_t buf_dw = CR * st.row_dw;  // two chunk buffers
    const uint32_t lane_rd = lds_address(lds) + static_cast<uint32_t>(lane) * 16u * (S == 1 ? 1u : S + 1u);

    // Records travel in groups of G = CR/2 rows, two per chunk, held in two
    // register sets used alternately (set 0: rows 0..G-1, set 1: rows
    // G..CR-1), so no copies are needed.  While one set is in use the other
    // is refilled with the next group, requested right after the LDS wait of
    // the current group's first row.
    constexpr int G = CR / 2;
    static_assert(CR % 2 == 0, "two record groups per chunk");
    const int32_t n_groups = c_hi * 2;
    uint32_t rs0[G * RD], rs1[G * RD];
    auto load_recs = [&](uint32_t (&r)[G * RD], int32_t g, int dep) {
        ctab *p = rec_tile + static_cast<int64_t>(g - 2 * c_first) * (G * RD) + dep;
#pragma unroll
        for (int i = 0; i < G * RD; ++i)
            r[i] = static_cast<uint32_t>(p[i]);
    };

    if (c_lo < c_hi) {  // uniform over the work-group
    st.fetch(c_lo);
    st.store(c_lo, lds + (c_lo & 1) * buf_dw);
    if (c_lo + 1 < c_hi)
        st.fetch(c_lo + 1);
    load_recs(rs0, 2 * c_lo, 0);
    __syncthreads();  // first chunk staged
    for (int32_t c = c_lo; c < c_hi; ++c) {
        const int32_t r0 = c * CR;
        const int32_t nr = min(CR, d.r_end - r0);
        const uint32_t chunk_rd = lane_rd + static_cast<uint32_t>((c & 1) * buf_dw) * 4u;
#pragma unroll
        for (int rr = 0; rr < CR; ++rr) {
            if (rr >= nr)
                break;
            const int gi = rr % G;
            const bool second = rr >= G;  // which record set holds this row
            uint32_t(&cur)[G * RD] = second ? rs1 : rs0;
            uint32_t(&oth)[G * RD] = second ? rs0 : rs1;
            const uint32_t rec = __builtin_amdgcn_readfirstlane(cur[gi * RD]);
            const uint32_t addr = chunk_rd + static_cast<uint32_t>(rr * st.row_dw) * 4u + (rec & 0xfffffu);
            typename RW::Win w;
            int dep;
            uint32_t pk[TDW / 4];
#pragma unroll
            for (int k = 0; k < TDW / 4; ++k)
                pk[k] = __builtin_amdgcn_readfirstlane(cur[gi * RD + 1 + k]);
            int o[TDW];
            RW::load(w, addr, static_cast<int>(rec >> 20), pk, o, dep);
            const int32_t g = 2 * c + (second ? 1 : 0);
            if (gi == 0 && g + 1 < n_groups)
                load_recs(oth, g + 1, __builtin_amdgcn_readfirstlane(dep));
            RW::add(acc, w, o);
        }
        if (c + 1 < c_hi) {
            // The other buffer was last read in chunk c-1, which every wave
            // finished before the previous barrier.
            st.store(c + 1, lds + ((c + 1) & 1) * buf_dw);
            if (c + 2 < c_hi)
                st.fetch(c + 2);
            __syncthreads();  // chunk c+1 staged; chunk c consumed by every wave
        }
    }
    }
    store_acc<RW, IT, TDW, TA>(acc, out, d, t0, tile_a, wave, lane);
}

// LDS form with prefetch: the staging of srs_tile_regwin (bounds-checked
// buffer loads two chunks ahead into registers, two LDS chunk buffers, one
// barrier per chunk; unpadded rows of wcap samples) and the addition of
// srs_tile_lds (lane l owns samples t0 + l + 64j; every addition reads its
// operand from LDS at a wave-uniform offset, 64 consecutive words per read).
template <typename TIn, int IT, int TDW, int NW, int RPW, int KMAX>
__device__ __forceinline__ void srs_tile_ldsp(const TIn *__restrict__ in, float *__restrict__ out,
                                              ctab *__restrict__ rel, ctab *__restrict__ base, ctab *span,
                                              const SrsDims &d, int32_t tile_t, int32_t tile_a, float *lds) {
    constexpr int TT = 64 * IT;
    constexpr int TA = TDW * NW;
    constexpr int CR = NW * RPW;
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int64_t t0 = static_cast<int64_t>(tile_t) * TT;
    // The tables hold this launch's block of rows, [r_begin, r_end).
    const int32_t nb = d.r_end - d.r_begin;
    ctab *base_tile = base + static_cast<int64_t>(tile_a) * nb;
    ctab *rel_tile = rel + static_cast<int64_t>(tile_a) * nb * TA + wave * TDW;
    const int32_t nk = d.wcap >> 6;
    const int32_t buf_dw = CR * d.wcap;

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

    float pre[RPW][KMAX];
    // This launch's block of rows: chunks [c_first, n_chunks).
    const int32_t c_first = d.r_begin / CR;
    const int32_t n_chunks = (d.r_end + CR - 1) / CR;
    auto fetch_chunk = [&](int32_t c) {
#pragma unroll
        for (int q = 0; q < RPW; ++q) {
            const int32_t row = c * CR + wave * RPW + q;
            if (row < d.r_end)
                fetch_row<TIn, KMAX>(in, d.in_stride, d.in_valid, row, t0 + base_tile[row - d.r_begin], nk, lane,
                                     pre[q]);
        }
    };
    auto store_chunk = [&](int32_t c) {
#pragma unroll
        for (int q = 0; q < RPW; ++q) {
            const int32_t rr = wave * RPW + q;
            if (c * CR + rr < d.r_end) {
                float *dst = lds + (c & 1) * buf_dw + rr * d.wcap + lane;
#pragma unroll
                for (int k = 0; k < KMAX; ++k)
                    if (k < nk)
                        dst[64 * k] = pre[q][k];
            }
        }
    };

    // This wave's offsets for a chunk (CR rows x TDW accumulator rows) come in
    // with wave-uniform vector loads (every lane the same address), held in
    // VGPRs (scalar registers would run out), two chunks ahead like the
    // staging data, so no row waits for them.
    const __amdgpu_buffer_rsrc_t rel_rs = __builtin_amdgcn_make_buffer_rsrc(
        const_cast<int32_t *>(reinterpret_cast<const int32_t *>(reinterpret_cast<uintptr_t>(rel_tile))), 0,
        0x7fffffff, kBufferFlags);
    // Small chunks only (CR*TDW <= 16): larger ones read each row's offsets
    // with scalar loads as they go.
    constexpr bool PREF = CR * TDW <= 16;
    constexpr int OR = PREF ? CR : 1, OK = PREF ? TDW : 1;
    int32_t ocur[OR][OK], onxt[OR][OK], onxt2[OR][OK];
    auto load_offsets = [&](int32_t (&o)[OR][OK], int32_t c) {
        if constexpr (PREF) {
#pragma unroll
        for (int rr = 0; rr < CR; ++rr) {
            const int32_t r = min(c * CR + rr, d.r_end - 1) - d.r_begin;
            const uint32_t off = static_cast<uint32_t>(r * TA) * 4u;  // within this tile's table
            if constexpr (TDW % 4 == 0) {
#pragma unroll
                for (int k = 0; k < TDW; k += 4) {
                    const v4i v = __builtin_bit_cast(v4i, __builtin_amdgcn_raw_buffer_load_b128(rel_rs, off + 4u * k, 0, 0));
                    o[rr][k] = v.x;
                    o[rr][k + 1] = v.y;
                    o[rr][k + 2] = v.z;
                    o[rr][k + 3] = v.w;
                }
            } else {
#pragma unroll
                for (int k = 0; k < TDW; ++k)
                    o[rr][k] = static_cast<int32_t>(__builtin_amdgcn_raw_buffer_load_b32(rel_rs, off + 4u * k, 0, 0));
            }
        }
        }
    };

    // Chunks [c_lo, c_hi): with a span, only those holding rows with an
    // operand inside the input for this tile (the rest would add only zeros;
    // span: null = all rows).
    int32_t c_lo = c_first, c_hi = n_chunks;
    if (span) {
        const int64_t k = 2 * (static_cast<int64_t>(tile_a) * d.n_t_tiles + tile_t);
        c_lo = max(c_lo, __builtin_amdgcn_readfirstlane(span[k]) / CR);
        c_hi = min(c_hi, (__builtin_amdgcn_readfirstlane(span[k + 1]) + CR - 1) / CR);
    }

    if (c_lo < c_hi) {  // uniform over the work-group
    fetch_chunk(c_lo);
    store_chunk(c_lo);
    if (c_lo + 1 < c_hi)
        fetch_chunk(c_lo + 1);
    if constexpr (PREF) {
        load_offsets(onxt, c_lo);
        if (c_lo + 1 < c_hi)
            load_offsets(onxt2, c_lo + 1);
    }
    __syncthreads();
    for (int32_t c = c_lo; c < c_hi; ++c) {
        const int32_t r0 = c * CR;
        const int32_t nr = min(CR, d.r_end - r0);
        const float *buf = lds + (c & 1) * buf_dw + lane;
#pragma unroll
        for (int rr = 0; rr < OR; ++rr)
#pragma unroll
            for (int k = 0; k < OK; ++k) {
                ocur[rr][k] = onxt[rr][k];
                onxt[rr][k] = onxt2[rr][k];
            }
#pragma unroll
        for (int rr = 0; rr < CR; ++rr) {
            if (rr >= nr)
                break;
            const float *row = buf + rr * d.wcap;
#pragma unroll
            for (int k = 0; k < TDW; ++k) {
                int32_t ok;
                if constexpr (PREF)
                    ok = ocur[rr % OR][k % OK];
                else
                    ok = __builtin_amdgcn_readfirstlane(rel_tile[static_cast<int64_t>(r0 - d.r_begin + rr) * TA + k]);
                const float *p = row + ok;
#pragma unroll
                for (int j = 0; j < IT; ++j)
                    acc[k][j] += p[64 * j];
            }
        }
        if (c + 1 < c_hi) {
            store_chunk(c + 1);
            if (c + 2 < c_hi) {
                // Chunk c+2's offsets go out just ahead of its staging loads;
                // they are used after that staging data has been stored, so
                // waiting for them never waits on newer loads.
                if constexpr (PREF) {
                    load_offsets(onxt2, c + 2);
                    __builtin_amdgcn_sched_barrier(0);
                }
                fetch_chunk(c + 2);
            }
            __syncthreads();
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

// Direct form, for shifted-row sums with no reuse between accumulator rows
// (e.g. the adjoint of a low-frequency setup, where neighbouring channels'
// delays differ by thousands of samples): each wave owns one accumulator row
// and reads every operand straight from memory with bounds-checked buffer
// loads (lane l: samples t0 + l + 64j, coalesced), U input rows in flight.
//
// Rows [r_begin, r_end) are summed.  With CARRY the sums continue the
// partial sums already in `out` (a previous launch's rows), so the rows can
// be split over successive launches with the same result, and the time tiles
// of each accumulator tile are rotated by the offset of the block's middle
// row: at that row every accumulator tile of a contiguous run of logical
// tiles (one XCD's share) reads the same input samples, rather than samples
// up to the largest delay apart, so their reads share the XCD's L2.  A
// rotation of the time tiles: every tile is still computed exactly once.
template <typename TIn, int IT, int NW, int U, bool CARRY>
__device__ __forceinline__ void srs_tile_direct(const TIn *__restrict__ in, float *__restrict__ out,
                                                ctab *__restrict__ rel, ctab *__restrict__ base, ctab *span,
                                                const SrsDims &d, int32_t tile_t, int32_t tile_a, int32_t r_begin,
                                                int32_t r_end) {
    constexpr int TT = 64 * IT;
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    ctab *base_tile = base + static_cast<int64_t>(tile_a) * d.n_rows;
    ctab *rel_tile = rel + static_cast<int64_t>(tile_a) * d.n_rows * NW + wave;
    if constexpr (CARRY) {
        const int32_t mid = __builtin_amdgcn_readfirstlane(base_tile[r_begin + (r_end - r_begin) / 2]);
        const int32_t shift = (mid >= 0 ? mid / TT : -((-mid + TT - 1) / TT)) % d.n_t_tiles;  // (-n, n)
        tile_t -= shift;
        if (tile_t < 0)
            tile_t += d.n_t_tiles;
        else if (tile_t >= d.n_t_tiles)
            tile_t -= d.n_t_tiles;
    }
    const int64_t t0 = static_cast<int64_t>(tile_t) * TT;
    const int32_t n_bytes = static_cast<int32_t>(d.in_valid * static_cast<int64_t>(sizeof(TIn)));
    const int32_t ag = tile_a * NW + wave;
    float *dst = out + static_cast<int64_t>(min(ag, d.n_acc - 1)) * d.out_stride;
    float acc[IT];
#pragma unroll
    for (int j = 0; j < IT; ++j) {
        const int64_t t = t0 + lane + 64 * j;
        acc[j] = (CARRY && r_begin > 0 && ag < d.n_acc && t < d.n_t) ? dst[t] : 0.f;
    }
    // Rows outside [span lo, span hi) add only zeros to this tile.
    int32_t r_from = r_begin, r_to = r_end;
    if (span) {
        const int64_t k = 2 * (static_cast<int64_t>(tile_a) * d.n_t_tiles + tile_t);
        r_from = max(r_from, __builtin_amdgcn_readfirstlane(span[k]));
        r_to = min(r_to, __builtin_amdgcn_readfirstlane(span[k + 1]));
    }
    for (int32_t r0 = r_from; r0 < r_to; r0 += U) {
        float v[U][IT];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int32_t r = min(r0 + u, r_to - 1);
            const int64_t g0 = t0 + __builtin_amdgcn_readfirstlane(base_tile[r]) +
                               __builtin_amdgcn_readfirstlane(rel_tile[static_cast<int64_t>(r) * NW]);
            const TIn *rp = in + static_cast<int64_t>(r) * d.in_stride;
            const __amdgpu_buffer_rsrc_t rs =
                __builtin_amdgcn_make_buffer_rsrc(const_cast<TIn *>(rp), 0, n_bytes, kBufferFlags);
#pragma unroll
            for (int j = 0; j < IT; ++j) {
                const int64_t g = g0 + lane + 64 * j;
                const uint32_t off = g >= 0 ? static_cast<uint32_t>(g) * sizeof(TIn) : kOutOfRange;
                v[u][j] = (r0 + u < r_to) ? buffer_ld<TIn>(rs, off) : 0.f;
            }
        }
#pragma unroll
        for (int u = 0; u < U; ++u)
#pragma unroll
            for (int j = 0; j < IT; ++j)
                acc[j] += v[u][j];
    }
    if (ag < d.n_acc) {
        const bool last = !CARRY || r_end >= d.n_rows;  // the next launch re-reads partial sums
#pragma unroll
        for (int j = 0; j < IT; ++j) {
            const int64_t t = t0 + lane + 64 * j;
            if (t < d.n_t) {
                if (last)
                    __builtin_nontemporal_store(acc[j], dst + t);
                else
                    dst[t] = acc[j];
            }
        }
    }
}

// Direct form with consecutive ownership, float32 input: lane l owns samples
// t0 + 4l + 256q + i (q < IT/4, i < 4) and reads each row's operands with
// 16-byte buffer loads (one per q), a quarter of the load instructions of
// srs_tile_direct.  Rows whose window starts before sample 0 fall back to
// per-sample loads.  Same rows, same order, same partial-sum carry and tile
// rotation as srs_tile_direct, so the sums are bit-identical to it.
template <int IT, int NW, int U, bool CARRY>
__device__ __forceinline__ void srs_tile_direct_vec(const float *__restrict__ in, float *__restrict__ out,
                                                    ctab *__restrict__ rel, ctab *__restrict__ base, ctab *span,
                                                    const SrsDims &d, int32_t tile_t, int32_t tile_a,
                                                    int32_t r_begin, int32_t r_end) {
    static_assert(IT % 4 == 0, "16-byte pieces");
    constexpr int TT = 64 * IT;
    constexpr int Q = IT / 4;
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    ctab *base_tile = base + static_cast<int64_t>(tile_a) * d.n_rows;
    ctab *rel_tile = rel + static_cast<int64_t>(tile_a) * d.n_rows * NW + wave;
    if constexpr (CARRY) {
        const int32_t mid = __builtin_amdgcn_readfirstlane(base_tile[r_begin + (r_end - r_begin) / 2]);
        const int32_t shift = (mid >= 0 ? mid / TT : -((-mid + TT - 1) / TT)) % d.n_t_tiles;  // (-n, n)
        tile_t -= shift;
        if (tile_t < 0)
            tile_t += d.n_t_tiles;
        else if (tile_t >= d.n_t_tiles)
            tile_t -= d.n_t_tiles;
    }
    const int64_t t0 = static_cast<int64_t>(tile_t) * TT;
    const int32_t n_bytes = static_cast<int32_t>(d.in_valid * 4);
    const int32_t ag = tile_a * NW + wave;
    float *dst = out + static_cast<int64_t>(min(ag, d.n_acc - 1)) * d.out_stride;
    // Output row as a buffer clipped to [0, n_t): out-of-range dwords read 0.
    const __amdgpu_buffer_rsrc_t out_rs =
        __builtin_amdgcn_make_buffer_rsrc(dst, 0, static_cast<int32_t>(d.n_t * 4), kBufferFlags);
    const uint32_t lane_off = static_cast<uint32_t>(t0 + 4 * lane) * 4u;  // < 2^31: t0 < n_t < 2^29
    v4f acc[Q];
#pragma unroll
    for (int q = 0; q < Q; ++q) {
        if (CARRY && r_begin > 0 && ag < d.n_acc)
            acc[q] = __builtin_bit_cast(v4f, __builtin_amdgcn_raw_buffer_load_b128(out_rs, lane_off + q * 1024u, 0, 0));
        else
            acc[q] = v4f{0.f, 0.f, 0.f, 0.f};
    }
    int32_t r_from = r_begin, r_to = r_end;
    if (span) {
        const int64_t k = 2 * (static_cast<int64_t>(tile_a) * d.n_t_tiles + tile_t);
        r_from = max(r_from, __builtin_amdgcn_readfirstlane(span[k]));
        r_to = min(r_to, __builtin_amdgcn_readfirstlane(span[k + 1]));
    }
    for (int32_t r0 = r_from; r0 < r_to; r0 += U) {
        v4f v[U][Q];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int32_t r = min(r0 + u, r_to - 1);
            const int64_t g0 = t0 + __builtin_amdgcn_readfirstlane(base_tile[r]) +
                               __builtin_amdgcn_readfirstlane(rel_tile[static_cast<int64_t>(r) * NW]);
            const float *rp = in + static_cast<int64_t>(r) * d.in_stride;
            const __amdgpu_buffer_rsrc_t rs =
                __builtin_amdgcn_make_buffer_rsrc(const_cast<float *>(rp), 0, n_bytes, kBufferFlags);
            if (r0 + u >= r_to) {
#pragma unroll
                for (int q = 0; q < Q; ++q)
                    v[u][q] = v4f{0.f, 0.f, 0.f, 0.f};
            } else if (g0 >= 0) {  // wave-uniform
                const uint32_t voff = static_cast<uint32_t>(g0 + 4 * lane) * 4u;
#pragma unroll
                for (int q = 0; q < Q; ++q)
                    v[u][q] = __builtin_bit_cast(v4f, __builtin_amdgcn_raw_buffer_load_b128(rs, voff + q * 1024u, 0, 0));
            } else {
#pragma unroll
                for (int q = 0; q < Q; ++q)
#pragma unroll
                    for (int i = 0; i < 4; ++i) {
                        const int64_t g = g0 + 4 * lane + 256 * q + i;
                        v[u][q][i] = buffer_ld<float>(rs, g >= 0 ? static_cast<uint32_t>(g) * 4u : kOutOfRange);
                    }
            }
        }
#pragma unroll
        for (int u = 0; u < U; ++u)
#pragma unroll
            for (int q = 0; q < Q; ++q)
                acc[q] += v[u][q];
    }
    if (ag < d.n_acc) {
#pragma unroll
        for (int q = 0; q < Q; ++q) {
            const int64_t t = t0 + 4 * lane + 256 * q;
            if (t + 3 < d.n_t) {
                __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(v4i, acc[q]), out_rs, lane_off + q * 1024u, 0,
                                                       0);
            } else {
#pragma unroll
                for (int i = 0; i < 4; ++i)
                    if (t + i < d.n_t)
                        dst[t + i] = acc[q][i];
            }
        }
    }
}

}  // namespace dev
}  // namespace dd
