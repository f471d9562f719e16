// The table of compiled tile variants and the dispatch of single-beam
// launches to the per-input-type instantiation units.
#include <hip/hip_runtime.h>

#include <vector>

#include "internal.h"
#include "srs_dims.h"
#ifdef DD_STUDY
#include "study_variants.def"
#else
#include "srs_variants.def"
#endif

namespace dd {

#ifdef DD_STUDY
// Study library: float32 single-beam kernels only, compiled in slices.
static_assert(DD_STUDY_N_SLICES == 8, "eight study slices");
extern const StudyEntry *study_slice_0, *study_slice_1, *study_slice_2, *study_slice_3, *study_slice_4,
    *study_slice_5, *study_slice_6, *study_slice_7;
extern const int32_t study_slice_n_0, study_slice_n_1, study_slice_n_2, study_slice_n_3, study_slice_n_4,
    study_slice_n_5, study_slice_n_6, study_slice_n_7;
static const LaunchFn *study_launchers() {
    static const std::vector<LaunchFn> table = [] {
        const StudyEntry *s[] = {study_slice_0, study_slice_1, study_slice_2, study_slice_3,
                                 study_slice_4, study_slice_5, study_slice_6, study_slice_7};
        const int32_t n[] = {study_slice_n_0, study_slice_n_1, study_slice_n_2, study_slice_n_3,
                             study_slice_n_4, study_slice_n_5, study_slice_n_6, study_slice_n_7};
        std::vector<LaunchFn> t;
        for (int k = 0; k < 8; ++k)
            for (int32_t i = 0; i < n[k]; ++i) {
                if (static_cast<size_t>(s[k][i].id) >= t.size())
                    t.resize(s[k][i].id + 1, nullptr);
                t[s[k][i].id] = s[k][i].fn;
            }
        return t;
    }();
    return table.data();
}
static const LaunchFn *launchers_of(int32_t in_type) { return in_type == DD_F32 ? study_launchers() : nullptr; }
static const void *const *multis_of(int32_t) { return nullptr; }
#else
extern const LaunchFn *launchers_f32, *launchers_f16, *launchers_u8;
extern const void *const *multis_f32, *const *multis_f16, *const *multis_u8;
static const LaunchFn *launchers_of(int32_t in_type) {
    return in_type == DD_F32 ? launchers_f32 : in_type == DD_F16 ? launchers_f16 : launchers_u8;
}
static const void *const *multis_of(int32_t in_type) {
    return in_type == DD_F32 ? multis_f32 : in_type == DD_F16 ? multis_f16 : multis_u8;
}
#endif

namespace {

#define X_LDS(ID, IT, TDW, NW, RATE) {ID, IT, TDW, NW, KIND_LDS, 0, 0, 0, RATE},
#define X_LDSP(ID, IT, TDW, NW, RPW, KMAX, RATE) {ID, IT, TDW, NW, KIND_LDS, RPW, 0, KMAX, RATE},
#define X_DIRECT(ID, IT, NW, U, RB, V, RATE) {ID, IT, 1, NW, KIND_DIRECT, U, 0, 0, RATE},
#define X_RW(ID, IT, TDW, NWR, NW, RPW, KMAX, RATE) {ID, IT, TDW, NW, KIND_REGWIN, RPW, NWR, KMAX, RATE},
#define X_RWO(ID, IT, TDW, NWR, NW, RPW, KMAX, OCC, RATE) {ID, IT, TDW, NW, KIND_REGWIN, RPW, NWR, KMAX, RATE},
const Variant kVariants[] = {DD_VARIANT_LIST};
constexpr int32_t kNumVariants = sizeof(kVariants) / sizeof(kVariants[0]);

bool ids_match_positions() {
    for (int32_t i = 0; i < kNumVariants; ++i)
        if (kVariants[i].id != i)
            return false;
    return true;
}

}  // namespace

const Variant *variants(int32_t *count) {
    static const bool ok = ids_match_positions();
    *count = ok ? kNumVariants : 0;
    return kVariants;
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

const void *multi_kernel(const Variant &v, int32_t in_type) {
    const void *const *t = multis_of(in_type);
    return t ? t[v.id] : nullptr;
}

bool has_kernel(const Variant &v, int32_t in_type) {
    const LaunchFn *t = launchers_of(in_type);
    return t && t[v.id];
}

hipError_t launch_srs(const Variant &v, int32_t in_type, const SrsArgs &a, hipStream_t stream) {
    dev::SrsDims d;
    d.in_stride = a.in_stride;
    d.in_valid = a.in_valid;
    d.out_stride = a.out_stride;
    d.n_t = a.n_t;
    d.n_acc = a.n_acc;
    d.n_rows = a.n_rows;
    d.wcap = a.wcap;
    d.rows_per_chunk = a.rows_per_chunk;
    d.r_begin = a.r_begin;
    d.r_end = a.r_end;
    d.carry = a.carry;
    d.skew = a.skew;
    d.n_t_tiles = a.n_t_tiles > 0 ? a.n_t_tiles : static_cast<int32_t>((a.n_t + v.tt() - 1) / v.tt());
    d.n_acc_tiles = (a.n_acc + v.ta() - 1) / v.ta();
    const uint64_t blocks = static_cast<uint64_t>(d.n_t_tiles) * d.n_acc_tiles;
    if (blocks == 0)
        return hipSuccess;
    if (blocks > 0x7fffffffull)
        return hipErrorInvalidConfiguration;
    const LaunchFn *t = launchers_of(in_type);
    if (!t || !t[v.id])
        return hipErrorInvalidDeviceFunction;  // callers check has_kernel first
    return t[v.id](a, d, static_cast<uint32_t>(blocks), static_cast<size_t>(a.lds_bytes), stream);
}

}  // namespace dd
