// C ABI entry points for single-beam forward / adjoint dedispersion and tile
// selection.  Every check runs before any GPU work is enqueued.
#include <cstdint>
#include <cstring>

#include "internal.h"

using namespace dd;

namespace {

size_t elem_size(int32_t t) { return t == DD_F32 ? 4 : t == DD_F16 ? 2 : 1; }

bool overlaps(const void *a, size_t na, const void *b, size_t nb) {
    const uintptr_t a0 = reinterpret_cast<uintptr_t>(a), b0 = reinterpret_cast<uintptr_t>(b);
    return a0 < b0 + nb && b0 < a0 + na;
}

int resolve_variant(const dd_plan *p, int direction, int32_t in_type, const Variant **out) {
    const Variant *v = find_variant(resolved_variant(p, direction, in_type));
    if (!v)
        return fail(DD_EUNSUPPORTED, "no tile variant can serve this plan");
    *out = v;
    return DD_OK;
}

}  // namespace

namespace dd {

// Shared by the public calls and the tuner: checks done by the caller.
int run_direction(const dd_plan *p, int direction, int32_t in_type, const Variant &v, const void *in,
                  int64_t in_stride, float *out, int64_t out_stride, hipStream_t stream) {
    if (!has_kernel(v, direction == DD_FORWARD ? in_type : (int32_t)DD_F32))
        return fail(DD_EUNSUPPORTED, "this library has no kernel of tile variant %d for this input type", v.id);
    SrsArgs a;
    int rc = make_args(p, direction, v, in, in_stride, out, out_stride, &a);
    if (rc != DD_OK)
        return rc;
    hipError_t e = launch_srs(v, direction == DD_FORWARD ? in_type : (int32_t)DD_F32, a, stream);
    if (e != hipSuccess)
        return fail(DD_EHIP, "kernel launch failed: %s", hipGetErrorString(e));
    return DD_OK;
}

// Argument checks of the forward (shared with the allocation-free entry).
int check_forward_args(const dd_plan *p, const void *d_in, int32_t in_type, int64_t in_stride, const float *d_out,
                       int64_t out_stride) {
    if (!p)
        return fail(DD_EINVAL, "plan is NULL");
    if (!d_in || !d_out)
        return fail(DD_EINVAL, "NULL data pointer");
    if (in_type != DD_F32 && in_type != DD_F16 && in_type != DD_U8)
        return fail(DD_EINVAL, "unknown input dtype %d", (int)in_type);
    if (in_stride < p->T_in)
        return fail(DD_ESHAPE, "in_stride %lld < input samples %lld (n_samples + max delay)",
                    (long long)in_stride, (long long)p->T_in);
    if (out_stride < p->S)
        return fail(DD_ESHAPE, "out_stride %lld < n_samples %lld", (long long)out_stride, (long long)p->S);
    const size_t es = elem_size(in_type);
    if (reinterpret_cast<uintptr_t>(d_in) % es != 0 || reinterpret_cast<uintptr_t>(d_out) % 4 != 0)
        return fail(DD_ESHAPE, "data pointers must be aligned to their element size");
    const size_t in_bytes = (static_cast<size_t>(p->C - 1) * in_stride + p->T_in) * es;
    const size_t out_bytes = (static_cast<size_t>(p->D - 1) * out_stride + p->S) * 4;
    if (overlaps(d_in, in_bytes, d_out, out_bytes))
        return fail(DD_ESHAPE, "input and output buffers overlap");
    return DD_OK;
}

}  // namespace dd

extern "C" {

int dd_dedisperse(const dd_plan *p, const void *d_in, dd_dtype in_type, int64_t in_stride, float *d_out,
                  int64_t out_stride, void *stream) {
    clear_error();
    int rc = check_forward_args(p, d_in, in_type, in_stride, d_out, out_stride);
    if (rc != DD_OK)
        return rc;
    const Variant *v = nullptr;
    rc = resolve_variant(p, DD_FORWARD, in_type, &v);
    if (rc != DD_OK)
        return rc;
    return run_direction(p, DD_FORWARD, in_type, *v, d_in, in_stride, d_out, out_stride,
                         static_cast<hipStream_t>(stream));
}

int dd_dedisperse_adjoint(const dd_plan *p, const float *d_grad_out, int64_t out_stride, float *d_grad_in,
                          int64_t in_stride, void *stream) {
    clear_error();
    if (!p)
        return fail(DD_EINVAL, "plan is NULL");
    if (!d_grad_out || !d_grad_in)
        return fail(DD_EINVAL, "NULL data pointer");
    if (out_stride < p->S)
        return fail(DD_ESHAPE, "out_stride %lld < n_samples %lld", (long long)out_stride, (long long)p->S);
    if (in_stride < p->T_in)
        return fail(DD_ESHAPE, "in_stride %lld < input samples %lld", (long long)in_stride, (long long)p->T_in);
    if (reinterpret_cast<uintptr_t>(d_grad_out) % 4 != 0 || reinterpret_cast<uintptr_t>(d_grad_in) % 4 != 0)
        return fail(DD_ESHAPE, "data pointers must be 4-byte aligned");
    const size_t go_bytes = (static_cast<size_t>(p->D - 1) * out_stride + p->S) * 4;
    const size_t gi_bytes = (static_cast<size_t>(p->C - 1) * in_stride + p->T_in) * 4;
    if (overlaps(d_grad_out, go_bytes, d_grad_in, gi_bytes))
        return fail(DD_ESHAPE, "gradient buffers overlap");
    const Variant *v = nullptr;
    int rc = resolve_variant(p, DD_ADJOINT, DD_F32, &v);
    if (rc != DD_OK)
        return rc;
    // The adjoint reads rows of grad_out (stride out_stride) and writes rows
    // of grad_in (stride in_stride).
    return run_direction(p, DD_ADJOINT, DD_F32, *v, d_grad_out, out_stride, d_grad_in, in_stride,
                         static_cast<hipStream_t>(stream));
}

int dd_plan_prepare(dd_plan *p, dd_direction direction, dd_dtype in_type) {
    clear_error();
    if (!p)
        return fail(DD_EINVAL, "plan is NULL");
    if (direction != DD_FORWARD && direction != DD_ADJOINT)
        return fail(DD_EINVAL, "unknown direction %d", (int)direction);
    if (in_type != DD_F32 && in_type != DD_F16 && in_type != DD_U8)
        return fail(DD_EINVAL, "unknown input dtype %d", (int)in_type);
    const Variant *v = nullptr;
    int rc = resolve_variant(p, direction, direction == DD_FORWARD ? in_type : DD_F32, &v);
    if (rc != DD_OK)
        return rc;
    const TileTables *t = nullptr;
    return plan_tables(p, direction, *v, &t);
}

int dd_tile_count(int32_t *n_variants) {
    clear_error();
    if (!n_variants)
        return fail(DD_EINVAL, "NULL argument");
    variants(n_variants);
    return DD_OK;
}

int dd_tile_info(int32_t variant, int32_t *items_t, int32_t *items_acc, int32_t *waves, int32_t *kind) {
    clear_error();
    const Variant *v = find_variant(variant);
    if (!v)
        return fail(DD_EINVAL, "unknown tile variant %d", variant);
    if (items_t)
        *items_t = v->items_t;
    if (items_acc)
        *items_acc = v->items_acc;
    if (waves)
        *waves = v->waves;
    if (kind)
        *kind = v->kind;
    return DD_OK;
}

int dd_plan_set_tile(dd_plan *p, dd_direction direction, dd_dtype in_type, int32_t variant) {
    clear_error();
    if (!p)
        return fail(DD_EINVAL, "plan is NULL");
    if (direction != DD_FORWARD && direction != DD_ADJOINT)
        return fail(DD_EINVAL, "unknown direction %d", (int)direction);
    if (in_type != DD_F32 && in_type != DD_F16 && in_type != DD_U8)
        return fail(DD_EINVAL, "unknown input dtype %d", (int)in_type);
    if (variant != -1) {
        const Variant *v = find_variant(variant);
        if (!v)
            return fail(DD_EINVAL, "unknown tile variant %d", variant);
        if (!has_kernel(*v, direction == DD_FORWARD ? (int32_t)in_type : (int32_t)DD_F32))
            return fail(DD_EUNSUPPORTED, "this library has no kernel of tile variant %d for this input type",
                        variant);
        if (!variant_fits(p, direction, *v))
            return fail(DD_EUNSUPPORTED, "tile variant %d cannot serve this plan (LDS window too large)",
                        variant);
    }
    std::lock_guard<std::mutex> lock(p->mu);
    p->forced[direction][in_type] = variant;
    return DD_OK;
}

int dd_plan_get_tile(const dd_plan *p, dd_direction direction, dd_dtype in_type, int32_t *variant) {
    clear_error();
    if (!p || !variant)
        return fail(DD_EINVAL, "NULL argument");
    if (direction != DD_FORWARD && direction != DD_ADJOINT)
        return fail(DD_EINVAL, "unknown direction %d", (int)direction);
    if (in_type != DD_F32 && in_type != DD_F16 && in_type != DD_U8)
        return fail(DD_EINVAL, "unknown input dtype %d", (int)in_type);
    const Variant *v = nullptr;
    int rc = resolve_variant(p, direction, in_type, &v);
    if (rc != DD_OK)
        return rc;
    *variant = v->id;
    return DD_OK;
}

}  // extern "C"
