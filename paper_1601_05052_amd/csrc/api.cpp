// C ABI entry points for single-beam forward / adjoint dedispersion and tile
// selection.  Every check runs before any GPU work is enqueued.
#include <cstdint>
#include <cstring>
#include <vector>

#include "internal.h"

using namespace dd;

namespace {

size_t elem_size(int32_t t) { return t == DD_F32 ? 4 : t == DD_F16 ? 2 : 1; }

bool overlaps(const void *a, size_t na, const void *b, size_t nb) {
    const uintptr_t a0 = reinterpret_cast<uintptr_t>(a), b0 = reinterpret_cast<uintptr_t>(b);
    return a0 < b0 + nb && b0 < a0 + na;
}

int resolve_blocks(const dd_plan *p, int direction, int32_t in_type, std::vector<Block> *out) {
    *out = launch_list(p, direction, in_type);
    if (out->empty())
        return fail(DD_EUNSUPPORTED, "no tile variant can serve this plan");
    return DD_OK;
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
int run_blocks(const dd_plan *p, int direction, int32_t in_type, const std::vector<Block> &blocks, const void *in,
               int64_t in_stride, float *out, int64_t out_stride, hipStream_t stream) {
    const int32_t kt = direction == DD_FORWARD ? in_type : (int32_t)DD_F32;
    for (const Block &b : blocks) {
        const Variant *v = find_variant(b.variant);
        if (!v || !has_kernel(*v, kt))
            return fail(DD_EUNSUPPORTED, "this library has no kernel of tile variant %d for this input type",
                        b.variant);
        SrsArgs a;
        int rc = make_args(p, direction, *v, in, in_stride, out, out_stride, &a, b.r0, b.r1);
        if (rc != DD_OK)
            return rc;
        hipError_t e = launch_srs(*v, kt, a, stream);
        if (e != hipSuccess)
            return fail(DD_EHIP, "kernel launch failed: %s", hipGetErrorString(e));
    }
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
    std::vector<Block> blocks;
    rc = resolve_blocks(p, DD_FORWARD, in_type, &blocks);
    if (rc != DD_OK)
        return rc;
    return run_blocks(p, DD_FORWARD, in_type, blocks, d_in, in_stride, d_out, out_stride,
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
    std::vector<Block> blocks;
    int rc = resolve_blocks(p, DD_ADJOINT, DD_F32, &blocks);
    if (rc != DD_OK)
        return rc;
    // The adjoint reads rows of grad_out (stride out_stride) and writes rows
    // of grad_in (stride in_stride).
    return run_blocks(p, DD_ADJOINT, DD_F32, blocks, d_grad_out, out_stride, d_grad_in, in_stride,
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
    std::vector<Block> blocks;
    int rc = resolve_blocks(p, direction, direction == DD_FORWARD ? in_type : DD_F32, &blocks);
    if (rc != DD_OK)
        return rc;
    for (const Block &b : blocks) {
        const TileTables *t = nullptr;
        rc = plan_tables(p, direction, *find_variant(b.variant), &t, b.r0, b.r1);
        if (rc != DD_OK)
            return rc;
    }
    return DD_OK;
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
    if (direction == DD_ADJOINT && in_type != DD_F32)
        return fail(DD_EINVAL, "the adjoint works on float32 only");
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
    p->blocks[direction][in_type].clear();
    return DD_OK;
}

int dd_plan_set_blocks(dd_plan *p, dd_direction direction, dd_dtype in_type, int32_t n_blocks,
                       const int32_t *row_starts, const int32_t *variants) {
    clear_error();
    if (!p)
        return fail(DD_EINVAL, "plan is NULL");
    if (direction != DD_FORWARD && direction != DD_ADJOINT)
        return fail(DD_EINVAL, "unknown direction %d", (int)direction);
    if (in_type != DD_F32 && in_type != DD_F16 && in_type != DD_U8)
        return fail(DD_EINVAL, "unknown input dtype %d", (int)in_type);
    if (direction == DD_ADJOINT && in_type != DD_F32)
        return fail(DD_EINVAL, "the adjoint works on float32 only");
    if (n_blocks < 1 || n_blocks > DD_MAX_BLOCKS || !row_starts || !variants)
        return fail(DD_EINVAL, "need 1 <= n_blocks <= %d and both arrays", DD_MAX_BLOCKS);
    const int32_t R = plan_rows(p, direction);
    if (row_starts[0] != 0)
        return fail(DD_EINVAL, "the first block must start at row 0");
    std::vector<Block> blocks;
    for (int32_t b = 0; b < n_blocks; ++b) {
        const int32_t r0 = row_starts[b], r1 = b + 1 < n_blocks ? row_starts[b + 1] : R;
        if (r1 <= r0 || r1 > R)
            return fail(DD_EINVAL, "row starts must increase and stay below %d", R);
        const Variant *v = find_variant(variants[b]);
        if (!v)
            return fail(DD_EINVAL, "unknown tile variant %d", variants[b]);
        if (n_blocks > 1 && !block_capable(*v))
            return fail(DD_EUNSUPPORTED, "tile variant %d cannot run a block of rows (direct kind)", v->id);
        if (!has_kernel(*v, direction == DD_FORWARD ? (int32_t)in_type : (int32_t)DD_F32))
            return fail(DD_EUNSUPPORTED, "this library has no kernel of tile variant %d for this input type", v->id);
        if (!variant_fits(p, direction, *v, r0, r1))
            return fail(DD_EUNSUPPORTED, "tile variant %d cannot serve rows [%d, %d) of this plan", v->id, r0, r1);
        blocks.push_back(Block{r0, r1, v->id});
    }
    std::lock_guard<std::mutex> lock(p->mu);
    p->forced[direction][in_type] = -1;
    p->blocks[direction][in_type] = blocks;
    return DD_OK;
}

int dd_plan_get_blocks(const dd_plan *p, dd_direction direction, dd_dtype in_type, int32_t *n_blocks,
                       int32_t *row_starts, int32_t *variants) {
    clear_error();
    if (!p || !n_blocks)
        return fail(DD_EINVAL, "NULL argument");
    if (direction != DD_FORWARD && direction != DD_ADJOINT)
        return fail(DD_EINVAL, "unknown direction %d", (int)direction);
    if (in_type != DD_F32 && in_type != DD_F16 && in_type != DD_U8)
        return fail(DD_EINVAL, "unknown input dtype %d", (int)in_type);
    std::vector<Block> blocks;
    int rc = resolve_blocks(p, direction, direction == DD_FORWARD ? in_type : DD_F32, &blocks);
    if (rc != DD_OK)
        return rc;
    *n_blocks = static_cast<int32_t>(blocks.size());
    for (size_t b = 0; b < blocks.size(); ++b) {
        if (row_starts)
            row_starts[b] = blocks[b].r0;
        if (variants)
            variants[b] = blocks[b].variant;
    }
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
    std::vector<Block> blocks;  // with a row split: the variant of its largest block
    int rc = resolve_blocks(p, direction, direction == DD_FORWARD ? in_type : DD_F32, &blocks);
    if (rc != DD_OK)
        return rc;
    const Block *big = &blocks[0];
    for (const Block &b : blocks)
        if (b.r1 - b.r0 > big->r1 - big->r0)
            big = &b;
    *variant = big->variant;
    return DD_OK;
}

}  // extern "C"
