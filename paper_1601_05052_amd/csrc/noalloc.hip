// Allocation-free forward dedispersion for callers that cannot allocate
// device memory (code under HIP graph capture, tight serving loops, harnesses
// that forbid hipMalloc).
//
// dd_dedisperse reads its tile tables (staged-row starts, window records or
// offsets) from device memory the plan allocates on first use.  This entry
// stages the same tables, from the plan's host copy, into one fixed device
// array, `scratch`, with asynchronous copies on the caller's stream, and runs
// the same kernels on them.  It calls no hipMalloc, hipFree or other
// allocating routine.
//
// `scratch` is a file-scope device array: in host code its name is only a
// stand-in, so its device address is looked up once per device
// (hipGetSymbolAddress, with that device current) and only that address is
// used for copies and kernel arguments.  Every call on a device shares the
// array: calls that overlap on one device (several host threads, or several
// streams without ordering between them) race on it.
#include <hip/hip_runtime.h>

#include <cstdint>
#include <mutex>
#include <vector>

#include "internal.h"

namespace dd {

constexpr size_t kScratchBytes = size_t(16) << 20;  // largest table set one call can stage
constexpr size_t kAlign = 256;                      // each table starts on a 256-byte boundary

static __device__ __align__(256) int32_t scratch[kScratchBytes / sizeof(int32_t)];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_mu;
int32_t *g_scratch[kMaxDevices];  // device address of `scratch` on each device; null until looked up

// The device address of `scratch` on the current device `dev`.
int scratch_address(int dev, int32_t **out) {
    if (dev < 0 || dev >= kMaxDevices)
        return fail(DD_EINVAL, "device %d out of range", dev);
    std::lock_guard<std::mutex> lock(g_mu);
    if (!g_scratch[dev]) {
        void *ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !ptr)
            return fail(DD_EHIP, "looking up the scratch array failed: %s", hipGetErrorString(e));
        g_scratch[dev] = static_cast<int32_t *>(ptr);
    }
    *out = g_scratch[dev];
    return DD_OK;
}

size_t aligned_bytes(const std::vector<int32_t> &v) {
    return (v.size() * sizeof(int32_t) + kAlign - 1) / kAlign * kAlign;
}

// Copy one host table into scratch at byte offset *off (advanced past it);
// null device pointer for an empty table.
int stage(const std::vector<int32_t> &h, int32_t *base, size_t *off, hipStream_t stream, const int32_t **dst) {
    *dst = nullptr;
    if (h.empty())
        return DD_OK;
    int32_t *d = base + *off / sizeof(int32_t);
    const hipError_t e = hipMemcpyAsync(d, h.data(), h.size() * sizeof(int32_t), hipMemcpyHostToDevice, stream);
    if (e != hipSuccess)
        return fail(DD_EHIP, "staging the tile tables failed: %s", hipGetErrorString(e));
    *off += aligned_bytes(h);
    *dst = d;
    return DD_OK;
}

}  // namespace
}  // namespace dd

using namespace dd;

extern "C" int dd_dedisperse_noalloc(const dd_plan *p, const void *d_in, dd_dtype in_type, int64_t in_stride,
                                     float *d_out, int64_t out_stride, void *stream_v) {
    clear_error();
    int rc = check_forward_args(p, d_in, in_type, in_stride, d_out, out_stride);
    if (rc != DD_OK)
        return rc;
    const std::vector<Block> blocks = launch_list(p, DD_FORWARD, in_type);
    if (blocks.empty())
        return fail(DD_EUNSUPPORTED, "no tile variant can serve this plan");
    // Every launch's tables (one per block of rows when the plan splits them).
    std::vector<const Layout *> lays;
    size_t need = 0;
    for (const Block &b : blocks) {
        const Variant *v = find_variant(b.variant);
        if (!has_kernel(*v, in_type))
            return fail(DD_EUNSUPPORTED, "this library has no kernel of tile variant %d for this input type", v->id);
        const Layout *L = plan_host_layout(p, DD_FORWARD, v->id, b.r0, b.r1);
        if (!L)
            return fail(DD_EINVAL,
                        "the plan's forward tables for tile variant %d are not built: call dd_plan_prepare (or "
                        "dd_dedisperse) once beforehand, where allocation is allowed", v->id);
        lays.push_back(L);
        need += aligned_bytes(L->base) + aligned_bytes(L->rel) + aligned_bytes(L->recs) + aligned_bytes(L->span) +
                aligned_bytes(L->skew);
    }
    if (need > kScratchBytes)
        return fail(DD_EUNSUPPORTED, "the tile tables need %zu bytes; the allocation-free entry holds at most %zu",
                    need, kScratchBytes);
    int dev = 0;
    DD_HIP_TRY(hipGetDevice(&dev));
    int32_t *base = nullptr;
    rc = scratch_address(dev, &base);
    if (rc != DD_OK)
        return rc;
    hipStream_t stream = static_cast<hipStream_t>(stream_v);
    size_t off = 0;
    for (size_t i = 0; i < blocks.size(); ++i) {
        const Layout *L = lays[i];
        SrsArgs a;
        args_dims(p, DD_FORWARD, d_in, in_stride, d_out, out_stride, &a);
        a.r_begin = blocks[i].r0;
        a.r_end = blocks[i].r1;
        a.carry = blocks[i].r0 > 0 ? 1 : 0;
        if ((rc = stage(L->base, base, &off, stream, &a.base)) != DD_OK ||
            (rc = stage(L->rel, base, &off, stream, &a.rel)) != DD_OK ||
            (rc = stage(L->recs, base, &off, stream, &a.recs)) != DD_OK ||
            (rc = stage(L->span, base, &off, stream, &a.span)) != DD_OK ||
            (rc = stage(L->skew, base, &off, stream, &a.skew)) != DD_OK)
            return rc;
        a.n_t_tiles = L->n_t_tiles;
        a.wcap = L->wcap;
        a.rows_per_chunk = L->rows_per_chunk;
        a.lds_bytes = L->lds_bytes;
        const hipError_t e = launch_srs(*find_variant(blocks[i].variant), in_type, a, stream);
        if (e != hipSuccess)
            return fail(DD_EHIP, "kernel launch failed: %s", hipGetErrorString(e));
    }
    return DD_OK;
}
