// Real-time (streaming) dedispersion of one beam.
//
// The method dedisperses one second of data at a time: the input of one step
// holds the s samples of that second plus the samples the largest delay reaches
// past it (Sec. III-A), and real time means one second of data is dedispersed
// in under a second (Sec. V; Sec. V-D sizes the Apertif beams per GPU from
// it).  A dd_realtime object keeps the last T_in = S + max_delay input samples
// of every channel on the device.  Each push appends S new samples from host
// memory and dedisperses the window, so consecutive outputs tile the time axis
// with no gap or overlap.
//
// Two window buffers alternate.  For push k, on the object's own copy stream
// (once the kernels of push k-2 have left window k % 2): the host chunk is
// copied straight into the chunk columns of window k % 2, and a copy kernel
// moves the last max_delay samples of the other window into its head.  The
// compute stream waits for those copies and runs the forward.  The copies of
// chunk k thus overlap the forward of chunk k-1.
//
// Window row layout (elements): `lead` unused columns, then max_delay tail
// samples, then the S chunk samples, which start on a multiple of 64 elements
// so that the host copy lands aligned.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>

#include "internal.h"

struct dd_realtime {
    const dd_plan *plan = nullptr;
    int device = 0;
    int32_t in_type = DD_F32;
    size_t es = 4;
    int64_t lead = 0;   // first used column of a window row
    int64_t pitch = 0;  // elements per window row
    void *win[2] = {nullptr, nullptr};  // [C][pitch]
    hipStream_t compute = nullptr;      // caller's stream, bound at create
    hipStream_t copy = nullptr;         // own stream for the window copies
    hipEvent_t copied[2] = {nullptr, nullptr};  // window s is complete
    hipEvent_t freed[2] = {nullptr, nullptr};   // the forward has finished reading window s
    bool used[2] = {false, false};
    int64_t pushed = 0;
};

namespace dd {
namespace {

// dst[ch][i] = src[ch][i] for i < n: one row per blockIdx.y (T is the storage
// type; the samples are only moved).
template <typename T>
__global__ __launch_bounds__(256) void copy_rows(T *__restrict__ dst, const T *__restrict__ src, int64_t pitch,
                                                 int64_t n) {
    const int64_t ch = blockIdx.y;
    T *d = dst + ch * pitch;
    const T *s = src + ch * pitch;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        d[i] = s[i];
}

// Byte rows whose source and destination have the same address modulo 4:
// up to three head bytes, whole 4-byte words, up to three tail bytes.
__global__ __launch_bounds__(256) void copy_rows_words(char *__restrict__ dst, const char *__restrict__ src,
                                                       int64_t pitch_bytes, int64_t n_bytes) {
    const int64_t ch = blockIdx.y;
    char *d = dst + ch * pitch_bytes;
    const char *s = src + ch * pitch_bytes;
    const int64_t head = min<int64_t>((4 - (reinterpret_cast<uintptr_t>(d) & 3)) & 3, n_bytes);
    const int64_t words = (n_bytes - head) / 4;
    const int64_t tail = head + 4 * words;
    const int64_t tid = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (tid < head)
        d[tid] = s[tid];
    uint32_t *dw = reinterpret_cast<uint32_t *>(d + head);
    const uint32_t *sw = reinterpret_cast<const uint32_t *>(s + head);
    for (int64_t w = tid; w < words; w += static_cast<int64_t>(gridDim.x) * blockDim.x)
        dw[w] = sw[w];
    if (tid < n_bytes - tail)
        d[tail + tid] = s[tail + tid];
}

size_t elem_size(int32_t t) { return t == DD_F32 ? 4 : t == DD_F16 ? 2 : 1; }

void rt_free(dd_realtime *r) {
    if (!r)
        return;
    int cur = 0;
    const bool have = hipGetDevice(&cur) == hipSuccess;
    if (have)
        (void)hipSetDevice(r->device);
    if (r->copy)
        (void)hipStreamSynchronize(r->copy);
    // freed[s] is recorded after the last forward that read window s.
    for (int s = 0; s < 2; ++s) {
        if (r->freed[s]) {
            if (r->used[s])
                (void)hipEventSynchronize(r->freed[s]);
            (void)hipEventDestroy(r->freed[s]);
        }
        if (r->copied[s])
            (void)hipEventDestroy(r->copied[s]);
    }
    for (int s = 0; s < 2; ++s)
        (void)hipFree(r->win[s]);
    if (r->copy)
        (void)hipStreamDestroy(r->copy);
    if (have)
        (void)hipSetDevice(cur);
    delete r;
}

hipError_t launch_tail(const dd_realtime *r, int s) {
    const dd_plan *p = r->plan;
    const int64_t n = p->max_delay;
    const size_t off = static_cast<size_t>(r->lead) * r->es;
    const size_t src_off = static_cast<size_t>(r->lead + p->S) * r->es;
    char *dst = static_cast<char *>(r->win[s]) + off;
    const char *src = static_cast<const char *>(r->win[1 - s]) + src_off;
    if (r->es != 4 && (static_cast<int64_t>(p->S) * static_cast<int64_t>(r->es)) % 4 == 0) {
        // Window bases and rows are 64-byte aligned, so source and destination
        // differ by S * es bytes modulo 4: here a multiple of 4.
        const int64_t n_bytes = n * static_cast<int64_t>(r->es);
        const dim3 grid_w(static_cast<uint32_t>(std::min<int64_t>((n_bytes / 4 + 255) / 256, 32)) + 1u,
                          static_cast<uint32_t>(p->C));
        hipLaunchKernelGGL(copy_rows_words, grid_w, dim3(256), 0, r->copy, dst, src,
                           static_cast<int64_t>(r->pitch * r->es), n_bytes);
        return hipGetLastError();
    }
    const dim3 grid(static_cast<uint32_t>(std::min<int64_t>((n + 255) / 256, 32)), static_cast<uint32_t>(p->C));
    if (r->es == 4)
        hipLaunchKernelGGL(copy_rows<uint32_t>, grid, dim3(256), 0, r->copy, reinterpret_cast<uint32_t *>(dst),
                           reinterpret_cast<const uint32_t *>(src), r->pitch, n);
    else if (r->es == 2)
        hipLaunchKernelGGL(copy_rows<uint16_t>, grid, dim3(256), 0, r->copy, reinterpret_cast<uint16_t *>(dst),
                           reinterpret_cast<const uint16_t *>(src), r->pitch, n);
    else
        hipLaunchKernelGGL(copy_rows<uint8_t>, grid, dim3(256), 0, r->copy, reinterpret_cast<uint8_t *>(dst),
                           reinterpret_cast<const uint8_t *>(src), r->pitch, n);
    return hipGetLastError();
}

}  // namespace
}  // namespace dd

using namespace dd;

extern "C" int dd_realtime_create(dd_realtime **out, const dd_plan *plan, dd_dtype in_type, void *stream) {
    clear_error();
    if (!out || !plan)
        return fail(DD_EINVAL, "NULL argument");
    *out = nullptr;
    if (in_type != DD_F32 && in_type != DD_F16 && in_type != DD_U8)
        return fail(DD_EINVAL, "unknown input dtype %d", (int)in_type);
    int device = 0;
    DD_HIP_TRY(hipGetDevice(&device));
    dd_realtime *r = new dd_realtime();
    r->plan = plan;
    r->device = device;
    r->in_type = in_type;
    r->es = elem_size(in_type);
    r->lead = (64 - plan->max_delay % 64) % 64;
    r->pitch = (r->lead + plan->T_in + 63) / 64 * 64;
    r->compute = static_cast<hipStream_t>(stream);
    const size_t win_bytes = static_cast<size_t>(plan->C) * r->pitch * r->es;
    for (int s = 0; s < 2; ++s) {
        if (hipMalloc(&r->win[s], win_bytes) != hipSuccess) {
            (void)hipGetLastError();
            rt_free(r);
            return fail(DD_ENOMEM, "device allocation for the real-time windows failed");
        }
    }
    hipError_t e = hipStreamCreateWithFlags(&r->copy, hipStreamNonBlocking);
    for (int s = 0; s < 2 && e == hipSuccess; ++s) {
        e = hipEventCreateWithFlags(&r->copied[s], hipEventDisableTiming);
        if (e == hipSuccess)
            e = hipEventCreateWithFlags(&r->freed[s], hipEventDisableTiming);
    }
    // Samples before the first push are zero.  Cleared on the copy stream,
    // ahead of every later copy; the forward only reads a window after
    // waiting for a copy event.
    for (int s = 0; s < 2 && e == hipSuccess; ++s)
        e = hipMemsetAsync(r->win[s], 0, win_bytes, r->copy);
    if (e != hipSuccess) {
        rt_free(r);
        return fail(DD_EHIP, "real-time set-up failed: %s", hipGetErrorString(e));
    }
    // Build the plan's forward tables now, outside any later graph capture.
    int rc = dd_plan_prepare(const_cast<dd_plan *>(plan), DD_FORWARD, in_type);
    if (rc != DD_OK) {
        rt_free(r);
        return rc;
    }
    clear_error();
    *out = r;
    return DD_OK;
}

extern "C" int dd_realtime_push(dd_realtime *r, const void *h_chunk, int64_t h_stride, float *d_out,
                                int64_t out_stride) {
    clear_error();
    if (!r || !h_chunk || !d_out)
        return fail(DD_EINVAL, "NULL argument");
    const dd_plan *p = r->plan;
    if (h_stride < p->S)
        return fail(DD_ESHAPE, "h_stride %lld < n_samples %lld", (long long)h_stride, (long long)p->S);
    if (out_stride < p->S)
        return fail(DD_ESHAPE, "out_stride %lld < n_samples %lld", (long long)out_stride, (long long)p->S);
    if (reinterpret_cast<uintptr_t>(h_chunk) % r->es != 0 || reinterpret_cast<uintptr_t>(d_out) % 4 != 0)
        return fail(DD_ESHAPE, "pointers must be aligned to their element size");
    int dev = 0;
    DD_HIP_TRY(hipGetDevice(&dev));
    if (dev != r->device)
        return fail(DD_EINVAL, "object was created on device %d, current device is %d", r->device, dev);
    const int s = static_cast<int>(r->pushed & 1);
    // The previous chunk's host buffer may be reused once this call returns.
    if (r->pushed > 0)
        DD_HIP_TRY(hipEventSynchronize(r->copied[1 - s]));
    // Window s is rewritten once the forward of push k-2 has read it.
    if (r->used[s])
        DD_HIP_TRY(hipStreamWaitEvent(r->copy, r->freed[s], 0));
    char *win = static_cast<char *>(r->win[s]);
    const size_t row = static_cast<size_t>(p->S) * r->es;
    DD_HIP_TRY(hipMemcpy2DAsync(win + static_cast<size_t>(r->lead + p->max_delay) * r->es, r->pitch * r->es, h_chunk,
                                static_cast<size_t>(h_stride) * r->es, row, p->C, hipMemcpyHostToDevice, r->copy));
    // Window k-1 is complete here: its copies precede on the same stream.
    if (p->max_delay > 0) {
        hipError_t e = launch_tail(r, s);
        if (e != hipSuccess)
            return fail(DD_EHIP, "tail copy launch failed: %s", hipGetErrorString(e));
    }
    DD_HIP_TRY(hipEventRecord(r->copied[s], r->copy));
    DD_HIP_TRY(hipStreamWaitEvent(r->compute, r->copied[s], 0));
    int rc = dd_dedisperse(p, win + static_cast<size_t>(r->lead) * r->es, static_cast<dd_dtype>(r->in_type), r->pitch,
                           d_out, out_stride, r->compute);
    // Record even after a failed launch, so that later pushes never wait on
    // a stale event; the window is not read then.
    DD_HIP_TRY(hipEventRecord(r->freed[s], r->compute));
    r->used[s] = true;
    ++r->pushed;
    return rc;
}

extern "C" int dd_realtime_pushed(const dd_realtime *r, int64_t *n_pushed) {
    clear_error();
    if (!r || !n_pushed)
        return fail(DD_EINVAL, "NULL argument");
    *n_pushed = r->pushed;
    return DD_OK;
}

extern "C" int dd_realtime_destroy(dd_realtime *r) {
    clear_error();
    rt_free(r);
    return DD_OK;
}
