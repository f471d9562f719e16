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
// Two window buffers alternate: push k assembles window k % 2 from the tail of
// the other window and the new chunk, then runs the forward on it.  The host
// copy of chunk k runs on the object's own copy stream, into one of two staging
// buffers, while the compute stream may still run chunk k-1.  Events order the
// two streams.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>

#include "internal.h"

struct dd_realtime {
    const dd_plan *plan = nullptr;
    int device = 0;
    int32_t in_type = DD_F32;
    size_t es = 4;
    int64_t pitch = 0;  // elements per window row
    void *win[2] = {nullptr, nullptr};    // [C][pitch]
    void *stage[2] = {nullptr, nullptr};  // [C][S], contiguous
    hipStream_t compute = nullptr;        // caller's stream, bound at create
    hipStream_t copy = nullptr;           // own stream for host-to-device copies
    hipEvent_t copied[2] = {nullptr, nullptr};  // chunk in stage[s] has arrived
    hipEvent_t freed[2] = {nullptr, nullptr};   // stage[s] has been consumed
    bool used[2] = {false, false};
    int64_t pushed = 0;
};

namespace dd {
namespace {

// dst[ch][i] for i < T_in: the tail of the previous window for i < max_delay,
// then the new chunk.  T is the storage type (no arithmetic on the samples).
template <typename T>
__global__ __launch_bounds__(256) void assemble_window(T *__restrict__ dst, const T *__restrict__ prev,
                                                       const T *__restrict__ stage, int64_t pitch,
                                                       int64_t max_delay, int64_t S) {
    const int64_t ch = blockIdx.y;
    const int64_t T_in = S + max_delay;
    T *d = dst + ch * pitch;
    const T *p = prev + ch * pitch + S;
    const T *c = stage + ch * S - max_delay;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < T_in; i += (int64_t)gridDim.x * blockDim.x)
        d[i] = i < max_delay ? p[i] : c[i];
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
    for (int s = 0; s < 2; ++s) {
        if (r->freed[s]) {
            (void)hipEventSynchronize(r->freed[s]);
            (void)hipEventDestroy(r->freed[s]);
        }
        if (r->copied[s])
            (void)hipEventDestroy(r->copied[s]);
    }
    // The last dedispersion reads a window after its freed event: wait for
    // the bound stream before releasing the windows.
    if (r->pushed)
        (void)hipStreamSynchronize(r->compute);
    for (int s = 0; s < 2; ++s) {
        (void)hipFree(r->win[s]);
        (void)hipFree(r->stage[s]);
    }
    if (r->copy)
        (void)hipStreamDestroy(r->copy);
    if (have)
        (void)hipSetDevice(cur);
    delete r;
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
    r->pitch = (plan->T_in + 63) / 64 * 64;
    r->compute = static_cast<hipStream_t>(stream);
    const size_t win_bytes = static_cast<size_t>(plan->C) * r->pitch * r->es;
    const size_t stage_bytes = static_cast<size_t>(plan->C) * plan->S * r->es;
    for (int s = 0; s < 2; ++s) {
        if (hipMalloc(&r->win[s], win_bytes) != hipSuccess || hipMalloc(&r->stage[s], stage_bytes) != hipSuccess) {
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
    // Samples before the first push are zero (cleared on the bound stream,
    // ahead of the first window assembly).
    for (int s = 0; s < 2 && e == hipSuccess; ++s)
        e = hipMemsetAsync(r->win[s], 0, win_bytes, r->compute);
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
    // Host copy into stage[s] once the chunk two pushes back has left it.
    if (r->used[s])
        DD_HIP_TRY(hipStreamWaitEvent(r->copy, r->freed[s], 0));
    const size_t row = static_cast<size_t>(p->S) * r->es;
    if (h_stride == p->S)
        DD_HIP_TRY(hipMemcpyAsync(r->stage[s], h_chunk, row * p->C, hipMemcpyHostToDevice, r->copy));
    else
        DD_HIP_TRY(hipMemcpy2DAsync(r->stage[s], row, h_chunk, static_cast<size_t>(h_stride) * r->es, row, p->C,
                                    hipMemcpyHostToDevice, r->copy));
    DD_HIP_TRY(hipEventRecord(r->copied[s], r->copy));
    r->used[s] = true;
    // Compute stream: assemble window s, release the stage, dedisperse.
    DD_HIP_TRY(hipStreamWaitEvent(r->compute, r->copied[s], 0));
    const int64_t T_in = p->T_in;
    const dim3 grid(static_cast<uint32_t>(std::min<int64_t>((T_in + 255) / 256, 64)), static_cast<uint32_t>(p->C));
    if (r->es == 4)
        hipLaunchKernelGGL(assemble_window<uint32_t>, grid, dim3(256), 0, r->compute,
                           static_cast<uint32_t *>(r->win[s]), static_cast<const uint32_t *>(r->win[1 - s]),
                           static_cast<const uint32_t *>(r->stage[s]), r->pitch, (int64_t)p->max_delay, p->S);
    else if (r->es == 2)
        hipLaunchKernelGGL(assemble_window<uint16_t>, grid, dim3(256), 0, r->compute,
                           static_cast<uint16_t *>(r->win[s]), static_cast<const uint16_t *>(r->win[1 - s]),
                           static_cast<const uint16_t *>(r->stage[s]), r->pitch, (int64_t)p->max_delay, p->S);
    else
        hipLaunchKernelGGL(assemble_window<uint8_t>, grid, dim3(256), 0, r->compute,
                           static_cast<uint8_t *>(r->win[s]), static_cast<const uint8_t *>(r->win[1 - s]),
                           static_cast<const uint8_t *>(r->stage[s]), r->pitch, (int64_t)p->max_delay, p->S);
    DD_HIP_TRY(hipGetLastError());
    DD_HIP_TRY(hipEventRecord(r->freed[s], r->compute));
    ++r->pushed;
    return dd_dedisperse(p, r->win[s], static_cast<dd_dtype>(r->in_type), r->pitch, d_out, out_stride, r->compute);
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
