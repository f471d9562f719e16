// Batched dedispersion: many independent beams (Sclocco et al., Sec. III-A,
// "all results can be applied to the case of multiple beams"; Sec. II, beams
// are independent) in ONE persistent kernel launch, replayed from a HIP graph.
//
// Work items are (beam, DM tile, time tile) triples ordered by cost, largest
// first, and handed out by an atomic counter; every beam keeps its own tile
// shape (chosen per plan, e.g. by dd_autotune) from the family of 4-wave
// variants compiled into the kernel.  Per-run pointers travel as a by-value
// kernel argument that dd_batch_run patches into the graph before launch, so
// no host-to-device copy is needed per run.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <numeric>
#include <vector>

#include "internal.h"
#include "srs_regwin.h"
#include "srs_tile.h"

namespace dd {
namespace {

constexpr int kMaxBeams = 96;

struct BeamPtrs {
    const void *in;
    float *out;
    int64_t in_stride;
    int64_t out_stride;
};

struct BatchPtrs {
    BeamPtrs b[kMaxBeams];
};

struct BeamDesc {
    const int32_t *rel;
    const int32_t *base;
    const int32_t *wrec;
    const int32_t *woff;
    dev::SrsDims d;
    int32_t slot;
    int32_t pad;
};

}  // namespace
}  // namespace dd

namespace dd {

// The batch kernel's tile family: 4-wave variants whose register footprints
// are close, so one kernel serves them all at the occupancy of the largest.
// Index = slot, value = variant id (see srs_kernels.hip).
const int32_t kBatchFamily[] = {17, 19, 14, 21, 20, 24, 25, 7};
const int32_t kBatchFamilySize = sizeof(kBatchFamily) / sizeof(kBatchFamily[0]);

int32_t batch_slot_of_variant(int32_t v) {
    for (int32_t s = 0; s < kBatchFamilySize; ++s)
        if (kBatchFamily[s] == v)
            return s;
    return -1;
}

}  // namespace dd

namespace dd {
namespace {

int32_t slot_of_variant(int32_t v) { return batch_slot_of_variant(v); }

__global__ void reset_counter(uint32_t *counter) { *counter = 0u; }

template <typename TIn>
__global__ void __launch_bounds__(256)
    batch_kernel(BatchPtrs ptrs, const BeamDesc *__restrict__ descs, const uint32_t *__restrict__ items,
                 uint32_t n_items, uint32_t *__restrict__ counter) {
    extern __shared__ __attribute__((aligned(16))) float lds[];
    __shared__ uint32_t s_item;
    for (;;) {
        if (threadIdx.x == 0)
            s_item = atomicAdd(counter, 1u);
        __syncthreads();
        const uint32_t item = __builtin_amdgcn_readfirstlane(s_item);
        __syncthreads();  // everyone has read s_item before it is reused
        if (item >= n_items)
            break;  // every work-group leaves once the list is exhausted
        const uint32_t w = items[item];
        const uint32_t beam = w >> 24, tile = w & 0xffffffu;
        const BeamDesc &bd = descs[beam];
        const BeamPtrs bp = ptrs.b[beam];
        dev::SrsDims d = bd.d;
        d.in_stride = bp.in_stride;
        d.out_stride = bp.out_stride;
        const int32_t tile_a = static_cast<int32_t>(tile % static_cast<uint32_t>(d.n_acc_tiles));
        const int32_t tile_t = static_cast<int32_t>(tile / static_cast<uint32_t>(d.n_acc_tiles));
        const TIn *in = static_cast<const TIn *>(bp.in);
        // Slot -> tile routine; must match kBatchFamily.
        switch (bd.slot) {
        case 0:
            dev::srs_tile_regwin<TIn, 8, 8, 40, 4, 1, 12, false>(in, bp.out, bd.base, bd.wrec, bd.woff, d, tile_t,
                                                               tile_a, lds);
            break;
        case 1:
            dev::srs_tile_regwin<TIn, 8, 4, 32, 4, 1, 12, false>(in, bp.out, bd.base, bd.wrec, bd.woff, d, tile_t,
                                                               tile_a, lds);
            break;
        case 2:
            dev::srs_tile_regwin<TIn, 4, 8, 32, 4, 2, 12, false>(in, bp.out, bd.base, bd.wrec, bd.woff, d, tile_t,
                                                               tile_a, lds);
            break;
        case 3: dev::srs_tile_ldsp<TIn, 4, 4, 4, 1, 16>(in, bp.out, bd.rel, bd.base, d, tile_t, tile_a, lds); break;
        case 4: dev::srs_tile_ldsp<TIn, 4, 8, 4, 1, 24>(in, bp.out, bd.rel, bd.base, d, tile_t, tile_a, lds); break;
        case 5: dev::srs_tile_ldsp<TIn, 4, 2, 4, 2, 12>(in, bp.out, bd.rel, bd.base, d, tile_t, tile_a, lds); break;
        case 6: dev::srs_tile_ldsp<TIn, 4, 1, 4, 2, 8>(in, bp.out, bd.rel, bd.base, d, tile_t, tile_a, lds); break;
        default:  // direct staging: fits spreads up to the LDS size
            dev::srs_tile_lds<TIn, 4, 1, 4>(in, bp.out, bd.rel, bd.base, d, tile_t, tile_a, lds);
            break;
        }
    }
}

const void *batch_fn(int32_t in_type) {
    switch (in_type) {
    case DD_F32: return reinterpret_cast<const void *>(batch_kernel<float>);
    case DD_F16: return reinterpret_cast<const void *>(batch_kernel<_Float16>);
    default: return reinterpret_cast<const void *>(batch_kernel<uint8_t>);
    }
}

}  // namespace
}  // namespace dd

using namespace dd;

struct dd_batch {
    int device = 0;
    int32_t n_beams = 0;
    int32_t in_type = DD_F32;
    std::vector<const dd_plan *> plans;
    double adds = 0;
    BeamDesc *d_descs = nullptr;
    uint32_t *d_items = nullptr;
    uint32_t *d_counter = nullptr;
    uint32_t n_items = 0;
    uint32_t grid = 0;
    size_t lds = 0;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    hipGraphNode_t node = nullptr;
    // Kernel-argument storage for the batch node (kernelParams points here).
    BatchPtrs ptrs;
    const BeamDesc *a_descs = nullptr;
    const uint32_t *a_items = nullptr;
    uint32_t a_n_items = 0;
    uint32_t *a_counter = nullptr;
    void *params[5] = {};
    uint32_t *r_counter = nullptr;
    void *r_params[1] = {};
};

static void batch_free(dd_batch *b) {
    if (!b)
        return;
    int cur = 0;
    bool have = hipGetDevice(&cur) == hipSuccess;
    if (have)
        (void)hipSetDevice(b->device);
    if (b->exec)
        (void)hipGraphExecDestroy(b->exec);
    if (b->graph)
        (void)hipGraphDestroy(b->graph);
    (void)hipFree(b->d_descs);
    (void)hipFree(b->d_items);
    (void)hipFree(b->d_counter);
    if (have)
        (void)hipSetDevice(cur);
    delete b;
}

extern "C" int dd_batch_create(dd_batch **out, const dd_plan *const *plans, int32_t n_beams, dd_dtype in_type) {
    clear_error();
    if (!out || !plans)
        return fail(DD_EINVAL, "NULL argument");
    *out = nullptr;
    if (n_beams < 1 || n_beams > kMaxBeams)
        return fail(DD_EINVAL, "n_beams must be in [1, %d] (got %d)", kMaxBeams, n_beams);
    if (in_type != DD_F32 && in_type != DD_F16 && in_type != DD_U8)
        return fail(DD_EINVAL, "unknown input dtype %d", (int)in_type);
    for (int32_t b = 0; b < n_beams; ++b)
        if (!plans[b])
            return fail(DD_EINVAL, "plan %d is NULL", b);

    int device = 0;
    DD_HIP_TRY(hipGetDevice(&device));
    dd_batch *B = new dd_batch();
    B->device = device;
    B->n_beams = n_beams;
    B->in_type = in_type;
    B->plans.assign(plans, plans + n_beams);

    std::vector<BeamDesc> descs(n_beams);
    std::vector<uint64_t> cost(n_beams);
    uint64_t total_items = 0;
    for (int32_t b = 0; b < n_beams; ++b) {
        const dd_plan *p = plans[b];
        B->adds += static_cast<double>(p->D) * static_cast<double>(p->S) * p->C;
        // The plan's batch-tuned choice, else its own choice if it is in the
        // batch family, else the family member the cost model prefers.
        int32_t vid = batch_variant(p, in_type);
        if (vid < 0) {
            batch_free(B);
            return fail(DD_EUNSUPPORTED, "beam %d: no batched tile variant fits its delay spread", b);
        }
        const Variant &v = *find_variant(vid);
        SrsArgs a;
        int rc = make_args(p, DD_FORWARD, v, nullptr, 0, nullptr, 0, &a);
        if (rc != DD_OK) {
            batch_free(B);
            return rc;
        }
        BeamDesc &bd = descs[b];
        std::memset(&bd, 0, sizeof(bd));
        bd.rel = a.rel;
        bd.base = a.base;
        bd.wrec = a.wrec;
        bd.woff = a.woff;
        bd.d.in_valid = a.in_valid;
        bd.d.n_t = a.n_t;
        bd.d.n_acc = a.n_acc;
        bd.d.n_rows = a.n_rows;
        bd.d.wcap = a.wcap;
        bd.d.rows_per_chunk = a.rows_per_chunk;
        bd.d.n_t_tiles = static_cast<int32_t>((a.n_t + v.tt() - 1) / v.tt());
        bd.d.n_acc_tiles = (a.n_acc + v.ta() - 1) / v.ta();
        bd.slot = slot_of_variant(vid);
        const uint64_t n = static_cast<uint64_t>(bd.d.n_t_tiles) * bd.d.n_acc_tiles;
        if (n >= (1u << 24)) {
            batch_free(B);
            return fail(DD_EUNSUPPORTED, "beam %d has %llu tiles (limit 2^24)", b, (unsigned long long)n);
        }
        total_items += n;
        cost[b] = static_cast<uint64_t>(v.tt()) * v.ta() * p->C;
        B->lds = std::max(B->lds, static_cast<size_t>(a.lds_bytes));
    }
    if (total_items >= (1ull << 32)) {
        batch_free(B);
        return fail(DD_EUNSUPPORTED, "too many work items");
    }
    // Work list: beams by descending per-item cost (longest items first).
    std::vector<int32_t> order(n_beams);
    std::iota(order.begin(), order.end(), 0);
    std::stable_sort(order.begin(), order.end(), [&](int32_t x, int32_t y) { return cost[x] > cost[y]; });
    std::vector<uint32_t> items;
    items.reserve(total_items);
    for (int32_t b : order) {
        const uint32_t n = static_cast<uint32_t>(descs[b].d.n_t_tiles) * descs[b].d.n_acc_tiles;
        for (uint32_t t = 0; t < n; ++t)
            items.push_back((static_cast<uint32_t>(b) << 24) | t);
    }
    B->n_items = static_cast<uint32_t>(items.size());

    const void *fn = batch_fn(in_type);
    hipError_t e = hipSuccess;
    if (B->lds > 65536)
        e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(B->lds));
    int per_cu = 0, n_cu = 0;
    if (e == hipSuccess)
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, 256, B->lds);
    if (e == hipSuccess)
        e = hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, B->device);
    if (e != hipSuccess) {
        batch_free(B);
        return fail(DD_EHIP, "occupancy query failed: %s", hipGetErrorString(e));
    }
    per_cu = std::max(per_cu, 1);
    B->grid = static_cast<uint32_t>(std::min<uint64_t>(static_cast<uint64_t>(per_cu) * n_cu, B->n_items));

    if (hipMalloc(&B->d_descs, descs.size() * sizeof(BeamDesc)) != hipSuccess ||
        hipMalloc(&B->d_items, items.size() * sizeof(uint32_t)) != hipSuccess ||
        hipMalloc(&B->d_counter, sizeof(uint32_t)) != hipSuccess) {
        (void)hipGetLastError();
        batch_free(B);
        return fail(DD_ENOMEM, "device allocation for the batch failed");
    }
    if (hipMemcpy(B->d_descs, descs.data(), descs.size() * sizeof(BeamDesc), hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(B->d_items, items.data(), items.size() * sizeof(uint32_t), hipMemcpyHostToDevice) != hipSuccess) {
        batch_free(B);
        return fail(DD_EHIP, "upload of the batch tables failed");
    }

    // Graph: counter reset (a kernel, not a memset node) -> persistent kernel.
    std::memset(&B->ptrs, 0, sizeof(B->ptrs));
    B->a_descs = B->d_descs;
    B->a_items = B->d_items;
    B->a_n_items = B->n_items;
    B->a_counter = B->d_counter;
    B->params[0] = &B->ptrs;
    B->params[1] = &B->a_descs;
    B->params[2] = &B->a_items;
    B->params[3] = &B->a_n_items;
    B->params[4] = &B->a_counter;
    B->r_counter = B->d_counter;
    B->r_params[0] = &B->r_counter;

    hipGraphNode_t reset = nullptr;
    hipKernelNodeParams rp;
    std::memset(&rp, 0, sizeof(rp));
    rp.func = reinterpret_cast<void *>(reset_counter);
    rp.gridDim = dim3(1);
    rp.blockDim = dim3(1);
    rp.kernelParams = B->r_params;
    hipKernelNodeParams kp;
    std::memset(&kp, 0, sizeof(kp));
    kp.func = const_cast<void *>(fn);
    kp.gridDim = dim3(B->grid);
    kp.blockDim = dim3(256);
    kp.sharedMemBytes = static_cast<unsigned int>(B->lds);
    kp.kernelParams = B->params;
    if ((e = hipGraphCreate(&B->graph, 0)) != hipSuccess ||
        (e = hipGraphAddKernelNode(&reset, B->graph, nullptr, 0, &rp)) != hipSuccess ||
        (e = hipGraphAddKernelNode(&B->node, B->graph, &reset, 1, &kp)) != hipSuccess ||
        (e = hipGraphInstantiate(&B->exec, B->graph, nullptr, nullptr, 0)) != hipSuccess) {
        batch_free(B);
        return fail(DD_EHIP, "building the batch graph failed: %s", hipGetErrorString(e));
    }
    *out = B;
    return DD_OK;
}

extern "C" int dd_batch_run(dd_batch *B, const void *const *d_in, const int64_t *in_strides, float *const *d_out,
                            const int64_t *out_strides, void *stream) {
    clear_error();
    if (!B || !d_in || !in_strides || !d_out || !out_strides)
        return fail(DD_EINVAL, "NULL argument");
    const size_t es = B->in_type == DD_F32 ? 4 : B->in_type == DD_F16 ? 2 : 1;
    for (int32_t b = 0; b < B->n_beams; ++b) {
        const dd_plan *p = B->plans[b];
        if (!d_in[b] || !d_out[b])
            return fail(DD_EINVAL, "beam %d: NULL data pointer", b);
        if (in_strides[b] < p->T_in)
            return fail(DD_ESHAPE, "beam %d: in_stride %lld < input samples %lld", b, (long long)in_strides[b],
                        (long long)p->T_in);
        if (out_strides[b] < p->S)
            return fail(DD_ESHAPE, "beam %d: out_stride %lld < n_samples %lld", b, (long long)out_strides[b],
                        (long long)p->S);
        if (reinterpret_cast<uintptr_t>(d_in[b]) % es || reinterpret_cast<uintptr_t>(d_out[b]) % 4)
            return fail(DD_ESHAPE, "beam %d: misaligned data pointer", b);
    }
    int dev = 0;
    DD_HIP_TRY(hipGetDevice(&dev));
    if (dev != B->device)
        return fail(DD_EINVAL, "batch was created on device %d, current device is %d", B->device, dev);
    for (int32_t b = 0; b < B->n_beams; ++b) {
        B->ptrs.b[b].in = d_in[b];
        B->ptrs.b[b].out = d_out[b];
        B->ptrs.b[b].in_stride = in_strides[b];
        B->ptrs.b[b].out_stride = out_strides[b];
    }
    hipKernelNodeParams kp;
    std::memset(&kp, 0, sizeof(kp));
    kp.func = const_cast<void *>(batch_fn(B->in_type));
    kp.gridDim = dim3(B->grid);
    kp.blockDim = dim3(256);
    kp.sharedMemBytes = static_cast<unsigned int>(B->lds);
    kp.kernelParams = B->params;
    DD_HIP_TRY(hipGraphExecKernelNodeSetParams(B->exec, B->node, &kp));
    DD_HIP_TRY(hipGraphLaunch(B->exec, static_cast<hipStream_t>(stream)));
    return DD_OK;
}

extern "C" int dd_batch_adds(const dd_batch *B, double *adds) {
    clear_error();
    if (!B || !adds)
        return fail(DD_EINVAL, "NULL argument");
    *adds = B->adds;
    return DD_OK;
}

extern "C" int dd_batch_destroy(dd_batch *B) {
    clear_error();
    batch_free(B);
    return DD_OK;
}
