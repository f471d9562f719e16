// Batched dedispersion: many independent beams (the method is described for
// one beam and applies unchanged to each of many; beams share nothing,
// Sec. II / III-A) run from ONE HIP graph launch.
//
// Every beam keeps the tile variant its plan would use on its own (forced,
// tuned by dd_autotune / dd_batch_autotune, or the cost model's choice).
// Beams that share a variant form a group served by one launch of that
// variant's multi-beam kernel, so each kernel keeps the register footprint
// and occupancy of the single-beam kernel.  The groups' launches are chained
// in the graph; per-run pointers travel as a by-value kernel argument that
// dd_batch_run patches into the instantiated graph before each launch.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <map>
#include <memory>
#include <numeric>
#include <vector>

#include "batch_desc.h"
#include "internal.h"

namespace dd {
namespace {

struct Group {
    int32_t variant = -1;
    std::vector<int32_t> beams;
    const void *fn = nullptr;
    uint32_t threads = 0;
    uint32_t grid = 0;
    uint32_t item_offset = 0;
    size_t lds = 0;
    // Kernel-argument storage (kernelParams point here).
    const BeamDesc *a_descs = nullptr;
    const uint32_t *a_items = nullptr;
    void *params[3] = {};
    hipGraphNode_t node = nullptr;
};

// Work list of one group.  Work-groups are dealt to the 8 XCDs round-robin
// (work-group g runs on XCD g % 8), so the list gives XCD x the entries
// g = 8j + x.  Every beam's logical tiles (accumulator tile fastest) are cut
// into 8 contiguous runs, one per XCD -- the same order as the single-beam
// kernel, so an XCD's resident work-groups share input windows in its L2 --
// and XCD x walks run x of each beam in turn, costliest beams first.  The
// remainders of uneven beams are dealt to XCDs in rotation; slots past the
// end of an XCD's list hold kNoItem.
std::vector<uint32_t> group_items(const std::vector<int32_t> &beams, const std::vector<BeamDesc> &descs) {
    std::vector<std::vector<uint32_t>> per_xcd(8);
    uint32_t rot = 0;
    for (int32_t b : beams) {
        const uint32_t n = static_cast<uint32_t>(descs[b].d.n_t_tiles) * static_cast<uint32_t>(descs[b].d.n_acc_tiles);
        const uint32_t per = n / 8u, extra = n % 8u;
        uint32_t start = 0;
        for (uint32_t x = 0; x < 8u; ++x) {
            const uint32_t len = per + (((x + 8u - rot) % 8u) < extra ? 1u : 0u);
            for (uint32_t k = 0; k < len; ++k)
                per_xcd[x].push_back((static_cast<uint32_t>(b) << 24) | (start + k));
            start += len;
        }
        rot = (rot + extra) % 8u;
    }
    size_t longest = 0;
    for (const auto &l : per_xcd)
        longest = std::max(longest, l.size());
    std::vector<uint32_t> items(8 * longest, kNoItem);
    for (uint32_t x = 0; x < 8u; ++x)
        for (size_t j = 0; j < per_xcd[x].size(); ++j)
            items[8 * j + x] = per_xcd[x][j];
    return items;
}

}  // namespace
}  // namespace dd

using namespace dd;

struct dd_batch {
    int device = 0;
    int32_t n_beams = 0;
    int32_t in_type = DD_F32;
    std::vector<const dd_plan *> plans;
    std::vector<int32_t> beam_variant;
    double adds = 0;
    BeamDesc *d_descs = nullptr;
    uint32_t *d_items = nullptr;
    std::vector<std::unique_ptr<Group>> groups;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    BatchPtrs ptrs;  // per-run pointers, copied into every node's arguments
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
    B->beam_variant.assign(n_beams, -1);

    std::vector<BeamDesc> descs(n_beams);
    std::vector<size_t> lds(n_beams, 0);
    std::map<int32_t, size_t> group_of;  // variant id -> index in B->groups
    for (int32_t b = 0; b < n_beams; ++b) {
        const dd_plan *p = plans[b];
        B->adds += static_cast<double>(p->D) * static_cast<double>(p->S) * p->C;
        const Variant *v = find_variant(resolved_variant(p, DD_FORWARD, in_type));
        if (!v) {
            batch_free(B);
            return fail(DD_EUNSUPPORTED, "beam %d: no tile variant can serve this plan", b);
        }
        SrsArgs a;
        int rc = make_args(p, DD_FORWARD, *v, nullptr, 0, nullptr, 0, &a);
        if (rc != DD_OK) {
            batch_free(B);
            return rc;
        }
        BeamDesc &bd = descs[b];
        std::memset(&bd, 0, sizeof(bd));
        bd.rel = a.rel;
        bd.base = a.base;
        bd.recs = a.recs;
        bd.d.in_valid = a.in_valid;
        bd.d.n_t = a.n_t;
        bd.d.n_acc = a.n_acc;
        bd.d.n_rows = a.n_rows;
        bd.d.wcap = a.wcap;
        bd.d.rows_per_chunk = a.rows_per_chunk;
        bd.d.n_t_tiles = a.n_t_tiles > 0 ? a.n_t_tiles : static_cast<int32_t>((a.n_t + v->tt() - 1) / v->tt());
        bd.d.n_acc_tiles = (a.n_acc + v->ta() - 1) / v->ta();
        bd.d.r_begin = 0;
        bd.d.r_end = a.n_rows;
        bd.d.carry = 0;
        bd.d.skew = a.skew;
        const uint64_t n = static_cast<uint64_t>(bd.d.n_t_tiles) * bd.d.n_acc_tiles;
        if (n >= (1u << 24)) {
            batch_free(B);
            return fail(DD_EUNSUPPORTED, "beam %d has %llu tiles (limit 2^24)", b, (unsigned long long)n);
        }
        lds[b] = static_cast<size_t>(a.lds_bytes);
        B->beam_variant[b] = v->id;
        auto it = group_of.find(v->id);
        if (it == group_of.end()) {
            it = group_of.emplace(v->id, B->groups.size()).first;
            B->groups.emplace_back(new Group());
            B->groups.back()->variant = v->id;
        }
        B->groups[it->second]->beams.push_back(b);
    }

    // Work lists; groups with the most additions first.
    std::vector<uint32_t> items;
    std::vector<double> group_adds(B->groups.size(), 0.0);
    for (size_t g = 0; g < B->groups.size(); ++g) {
        Group &G = *B->groups[g];
        for (int32_t b : G.beams)
            group_adds[g] += static_cast<double>(plans[b]->D) * static_cast<double>(plans[b]->S) * plans[b]->C;
        std::stable_sort(G.beams.begin(), G.beams.end(),
                         [&](int32_t x, int32_t y) { return descs[x].d.n_rows > descs[y].d.n_rows; });
    }
    std::vector<size_t> gorder(B->groups.size());
    std::iota(gorder.begin(), gorder.end(), 0);
    std::stable_sort(gorder.begin(), gorder.end(), [&](size_t x, size_t y) { return group_adds[x] > group_adds[y]; });
    std::vector<std::unique_ptr<Group>> sorted;
    for (size_t g : gorder)
        sorted.push_back(std::move(B->groups[g]));
    B->groups = std::move(sorted);
    for (auto &gp : B->groups) {
        Group &G = *gp;
        const Variant &v = *find_variant(G.variant);
        std::vector<uint32_t> gi = group_items(G.beams, descs);
        if (items.size() + gi.size() >= (1ull << 32) || gi.size() > 0x7fffffffu) {
            batch_free(B);
            return fail(DD_EUNSUPPORTED, "too many work items");
        }
        G.item_offset = static_cast<uint32_t>(items.size());
        G.grid = static_cast<uint32_t>(gi.size());
        items.insert(items.end(), gi.begin(), gi.end());
        G.fn = multi_kernel(v, in_type);
        if (!G.fn) {
            batch_free(B);
            return fail(DD_EUNSUPPORTED, "this library has no multi-beam kernel for tile variant %d", v.id);
        }
        G.threads = static_cast<uint32_t>(64 * v.waves);
        for (int32_t b : G.beams)
            G.lds = std::max(G.lds, lds[b]);
        if (G.lds > 65536) {
            hipError_t e = hipFuncSetAttribute(G.fn, hipFuncAttributeMaxDynamicSharedMemorySize,
                                               static_cast<int>(G.lds));
            if (e != hipSuccess) {
                batch_free(B);
                return fail(DD_EHIP, "setting the LDS limit failed: %s", hipGetErrorString(e));
            }
        }
    }

    if (hipMalloc(&B->d_descs, descs.size() * sizeof(BeamDesc)) != hipSuccess ||
        hipMalloc(&B->d_items, items.size() * sizeof(uint32_t)) != hipSuccess) {
        (void)hipGetLastError();
        batch_free(B);
        return fail(DD_ENOMEM, "device allocation for the batch failed");
    }
    if (hipMemcpy(B->d_descs, descs.data(), descs.size() * sizeof(BeamDesc), hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(B->d_items, items.data(), items.size() * sizeof(uint32_t), hipMemcpyHostToDevice) != hipSuccess) {
        batch_free(B);
        return fail(DD_EHIP, "upload of the batch tables failed");
    }

    // Graph: one kernel node per group, chained.
    std::memset(&B->ptrs, 0, sizeof(B->ptrs));
    hipError_t e = hipGraphCreate(&B->graph, 0);
    hipGraphNode_t prev = nullptr;
    for (auto &gp : B->groups) {
        if (e != hipSuccess)
            break;
        Group &G = *gp;
        G.a_descs = B->d_descs;
        G.a_items = B->d_items + G.item_offset;
        G.params[0] = &B->ptrs;
        G.params[1] = &G.a_descs;
        G.params[2] = &G.a_items;
        hipKernelNodeParams kp;
        std::memset(&kp, 0, sizeof(kp));
        kp.func = const_cast<void *>(G.fn);
        kp.gridDim = dim3(G.grid);
        kp.blockDim = dim3(G.threads);
        kp.sharedMemBytes = static_cast<unsigned int>(G.lds);
        kp.kernelParams = G.params;
        e = hipGraphAddKernelNode(&G.node, B->graph, prev ? &prev : nullptr, prev ? 1 : 0, &kp);
        prev = G.node;
    }
    if (e == hipSuccess)
        e = hipGraphInstantiate(&B->exec, B->graph, nullptr, nullptr, 0);
    if (e != hipSuccess) {
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
    for (auto &gp : B->groups) {
        const Group &G = *gp;
        hipKernelNodeParams kp;
        std::memset(&kp, 0, sizeof(kp));
        kp.func = const_cast<void *>(G.fn);
        kp.gridDim = dim3(G.grid);
        kp.blockDim = dim3(G.threads);
        kp.sharedMemBytes = static_cast<unsigned int>(G.lds);
        kp.kernelParams = const_cast<void **>(G.params);
        DD_HIP_TRY(hipGraphExecKernelNodeSetParams(B->exec, G.node, &kp));
    }
    DD_HIP_TRY(hipGraphLaunch(B->exec, static_cast<hipStream_t>(stream)));
    return DD_OK;
}

extern "C" int dd_batch_variants(const dd_batch *B, int32_t *variants) {
    clear_error();
    if (!B || !variants)
        return fail(DD_EINVAL, "NULL argument");
    for (int32_t b = 0; b < B->n_beams; ++b)
        variants[b] = B->beam_variant[b];
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
