// Descriptors shared by the batched (multi-beam) kernels and their host side.
//
// A batch runs many independent beams (the method is described for one beam
// and applies unchanged to each; beams share nothing, Sec. II / III-A).  Beams that use
// the same tile variant are served by one launch of that variant's multi-beam
// kernel: work-group g reads items[g] = (beam << 24) | tile and runs the same
// tile routine as the single-beam kernel on that beam's tables and pointers.
#pragma once

#include <cstdint>

#include "srs_tile.h"

namespace dd {

constexpr int kMaxBeams = 96;
constexpr uint32_t kNoItem = 0xffffffffu;  // padding slot: the work-group exits at once

// Per-run data of one beam (patched into the graph's kernel arguments).
struct BeamPtrs {
    const void *in;
    float *out;
    int64_t in_stride;
    int64_t out_stride;
};

struct BatchPtrs {
    BeamPtrs b[kMaxBeams];
};

// Per-plan data of one beam (device resident, fixed when the batch is built).
struct BeamDesc {
    const int32_t *rel;
    const int32_t *base;
    const int32_t *recs;
    dev::SrsDims d;  // in_stride / out_stride are taken from BeamPtrs
};

}  // namespace dd
