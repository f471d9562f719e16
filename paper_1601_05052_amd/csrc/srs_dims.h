// Sizes of one shifted-row-sum launch, passed by value to the kernels (plain
// data, shared by host and device code).
#pragma once

#include <cstdint>

namespace dd {
namespace dev {

struct SrsDims {
    int64_t in_stride;
    int64_t in_valid;
    int64_t out_stride;
    int64_t n_t;
    int32_t n_acc;
    int32_t n_rows;
    int32_t wcap;
    int32_t rows_per_chunk;
    int32_t n_t_tiles;
    int32_t n_acc_tiles;
};

}  // namespace dev
}  // namespace dd
