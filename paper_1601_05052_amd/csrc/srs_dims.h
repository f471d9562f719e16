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
    // Input rows [r_begin, r_end) are summed (a block of a plan whose rows are
    // split over several launches; r_begin is a multiple of the variant's rows
    // per chunk).  carry: the sums continue the partial sums in the output.
    int32_t r_begin;
    int32_t r_end;
    int32_t carry;
    // Per accumulator row, the skew of its tiles (null: none): a tile's
    // sample tau holds output sample tau - skew[a] of row a, so every
    // accumulator row of a tile can follow the delay curve and the rows'
    // windows line up.  The tables hold offsets O[r][a] - skew[a].
    const int32_t *skew;
};

}  // namespace dev
}  // namespace dd
