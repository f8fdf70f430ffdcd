// sid_sketch_f64.hpp -- W = Psi A and Y = A Omega in FP64 over all rows
// (register-tiled).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace sid {

// W (lq x n, ld lq, FP64) from A (N x n, column-major, ld lda, FP32 promoted
// exactly or FP64); part: nchunks lq n doubles of per-chunk partials, summed
// in chunk order.  Bitwise equal to the general F64 sketch with the same
// nchunks.
hipError_t launch_sketch_w_f64(hipStream_t st, const void* A, bool a_is_f64, int64_t lda,
                               int64_t N, int64_t n, int lq, uint64_t seed, int64_t nchunks,
                               double* part, double* W);

// Y (N x l, row-major FP64) = A Omega, Omega (n x l, row-major) the
// single-precision draws.  Bitwise equal to the general F64 sketch.
hipError_t launch_sketch_y_f64(hipStream_t st, const void* A, bool a_is_f64, int64_t lda,
                               int64_t N, int64_t n, const float* omega, int l, double* Y);

}  // namespace sid
