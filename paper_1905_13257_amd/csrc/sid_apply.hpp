// sid_apply.hpp -- AJ = Y T for the bfloat16 sketch precisions with the
// output stored in long column runs.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace sid {

// Y: N x l row-major FP32; Tm: l x k FP64 (column-major, ld l); AJ: N x k
// FP32 column-major (ld ldaj >= N).  k <= 128 and l <= 128, or k <= 160 and
// l <= 192 with l % 4 == 0.
bool apply_t_bf16_runs_supported(int k, int l);
hipError_t launch_apply_t_bf16_runs(hipStream_t st, const float* Y, int64_t N, int l,
                                    const double* Tm, int k, float* AJ, int64_t ldaj, int num_cu);

}  // namespace sid
