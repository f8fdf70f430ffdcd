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

// One problem of the batched launch: Y (N x l), T (l x k) and AJ (ld ldaj)
// as above, l <= 128, k <= 128; al: l % 4 == 0; vec: AJ and ldaj 16-byte
// aligned; nwg: its workgroups (apply_batch_workgroups).
struct ApplyJob {
  const float* Y;
  const double* T;
  float* AJ;
  int64_t N, ldaj;
  int l, k, al, vec, nwg, pad_;
};
constexpr int APPLY_MIN_BLOCKS = 8;  // blocks of 64 rows per workgroup, at least
int apply_batch_workgroups(int64_t N, int num_cu);
// every job's AJ = Y T in one launch (device table of njobs jobs; max_nwg:
// the largest nwg; kmax: the largest k); each entry has the bits of the
// one-problem launch
hipError_t launch_apply_t_bf16_runs_batch(hipStream_t st, const ApplyJob* jobs, int njobs,
                                          int max_nwg, int kmax);

}  // namespace sid
