// sid_interp.hpp -- single-pass ID with interpolation (Alg. 6): launchers of
// the coarse skeleton gather and of the coarse-to-fine reconstruction.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace sid {

// The trilinear coarse-to-fine operator as three 1-D tables, indexed by the
// fine index of x (0 .. nx-1), then y (nx ..), then z (nx + ny ..): the two
// coarse nodes a fine index lies between and the weight of the second one
// (the first one weighs 1 - w).
struct InterpDev {
  const int32_t* lo;
  const int32_t* hi;
  const float* w32;
  const double* w64;
  int32_t nx, ny, nz, mx, my, mz, ncomp;
  int64_t N, Nc;
};

// AC(s, t) = A(rows[s], piv[t]) for t < keff, 0 beyond (|S| x kcap, ldd)
hipError_t launch_gather_coarse_skeleton(hipStream_t st, const void* A, bool f64, int64_t lda,
                                         const int64_t* rows, int64_t Ns, const int64_t* piv,
                                         const int64_t* keff, int kcap, void* dst, int64_t ldd);

// B = Mf ACJ (N x k, ldb), element type of ACJ (FP64 weights for FP64)
hipError_t launch_interp_apply(hipStream_t st, const InterpDev& t, bool f64, const void* ACJ,
                               int64_t ldacj, int k, void* B, int64_t ldb);

// Matrix-core path (FP32, k <= 128): kp = k rounded up to 16.
//   acjt: Nc x kp row-major FP32 copy of ACJ (zero padded)
//   pb:   P packed as bfloat16 hi/lo operand tiles, (ceil(n/32) + 3) * kp/16 * 2 KiB
size_t interp_pb_bytes(int64_t n, int kp);
hipError_t launch_interp_pack(hipStream_t st, const float* ACJ, int64_t ldacj, int64_t Nc, int k,
                              int kp, float* acjt, const float* P, int64_t ldp, int64_t n,
                              void* pb);
// out = Mf ACJ P (out != NULL), or, with A != NULL, 4 error partials per
// row block (interp_mfma_blocks) into part (part_cap entries of 4) reduced
// into out4.
int64_t interp_mfma_blocks(int64_t N);
hipError_t launch_interp_mfma(hipStream_t st, const InterpDev& t, int kp, const float* acjt,
                              const void* pb, int64_t n, float* out, int64_t ldo, const float* A,
                              int64_t lda, double* part, int64_t part_cap, double* out4);

// The plain ID on the same kernel (eq. (ID)): Ahat = AJ P with AJ the
// column-major N x k skeleton (FP32, k <= kp <= 128), P packed by
// launch_pack_p into pb (interp_pb_bytes(n, kp)); out, or the error
// partials and out4 as above.
hipError_t launch_pack_p(hipStream_t st, const float* P, int64_t ldp, int k, int kp, int64_t n,
                         void* pb);
hipError_t launch_id_mfma(hipStream_t st, const float* AJ, int64_t ldaj, int64_t N, int k, int kp,
                          const void* pb, int64_t n, float* out, int64_t ldo, const float* A,
                          int64_t lda, double* part, int64_t part_cap, double* out4);

}  // namespace sid
