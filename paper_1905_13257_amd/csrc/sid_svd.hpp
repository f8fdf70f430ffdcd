// sid_svd.hpp -- small FP64 kernels of SBR-SVD (Alg. 2).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace sid {

// in-place thin QR (CGS2) of Y (n x b, ld n), R (b x b, ld b); b <= 64
hipError_t launch_small_qr(hipStream_t st, double* Y, int n, int b, double* R);
// R = Rt R for b x b upper triangular factors (ld b); min |R(c, c)| into *mindiag.
// The block loop's stop test on the device: state[0] = columns of the basis
// so far, state[1] = 1 once a block was rank deficient (reset at blk = 0);
// block blk counts (state[0] = (blk + 1) b) unless min |R(c, c)| <=
// 1e-12 sqrt(*g2), which stops the loop at blk b columns for good.
hipError_t launch_trmul(hipStream_t st, const double* Rt, double* R, int b, double* mindiag,
                        const double* g2, int64_t blk, int64_t* state);
// Jacobi eigensolver of a symmetric m x m matrix (ld m, m <= 256; the upper
// triangle is read): M becomes
// diagonal (eigenvalues), V (m x m, ld m) the eigenvectors; work: (m rounded
// up to even)^2 doubles, used when that exceeds 128 (else may be NULL); rot:
// jacobi_rot_doubles(m) doubles of rotation records; nsweeps: one int
size_t jacobi_rot_doubles(int m);
hipError_t launch_jacobi(hipStream_t st, double* M, int m, double* V, double* work, double* rot,
                         int* nsweeps);
// S[0:k] = sqrt of the eigenvalues in descending order (0 past m); Uv (m x k)
// the matching eigenvectors, Us = Uv / S column by column (0 where S = 0)
hipError_t launch_eig_sort(hipStream_t st, const double* M, int m, const double* V, int k,
                           double* S, double* Us, double* Uv);
// dst = src (rows x cols), element type conversion between FP32 / FP64
hipError_t launch_convert(hipStream_t st, const void* src, bool src_f64, int64_t rows,
                          int64_t cols, int64_t lds, void* dst, bool dst_f64, int64_t ldd);
// H (N x l, ld ldh) = A W^T, or H += A W^T with accumulate (continuing each
// sum from H's entry: column blocks in order give the bits of one call), in
// FP64 (A: N x n, ld lda, FP32 promoted exactly or FP64; W: l x n FP64, ld
// ldw >= l rounded up to 16, the rows past l read but unused); l <= 256
hipError_t launch_h_gemm(hipStream_t st, const void* A, bool a_f64, int64_t lda, int64_t N, int n,
                         const double* W, int64_t ldw, int l, double* H, int64_t ldh,
                         bool accumulate);
// Bi (N x b, ld N) = (Hi - Bt(:, 0:j) M) R^-1: Bt, Hi column-major with ld N,
// M j x b (ld ldm), R b x b upper triangular (ld b, nonzero diagonal);
// b <= 64; Bi must not overlap Bt(:, 0:j) or Hi
hipError_t launch_block_update(hipStream_t st, const double* Bt, int64_t N, int j,
                               const double* Hi, const double* M, int64_t ldm, const double* R,
                               int b, double* Bi);
// dst (cols x rows, ld ldd) = src^T (rows x cols, ld lds), FP64
hipError_t launch_transpose64(hipStream_t st, const double* src, int64_t rows, int64_t cols,
                              int64_t lds, double* dst, int64_t ldd);

// C (p x q, ld ldc) = alpha X^T Y + beta C over N rows (beta = 0: C is not
// read): X N x p column-major (ld ldx); Y N x q with entry (r, c) at
// Y[r ysr + c ysc]; p, q <= 128; part: tsmm_blocks(N, num_cu) x p x q
// doubles of scratch.  FP64, fixed summation order.
int64_t tsmm_blocks(int64_t N, int num_cu, int64_t* rows_per_block);
hipError_t launch_tsmm(hipStream_t st, const double* X, int64_t ldx, const double* Y, int64_t ysr,
                       int64_t ysc, int64_t N, int p, int q, double alpha, double beta, double* C,
                       int64_t ldc, double* part, int num_cu);
// out (N x k, ld ldo, FP32 or FP64) = X (N x j, ld ldx) S (j x k) in FP64;
// k <= 128; S given row by row: St[c ldst + t] = S(c, t), ldst >= 128 (the
// entries past k are read and their results dropped)
hipError_t launch_tall_mul(hipStream_t st, const double* X, int64_t ldx, int64_t N, int j,
                           const double* St, int64_t ldst, int k, void* out, bool out_f64,
                           int64_t ldo);
// out[0] = sum of squares of x[0:count] (fixed order)
hipError_t launch_sumsq(hipStream_t st, const double* x, int64_t count, double* out);

}  // namespace sid
