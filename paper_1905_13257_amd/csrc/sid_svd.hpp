// sid_svd.hpp -- small FP64 kernels of SBR-SVD (Alg. 2).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace sid {

// in-place thin QR (CGS2) of Y (n x b, ld n), R (b x b, ld b); b <= 64
hipError_t launch_small_qr(hipStream_t st, double* Y, int n, int b, double* R);
// R = Rt R for b x b upper triangular factors (ld b); min |R(c, c)| into *mindiag
hipError_t launch_trmul(hipStream_t st, const double* Rt, double* R, int b, double* mindiag);
// Jacobi eigensolver of a symmetric m x m matrix (ld m, m <= 256): M becomes
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
// C (p x q, ld ldc) = X^T Y over N rows, X(g, i) = X[g + ldx i],
// Y(g, c) = Y[g ysg + c ysc]; split over tsprod_blocks(N) row slices with
// partials (part: tsprod_blocks(N) p q doubles) summed in a fixed order.
// p <= 256, q <= 64.
int64_t tsprod_blocks(int64_t N);
hipError_t launch_tsprod(hipStream_t st, const double* X, int64_t ldx, int p, const double* Y,
                         int64_t ysg, int64_t ysc, int q, int64_t N, double* part, double* C,
                         int64_t ldc);
// H (N x l, ld ldh) = A W^T in FP64 (A: N x n, ld lda, FP32 promoted exactly
// or FP64; W: l x n FP64, ld ldw >= l rounded up to 16, the rows past l read
// but unused); l <= 256
hipError_t launch_h_gemm(hipStream_t st, const void* A, bool a_f64, int64_t lda, int64_t N, int n,
                         const double* W, int64_t ldw, int l, double* H, int64_t ldh);
// dst (cols x rows, ld ldd) = src^T (rows x cols, ld lds), FP64
hipError_t launch_transpose64(hipStream_t st, const double* src, int64_t rows, int64_t cols,
                              int64_t lds, double* dst, int64_t ldd);

}  // namespace sid
