// sid_kernels.hpp -- launchers of the gfx950 kernels (internal to libsid).
#pragma once
#include <type_traits>
#include "sid_device.hpp"

namespace sid {

// One matrix of the batched sketch pass (device table, one entry per matrix
// in queue order).  A: FP32 column-major N x n (lda); its shares are the row
// ranges of rows_per_wg rows the single-matrix launch gives its workgroups;
// share0: the queue index of its first share in its layout class; cls: the
// class (fused_bf16_batch_class).  Outputs: part (nshares x lq
// x n FP32 partials), W (lq x n FP64, column-major), and with Y: omega (n x l
// FP32 values, row-major), omT (128 x 512 bfloat16), Y (N x l FP32,
// row-major).
struct FbBatchEntry {
  const float* A;
  int64_t lda, N;
  int n, lq, l, cls;
  uint64_t seed;
  int64_t rows_per_wg, share0, nshares;
  float* part;
  double* W;
  float* omega;
  __bf16* omT;
  float* Y;
};

hipError_t launch_fill_gaussian(hipStream_t st, uint64_t seed, uint32_t stream, int64_t major0,
                                int64_t nmajor, int64_t minor0, int64_t nminor, float* out);
hipError_t launch_sketch(hipStream_t st, int prec, bool a_is_f64, const void* A, int64_t lda,
                         int64_t N, int64_t n, const int64_t* rows, int64_t Ns, int lq,
                         uint64_t seed, int64_t nchunks, double* part, double* W,
                         const float* omega, int l, void* Y);
// mgsqr (k_cpqr_l2 / k_cpqr_coop / k_cpqr_wg).  forced (device, kmax
// entries, optional): step i takes column forced[i] as its pivot instead of
// the largest residual (a negative entry ends the factorization there)
hipError_t launch_cpqr(hipStream_t st, const double* X, int64_t ldx, int m, int nc, int kmax,
                       double rank_tol, double* Wr, double* nrm2, int64_t* piv, double* R,
                       double* Q, int64_t* keff, double* stats, const int64_t* forced = nullptr);
hipError_t launch_backsolve(hipStream_t st, const double* R, const int64_t* piv,
                            const int64_t* keff, int kcap, int nc, double* Pd, void* P,
                            int64_t ldp, bool p_is_f64);
hipError_t launch_fit_residual(hipStream_t st, const double* W, int lq, int r0, int q, int nc,
                               const int64_t* piv, const int64_t* keff, const double* Pd, int kcap,
                               const double* mix, double* part /* 2 * ceil(q nc / 256) */,
                               double* out);
hipError_t launch_omega_values(hipStream_t st, int prec, const float* z, int64_t count,
                               double* out);
hipError_t launch_ratio_sqrt(hipStream_t st, const double* stats, double* out);
hipError_t launch_gemm64(hipStream_t st, int M, int Nn, int K, const double* A, int64_t lda,
                         int tA, const double* B, int64_t ldb, int tB, double* C, int64_t ldc);
// C = alpha op(A) op(B) + beta C (beta = 0: C is not read)
// batched forms of launch_omega_values and launch_gemm64(_ab): one job per
// product, the same arithmetic as the single launch
struct OmegaJob {
  const float* z;
  int64_t count;
  double* out;
};
hipError_t launch_omega_values_batch(hipStream_t st, int prec, const OmegaJob* jobs, int njobs,
                                     int64_t max_count);
struct Gemm64Job {
  int M, Nn, K, tA, tB, pad_;
  const double* A;
  int64_t lda;
  const double* B;
  int64_t ldb;
  double* C;
  int64_t ldc;
  double alpha, beta;
};
hipError_t launch_gemm64_batch(hipStream_t st, const Gemm64Job* jobs, int njobs, int max_m,
                               int max_n);
// batched forms of the small steps after mgsqr (one job per problem, job
// blockIdx.y; the single launch's arithmetic)
struct GatherR11Job {
  const double* R;
  int64_t ldr;
  const int64_t* piv;
  const int64_t* keff;
  int kcap, pad_;
  double* R11;
};
hipError_t launch_gather_r11_batch(hipStream_t st, const GatherR11Job* jobs, int njobs);
// R11 x = rhs per column into out64 (the P solve: MODE 0; the single-pass T
// solve: MODE 1), no second output
struct TrsvJob {
  const double* R11;
  int kcap, ncols;
  const int64_t* keff;
  const int64_t* piv;
  const double* rhs;
  int64_t ldrhs;
  double* out64;
  int64_t ldo64;
};
hipError_t launch_trsv_batch(hipStream_t st, int mode, const TrsvJob* jobs, int njobs,
                             int max_kcap, int max_ncols);
struct RatioJob {
  const double* stats;
  double* out;
};
hipError_t launch_ratio_sqrt_batch(hipStream_t st, const RatioJob* jobs, int njobs);
struct GatherBlockJob {
  const double* W;
  int lq, r0, q, kcap;
  const int64_t* piv;
  const int64_t* keff;
  double* out;
};
hipError_t launch_gather_block_batch(hipStream_t st, const GatherBlockJob* jobs, int njobs,
                                     int max_total);
struct FitJob {
  const double* W;
  int lq, r0, q, nc, kcap, pad_;
  const int64_t* piv;
  const int64_t* keff;
  const double* Pd;
  const double* mix;
  double* part;
  double* out;
};
hipError_t launch_fit_residual_batch(hipStream_t st, const FitJob* jobs, int njobs,
                                     int max_qn);
hipError_t launch_gemm64_ab(hipStream_t st, int M, int Nn, int K, const double* A, int64_t lda,
                            int tA, const double* B, int64_t ldb, int tB, double alpha, double beta,
                            double* C, int64_t ldc);
hipError_t launch_add_inplace(hipStream_t st, bool f64, void* y, const void* x, int64_t count,
                              int num_cu);
// J = piv (k entries), *k_eff = *keff, err[0:2] = werr[0:2]; NULL destinations skipped
hipError_t launch_copy_results(hipStream_t st, int64_t* J, const int64_t* piv, int k,
                               int64_t* k_eff, const int64_t* keff, double* err,
                               const double* werr);
hipError_t launch_gather_r11(hipStream_t st, const double* R, int nc, const int64_t* piv,
                             const int64_t* keff, int kcap, double* R11);
hipError_t launch_gather_cols(hipStream_t st, const void* src, bool src_f64, int64_t lds,
                              int64_t rows, const int64_t* piv, const int64_t* keff, int kcap,
                              void* dst, bool dst_f64, int64_t ldd);
hipError_t launch_fp8_quantize(hipStream_t st, const void* A, bool f64, int64_t lda, int64_t N,
                               int64_t n, float* out, int64_t ldo);
hipError_t launch_gather_rows(hipStream_t st, const void* A, bool f64, int64_t lda,
                              const int64_t* rows, int64_t Ns, int64_t n, bool to_f32, double* W,
                              int64_t ldw);
hipError_t launch_gather_block(hipStream_t st, const double* W, int lq, int r0, int q,
                               const int64_t* piv, const int64_t* keff, int kcap, double* out);
hipError_t launch_small_backsolve(hipStream_t st, const double* RM, const int64_t* pivM,
                                  const int64_t* rM, int l, const double* Cm, int64_t ldc, int kc,
                                  double* Tm);
hipError_t launch_apply_t(hipStream_t st, const void* Y, bool y_f64, int64_t N, int l,
                          const double* Tm, int k, void* AJ, bool aj_f64, int64_t ldaj);
hipError_t launch_reconstruct(hipStream_t st, bool f64, const void* AJ, int64_t ldaj,
                              const void* P, int64_t ldp, int64_t N, int k, int64_t n, void* out,
                              int64_t ldo);
hipError_t launch_error_norms(hipStream_t st, bool f64, const void* A, int64_t lda,
                              const void* AJ, int64_t ldaj, const void* P, int64_t ldp, int64_t N,
                              int k, int64_t n, double* part, int64_t part_cap, double* out4);

}  // namespace sid

namespace sid {
// how the fused pass feeds the data to the bf16 matrix products
enum FusedData : int { FB_BF16 = 0, FB_BF16X2 = 1, FB_FP8 = 2 };
bool fused_bf16_supported(int64_t n, int lq, int l, int64_t lda, const void* A, bool has_rows);
// the 32x32x16 pass over workgroup pairs (sid_sketch_v2.*): widest column
// slab for a shape (0: does not apply), applicability, Omega^T size, pairs
int sketch_v2_slab(int lq, int l, bool wanty);
bool sketch_v2_supported(int64_t n, int lq, int l, bool wanty, int64_t lda, const void* A);
size_t sketch_v2_omt_elems(int l, int n);
int64_t sketch_v2_pairs(int64_t N, int num_cu, int64_t* rows_per_pair);
// y_add: Y += A Omega (the sums a separate Y + part pass would form) instead
// of Y = A Omega
hipError_t launch_sketch_v2(hipStream_t st, int dmode, const float* A, int64_t lda, int64_t N,
                            int n, int lq, int l, uint64_t seed, const float* omega, __bf16* omT,
                            int num_cu, float* part, double* W, float* Y, int64_t* nparts_out,
                            bool y_add = false, const __bf16* psi_img = nullptr);
// Psi images for launch_sketch_v2 (psi_img): the half-panel LDS images of
// Psi that the pass would generate, formed once and read by every launch
// over the same rows, seed and lq (a matrix wider than one slab, a stream's
// flushes); the bits are those of the generating pass.  0 bytes (images not
// taken) unless the shape has 4 W row tiles per half.
size_t sketch_v2_psi_image_bytes(int64_t N, int lq);
hipError_t launch_sketch_v2_psi_image(hipStream_t st, int dmode, uint64_t seed, int64_t N, int lq,
                                      __bf16* img);
int64_t fused_bf16_grid(int64_t N, int num_cu, int64_t* rows_per_wg);
bool fused_bf16_batch_supported(int64_t n, int lq, int l, int64_t lda, const void* A);
// Layout classes of the batched sketch pass (the register and LDS layout a
// matrix's shares run with): 0: W row tiles MT = 10, Y column tiles LT = 8;
// 1: MT = 10, LT = 4 (l <= 64); 2: MT = 4, LT = 4 (lq <= 64).  Without Y
// every matrix takes class 0.  The layout bounds only the register state,
// so every class gives the bits of the single-matrix pass.
constexpr int FB_NCLASS = 3;
int fused_bf16_batch_class(int lq, int l, bool want_y);
// One class of the table: entries [first, first + count), whose shares are
// numbered from 0 (share0 relative to the class), nshares in all.
struct FbBatchClass {
  int cls, first, count;
  int64_t nshares;
};
// The batched sketch pass over d_tab (count entries grouped by class; queue:
// FB_NCLASS counters): the setup (every Omega and Omega^T with Y, the
// counters cleared), one persistent launch per class (the classes may run on
// different streams once the setup is done), then the FP64 sums of every
// matrix's partials (max_n / max_lqn: the largest n and lq n of the batch).
hipError_t launch_sketch_batch_setup(hipStream_t st, int dmode, bool want_y,
                                     const FbBatchEntry* d_tab, int count, int max_n,
                                     unsigned int* queue);
hipError_t launch_sketch_batch_class(hipStream_t st, int dmode, bool want_y,
                                     const FbBatchEntry* d_tab, const FbBatchClass& k,
                                     unsigned int* queue, int num_cu);
hipError_t launch_reduce_partials_batch(hipStream_t st, const FbBatchEntry* d_tab, int count,
                                        int64_t max_lqn);
hipError_t launch_sketch_fused_bf16(hipStream_t st, int dmode, const float* A, int64_t lda,
                                    int64_t N, int n, int lq, int l, uint64_t seed,
                                    const float* omega, __bf16* omT, int num_cu, float* part,
                                    double* W, float* Y, int64_t* nparts_out,
                                    const int64_t* rows = nullptr);
hipError_t launch_sketch_fused_f32(hipStream_t st, const float* A, int64_t lda, int64_t N, int n,
                                   int lq, int l, uint64_t seed, const float* omega, float* omP,
                                   int num_cu, float* part, double* W, float* Y);
bool apply_t_mfma_supported(int k, int l, bool y_f64);
bool cpqr_coop_supported(int m, int nc);
size_t cpqr_coop_scratch_bytes(int m, int nc);
hipError_t launch_cpqr_coop(hipStream_t st, const double* X, int64_t ldx, int m, int nc, int kmax,
                            double rank_tol, void* scratch, unsigned int* sync2, int64_t* piv,
                            double* R, double* Q, int64_t* keff, double* stats,
                            bool cooperative, unsigned int* sticky,
                            const int64_t* forced = nullptr);
hipError_t launch_id_coefficients(hipStream_t st, const double* R, int nc, const int64_t* piv,
                                  const int64_t* keff, int kcap, double* R11, double* Pd,
                                  void* P, int64_t ldp, bool p_is_f64);
hipError_t launch_small_solve(hipStream_t st, const double* RM, int l, const int64_t* pivM,
                              const int64_t* rM, double* R11, const double* C, int64_t ldc, int kc,
                              double* T);
hipError_t launch_apply_t_mfma(hipStream_t st, const void* Y, bool y_f64, int64_t N, int l,
                               const double* Tm, int k, void* AJ, bool aj_f64, int64_t ldaj, int num_cu);
bool apply_t_bf16_supported(int k, int l);
hipError_t launch_apply_t_bf16(hipStream_t st, const float* Y, int64_t N, int l, const double* Tm,
                               int k, void* AJ, bool aj_f64, int64_t ldaj, int num_cu);
bool cpqr_wg_supported(int m, int nc);
// one workgroup of 512 threads, part of the residual in LDS: nc <= 512,
// m <= 134
bool cpqr_wgl_supported(int m, int nc);
hipError_t launch_cpqr_wgl(hipStream_t st, const double* X, int64_t ldx, int m, int nc, int kmax,
                           double rank_tol, int64_t* piv, double* R, double* Q, int64_t* keff,
                           double* stats, const int64_t* forced = nullptr);
hipError_t launch_cpqr_wg(hipStream_t st, const double* X, int64_t ldx, int m, int nc, int kmax,
                          double rank_tol, int64_t* piv, double* R, double* Q, int64_t* keff,
                          double* stats, const int64_t* forced = nullptr);
// One mgsqr of a batch: the arguments of launch_cpqr_wg / launch_cpqr_wgl
// (no forced order).  A batched launch runs one job per workgroup with the
// kernel instance that the single launch would pick for each of its jobs
// (cpqr_batch_instance), so every job gets the single launch's bits.
struct CpqrJob {
  const double* X;
  int64_t ldx;
  int m, nc, kmax, inst;  // inst: cpqr_batch_instance of (m, nc)
  double rank_tol;
  int64_t* piv;
  double* R;
  double* Q;
  int64_t* keff;
  double* stats;
};
// kernel instance of an (m x nc) mgsqr: > 0 for the register kernel, < 0
// for the LDS kernel (wgl = true), 0 if neither takes the shape
int cpqr_batch_instance(int m, int nc, bool wgl);
// launch_cpqr_batch's instance for jobs of any register-kernel instance
// (each job's inst field picks it), all in one launch
constexpr int CPQR_BATCH_ANY_WG = 1000;
hipError_t launch_cpqr_batch(hipStream_t st, int instance, const CpqrJob* jobs, int njobs);
// measurement probes (sid_probe): kind 0 read / 1 column stores / 2
// sequential fill of an N x n FP32 buffer, 3 / 4 the 16x16x32 / 32x32x16
// bf16 matrix-instruction loop of N rounds; sink: 8 num_cu floats
hipError_t launch_probe(hipStream_t st, int kind, void* buf, int64_t N, int64_t n, int num_cu,
                        float* sink);
}  // namespace sid
