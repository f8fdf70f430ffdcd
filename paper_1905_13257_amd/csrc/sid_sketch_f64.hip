// sid_sketch_f64.hip -- the sketches W = Psi A and Y = A Omega in FP64
// arithmetic (the F64 sketch precision over all rows), register-tiled on the
// vector units.
//
// W's row chunks are split over the grid exactly as in the general sketch
// kernels (chunk = ceil(N / nchunks) rows, 16 rows of A staged at a time, a
// zero-padded last step), each per-chunk partial of W(r, c) is summed over
// its rows in order with fma(Psi(r, s), A(s, c), acc), and the partials are
// added in chunk order in FP64: W is the one those kernels give, bit for
// bit.  What differs is the tiling: a 256-thread block owns 128 rows of W
// (Psi's rows; 160 when that covers the rest, a last tile of 16, 32 or 64
// otherwise) by 128 columns and each thread an 8 x 8 (10 x 8) tile of them,
// so a step over one row of A reads 16 operands from LDS for 64 FMAs, and
// Psi's entries for a block of A's rows are drawn once per 128 columns.
// Psi(r, s) = G(seed, 1, s, r) (Philox4x32-10, Box-Muller in single
// precision), keyed by the row s of A.
#include "sid_device.hpp"
#include "sid_sketch_f64.hpp"

namespace sid {

namespace {

constexpr int SF_THREADS = 256;
constexpr int SF_RT = 128;  // rows of W per block
constexpr int SF_CT = 128;  // columns of W per block
constexpr int SF_RB = 16;   // rows of A per step
constexpr int SF_TI = 8;    // rows of W per thread (stride 16)
constexpr int SF_TJ = 8;    // columns of W per thread (stride 16)

// TI rows of W per thread: the block covers rows r0 .. r0 + 16 TI - 1 (a
// last, shorter row tile when lq is not a multiple of 128)
template <typename In, int TI>
__global__ __launch_bounds__(SF_THREADS) void k_sketch_w_f64_tiled(
    const In* __restrict__ A, int64_t lda, int64_t n, int64_t N, int64_t chunk, int lq, int r0,
    uint64_t seed, double* __restrict__ part) {
  constexpr int RT = 16 * TI;
  __shared__ double s_psi[SF_RB][RT];
  __shared__ double s_a[SF_RB][SF_CT];
  const int tid = threadIdx.x;
  const int tr = tid & 15, tc = tid >> 4;
  const int64_t c0 = (int64_t)blockIdx.x * SF_CT;
  const int64_t s_begin = (int64_t)blockIdx.z * chunk;
  const int64_t s_end = s_begin + chunk < N ? s_begin + chunk : N;
  double acc[TI][SF_TJ];
#pragma unroll
  for (int i = 0; i < TI; ++i)
#pragma unroll
    for (int j = 0; j < SF_TJ; ++j) acc[i][j] = 0.0;
  for (int64_t s0 = s_begin; s0 < s_end; s0 += SF_RB) {
    const int nb = (int)(s_end - s0 < SF_RB ? s_end - s0 : SF_RB);
    // Psi(r0 .. r0 + RT - 1, s0 .. s0 + 15): RT / 4 groups of 4 rows per row
    // of A
    for (int w = tid; w < SF_RB * (RT / 4); w += SF_THREADS) {
      const int ss = w / (RT / 4), g = w - ss * (RT / 4);
      float z[4] = {0.f, 0.f, 0.f, 0.f};
      if (ss < nb) gauss4(seed, 1u, (uint64_t)(s0 + ss), (uint32_t)(r0 / 4 + g), z);
#pragma unroll
      for (int e = 0; e < 4; ++e) s_psi[ss][4 * g + e] = (double)gauss_value<P_F64>(z[e]);
    }
    // A(s0 .. s0 + 15, c0 .. c0 + 127): 16 consecutive rows of a column per
    // 16 threads
    for (int w = tid; w < SF_RB * SF_CT; w += SF_THREADS) {
      const int ss = w % SF_RB, cc = w / SF_RB;
      double v = 0.0;
      if (ss < nb && c0 + cc < n) v = data_value<P_F64, double>(A[(s0 + ss) + lda * (c0 + cc)]);
      s_a[ss][cc] = v;
    }
    __syncthreads();
#pragma unroll 2
    for (int ss = 0; ss < SF_RB; ++ss) {
      double p[TI], a[SF_TJ];
#pragma unroll
      for (int i = 0; i < TI; ++i) p[i] = s_psi[ss][tr + 16 * i];
#pragma unroll
      for (int j = 0; j < SF_TJ; ++j) a[j] = s_a[ss][tc + 16 * j];
#pragma unroll
      for (int i = 0; i < TI; ++i)
#pragma unroll
        for (int j = 0; j < SF_TJ; ++j) acc[i][j] = fma(p[i], a[j], acc[i][j]);
    }
    __syncthreads();
  }
  double* dst = part + (int64_t)blockIdx.z * lq * n;
#pragma unroll
  for (int i = 0; i < TI; ++i) {
    const int r = r0 + tr + 16 * i;
#pragma unroll
    for (int j = 0; j < SF_TJ; ++j) {
      const int64_t c = c0 + tc + 16 * j;
      if (r < lq && c < n) dst[r + (int64_t)lq * c] = acc[i][j];
    }
  }
}

// Y (N x l, row-major FP64) = A Omega with Omega (n x l, row-major) the
// single-precision draws; each entry is one FMA chain over k = 0, 1, ...,
// n - 1 (zero-padded to a multiple of 16) in order, as in the general
// kernel, so Y is the same bits.  A 256-thread block owns 128 rows x 128
// columns of Y (block y: columns 128 y ..), each thread an 8 x 8 tile
// (columns tc + 16 j, so that a row's stores run along Y's rows).
template <typename In>
__global__ __launch_bounds__(SF_THREADS) void k_sketch_y_f64_tiled(
    const In* __restrict__ A, int64_t lda, int64_t N, int64_t n, const float* __restrict__ omega,
    int l, double* __restrict__ Y) {
  __shared__ double s_a[SF_RB][SF_RT];
  __shared__ double s_om[SF_RB][SF_CT];
  const int tid = threadIdx.x;
  const int tc = tid & 15, tr = tid >> 4;
  const int64_t i0 = (int64_t)blockIdx.x * SF_RT;
  const int cb = blockIdx.y * SF_CT;
  double acc[SF_TI][SF_TJ];
#pragma unroll
  for (int i = 0; i < SF_TI; ++i)
#pragma unroll
    for (int j = 0; j < SF_TJ; ++j) acc[i][j] = 0.0;
  for (int64_t k0 = 0; k0 < n; k0 += SF_RB) {
    for (int w = tid; w < SF_RB * SF_RT; w += SF_THREADS) {
      const int kk = w / SF_RT, ii = w - kk * SF_RT;
      double v = 0.0;
      if (k0 + kk < n && i0 + ii < N)
        v = data_value<P_F64, double>(A[(i0 + ii) + lda * (k0 + kk)]);
      s_a[kk][ii] = v;
    }
    for (int w = tid; w < SF_RB * SF_CT; w += SF_THREADS) {
      const int kk = w / SF_CT, cc = w - kk * SF_CT;
      double v = 0.0;
      if (k0 + kk < n && cb + cc < l) v = (double)gauss_value<P_F64>(omega[(k0 + kk) * l + cb + cc]);
      s_om[kk][cc] = v;
    }
    __syncthreads();
#pragma unroll 2
    for (int kk = 0; kk < SF_RB; ++kk) {
      double a[SF_TI], o[SF_TJ];
#pragma unroll
      for (int i = 0; i < SF_TI; ++i) a[i] = s_a[kk][tr + 16 * i];
#pragma unroll
      for (int j = 0; j < SF_TJ; ++j) o[j] = s_om[kk][tc + 16 * j];
#pragma unroll
      for (int i = 0; i < SF_TI; ++i)
#pragma unroll
        for (int j = 0; j < SF_TJ; ++j) acc[i][j] = fma(a[i], o[j], acc[i][j]);
    }
    __syncthreads();
  }
#pragma unroll
  for (int i = 0; i < SF_TI; ++i) {
    const int64_t row = i0 + tr + 16 * i;
#pragma unroll
    for (int j = 0; j < SF_TJ; ++j) {
      const int c = cb + tc + 16 * j;
      if (row < N && c < l) Y[row * (int64_t)l + c] = acc[i][j];
    }
  }
}

// W(e) = sum of the nparts partials in order (FP64)
__global__ void k_sum_partials_f64(const double* __restrict__ part, int64_t nparts, int64_t count,
                                   double* __restrict__ out) {
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < count;
       e += (int64_t)gridDim.x * blockDim.x) {
    double s = 0.0;
    for (int64_t g = 0; g < nparts; ++g) s += part[g * count + e];
    out[e] = s;
  }
}

}  // namespace

hipError_t launch_sketch_y_f64(hipStream_t st, const void* A, bool a_is_f64, int64_t lda,
                               int64_t N, int64_t n, const float* omega, int l, double* Y) {
  if (N < 1 || n < 1 || l < 1 || lda < N) return hipErrorInvalidValue;
  const dim3 grid((unsigned)((N + SF_RT - 1) / SF_RT), (unsigned)((l + SF_CT - 1) / SF_CT));
  if (a_is_f64)
    hipLaunchKernelGGL(k_sketch_y_f64_tiled<double>, grid, dim3(SF_THREADS), 0, st,
                       (const double*)A, lda, N, n, omega, l, Y);
  else
    hipLaunchKernelGGL(k_sketch_y_f64_tiled<float>, grid, dim3(SF_THREADS), 0, st,
                       (const float*)A, lda, N, n, omega, l, Y);
  return hipGetLastError();
}

hipError_t launch_sketch_w_f64(hipStream_t st, const void* A, bool a_is_f64, int64_t lda,
                               int64_t N, int64_t n, int lq, uint64_t seed, int64_t nchunks,
                               double* part, double* W) {
  if (N < 1 || n < 1 || lq < 1 || lda < N || nchunks < 1) return hipErrorInvalidValue;
  const int64_t chunk = (N + nchunks - 1) / nchunks;
  const dim3 grid((unsigned)((n + SF_CT - 1) / SF_CT), 1u, (unsigned)nchunks);
  // row tiles of 128, the last one of 16, 32, 64 or 128 rows, or one of 160
  // when 128 to 160 remain (A is read once per row tile)
  for (int r0 = 0; r0 < lq;) {
    const int left = lq - r0;
    const int ti = (left > 128 && left <= 160) ? 10
                   : left > 64 ? 8 : left > 32 ? 4 : left > 16 ? 2 : 1;
#define SID_SW(TI_)                                                                           \
  case TI_:                                                                                   \
    if (a_is_f64)                                                                             \
      hipLaunchKernelGGL((k_sketch_w_f64_tiled<double, TI_>), grid, dim3(SF_THREADS), 0, st,  \
                         (const double*)A, lda, n, N, chunk, lq, r0, seed, part);             \
    else                                                                                      \
      hipLaunchKernelGGL((k_sketch_w_f64_tiled<float, TI_>), grid, dim3(SF_THREADS), 0, st,   \
                         (const float*)A, lda, n, N, chunk, lq, r0, seed, part);              \
    break;
    switch (ti) { SID_SW(1) SID_SW(2) SID_SW(4) SID_SW(8) SID_SW(10) }
#undef SID_SW
    r0 += 16 * ti;
  }
  const int64_t count = (int64_t)lq * n;
  int64_t blocks = (count + 255) / 256;
  if (blocks > 4096) blocks = 4096;
  hipLaunchKernelGGL(k_sum_partials_f64, dim3((unsigned)blocks), dim3(256), 0, st, part, nchunks,
                     count, W);
  return hipGetLastError();
}

}  // namespace sid
