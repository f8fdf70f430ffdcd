// sid_sketch_f64.hip -- the Gaussian sketch W = Psi A in FP64 arithmetic
// (the F64 sketch precision over all rows, W only: the two-pass ID and the
// pass forming G of SBR-SVD), register-tiled on the vector units.
//
// W's row chunks are split over the grid exactly as in the general sketch
// kernels (chunk = ceil(N / nchunks) rows, 16 rows of A staged at a time, a
// zero-padded last step), each per-chunk partial of W(r, c) is summed over
// its rows in order with fma(Psi(r, s), A(s, c), acc), and the partials are
// added in chunk order in FP64: W is the one those kernels give, bit for
// bit.  What differs is the tiling: a 256-thread block owns 128 rows of W
// (Psi's rows) by 128 columns and each thread an 8 x 8 tile of them, so a
// step over one row of A reads 16 operands from LDS for 64 FMAs, and Psi's
// entries for a block of A's rows are drawn once per 128 columns.
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

template <typename In>
__global__ __launch_bounds__(SF_THREADS) void k_sketch_w_f64_tiled(
    const In* __restrict__ A, int64_t lda, int64_t n, int64_t N, int64_t chunk, int lq,
    uint64_t seed, double* __restrict__ part) {
  __shared__ double s_psi[SF_RB][SF_RT];
  __shared__ double s_a[SF_RB][SF_CT];
  const int tid = threadIdx.x;
  const int tr = tid & 15, tc = tid >> 4;
  const int64_t c0 = (int64_t)blockIdx.x * SF_CT;
  const int r0 = blockIdx.y * SF_RT;
  const int64_t s_begin = (int64_t)blockIdx.z * chunk;
  const int64_t s_end = s_begin + chunk < N ? s_begin + chunk : N;
  double acc[SF_TI][SF_TJ];
#pragma unroll
  for (int i = 0; i < SF_TI; ++i)
#pragma unroll
    for (int j = 0; j < SF_TJ; ++j) acc[i][j] = 0.0;
  for (int64_t s0 = s_begin; s0 < s_end; s0 += SF_RB) {
    const int nb = (int)(s_end - s0 < SF_RB ? s_end - s0 : SF_RB);
    // Psi(r0 .. r0 + 127, s0 .. s0 + 15): 32 groups of 4 rows per row of A
    for (int w = tid; w < SF_RB * (SF_RT / 4); w += SF_THREADS) {
      const int ss = w / (SF_RT / 4), g = w - ss * (SF_RT / 4);
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
      double p[SF_TI], a[SF_TJ];
#pragma unroll
      for (int i = 0; i < SF_TI; ++i) p[i] = s_psi[ss][tr + 16 * i];
#pragma unroll
      for (int j = 0; j < SF_TJ; ++j) a[j] = s_a[ss][tc + 16 * j];
#pragma unroll
      for (int i = 0; i < SF_TI; ++i)
#pragma unroll
        for (int j = 0; j < SF_TJ; ++j) acc[i][j] = fma(p[i], a[j], acc[i][j]);
    }
    __syncthreads();
  }
  double* dst = part + (int64_t)blockIdx.z * lq * n;
#pragma unroll
  for (int i = 0; i < SF_TI; ++i) {
    const int r = r0 + tr + 16 * i;
#pragma unroll
    for (int j = 0; j < SF_TJ; ++j) {
      const int64_t c = c0 + tc + 16 * j;
      if (r < lq && c < n) dst[r + (int64_t)lq * c] = acc[i][j];
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

hipError_t launch_sketch_w_f64(hipStream_t st, const void* A, bool a_is_f64, int64_t lda,
                               int64_t N, int64_t n, int lq, uint64_t seed, int64_t nchunks,
                               double* part, double* W) {
  if (N < 1 || n < 1 || lq < 1 || lda < N || nchunks < 1) return hipErrorInvalidValue;
  const int64_t chunk = (N + nchunks - 1) / nchunks;
  const dim3 grid((unsigned)((n + SF_CT - 1) / SF_CT), (unsigned)((lq + SF_RT - 1) / SF_RT),
                  (unsigned)nchunks);
  if (a_is_f64)
    hipLaunchKernelGGL(k_sketch_w_f64_tiled<double>, grid, dim3(SF_THREADS), 0, st,
                       (const double*)A, lda, n, N, chunk, lq, seed, part);
  else
    hipLaunchKernelGGL(k_sketch_w_f64_tiled<float>, grid, dim3(SF_THREADS), 0, st,
                       (const float*)A, lda, n, N, chunk, lq, seed, part);
  const int64_t count = (int64_t)lq * n;
  int64_t blocks = (count + 255) / 256;
  if (blocks > 4096) blocks = 4096;
  hipLaunchKernelGGL(k_sum_partials_f64, dim3((unsigned)blocks), dim3(256), 0, st, part, nchunks,
                     count, W);
  return hipGetLastError();
}

}  // namespace sid
