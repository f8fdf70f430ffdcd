// sid_svd.hip -- small FP64 kernels of the single-pass blocked randomized
// SVD (SBR-SVD, Alg. 2): the thin QR of a block, the triangular product
// that combines two of them, the symmetric eigensolver of B B^T, and
// conversions.  The N-length products of the algorithm run as library GEMMs.
#include <hip/hip_runtime.h>

#include "sid_device.hpp"
#include "sid_svd.hpp"

namespace sid {

namespace {

constexpr int SV_THREADS = 256;

__device__ double block_sum(double v, double* red) {
  v = wave_sum(v);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) red[wave] = v;
  __syncthreads();
  double s = 0.0;
  for (int w = 0; w < SV_THREADS / 64; ++w) s += red[w];
  return s;
}

// In-place thin QR of Y (n x b, column-major, ld n) by Gram-Schmidt with one
// reorthogonalization per column (CGS2): Y becomes Q, R (b x b, ld b) upper
// triangular.  A column whose norm after the projections is zero gets a
// zero Q column and R(c, c) = 0.
__global__ __launch_bounds__(SV_THREADS) void k_small_qr(double* __restrict__ Y, int n, int b,
                                                         double* __restrict__ R) {
  __shared__ double red[SV_THREADS / 64];
  for (int e = threadIdx.x; e < b * b; e += SV_THREADS) R[e] = 0.0;
  __syncthreads();
  for (int c = 0; c < b; ++c) {
    double* y = Y + (int64_t)n * c;
    for (int pass = 0; pass < 2; ++pass) {
      for (int d = 0; d < c; ++d) {
        const double* qd = Y + (int64_t)n * d;
        double s = 0.0;
        for (int r = threadIdx.x; r < n; r += SV_THREADS) s = fma(qd[r], y[r], s);
        s = block_sum(s, red);
        for (int r = threadIdx.x; r < n; r += SV_THREADS) y[r] = fma(-s, qd[r], y[r]);
        if (threadIdx.x == 0) R[d + b * c] += s;
        __syncthreads();
      }
    }
    double s = 0.0;
    for (int r = threadIdx.x; r < n; r += SV_THREADS) s = fma(y[r], y[r], s);
    const double nrm = sqrt(block_sum(s, red));
    const double inv = nrm > 0.0 ? 1.0 / nrm : 0.0;
    for (int r = threadIdx.x; r < n; r += SV_THREADS) y[r] *= inv;
    if (threadIdx.x == 0) R[c + b * c] = nrm;
    __syncthreads();
  }
}

// R = Rt R (both b x b upper triangular, column-major), in place in R;
// also the smallest |R(c, c)| into *mindiag
__global__ __launch_bounds__(SV_THREADS) void k_trmul(const double* __restrict__ Rt,
                                                      double* __restrict__ R, int b,
                                                      double* __restrict__ mindiag) {
  __shared__ double out[64 * 64];
  for (int e = threadIdx.x; e < b * b; e += SV_THREADS) {
    const int i = e % b, j = e / b;
    double s = 0.0;
    if (i <= j)
      for (int t = i; t <= j; ++t) s = fma(Rt[i + b * t], R[t + b * j], s);
    out[e] = s;
  }
  __syncthreads();
  for (int e = threadIdx.x; e < b * b; e += SV_THREADS) R[e] = out[e];
  if (threadIdx.x == 0) {
    double m = INFINITY;
    for (int c = 0; c < b; ++c) m = fmin(m, fabs(out[c + b * c]));
    *mindiag = m;
  }
}

// Cyclic Jacobi eigensolver of a symmetric M (m x m, column-major, ld m,
// m <= 256) in place, eigenvectors into V.  Each sweep visits every pair
// once in m' - 1 rounds of a round-robin tournament (m' = m rounded up to
// even; index m' - 1 is a dummy when m is odd), the pairs of a round being
// disjoint, so their rotations are applied in parallel: first to the rows
// of M, then to its columns and to the columns of V.  Stops when the
// off-diagonal Frobenius norm is below 1e-15 of the whole, or after 40
// sweeps.
__global__ __launch_bounds__(SV_THREADS) void k_jacobi(double* __restrict__ M, int m,
                                                       double* __restrict__ V) {
  __shared__ int pp[128], qq[128];
  __shared__ double cc[128], ss[128];
  __shared__ double red[SV_THREADS / 64];
  const int me = m + (m & 1);
  const int npairs = me / 2;
  for (int e = threadIdx.x; e < m * m; e += SV_THREADS) V[e] = (e % m == e / m) ? 1.0 : 0.0;
  __syncthreads();
  for (int sweep = 0; sweep < 40; ++sweep) {
    double off = 0.0, tot = 0.0;
    for (int e = threadIdx.x; e < m * m; e += SV_THREADS) {
      const double v = M[e];
      tot = fma(v, v, tot);
      if (e % m != e / m) off = fma(v, v, off);
    }
    off = block_sum(off, red);
    tot = block_sum(tot, red);
    if (off <= 1e-30 * tot || tot == 0.0) break;
    for (int round = 0; round < me - 1; ++round) {
      // tournament pairing: position 0 fixed, the others rotate
      for (int k = threadIdx.x; k < npairs; k += SV_THREADS) {
        auto slot = [&](int pos) { return pos == 0 ? 0 : 1 + (pos - 1 + round) % (me - 1); };
        int p = slot(k), q = slot(me - 1 - k);
        if (p > q) { const int t = p; p = q; q = t; }
        double c = 1.0, s = 0.0;
        if (q < m) {
          const double apq = M[p + (int64_t)m * q];
          if (apq != 0.0) {
            const double app = M[p + (int64_t)m * p], aqq = M[q + (int64_t)m * q];
            const double tau = (aqq - app) / (2.0 * apq);
            const double t = (tau >= 0.0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
            c = 1.0 / sqrt(1.0 + t * t);
            s = t * c;
          }
        }
        pp[k] = p;
        qq[k] = q;
        cc[k] = c;
        ss[k] = s;
      }
      __syncthreads();
      // rows p, q of M
      for (int e = threadIdx.x; e < npairs * m; e += SV_THREADS) {
        const int k = e / m, x = e - k * m;
        const int p = pp[k], q = qq[k];
        if (q >= m) continue;
        const double c = cc[k], s = ss[k];
        const double mp = M[p + (int64_t)m * x], mq = M[q + (int64_t)m * x];
        M[p + (int64_t)m * x] = c * mp - s * mq;
        M[q + (int64_t)m * x] = s * mp + c * mq;
      }
      __syncthreads();
      // columns p, q of M and of V
      for (int e = threadIdx.x; e < npairs * m; e += SV_THREADS) {
        const int k = e / m, x = e - k * m;
        const int p = pp[k], q = qq[k];
        if (q >= m) continue;
        const double c = cc[k], s = ss[k];
        const double mp = M[x + (int64_t)m * p], mq = M[x + (int64_t)m * q];
        M[x + (int64_t)m * p] = c * mp - s * mq;
        M[x + (int64_t)m * q] = s * mp + c * mq;
        const double vp = V[x + (int64_t)m * p], vq = V[x + (int64_t)m * q];
        V[x + (int64_t)m * p] = c * vp - s * vq;
        V[x + (int64_t)m * q] = s * vp + c * vq;
      }
      __syncthreads();
    }
  }
}

// Eigenvalues (diagonal of M) in descending order: S[j] = sqrt(max(lambda, 0))
// for j < k (0 beyond m), and Us (m x k) = the matching eigenvector columns of
// V divided by S[j] (0 where S[j] = 0), so that B^T Us = V_k.
__global__ __launch_bounds__(SV_THREADS) void k_eig_sort(const double* __restrict__ M, int m,
                                                         const double* __restrict__ V, int k,
                                                         double* __restrict__ S,
                                                         double* __restrict__ Us,
                                                         double* __restrict__ Uv) {
  __shared__ int order[256];
  __shared__ double lam[256];
  if (threadIdx.x == 0) {
    for (int i = 0; i < m; ++i) {
      lam[i] = M[i + (int64_t)m * i];
      order[i] = i;
    }
    for (int i = 0; i < m; ++i) {  // selection sort, descending (m <= 256)
      int best = i;
      for (int j = i + 1; j < m; ++j)
        if (lam[order[j]] > lam[order[best]]) best = j;
      const int t = order[i];
      order[i] = order[best];
      order[best] = t;
    }
  }
  __syncthreads();
  for (int j = threadIdx.x; j < k; j += SV_THREADS)
    S[j] = j < m ? sqrt(fmax(lam[order[j]], 0.0)) : 0.0;
  __syncthreads();
  for (int e = threadIdx.x; e < m * k; e += SV_THREADS) {
    const int i = e % m, j = e / m;
    const double v = j < m ? V[i + (int64_t)m * order[j]] : 0.0;
    const double sj = j < m ? sqrt(fmax(lam[order[j]], 0.0)) : 0.0;
    Uv[e] = v;
    Us[e] = sj > 0.0 ? v / sj : 0.0;
  }
}

template <typename TS, typename TD>
__global__ void k_convert(const TS* __restrict__ src, int64_t rows, int64_t cols, int64_t lds,
                          TD* __restrict__ dst, int64_t ldd) {
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < rows * cols;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t c = e / rows, r = e - c * rows;
    dst[r + ldd * c] = (TD)src[r + lds * c];
  }
}

// dst (cols x rows) = src^T (src rows x cols), both column-major
__global__ void k_transpose64(const double* __restrict__ src, int64_t rows, int64_t cols,
                              int64_t lds, double* __restrict__ dst, int64_t ldd) {
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < rows * cols;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t c = e / rows, r = e - c * rows;
    dst[c + ldd * r] = src[r + lds * c];
  }
}

unsigned grid_for(int64_t count) {
  int64_t g = (count + 255) / 256;
  if (g > 8192) g = 8192;
  if (g < 1) g = 1;
  return (unsigned)g;
}

}  // namespace

hipError_t launch_small_qr(hipStream_t st, double* Y, int n, int b, double* R) {
  if (b > 64) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_small_qr, dim3(1), dim3(SV_THREADS), 0, st, Y, n, b, R);
  return hipGetLastError();
}

hipError_t launch_trmul(hipStream_t st, const double* Rt, double* R, int b, double* mindiag) {
  if (b > 64) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_trmul, dim3(1), dim3(SV_THREADS), 0, st, Rt, R, b, mindiag);
  return hipGetLastError();
}

hipError_t launch_jacobi(hipStream_t st, double* M, int m, double* V) {
  if (m > 256) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_jacobi, dim3(1), dim3(SV_THREADS), 0, st, M, m, V);
  return hipGetLastError();
}

hipError_t launch_eig_sort(hipStream_t st, const double* M, int m, const double* V, int k,
                           double* S, double* Us, double* Uv) {
  if (m > 256) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_eig_sort, dim3(1), dim3(SV_THREADS), 0, st, M, m, V, k, S, Us, Uv);
  return hipGetLastError();
}

hipError_t launch_convert(hipStream_t st, const void* src, bool src_f64, int64_t rows,
                          int64_t cols, int64_t lds, void* dst, bool dst_f64, int64_t ldd) {
  const unsigned g = grid_for(rows * cols);
  if (src_f64 && dst_f64)
    hipLaunchKernelGGL((k_convert<double, double>), dim3(g), dim3(256), 0, st,
                       (const double*)src, rows, cols, lds, (double*)dst, ldd);
  else if (src_f64)
    hipLaunchKernelGGL((k_convert<double, float>), dim3(g), dim3(256), 0, st,
                       (const double*)src, rows, cols, lds, (float*)dst, ldd);
  else if (dst_f64)
    hipLaunchKernelGGL((k_convert<float, double>), dim3(g), dim3(256), 0, st,
                       (const float*)src, rows, cols, lds, (double*)dst, ldd);
  else
    hipLaunchKernelGGL((k_convert<float, float>), dim3(g), dim3(256), 0, st, (const float*)src,
                       rows, cols, lds, (float*)dst, ldd);
  return hipGetLastError();
}

hipError_t launch_transpose64(hipStream_t st, const double* src, int64_t rows, int64_t cols,
                              int64_t lds, double* dst, int64_t ldd) {
  hipLaunchKernelGGL(k_transpose64, dim3(grid_for(rows * cols)), dim3(256), 0, st, src, rows,
                     cols, lds, dst, ldd);
  return hipGetLastError();
}

}  // namespace sid
