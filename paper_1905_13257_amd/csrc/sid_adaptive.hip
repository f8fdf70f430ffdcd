// sid_adaptive.hip -- tolerance-driven rank (Remark 2.2) with the held-out
// probe rows as the error estimator.
//
// For the first k' pivots J' the ID coefficients are P' = R11'^-1 R' (R' the
// first k' rows of mgsqr's R, R11' = R'(:, J') upper triangular), so the
// probe fit is W_pr(:, J') P' = Z(:, 0:k') R' with Z = W_pr(:, J) R11^-1: the
// inverse of an upper triangular matrix restricted to its leading block is
// the leading block's inverse, so one Z serves every prefix.  Each prefix
// residual is then formed entry by entry.
#include <hip/hip_runtime.h>

#include "sid_adaptive.hpp"
#include "sid_device.hpp"

namespace sid {

namespace {

// R11(a, b) = R(a, piv[b]) for a <= b < keff (row-major kcap x kcap), else 0
__global__ void k_adapt_r11(const double* __restrict__ R, int n, const int64_t* __restrict__ piv,
                            const int64_t* __restrict__ keff_p, int kcap,
                            double* __restrict__ R11) {
  const int keff = (int)*keff_p;
  for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < kcap * kcap;
       e += gridDim.x * blockDim.x) {
    const int a = e / kcap, b = e - a * kcap;
    R11[e] = (a < keff && b < keff && b >= a) ? R[(int64_t)a * n + piv[b]] : 0.0;
  }
}

// Z(r, :) R11 = W_pr(r, J) by forward substitution, one block per probe row:
// the row sits in LDS, and once z_t is known every later entry u subtracts
// z_t R11(t, u) in parallel; each thread loads its R11 entry of the next
// step before the current step's barriers (Z column-major q x kcap;
// kcap <= 256)
__global__ __launch_bounds__(256) void k_adapt_z(const double* __restrict__ W, int lq, int r0,
                                                 int q, const int64_t* __restrict__ piv,
                                                 const int64_t* __restrict__ keff_p,
                                                 const double* __restrict__ R11, int kcap,
                                                 double* __restrict__ Z) {
  const int r = blockIdx.x;
  const int u = threadIdx.x;
  const int keff = (int)*keff_p;
  __shared__ double x[256];
  __shared__ double zt;
  if (u < keff) x[u] = W[(r0 + r) + (int64_t)lq * piv[u]];
  double rn = (u < keff && keff > 0) ? R11[u] : 0.0;  // R11(0, u)
  __syncthreads();
  for (int t = 0; t < keff; ++t) {
    const double rc = rn;
    if (t + 1 < keff && u < keff) rn = R11[(t + 1) * kcap + u];
    if (u == t) {
      zt = x[t] / rc;
      Z[r + (int64_t)q * t] = zt;
    }
    __syncthreads();
    if (u > t && u < keff) x[u] = fma(-zt, rc, x[u]);
    __syncthreads();
  }
}

// One pass over the probe entries: the thread of entry (r, j) walks the
// pivots once, acc_t = W_pr(r, j) - sum_{s<t} Z(r, s) R(s, j) being the
// residual after t of them, and its block adds acc_t^2 for every prefix t
// into its row of part (blocks x (kcap + 1)), summed in a fixed order.
__global__ __launch_bounds__(256) void k_adapt_prefix(const double* __restrict__ W, int lq, int r0,
                                                      int q, int n, const double* __restrict__ Z,
                                                      const double* __restrict__ R,
                                                      const int64_t* __restrict__ keff_p,
                                                      int kcap, double* __restrict__ part) {
  const int keff = (int)*keff_p;
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const bool live = e < (int64_t)q * n;
  const int j = live ? (int)(e / q) : 0;
  const int r = live ? (int)(e - (int64_t)j * q) : 0;
  double acc = live ? W[(r0 + r) + (int64_t)lq * j] : 0.0;
  __shared__ double red[2][4];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  for (int t = 0; t <= keff; ++t) {
    const double sq = wave_sum(acc * acc);
    if (lane == 0) red[t & 1][wave] = sq;
    // the next product is independent of the reduction
    if (t < keff && live) acc = fma(-Z[r + (int64_t)q * t], R[(int64_t)t * n + j], acc);
    __syncthreads();
    if (threadIdx.x == 0)
      part[(int64_t)blockIdx.x * (kcap + 1) + t] =
          red[t & 1][0] + red[t & 1][1] + red[t & 1][2] + red[t & 1][3];
  }
}

// e2[k'] = sum of the blocks' partials (fixed order); the chosen rank is the
// smallest k' >= 1 with e2[k'] <= tol^2 e2[0] (keff unchanged if none), and
// pivots past it are marked -1 as after an early mgsqr stop
__global__ __launch_bounds__(256) void k_adapt_select(const double* __restrict__ part, int nb,
                                                      int kcap, int64_t* __restrict__ keff_p,
                                                      int64_t* __restrict__ piv,
                                                      double* __restrict__ e2, double tol) {
  const int keff = (int)*keff_p;
  __shared__ double s_e0;
  __shared__ int s_best;
  if (threadIdx.x == 0) s_best = keff;
  for (int t = threadIdx.x; t <= keff; t += 256) {
    double s = 0.0;
    for (int b = 0; b < nb; ++b) s += part[(int64_t)b * (kcap + 1) + t];
    e2[t] = s;
    if (t == 0) s_e0 = s;
  }
  __syncthreads();
  const double thr = tol * tol * s_e0;
  for (int t = 1 + threadIdx.x; t <= keff; t += 256)
    if (e2[t] <= thr) atomicMin(&s_best, t);
  __syncthreads();
  const int chosen = s_best;
  if (threadIdx.x == 0) *keff_p = chosen;
  for (int t = chosen + threadIdx.x; t < kcap; t += 256) piv[t] = -1;
}

}  // namespace

int64_t probe_adapt_blocks(int q, int n) { return ((int64_t)q * n + 255) / 256; }

hipError_t launch_probe_adapt(hipStream_t st, const double* W, int lq, int r0, int q, int n,
                              int64_t* piv, int64_t* keff, const double* R, int kcap,
                              double* R11, double* Z, double* part, double* e2, double tol) {
  if (q < 1 || kcap < 1 || kcap > 256) return hipErrorInvalidValue;
  const int64_t nb = probe_adapt_blocks(q, n);
  hipLaunchKernelGGL(k_adapt_r11, dim3(64), dim3(256), 0, st, R, n, piv, keff, kcap, R11);
  hipLaunchKernelGGL(k_adapt_z, dim3((unsigned)q), dim3(256), 0, st, W, lq, r0, q, piv, keff, R11,
                     kcap, Z);
  hipLaunchKernelGGL(k_adapt_prefix, dim3((unsigned)nb), dim3(256), 0, st, W, lq, r0, q, n, Z, R,
                     keff, kcap, part);
  hipLaunchKernelGGL(k_adapt_select, dim3(1), dim3(256), 0, st, part, (int)nb, kcap, keff, piv, e2,
                     tol);
  return hipGetLastError();
}

}  // namespace sid
