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

// In-place thin QR of Y (n x b, column-major, ld n) by classical
// Gram-Schmidt applied twice per column (CGS2): Y becomes Q, R (b x b, ld b)
// upper triangular.  Per column and pass, the projections on all earlier
// columns are formed at once (wave w takes columns w, w + 16, ...) and then
// subtracted together.  Y is worked on in LDS when n b <= QR_LDS, else in
// place.  A column whose norm after the projections is zero gets a zero Q
// column and R(c, c) = 0.
constexpr int QR_THREADS = 1024;
constexpr int QR_LDS = 14336;  // doubles (112 KiB)

template <bool SH>
__global__ __launch_bounds__(QR_THREADS) void k_small_qr(double* __restrict__ Y, int n, int b,
                                                         double* __restrict__ R) {
  __shared__ double sy[SH ? QR_LDS : 1];
  __shared__ double sr[64 * 64];
  __shared__ double sd[64];
  __shared__ double red[QR_THREADS / 64];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  double* W = SH ? sy : Y;
  if (SH)
    for (int e = threadIdx.x; e < n * b; e += QR_THREADS) sy[e] = Y[e];
  for (int e = threadIdx.x; e < b * b; e += QR_THREADS) sr[e] = 0.0;
  __syncthreads();
  for (int c = 0; c < b; ++c) {
    double* y = W + (int64_t)n * c;
    for (int pass = 0; pass < 2 && c > 0; ++pass) {
      for (int d = wave; d < c; d += QR_THREADS / 64) {
        const double* qd = W + (int64_t)n * d;
        double t = 0.0;
        for (int r = lane; r < n; r += 64) t = fma(qd[r], y[r], t);
        t = wave_sum(t);
        if (lane == 0) {
          sd[d] = t;
          sr[d + b * c] += t;
        }
      }
      __syncthreads();
      for (int r = threadIdx.x; r < n; r += QR_THREADS) {
        double v = y[r];
        for (int d = 0; d < c; ++d) v = fma(-sd[d], W[r + (int64_t)n * d], v);
        y[r] = v;
      }
      __syncthreads();
    }
    double t = 0.0;
    for (int r = threadIdx.x; r < n; r += QR_THREADS) t = fma(y[r], y[r], t);
    t = wave_sum(t);
    if (lane == 0) red[wave] = t;
    __syncthreads();
    double ss = 0.0;
    for (int w = 0; w < QR_THREADS / 64; ++w) ss += red[w];
    const double nrm = sqrt(ss);
    const double inv = nrm > 0.0 ? 1.0 / nrm : 0.0;
    for (int r = threadIdx.x; r < n; r += QR_THREADS) y[r] *= inv;
    if (threadIdx.x == 0) sr[c + b * c] = nrm;
    __syncthreads();
  }
  if (SH)
    for (int e = threadIdx.x; e < n * b; e += QR_THREADS) Y[e] = sy[e];
  for (int e = threadIdx.x; e < b * b; e += QR_THREADS) R[e] = sr[e];
}

// R = Rt R (both b x b upper triangular, column-major), in place in R;
// also the smallest |R(c, c)| into *mindiag
__global__ __launch_bounds__(SV_THREADS) void k_trmul(const double* __restrict__ Rt,
                                                      double* __restrict__ R, int b,
                                                      double* __restrict__ mindiag,
                                                      const double* __restrict__ g2, int64_t blk,
                                                      int64_t* __restrict__ state) {
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
    // the stop test: A_p Omega of rank below the columns so far means the
    // blocks before this one span it
    const int64_t stopped = blk == 0 ? 0 : state[1];
    if (!stopped) {
      const bool deficient = !(m > 1e-12 * sqrt(*g2));
      state[0] = deficient ? blk * b : (blk + 1) * b;
      state[1] = deficient ? 1 : 0;
    }
  }
}

// Cyclic Jacobi eigenvalues of a symmetric M (m x m, column-major, ld m,
// m <= 256; only its upper triangle is read) in place.  The matrix is worked on padded to m' = m rounded up
// to even (index m' - 1 a zero dummy when m is odd, never rotated), in LDS
// when m' <= 128, else in `work` (m'^2 doubles).  A sweep visits every pair
// once in m' - 1 rounds of a round-robin tournament; the pairs of a round are
// disjoint, so each 2 x 2 block M(P, R) of two pairs P, R becomes
// R_P M(P, R) R_R^T independently of the others (one thread per block).  A
// pair is rotated only while |a_pq| > 1e-15 sqrt(|a_pp a_qq|) and
// |a_pq| > 1e-300; the loop ends after a sweep without rotations, or after
// JAC_SWEEPS sweeps.  Every round's (c, s) per pair goes to rot (round t,
// pair k at rot[2 (t npairs + k)]) and the number of sweeps to *nsweeps, for
// the eigenvectors.
constexpr int JAC_THREADS = 1024;
constexpr int JAC_SWEEPS = 40;

__device__ inline int jac_slot(int pos, int round, int me) {
  // (pos - 1 + round) mod (me - 1) with both terms below me - 1
  int v = pos - 1 + round;
  v = v >= me - 1 ? v - (me - 1) : v;
  return pos == 0 ? 0 : 1 + v;
}

template <bool SH>
__global__ __launch_bounds__(JAC_THREADS) void k_jacobi(double* __restrict__ M, int m,
                                                        double* __restrict__ work,
                                                        double* __restrict__ rot,
                                                        int* __restrict__ nsweeps) {
  __shared__ double sm[SH ? 128 * 128 : 1];
  __shared__ int2 pq[128];     // the pair (p, q) of slot k
  __shared__ double2 cs[128];  // its rotation (c, s)
  __shared__ int rotated;
  const int me = m + (m & 1);
  const int npairs = me / 2;
  double* W = SH ? sm : work;
  for (int e = threadIdx.x; e < me * me; e += JAC_THREADS) {
    const int i = e % me, j = e / me;
    W[e] = (i < m && j < m) ? M[(i < j ? i : j) + (int64_t)m * (i < j ? j : i)] : 0.0;
  }
  if (threadIdx.x == 0) rotated = 0;
  __syncthreads();
  int sweep = 0;
  while (sweep < JAC_SWEEPS) {
    for (int round = 0; round < me - 1; ++round) {
      double* rr = rot + 2 * ((int64_t)(sweep * (me - 1) + round) * npairs);
      for (int k = threadIdx.x; k < npairs; k += JAC_THREADS) {
        int p = jac_slot(k, round, me), q = jac_slot(me - 1 - k, round, me);
        if (p > q) { const int t = p; p = q; q = t; }
        double c = 1.0, sn = 0.0;
        const double apq = W[p + me * q];
        const double app = W[p + me * p], aqq = W[q + me * q];
        const double ab = fabs(apq);
        if (ab > 1e-300 && ab > 1e-15 * sqrt(fabs(app) * fabs(aqq))) {
          const double tau = (aqq - app) / (2.0 * apq);
          const double t = (tau >= 0.0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
          c = 1.0 / sqrt(1.0 + t * t);
          sn = t * c;
          rotated = 1;
        }
        pq[k] = make_int2(p, q);
        cs[k] = make_double2(c, sn);
        rr[2 * k] = c;
        rr[2 * k + 1] = sn;
      }
      __syncthreads();
      for (int e = threadIdx.x; e < npairs * npairs; e += JAC_THREADS) {
        const int a = e % npairs, b = e / npairs;
        const double2 ra = cs[a], rb = cs[b];
        const double c1 = ra.x, s1 = ra.y, c2 = rb.x, s2 = rb.y;
        if (s1 == 0.0 && s2 == 0.0) continue;
        const int2 pa = pq[a], pb = pq[b];
        const int p = pa.x, q = pa.y, r = pb.x, t = pb.y;
        const double xpr = W[p + me * r], xps = W[p + me * t];
        const double xqr = W[q + me * r], xqs = W[q + me * t];
        // left: rows p, q
        const double lpr = c1 * xpr - s1 * xqr, lqr = s1 * xpr + c1 * xqr;
        const double lps = c1 * xps - s1 * xqs, lqs = s1 * xps + c1 * xqs;
        // right: columns r, t
        double ypr = c2 * lpr - s2 * lps, yps = s2 * lpr + c2 * lps;
        double yqr = c2 * lqr - s2 * lqs, yqs = s2 * lqr + c2 * lqs;
        if (a == b) {  // the rotated pair's own block: off-diagonal annihilated
          yps = 0.0;
          yqr = 0.0;
        }
        W[p + me * r] = ypr;
        W[p + me * t] = yps;
        W[q + me * r] = yqr;
        W[q + me * t] = yqs;
      }
      __syncthreads();
    }
    ++sweep;
    const bool again = rotated != 0;
    __syncthreads();
    if (!again) break;
    if (threadIdx.x == 0) rotated = 0;
    __syncthreads();
  }
  for (int e = threadIdx.x; e < m * m; e += JAC_THREADS) {
    const int i = e % m, j = e / m;
    M[e] = W[i + me * j];
  }
  if (threadIdx.x == 0) *nsweeps = sweep;
}

// Eigenvectors from the recorded rotations: row x of V (block x, one wave)
// starts as e_x and turns through every round in order, V(x, p) <-
// c V(x, p) - s V(x, q), V(x, q) <- s V(x, p) + c V(x, q); the rotation
// records are staged JV_CHUNK rounds at a time in LDS.
constexpr int JV_CHUNK = 16;

__global__ __launch_bounds__(64) void k_jacobi_vectors(const double* __restrict__ rot,
                                                       const int* __restrict__ nsweeps, int m,
                                                       double* __restrict__ V) {
  __shared__ double row[256];
  __shared__ double cs[JV_CHUNK * 128 * 2];
  const int me = m + (m & 1);
  const int npairs = me / 2;
  const int x = blockIdx.x;
  for (int j = threadIdx.x; j < me; j += 64) row[j] = j == x ? 1.0 : 0.0;
  const int64_t total = (int64_t)(*nsweeps) * (me - 1);
  for (int64_t t0 = 0; t0 < total; t0 += JV_CHUNK) {
    const int nr = (int)(total - t0 < JV_CHUNK ? total - t0 : JV_CHUNK);
    __syncthreads();
    for (int e = threadIdx.x; e < nr * npairs * 2; e += 64) cs[e] = rot[2 * t0 * npairs + e];
    __syncthreads();
    for (int u = 0; u < nr; ++u) {
      const int round = (int)((t0 + u) % (me - 1));
      for (int k = threadIdx.x; k < npairs; k += 64) {
        const double c = cs[2 * (u * npairs + k)], sn = cs[2 * (u * npairs + k) + 1];
        if (sn != 0.0) {
          int p = jac_slot(k, round, me), q = jac_slot(me - 1 - k, round, me);
          if (p > q) { const int t = p; p = q; q = t; }
          const double vp = row[p], vq = row[q];
          row[p] = c * vp - sn * vq;
          row[q] = sn * vp + c * vq;
        }
      }
      __syncthreads();
    }
  }
  __syncthreads();
  for (int j = threadIdx.x; j < m; j += 64) V[x + (int64_t)m * j] = row[j];
}

// Eigenvalues (diagonal of M) in descending order: S[j] = sqrt(max(lambda, 0))
// for j < k (0 beyond m), and Us (m x k) = the matching eigenvector columns of
// V divided by S[j] (0 where S[j] = 0), so that B^T Us = V_k.  The position
// of eigenvalue i is the number of eigenvalues before it in that order (ties
// by index).
__global__ __launch_bounds__(SV_THREADS) void k_eig_sort(const double* __restrict__ M, int m,
                                                         const double* __restrict__ V, int k,
                                                         double* __restrict__ S,
                                                         double* __restrict__ Us,
                                                         double* __restrict__ Uv) {
  __shared__ int order[256];
  __shared__ double lam[256];
  for (int i = threadIdx.x; i < m; i += SV_THREADS) {
    lam[i] = M[i + (int64_t)m * i];
    order[i] = i;  // stays a valid index should NaNs make positions collide
  }
  __syncthreads();
  for (int i = threadIdx.x; i < m; i += SV_THREADS) {
    const double li = lam[i];
    int pos = 0;
    for (int j = 0; j < m; ++j) pos += (lam[j] > li) || (lam[j] == li && j < i);
    order[pos] = i;
  }
  __syncthreads();
  for (int j = threadIdx.x; j < k; j += SV_THREADS)
    S[j] = j < m ? sqrt(fmax(lam[order[j]], 0.0)) : 0.0;
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

// H (N x l, column-major, ld ldh) = A W^T (or H += A W^T) in FP64: A (N x n, column-major,
// ld lda, FP32 promoted exactly or FP64), W (l x n, column-major, ld ldw >=
// l rounded up to 16, FP64; the rows past l are read, not used).  A workgroup of eight waves owns 128 rows and 128 columns of H
// (block y: columns 128 y ..); wave v the columns 16 v .. 16 v + 15, each
// lane two consecutive rows of them (32 accumulators).  Every step over the
// n columns of A loads one pair of entries per lane and the 16 W entries of
// the wave through the scalar cache (uniform addresses), then does 32 FMAs
// per lane in the order c = 0, 1, ..., n - 1.
constexpr int HG_ROWS = 128;
constexpr int HG_COLS = 16;
constexpr int HG_PF = 8;

template <typename T>
__global__ __launch_bounds__(512) void k_h_gemm(const T* __restrict__ A, int64_t lda,
                                                int64_t N, int n, const double* __restrict__ W,
                                                int64_t ldw, int l, double* __restrict__ H,
                                                int64_t ldh, bool accumulate) {
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int col0 = blockIdx.y * 128 + wave * HG_COLS;
  if (col0 >= l) return;
  const int ncol = l - col0 < HG_COLS ? l - col0 : HG_COLS;
  const int64_t g = (int64_t)blockIdx.x * HG_ROWS + 2 * lane;
  const bool r0 = g < N, r1 = g + 1 < N;
  // branch-free loop: rows past N read row N - 1, and W's rows l .. (l
  // rounded up to 16) - 1 are read (in bounds, ldw >= that) but never stored
  const int64_t ga = r0 ? g : N - 1, gb = r1 ? g + 1 : N - 1;
  // accumulate: the sums continue from H's entries (so H += A W^T over
  // successive column blocks gives the bits of one call over all of them)
  double acc0[HG_COLS], acc1[HG_COLS];
#pragma unroll
  for (int j = 0; j < HG_COLS; ++j) {
    const double* h = H + ldh * (int64_t)(col0 + (j < ncol ? j : ncol - 1));
    acc0[j] = (accumulate && r0) ? h[g] : 0.0;
    acc1[j] = (accumulate && r1) ? h[g + 1] : 0.0;
  }
  const double* w = W + col0;
  // A's entries run HG_PF columns ahead of the FMAs (a register ring; the
  // column index is clamped to n - 1 past the end, so every load is in bounds
  // and the loop has no branch around a memory access)
  T ra[HG_PF], rb[HG_PF];
#pragma unroll
  for (int u = 0; u < HG_PF; ++u) {
    const int64_t cc = u < n ? u : n - 1;
    ra[u] = A[ga + lda * cc];
    rb[u] = A[gb + lda * cc];
  }
  const int nfull = n - n % HG_PF;
  for (int c0 = 0; c0 < nfull; c0 += HG_PF) {
#pragma unroll
    for (int u = 0; u < HG_PF; ++u) {
      const int c = c0 + u;
      const double a0 = (double)ra[u], a1 = (double)rb[u];
      const int64_t cn = c + HG_PF < n ? c + HG_PF : n - 1;
      ra[u] = A[ga + lda * cn];
      rb[u] = A[gb + lda * cn];
      const double* wc = w + ldw * (int64_t)c;
#pragma unroll
      for (int j = 0; j < HG_COLS; ++j) {
        acc0[j] = fma(a0, wc[j], acc0[j]);
        acc1[j] = fma(a1, wc[j], acc1[j]);
      }
    }
  }
  // the last n % HG_PF columns are already in the ring
#pragma unroll
  for (int u = 0; u < HG_PF; ++u) {
    if (nfull + u < n) {
      const double a0 = (double)ra[u], a1 = (double)rb[u];
      const double* wc = w + ldw * (int64_t)(nfull + u);
#pragma unroll
      for (int j = 0; j < HG_COLS; ++j) {
        acc0[j] = fma(a0, wc[j], acc0[j]);
        acc1[j] = fma(a1, wc[j], acc1[j]);
      }
    }
  }
#pragma unroll
  for (int j = 0; j < HG_COLS; ++j) {
    if (j < ncol) {
      double* h = H + ldh * (int64_t)(col0 + j) + g;
      if (r0) h[0] = acc0[j];
      if (r1) h[1] = acc1[j];
    }
  }
}

// One block row of B^T: Bi(g, :) = (Hi(g, :) - sum_{t<j} Bt(g, t) M(t, :)) R^-1
// for every row g (N rows; Bt, Hi, Bi column-major with ld N; M j x b with
// ld ldm; R b x b upper triangular with ld b and a nonzero diagonal).  One
// thread per row with b accumulators; M passes through LDS 64 rows at a
// time and R is held in LDS; the triangular solve is forward substitution
// over the columns.  Bi may not overlap Bt(:, 0:j) or Hi.
constexpr int BU_THREADS = 256;

template <int BMAX>
__global__ __launch_bounds__(BU_THREADS) void k_block_update(const double* __restrict__ Bt,
                                                             int64_t N, int j,
                                                             const double* __restrict__ Hi,
                                                             const double* __restrict__ M,
                                                             int64_t ldm,
                                                             const double* __restrict__ R, int b,
                                                             double* __restrict__ Bi) {
  __shared__ double sm[64 * BMAX];
  __shared__ double sr[BMAX * BMAX];
  for (int e = threadIdx.x; e < b * b; e += BU_THREADS) sr[e] = R[e];
  const int64_t g = (int64_t)blockIdx.x * BU_THREADS + threadIdx.x;
  const int64_t gl = g < N ? g : N - 1;  // rows past N compute on row N - 1, store nothing
  double x[BMAX];
#pragma unroll
  for (int c = 0; c < BMAX; ++c) x[c] = c < b ? Hi[gl + N * c] : 0.0;
  for (int t0 = 0; t0 < j; t0 += 64) {
    const int tn = j - t0 < 64 ? j - t0 : 64;
    __syncthreads();
    for (int e = threadIdx.x; e < tn * b; e += BU_THREADS) {
      const int t = e % tn, c = e / tn;
      sm[t * BMAX + c] = M[(t0 + t) + ldm * c];
    }
    __syncthreads();
    for (int t = 0; t < tn; ++t) {
      const double v = Bt[gl + N * (int64_t)(t0 + t)];
#pragma unroll
      for (int c = 0; c < BMAX; ++c) x[c] = fma(-v, sm[t * BMAX + c], x[c]);
    }
  }
  __syncthreads();
  // x R^-1 by forward substitution: y_c = (x_c - sum_{t<c} y_t R(t, c)) / R(c, c)
#pragma unroll
  for (int c = 0; c < BMAX; ++c) {
    if (c < b) {
      double v = x[c];
#pragma unroll
      for (int t = 0; t < c; ++t) v = fma(-x[t], sr[t + b * c], v);
      x[c] = v / sr[c + b * c];
    }
  }
  if (g < N)
#pragma unroll
    for (int c = 0; c < BMAX; ++c)
      if (c < b) Bi[g + N * c] = x[c];
}

unsigned grid_for(int64_t count) {
  int64_t g = (count + 255) / 256;
  if (g > 8192) g = 8192;
  if (g < 1) g = 1;
  return (unsigned)g;
}

}  // namespace

hipError_t launch_small_qr(hipStream_t st, double* Y, int n, int b, double* R) {
  if (b < 1 || b > 64 || n < 1) return hipErrorInvalidValue;
  if ((int64_t)n * b <= QR_LDS)
    hipLaunchKernelGGL(k_small_qr<true>, dim3(1), dim3(QR_THREADS), 0, st, Y, n, b, R);
  else
    hipLaunchKernelGGL(k_small_qr<false>, dim3(1), dim3(QR_THREADS), 0, st, Y, n, b, R);
  return hipGetLastError();
}

hipError_t launch_trmul(hipStream_t st, const double* Rt, double* R, int b, double* mindiag,
                        const double* g2, int64_t blk, int64_t* state) {
  if (b > 64 || !g2 || !state || blk < 0) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_trmul, dim3(1), dim3(SV_THREADS), 0, st, Rt, R, b, mindiag, g2, blk, state);
  return hipGetLastError();
}

size_t jacobi_rot_doubles(int m) {
  const int me = m + (m & 1);
  return (size_t)JAC_SWEEPS * (size_t)(me - 1) * (size_t)me;
}

hipError_t launch_jacobi(hipStream_t st, double* M, int m, double* V, double* work, double* rot,
                         int* nsweeps) {
  if (m < 1 || m > 256 || !rot || !nsweeps) return hipErrorInvalidValue;
  const int me = m + (m & 1);
  if (me <= 128)
    hipLaunchKernelGGL(k_jacobi<true>, dim3(1), dim3(JAC_THREADS), 0, st, M, m, work, rot,
                       nsweeps);
  else if (work)
    hipLaunchKernelGGL(k_jacobi<false>, dim3(1), dim3(JAC_THREADS), 0, st, M, m, work, rot,
                       nsweeps);
  else
    return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_jacobi_vectors, dim3((unsigned)m), dim3(64), 0, st, rot, nsweeps, m, V);
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

hipError_t launch_h_gemm(hipStream_t st, const void* A, bool a_f64, int64_t lda, int64_t N, int n,
                         const double* W, int64_t ldw, int l, double* H, int64_t ldh,
                         bool accumulate) {
  if (N < 1 || n < 1 || l < 1 || l > 256 || ldw < (l + 15) / 16 * 16 || ldh < N || lda < N)
    return hipErrorInvalidValue;
  const dim3 grid((unsigned)((N + HG_ROWS - 1) / HG_ROWS), (unsigned)((l + 127) / 128));
  if (a_f64)
    hipLaunchKernelGGL(k_h_gemm<double>, grid, dim3(512), 0, st, (const double*)A, lda, N, n, W,
                       ldw, l, H, ldh, accumulate);
  else
    hipLaunchKernelGGL(k_h_gemm<float>, grid, dim3(512), 0, st, (const float*)A, lda, N, n, W, ldw,
                       l, H, ldh, accumulate);
  return hipGetLastError();
}

hipError_t launch_block_update(hipStream_t st, const double* Bt, int64_t N, int j,
                               const double* Hi, const double* M, int64_t ldm, const double* R,
                               int b, double* Bi) {
  if (N < 1 || j < 0 || b < 1 || b > 64 || (j > 0 && ldm < j)) return hipErrorInvalidValue;
  const dim3 grid((unsigned)((N + BU_THREADS - 1) / BU_THREADS));
  if (b <= 8)
    hipLaunchKernelGGL(k_block_update<8>, grid, dim3(BU_THREADS), 0, st, Bt, N, j, Hi, M, ldm, R,
                       b, Bi);
  else if (b <= 16)
    hipLaunchKernelGGL(k_block_update<16>, grid, dim3(BU_THREADS), 0, st, Bt, N, j, Hi, M, ldm, R,
                       b, Bi);
  else if (b <= 20)
    hipLaunchKernelGGL(k_block_update<20>, grid, dim3(BU_THREADS), 0, st, Bt, N, j, Hi, M, ldm, R,
                       b, Bi);
  else if (b <= 32)
    hipLaunchKernelGGL(k_block_update<32>, grid, dim3(BU_THREADS), 0, st, Bt, N, j, Hi, M, ldm, R,
                       b, Bi);
  else
    hipLaunchKernelGGL(k_block_update<64>, grid, dim3(BU_THREADS), 0, st, Bt, N, j, Hi, M, ldm, R,
                       b, Bi);
  return hipGetLastError();
}

hipError_t launch_transpose64(hipStream_t st, const double* src, int64_t rows, int64_t cols,
                              int64_t lds, double* dst, int64_t ldd) {
  hipLaunchKernelGGL(k_transpose64, dim3(grid_for(rows * cols)), dim3(256), 0, st, src, rows,
                     cols, lds, dst, ldd);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Tall-skinny products over the N rows (SBR-SVD's B Omega_i and B B^T, Alg. 2
// steps "B Omega_i" and the SVD of B): C = alpha X^T Y (+ beta C), X: N x p
// column-major (ld ldx), Y: N x q with entry (r, c) at Y[r ysr + c ysc];
// p, q <= 128.  Split over row ranges: a block stages 32 rows of X and Y in
// LDS at a time and each thread accumulates an 8 x 8 tile of its range's
// partial in FP64 registers (threads beyond the tiles take every G-th row of
// the 32 and their tiles are summed in a fixed order at the end); a second
// launch sums the blocks' partials in a fixed order.  HBM traffic: X and Y
// once.
// ---------------------------------------------------------------------------
constexpr int TS_THREADS = 256;
constexpr int TS_SUB = 32;
// LDS layout of a staged slice: column c of row r at r * TS_LD + c + c / 8.
// The gap after every 8 columns puts the 8-column groups that the lanes of a
// wave read together (a lane reads 8 consecutive columns of one group) on
// different banks; the row stride makes the staging writes (32 rows of one
// column) conflict-free.
constexpr int TS_LD = 145;
__device__ __forceinline__ int ts_col(int c) { return c + (c >> 3); }

__global__ __launch_bounds__(TS_THREADS) void k_tsmm_part(
    const double* __restrict__ X, int64_t ldx, const double* __restrict__ Y, int64_t ysr,
    int64_t ysc, int64_t N, int p, int q, int64_t rows_per_block, double* __restrict__ part) {
  __shared__ double s_x[TS_SUB * TS_LD];
  __shared__ double s_y[TS_SUB * TS_LD];
  const int tid = threadIdx.x;
  const int tq = (q + 7) / 8, nt = ((p + 7) / 8) * tq;
  const int G = TS_THREADS / nt;  // >= 1: nt <= 256
  const int tile = tid % nt, grp = tid / nt;
  const bool active = grp < G;
  const int ti = tile / tq, tj = tile - ti * tq;
  double acc[8][8];
#pragma unroll
  for (int a = 0; a < 8; ++a)
#pragma unroll
    for (int b = 0; b < 8; ++b) acc[a][b] = 0.0;
  const int64_t r0 = (int64_t)blockIdx.x * rows_per_block;
  const int64_t r1 = r0 + rows_per_block < N ? r0 + rows_per_block : N;
  // this thread's share of a 32-row slice (16 entries of X and of Y), loaded
  // one slice ahead into registers so that the loads of the next slice are in
  // flight while this one is multiplied.  Rows fastest for column-major X
  // (and Y with ysr == 1): 256 contiguous bytes per column; columns fastest
  // for row-contiguous Y.
  constexpr int PER = TS_SUB * 128 / TS_THREADS;
  double px[PER], py[PER];
  auto gload = [&](int64_t s0) {
#pragma unroll
    for (int t = 0; t < PER; ++t) {
      const int e = tid + TS_THREADS * t;
      const int r = e % TS_SUB, c = e / TS_SUB;
      const int64_t row = s0 + r;
      px[t] = (row < r1 && c < p) ? X[row + ldx * c] : 0.0;
      int ry, cy;
      if (ysr == 1) { ry = r; cy = c; }
      else { cy = e % 128; ry = e / 128; }
      const int64_t rowy = s0 + ry;
      py[t] = (rowy < r1 && cy < q) ? Y[rowy * ysr + cy * ysc] : 0.0;
    }
  };
  if (r0 < r1) gload(r0);
  for (int64_t s0 = r0; s0 < r1; s0 += TS_SUB) {
    __syncthreads();  // the previous slice is consumed
#pragma unroll
    for (int t = 0; t < PER; ++t) {
      const int e = tid + TS_THREADS * t;
      const int r = e % TS_SUB, c = e / TS_SUB;
      s_x[r * TS_LD + ts_col(c)] = px[t];
      int ry, cy;
      if (ysr == 1) { ry = r; cy = c; }
      else { cy = e % 128; ry = e / 128; }
      s_y[ry * TS_LD + ts_col(cy)] = py[t];
    }
    __syncthreads();
    if (s0 + TS_SUB < r1) gload(s0 + TS_SUB);
    if (active) {
      for (int r = grp; r < TS_SUB; r += G) {
        double a[8], b[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
          a[u] = s_x[r * TS_LD + 9 * ti + u];
          b[u] = s_y[r * TS_LD + 9 * tj + u];
        }
#pragma unroll
        for (int u = 0; u < 8; ++u)
#pragma unroll
          for (int v = 0; v < 8; ++v) acc[u][v] = fma(a[u], b[v], acc[u][v]);
      }
    }
  }
  // the groups' tiles, summed in group order (G > 1 only when nt <= 128:
  // nt x 64 doubles fit the two staging arrays)
  // the two staging arrays serve as one buffer of 2 x 4640 doubles
  double* red = s_x;
  for (int g = 1; g < G; ++g) {
    __syncthreads();
    if (grp == g)
#pragma unroll
      for (int u = 0; u < 8; ++u)
#pragma unroll
        for (int v = 0; v < 8; ++v) {
          const int idx = tile * 64 + u * 8 + v;  // < nt * 64 <= 8192
          if (idx < TS_SUB * TS_LD) red[idx] = acc[u][v];
          else s_y[idx - TS_SUB * TS_LD] = acc[u][v];
        }
    __syncthreads();
    if (grp == 0)
#pragma unroll
      for (int u = 0; u < 8; ++u)
#pragma unroll
        for (int v = 0; v < 8; ++v) {
          const int idx = tile * 64 + u * 8 + v;
          acc[u][v] += idx < TS_SUB * TS_LD ? red[idx] : s_y[idx - TS_SUB * TS_LD];
        }
  }
  if (grp == 0) {
    double* dst = part + (int64_t)blockIdx.x * p * q;
#pragma unroll
    for (int u = 0; u < 8; ++u)
#pragma unroll
      for (int v = 0; v < 8; ++v) {
        const int a = 8 * ti + u, c = 8 * tj + v;
        if (a < p && c < q) dst[a + p * c] = acc[u][v];
      }
  }
}

// C (p x q, ld ldc) = alpha * (fixed-order sum of the nb partials) + beta C
__global__ void k_tsmm_reduce(const double* __restrict__ part, int64_t nb, int p, int q,
                              double alpha, double beta, double* __restrict__ C, int64_t ldc) {
  const int64_t count = (int64_t)p * q;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < count;
       e += (int64_t)gridDim.x * blockDim.x) {
    double sacc[8] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    int64_t g = 0;
    for (; g + 8 <= nb; g += 8)
#pragma unroll
      for (int u = 0; u < 8; ++u) sacc[u] += part[(g + u) * count + e];
    for (; g < nb; ++g) sacc[0] += part[g * count + e];
    const double v = ((sacc[0] + sacc[1]) + (sacc[2] + sacc[3])) +
                     ((sacc[4] + sacc[5]) + (sacc[6] + sacc[7]));
    const int a = (int)(e % p);
    const int64_t c = e / p;
    double* o = C + a + ldc * c;
    *o = beta != 0.0 ? fma(alpha, v, beta * *o) : alpha * v;
  }
}

int64_t tsmm_blocks(int64_t N, int num_cu, int64_t* rows_per_block) {
  int64_t nb = 2 * (int64_t)num_cu;
  int64_t rpb = (N + nb - 1) / nb;
  rpb = (rpb + TS_SUB - 1) / TS_SUB * TS_SUB;
  if (rpb < TS_SUB) rpb = TS_SUB;
  *rows_per_block = rpb;
  return (N + rpb - 1) / rpb;
}

hipError_t launch_tsmm(hipStream_t st, const double* X, int64_t ldx, const double* Y, int64_t ysr,
                       int64_t ysc, int64_t N, int p, int q, double alpha, double beta, double* C,
                       int64_t ldc, double* part, int num_cu) {
  if (p < 1 || q < 1 || p > 128 || q > 128 || N < 1) return hipErrorInvalidValue;
  int64_t rpb = 0;
  const int64_t nb = tsmm_blocks(N, num_cu, &rpb);
  hipLaunchKernelGGL(k_tsmm_part, dim3((unsigned)nb), dim3(TS_THREADS), 0, st, X, ldx, Y, ysr, ysc,
                     N, p, q, rpb, part);
  hipLaunchKernelGGL(k_tsmm_reduce, dim3((unsigned)(((int64_t)p * q + 255) / 256)), dim3(256), 0,
                     st, part, nb, p, q, alpha, beta, C, ldc);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// out (N x k, ld ldo, FP32 or FP64) = X (N x j, column-major, ld ldx) S (j x k,
// ld lds), FP64 arithmetic: SBR-SVD's V = B^T U~ S^-1 written straight in
// the output type.  A block covers 64 rows; wave w forms output columns
// [w kq, (w+1) kq) with kq = ceil(k / 4) <= 32, one row per lane; S's entries
// are the same for a whole wave (scalar loads), X's 64 rows are read by the
// four waves of the block (the later reads hit the cache).
// ---------------------------------------------------------------------------
template <typename OutT, int KQ>
__global__ __launch_bounds__(256) void k_tall_mul(const double* __restrict__ X, int64_t ldx,
                                                  int64_t N, int j, const double* __restrict__ St,
                                                  int64_t ldst, int k, OutT* __restrict__ out,
                                                  int64_t ldo) {
  const int lane = threadIdx.x & 63;
  // the wave index, made wave-uniform for the compiler: S's entries are then
  // scalar loads shared by the wave
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int64_t r = (int64_t)blockIdx.x * 64 + lane;
  const int c0 = wave * KQ;
  double acc[KQ];
#pragma unroll
  for (int u = 0; u < KQ; ++u) acc[u] = 0.0;
  const int64_t rr = r < N ? r : N - 1;
  for (int c = 0; c < j; ++c) {
    const double x = X[rr + ldx * c];
    // S^T stored row c = (S(c, 0), S(c, 1), ...) with stride ldst: the
    // wave's KQ entries are contiguous (entries past k are read, their
    // results dropped)
    const double* srow = St + ldst * c + c0;
#pragma unroll
    for (int u = 0; u < KQ; ++u) acc[u] = fma(x, srow[u], acc[u]);
  }
  if (r < N)
#pragma unroll
    for (int u = 0; u < KQ; ++u)
      if (c0 + u < k) out[r + ldo * (c0 + u)] = (OutT)acc[u];
}

hipError_t launch_tall_mul(hipStream_t st, const double* X, int64_t ldx, int64_t N, int j,
                           const double* St, int64_t ldst, int k, void* out, bool out_f64,
                           int64_t ldo) {
  const int kq = (k + 3) / 4;
  const int kqt = kq <= 8 ? 8 : kq <= 16 ? 16 : kq <= 25 ? 25 : 32;  // the instance below
  if (k < 1 || k > 128 || j < 1 || N < 1 || ldst < 4 * kqt) return hipErrorInvalidValue;
  const dim3 grid((unsigned)((N + 63) / 64));
#define SID_TM(KQ_)                                                                              \
  if (out_f64)                                                                                   \
    hipLaunchKernelGGL((k_tall_mul<double, KQ_>), grid, dim3(256), 0, st, X, ldx, N, j, St, ldst, \
                       k, (double*)out, ldo);                                                    \
  else                                                                                           \
    hipLaunchKernelGGL((k_tall_mul<float, KQ_>), grid, dim3(256), 0, st, X, ldx, N, j, St, ldst,  \
                       k, (float*)out, ldo);
  if (kq <= 8) { SID_TM(8) }
  else if (kq <= 16) { SID_TM(16) }
  else if (kq <= 25) { SID_TM(25) }
  else { SID_TM(32) }
#undef SID_TM
  return hipGetLastError();
}

// out[0] = sum of x[e]^2 over count entries (one block, fixed order)
__global__ __launch_bounds__(256) void k_sumsq(const double* __restrict__ x, int64_t count,
                                               double* __restrict__ out) {
  __shared__ double s[256];
  double a = 0.0;
  for (int64_t e = threadIdx.x; e < count; e += 256) a = fma(x[e], x[e], a);
  s[threadIdx.x] = a;
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if ((int)threadIdx.x < h) s[threadIdx.x] += s[threadIdx.x + h];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[0] = s[0];
}

hipError_t launch_sumsq(hipStream_t st, const double* x, int64_t count, double* out) {
  hipLaunchKernelGGL(k_sumsq, dim3(1), dim3(256), 0, st, x, count, out);
  return hipGetLastError();
}

}  // namespace sid
