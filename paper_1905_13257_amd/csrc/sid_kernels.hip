// sid_kernels.hip -- gfx950 kernels of the pass-efficient ID compressor.
//
// Orientation: A is N x n column-major (one snapshot per column); the column
// ID A ~ A(:, J) P is the paper's row ID (Sec. 2.4, eq. (ID)) transposed.
#include "sid_kernels.hpp"

namespace sid {

// ---------------------------------------------------------------------------
// Gaussian fill: out[t + nminor*s] = G(seed, stream, major0 + s, minor0 + t)
// ---------------------------------------------------------------------------
__global__ void k_fill_gaussian(uint64_t seed, uint32_t stream, int64_t major0, int64_t nmajor,
                                int64_t minor0, int64_t nminor, float* __restrict__ out) {
  const int64_t g0 = minor0 >> 2;
  const int64_t g1 = (minor0 + nminor + 3) >> 2;
  const int64_t ngroups = g1 - g0;
  const int64_t total = ngroups * nmajor;
  for (int64_t w = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; w < total;
       w += (int64_t)gridDim.x * blockDim.x) {
    const int64_t s = w / ngroups;
    const int64_t g = g0 + (w - s * ngroups);
    float z[4];
    gauss4(seed, stream, (uint64_t)(major0 + s), (uint32_t)g, z);
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int64_t minor = 4 * g + e;
      if (minor >= minor0 && minor < minor0 + nminor) out[(minor - minor0) + nminor * s] = z[e];
    }
  }
}

// ---------------------------------------------------------------------------
// Sketch W = Psi(:, S) A(S, :), v1 (VALU).  Grid: (column tiles of 64, row
// chunks).  Each block accumulates its chunk's partial (lq x 64) and writes
// it to part[chunk]; k_reduce_partials sums chunks in a fixed order (FP64),
// so the result is bitwise reproducible.
// Psi(r, i) = G(seed, 1, i, r) keyed by the global row i = rows[s] (or s).
// ---------------------------------------------------------------------------
template <int PREC, typename In, int RI>
__global__ __launch_bounds__(256) void k_sketch_w_v1(
    const In* __restrict__ A, int64_t lda, int64_t n, const int64_t* __restrict__ rows,
    int64_t Ns, int64_t chunk, int lq, uint64_t seed, double* __restrict__ part) {
  using T = typename std::conditional<PREC == P_F64, double, float>::type;
  constexpr int RB = (RI * sizeof(T) > 128) ? 16 : 32;
  constexpr int CT = 64;
  __shared__ T s_psi[RB][4 * RI];  // [s][r]
  __shared__ T s_a[RB][CT];        // [s][c]
  const int tid = threadIdx.x;
  const int c = tid & (CT - 1);
  const int rq = tid >> 6;  // 0..3
  const int64_t c0 = (int64_t)blockIdx.x * CT;
  const int64_t s_begin = (int64_t)blockIdx.y * chunk;
  const int64_t s_end = (s_begin + chunk < Ns) ? s_begin + chunk : Ns;
  const int lq4 = (lq + 3) >> 2;
  T acc[RI];
#pragma unroll
  for (int i = 0; i < RI; ++i) acc[i] = T(0);

  for (int64_t s0 = s_begin; s0 < s_end; s0 += RB) {
    const int nb = (int)((s_end - s0 < RB) ? s_end - s0 : RB);
    // Psi block: RB rows of A x lq sketch rows
    for (int w = tid; w < RB * lq4; w += 256) {
      const int ss = w / lq4, g = w - ss * lq4;
      float z[4] = {0.f, 0.f, 0.f, 0.f};
      if (ss < nb) {
        const int64_t gi = rows ? rows[s0 + ss] : s0 + ss;
        gauss4(seed, 1u, (uint64_t)gi, (uint32_t)g, z);
      }
#pragma unroll
      for (int e = 0; e < 4; ++e) s_psi[ss][4 * g + e] = (T)gauss_value<PREC>(z[e]);
    }
    // A block
    for (int w = tid; w < RB * CT; w += 256) {
      const int ss = w / CT, cc = w - ss * CT;
      T v = T(0);
      if (ss < nb && c0 + cc < n) {
        const int64_t gi = rows ? rows[s0 + ss] : s0 + ss;
        v = data_value<PREC, T>(A[gi + lda * (c0 + cc)]);
      }
      s_a[ss][cc] = v;
    }
    __syncthreads();
    for (int ss = 0; ss < RB; ++ss) {
      const T a = s_a[ss][c];
#pragma unroll
      for (int i = 0; i < RI; ++i) acc[i] = fma(s_psi[ss][rq + 4 * i], a, acc[i]);
    }
    __syncthreads();
  }
  if (c0 + c < n) {
    double* dst = part + (int64_t)blockIdx.y * lq * n;
#pragma unroll
    for (int i = 0; i < RI; ++i) {
      const int r = rq + 4 * i;
      if (r < lq) dst[r + (int64_t)lq * (c0 + c)] = (double)acc[i];
    }
  }
}

__global__ void k_reduce_partials(const double* __restrict__ part, int64_t nparts, int64_t count,
                                  double* __restrict__ out) {
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < count;
       e += (int64_t)gridDim.x * blockDim.x) {
    double s = 0.0;
    for (int64_t g = 0; g < nparts; ++g) s += part[g * count + e];
    out[e] = s;
  }
}

// ---------------------------------------------------------------------------
// Sketch Y = A Omega, v1 (VALU).  One block per 64-row panel; Y row-major
// (N x l), stored in T (FP64 for the F64 sketch, FP32 otherwise).  Omega is
// the n x l row-major matrix of single-precision draws; each precision maps
// it with gauss_value.
// ---------------------------------------------------------------------------
template <int PREC, typename In, int CJ>
__global__ __launch_bounds__(256) void k_sketch_y_v1(
    const In* __restrict__ A, int64_t lda, int64_t N, int64_t n,
    const float* __restrict__ omega, int l,
    typename std::conditional<PREC == P_F64, double, float>::type* __restrict__ Y) {
  using T = typename std::conditional<PREC == P_F64, double, float>::type;
  constexpr int RP = 64;
  constexpr int KC = (CJ * sizeof(T) > 128) ? 16 : 32;
  __shared__ T s_a[KC][RP];
  __shared__ T s_om[KC][4 * CJ];
  const int tid = threadIdx.x;
  const int ir = tid & (RP - 1);
  const int cq = tid >> 6;
  const int64_t i0 = (int64_t)blockIdx.x * RP;
  T acc[CJ];
#pragma unroll
  for (int j = 0; j < CJ; ++j) acc[j] = T(0);
  for (int64_t k0 = 0; k0 < n; k0 += KC) {
    for (int w = tid; w < KC * RP; w += 256) {
      const int kk = w / RP, ii = w - kk * RP;
      T v = T(0);
      if (k0 + kk < n && i0 + ii < N) v = data_value<PREC, T>(A[(i0 + ii) + lda * (k0 + kk)]);
      s_a[kk][ii] = v;
    }
    for (int w = tid; w < KC * 4 * CJ; w += 256) {
      const int kk = w / (4 * CJ), cc = w - kk * (4 * CJ);
      T v = T(0);
      if (k0 + kk < n && cc < l) v = (T)gauss_value<PREC>(omega[(k0 + kk) * l + cc]);
      s_om[kk][cc] = v;
    }
    __syncthreads();
    for (int kk = 0; kk < KC; ++kk) {
      const T a = s_a[kk][ir];
#pragma unroll
      for (int j = 0; j < CJ; ++j) acc[j] = fma(a, s_om[kk][cq + 4 * j], acc[j]);
    }
    __syncthreads();
  }
  if (i0 + ir < N) {
#pragma unroll
    for (int j = 0; j < CJ; ++j) {
      const int cc = cq + 4 * j;
      if (cc < l) Y[(i0 + ir) * (int64_t)l + cc] = acc[j];
    }
  }
}

// ---------------------------------------------------------------------------
// mgsqr: column-pivoted modified Gram-Schmidt of an m x nc matrix X (FP64,
// column-major, ld ldx), at most kmax steps (Sec. 2.4, Alg. 3-5 step 3).
// Single work-group; the residual lives in global scratch Wr (row-major
// m x nc, L2-resident at these sizes).  Step i: every live column's residual
// norm (recomputed during the previous update), argmax with ties to the
// smallest index, q_i = r_p / nu_p, R(i, j) = q_i^T r_j, r_j -= R(i, j) q_i.
// Stops early when nu_p == 0 or nu_p <= rank_tol * nu_first.
// Outputs: piv[kmax] (-1 past k_eff), R (kmax x nc row-major), Q (m x kmax
// column-major), *keff, stats[0] = sum of final residual norms^2 over live
// columns, stats[1] = ||X||_F^2.
// ---------------------------------------------------------------------------
constexpr int CPQR_THREADS = 1024;

__global__ __launch_bounds__(CPQR_THREADS) void k_cpqr_l2(
    const double* __restrict__ X, int64_t ldx, int m, int nc, int kmax, double rank_tol,
    double* __restrict__ Wr, double* __restrict__ nrm2, int64_t* __restrict__ piv,
    double* __restrict__ R, double* __restrict__ Q, int64_t* __restrict__ keff,
    double* __restrict__ stats, const int64_t* __restrict__ forced) {
  extern __shared__ double s_dyn[];
  double* s_q = s_dyn;  // m doubles
  __shared__ double s_wv[CPQR_THREADS / 64];
  __shared__ int s_wi[CPQR_THREADS / 64];
  __shared__ double s_red[CPQR_THREADS / 64];
  const int tid = threadIdx.x;
  const int lane = tid & 63, wid = tid >> 6;
  const int nw = CPQR_THREADS / 64;

  // load residual (row-major) and initial norms
  double local_tot = 0.0;
  for (int j = tid; j < nc; j += CPQR_THREADS) {
    double s = 0.0;
    for (int r = 0; r < m; ++r) {
      const double v = X[r + ldx * j];
      Wr[(int64_t)r * nc + j] = v;
      s = fma(v, v, s);
    }
    nrm2[j] = s;
    local_tot += s;
  }
  {
    double v = wave_sum(local_tot);
    if (lane == 0) s_red[wid] = v;
    __syncthreads();
    if (tid == 0) {
      double t = 0.0;
      for (int w = 0; w < nw; ++w) t += s_red[w];
      stats[1] = t;
    }
    __syncthreads();
  }
  if (tid == 0)
    for (int i = 0; i < kmax; ++i) piv[i] = -1;

  double first = -1.0;
  int k = 0;
  for (; k < kmax; ++k) {
    // argmax over live columns (dead columns carry nrm2 = -1; forced order:
    // the given column is the only candidate)
    double bv = -1.0;
    int bi = 0x7fffffff;
    const int64_t fk = forced ? forced[k] : -1;
    for (int j = tid; j < nc; j += CPQR_THREADS) {
      const double v = nrm2[j];
      if (forced && j != fk) continue;
      if (v > bv) { bv = v; bi = j; }  // j increasing: first max kept
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
      const double ov = __shfl_xor(bv, o, 64);
      const int oi = __shfl_xor(bi, o, 64);
      if (ov > bv || (ov == bv && oi < bi)) { bv = ov; bi = oi; }
    }
    if (lane == 0) { s_wv[wid] = bv; s_wi[wid] = bi; }
    __syncthreads();
    bv = s_wv[0];
    bi = s_wi[0];
    for (int w = 1; w < nw; ++w) {
      const double ov = s_wv[w];
      const int oi = s_wi[w];
      if (ov > bv || (ov == bv && oi < bi)) { bv = ov; bi = oi; }
    }
    if (bv <= 0.0) break;
    const double nu = sqrt(bv);
    if (first < 0.0) first = nu;
    else if (rank_tol > 0.0 && nu <= rank_tol * first) break;
    const int p = bi;
    const double inv = 1.0 / nu;
    for (int r = tid; r < m; r += CPQR_THREADS) {
      const double q = Wr[(int64_t)r * nc + p] * inv;
      s_q[r] = q;
      Q[r + (int64_t)m * k] = q;
    }
    __syncthreads();
    if (tid == 0) { piv[k] = p; }
    for (int j = tid; j < nc; j += CPQR_THREADS) {
      const double cur = nrm2[j];
      double coef = 0.0;
      if (j == p) {
        R[(int64_t)k * nc + j] = nu;
        for (int r = 0; r < m; ++r) Wr[(int64_t)r * nc + j] = 0.0;
        nrm2[j] = -1.0;
      } else if (cur < 0.0) {
        R[(int64_t)k * nc + j] = 0.0;
      } else {
        for (int r = 0; r < m; ++r) coef = fma(s_q[r], Wr[(int64_t)r * nc + j], coef);
        double s = 0.0;
        for (int r = 0; r < m; ++r) {
          const double v = fma(-coef, s_q[r], Wr[(int64_t)r * nc + j]);
          Wr[(int64_t)r * nc + j] = v;
          s = fma(v, v, s);
        }
        R[(int64_t)k * nc + j] = coef;
        nrm2[j] = s;
      }
    }
    __syncthreads();
  }
  // final residual energy over live columns
  double loc = 0.0;
  for (int j = tid; j < nc; j += CPQR_THREADS) {
    const double v = nrm2[j];
    if (v > 0.0) loc += v;
  }
  loc = wave_sum(loc);
  if (lane == 0) s_red[wid] = loc;
  __syncthreads();
  if (tid == 0) {
    double t = 0.0;
    for (int w = 0; w < nw; ++w) t += s_red[w];
    stats[0] = t;
    *keff = k;
  }
}

// ---------------------------------------------------------------------------
// ID coefficients (Alg. 3-5: C = R11^+ R12, P = Z [I | C]^T): for every
// non-pivot column j solve R11 x = R(0:keff, j) by back substitution, R11 =
// R(:, piv) upper triangular in pivot order; P(:, piv_i) = e_i.  One thread
// per column.  Pd: FP64 copy (k x nc, column-major ld k); P: output in
// OutT with leading dimension ldp (rows >= keff zero).
// ---------------------------------------------------------------------------
template <typename OutT>
__global__ void k_backsolve(const double* __restrict__ R, const int64_t* __restrict__ piv,
                            const int64_t* __restrict__ keff_p, int kcap, int nc,
                            double* __restrict__ Pd, OutT* __restrict__ P, int64_t ldp) {
  const int keff = (int)*keff_p;
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= nc) return;
  int pos = -1;
  for (int b = 0; b < keff; ++b)
    if (piv[b] == j) pos = b;
  double* x = Pd + (int64_t)kcap * j;
  if (pos >= 0) {
    for (int a = 0; a < kcap; ++a) x[a] = (a == pos) ? 1.0 : 0.0;
  } else {
    for (int a = keff; a < kcap; ++a) x[a] = 0.0;
    for (int a = keff - 1; a >= 0; --a) {
      const double* Ra = R + (int64_t)a * nc;
      double acc = Ra[j];
      for (int b = a + 1; b < keff; ++b) acc = fma(-Ra[piv[b]], x[b], acc);
      x[a] = acc / Ra[piv[a]];
    }
  }
  if (P) {
    for (int a = 0; a < kcap; ++a) P[a + ldp * j] = (OutT)x[a];
  }
}

// ---------------------------------------------------------------------------
// Relative residual of held-out rows: ||Wp - Wp(:, piv) Pd||_F / ||Wp||_F
// (Wp = rows [r0, r0+q) of W, lq x nc column-major), or, when `mix` is given
// (single pass), ||Wp - mix Pd||_F with mix (q x kcap, column-major ld q).
// Single block; result to *out.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_fit_residual_part(
    const double* __restrict__ W_, int lq, int r0, int q, int nc,
    const int64_t* __restrict__ piv_, const int64_t* __restrict__ keff_,
    const double* __restrict__ Pd_, int kcap, const double* __restrict__ mix_,
    double* __restrict__ part_ /* 2 x (q nc + 255) / 256 */, const FitJob* __restrict__ jobs) {
  if (jobs) {  // a batched launch: job blockIdx.y, its first (q nc + 255) / 256 blocks
    const FitJob jb = jobs[blockIdx.y];
    if ((int)blockIdx.x * 256 >= jb.q * jb.nc) return;
    W_ = jb.W;
    lq = jb.lq;
    r0 = jb.r0;
    q = jb.q;
    nc = jb.nc;
    piv_ = jb.piv;
    keff_ = jb.keff;
    Pd_ = jb.Pd;
    kcap = jb.kcap;
    mix_ = jb.mix;
    part_ = jb.part;
  }
  const auto W = to_global(W_);
  const auto piv = to_global(piv_);
  const auto keff_p = to_global(keff_);
  const auto Pd = to_global(Pd_);
  const auto mix = to_global(mix_);
  const auto part = to_global(part_);
  __shared__ double s_num[4], s_den[4];
  const int keff = (int)*keff_p;
  double num = 0.0, den = 0.0;
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e < q * nc) {
    const int j = e / q, r = r0 + (e - j * q);
    const double w = W[r + (int64_t)lq * j];
    const auto pj = Pd + (int64_t)kcap * j;
    double a0 = 0.0, a1 = 0.0;
    int t = 0;
    for (; t + 1 < keff; t += 2) {
      const double b0 = mix ? mix[(r - r0) + (int64_t)q * t] : W[r + (int64_t)lq * piv[t]];
      const double b1 = mix ? mix[(r - r0) + (int64_t)q * (t + 1)] : W[r + (int64_t)lq * piv[t + 1]];
      a0 = fma(b0, pj[t], a0);
      a1 = fma(b1, pj[t + 1], a1);
    }
    if (t < keff) {
      const double b0 = mix ? mix[(r - r0) + (int64_t)q * t] : W[r + (int64_t)lq * piv[t]];
      a0 = fma(b0, pj[t], a0);
    }
    const double d = w - (a0 + a1);
    num = d * d;
    den = w * w;
  }
  num = wave_sum(num);
  den = wave_sum(den);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  if (lane == 0) { s_num[wid] = num; s_den[wid] = den; }
  __syncthreads();
  if (threadIdx.x == 0) {
    double a = 0.0, b = 0.0;
    for (int u = 0; u < 4; ++u) { a += s_num[u]; b += s_den[u]; }
    part[2 * blockIdx.x] = a;
    part[2 * blockIdx.x + 1] = b;
  }
}

// partial sums in block order (fixed), then the ratio
__global__ void k_fit_residual_final(const double* __restrict__ part, int nparts, int q,
                                     double* __restrict__ out, const FitJob* __restrict__ jobs) {
  if (jobs) {  // a batched launch: job blockIdx.x
    const FitJob jb = jobs[blockIdx.x];
    part = jb.part;
    nparts = (jb.q * jb.nc + 255) / 256;
    q = jb.q;
    out = jb.out;
  }
  __shared__ double s_a[64], s_b[64];
  double a = 0.0, b = 0.0;
  for (int i = threadIdx.x; i < nparts; i += 64) { a += part[2 * i]; b += part[2 * i + 1]; }
  s_a[threadIdx.x] = a;
  s_b[threadIdx.x] = b;
  __syncthreads();
  if (threadIdx.x == 0) {
    double ta = 0.0, tb = 0.0;
    for (int u = 0; u < 64; ++u) { ta += s_a[u]; tb += s_b[u]; }
    *out = (q > 0 && tb > 0.0) ? sqrt(ta / tb) : (q > 0 ? 0.0 : __longlong_as_double(0x7ff8000000000000ll));
  }
}

__global__ void k_ratio_sqrt(const double* __restrict__ stats, double* __restrict__ out,
                             const RatioJob* __restrict__ jobs, int njobs) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (jobs) {  // a batched launch: job i
    if (i < njobs) {
      const RatioJob jb = jobs[i];
      *jb.out = jb.stats[1] > 0.0 ? sqrt(jb.stats[0] / jb.stats[1]) : 0.0;
    }
    return;
  }
  if (i == 0) *out = stats[1] > 0.0 ? sqrt(stats[0] / stats[1]) : 0.0;
}

// ---------------------------------------------------------------------------
// Small FP64 GEMM: C (M x Nn, col-major ldc) = alpha * opA(A) opB(B), with
// opX = transpose when tX != 0.  A: M x K (or K x M transposed), col-major.
// Used for the l x l and l x k products of the single-pass solve.
// ---------------------------------------------------------------------------
// one 16 x 16 tile (bx, by) of C = alpha op(A) op(B) + beta C
__device__ __forceinline__ void gemm64_tile(int bx, int by, int M, int Nn, int K,
                                            const __attribute__((address_space(1))) double* __restrict__ A,
                                            int64_t lda, int tA,
                                            const __attribute__((address_space(1))) double* __restrict__ B,
                                            int64_t ldb, int tB,
                                            __attribute__((address_space(1))) double* __restrict__ C,
                                            int64_t ldc, double alpha, double beta) {
  __shared__ double sa[16][17], sb[16][17];
  const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
  const int row = bx * 16 + tx;
  const int col = by * 16 + ty;
  double acc = 0.0;
  for (int k0 = 0; k0 < K; k0 += 16) {
    {
      const int r = bx * 16 + tx, kk = k0 + ty;
      double v = 0.0;
      if (r < M && kk < K) v = tA ? A[kk + lda * r] : A[r + lda * kk];
      sa[tx][ty] = v;
    }
    {
      const int kk = k0 + tx, c = by * 16 + ty;
      double v = 0.0;
      if (kk < K && c < Nn) v = tB ? B[c + ldb * kk] : B[kk + ldb * c];
      sb[tx][ty] = v;
    }
    __syncthreads();
#pragma unroll
    for (int t = 0; t < 16; ++t) acc = fma(sa[tx][t], sb[t][ty], acc);
    __syncthreads();
  }
  if (row < M && col < Nn) {
    __attribute__((address_space(1))) double* o = C + row + ldc * col;
    *o = beta != 0.0 ? fma(alpha, acc, beta * *o) : (alpha == 1.0 ? acc : alpha * acc);
  }
}

__global__ void k_gemm64(int M, int Nn, int K, const double* __restrict__ A, int64_t lda, int tA,
                         const double* __restrict__ B, int64_t ldb, int tB, double* __restrict__ C,
                         int64_t ldc, double alpha, double beta) {
  gemm64_tile(blockIdx.x, blockIdx.y, M, Nn, K, to_global(A), lda, tA, to_global(B), ldb, tB,
              to_global(C), ldc, alpha, beta);
}

// many products in one launch: job blockIdx.z, its tiles (bx, by) (blocks
// past a job's tile grid return)
__global__ void k_gemm64_batch(const Gemm64Job* __restrict__ jobs) {
  const Gemm64Job jb = jobs[blockIdx.z];
  if ((int)blockIdx.x * 16 >= jb.M || (int)blockIdx.y * 16 >= jb.Nn) return;
  gemm64_tile(blockIdx.x, blockIdx.y, jb.M, jb.Nn, jb.K, to_global(jb.A), jb.lda, jb.tA,
              to_global(jb.B), jb.ldb, jb.tB, to_global(jb.C), jb.ldc, jb.alpha, jb.beta);
}

// gather columns: dst(:, t) = src(:, piv[t]) for t < keff, zero for keff <= t < kcap
template <typename TS, typename TD>
__global__ void k_gather_cols(const TS* __restrict__ src, int64_t lds, int64_t rows,
                              const int64_t* __restrict__ piv, const int64_t* __restrict__ keff_p,
                              int kcap, TD* __restrict__ dst, int64_t ldd) {
  const int keff = (int)*keff_p;
  const int t = blockIdx.y;
  const TS* s = (t < keff) ? src + lds * piv[t] : nullptr;
  TD* d = dst + ldd * t;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < rows;
       i += (int64_t)gridDim.x * blockDim.x)
    d[i] = s ? (TD)s[i] : (TD)0;
}

// rows of the data as FP64 values: W(i, j) = A(rows[i], j) (rounded to
// single precision first when to_f32)
template <typename TS>
__global__ void k_gather_rows(const TS* __restrict__ A, int64_t lda, const int64_t* __restrict__ rows,
                              int64_t Ns, int64_t n, int to_f32, double* __restrict__ W, int64_t ldw) {
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < Ns * n;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t j = e / Ns, i = e - j * Ns;
    const TS a = A[rows[i] + lda * j];
    W[i + ldw * j] = to_f32 ? (double)(float)a : (double)a;
  }
}

// gather rows of a column-major FP64 matrix into a (q x k) block: out(r, t) = W(r0 + r, piv[t])
__global__ void k_gather_block(const double* __restrict__ W, int lq, int r0, int q,
                               const int64_t* __restrict__ piv, const int64_t* __restrict__ keff_p,
                               int kcap, double* __restrict__ out,
                               const GatherBlockJob* __restrict__ jobs) {
  if (jobs) {  // a batched launch: job blockIdx.y
    const GatherBlockJob jb = jobs[blockIdx.y];
    W = jb.W;
    lq = jb.lq;
    r0 = jb.r0;
    q = jb.q;
    piv = jb.piv;
    keff_p = jb.keff;
    kcap = jb.kcap;
    out = jb.out;
  }
  const int keff = (int)*keff_p;
  for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < q * kcap; e += gridDim.x * blockDim.x) {
    const int t = e / q, r = e - t * q;
    out[e] = (t < keff) ? W[(r0 + r) + (int64_t)lq * piv[t]] : 0.0;
  }
}

// T(K_b, :) = R_M11^{-1} C(b, :) for the pivoted rows of the small solve;
// rows of T not in K are zero.  C is rM x kc (col-major ld ldc_), R_M is the
// (kcapM x l) row-major R of mgsqr on M, pivots pivM.  One thread per column.
__global__ void k_small_backsolve(const double* __restrict__ RM, const int64_t* __restrict__ pivM,
                                  const int64_t* __restrict__ rM_p, int l,
                                  const double* __restrict__ Cm, int64_t ldc_, int kc,
                                  double* __restrict__ Tm /* l x kc col-major ld l */) {
  const int rM = (int)*rM_p;
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= kc) return;
  double* t = Tm + (int64_t)l * j;
  for (int a = 0; a < l; ++a) t[a] = 0.0;
  for (int a = rM - 1; a >= 0; --a) {
    double acc = Cm[a + ldc_ * j];
    for (int b = a + 1; b < rM; ++b) acc = fma(-RM[(int64_t)a * l + pivM[b]], t[pivM[b]], acc);
    t[pivM[a]] = acc / RM[(int64_t)a * l + pivM[a]];
  }
}

// ---------------------------------------------------------------------------
// Single-pass skeleton estimate AJ = Y T: Y (N x l row-major, TY), T (l x k
// col-major FP64, converted once to float in LDS for the FP32 path), AJ N x k
// column-major (ld ldaj) in OutT.  One thread per row i, all k columns.
// ---------------------------------------------------------------------------
template <typename TY, typename OutT>
__global__ __launch_bounds__(256) void k_apply_t(const TY* __restrict__ Y, int64_t N, int l,
                                                 const double* __restrict__ Tm, int k,
                                                 OutT* __restrict__ AJ, int64_t ldaj) {
  using TC = typename std::conditional<std::is_same<TY, double>::value, double, float>::type;
  constexpr int KB = 16;
  extern __shared__ unsigned char s_raw[];
  TC* s_t = reinterpret_cast<TC*>(s_raw);  // l x KB
  const int t0 = blockIdx.y * KB;
  for (int e = threadIdx.x; e < l * KB; e += blockDim.x) {
    const int c = e % l, u = e / l;
    s_t[e] = (t0 + u < k) ? (TC)Tm[c + (int64_t)l * (t0 + u)] : TC(0);
  }
  __syncthreads();
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= N) return;
  const TY* y = Y + i * l;
  TC acc[KB];
#pragma unroll
  for (int u = 0; u < KB; ++u) acc[u] = TC(0);
  for (int c = 0; c < l; ++c) {
    const TC yv = (TC)y[c];
#pragma unroll
    for (int u = 0; u < KB; ++u) acc[u] = fma(yv, s_t[c + l * u], acc[u]);
  }
#pragma unroll
  for (int u = 0; u < KB; ++u)
    if (t0 + u < k) AJ[i + ldaj * (t0 + u)] = (OutT)acc[u];
}

// ---------------------------------------------------------------------------
// Reconstruction Ahat = AJ P (eq. (ID)) and fused error norms.
// Block: 256 threads = 64 rows x 4 column groups; P tile in LDS.
// ---------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(256) void k_reconstruct(const T* __restrict__ AJ, int64_t ldaj,
                                                     const T* __restrict__ P, int64_t ldp,
                                                     int64_t N, int k, int64_t n,
                                                     T* __restrict__ out, int64_t ldo) {
  using TC = typename std::conditional<std::is_same<T, double>::value, double, float>::type;
  constexpr int CB = 32;
  extern __shared__ unsigned char s_raw[];
  TC* s_p = reinterpret_cast<TC*>(s_raw);  // k x CB
  const int64_t j0 = (int64_t)blockIdx.y * CB;
  for (int e = threadIdx.x; e < k * CB; e += blockDim.x) {
    const int t = e % k, c = e / k;
    s_p[t + k * c] = (j0 + c < n) ? (TC)P[t + ldp * (j0 + c)] : TC(0);
  }
  __syncthreads();
  const int64_t i = blockIdx.x * (int64_t)64 + (threadIdx.x & 63);
  const int cg = threadIdx.x >> 6;
  if (i >= N) return;
  // each AJ entry is loaded once for the lane's 8 columns (cg, cg + 4, ...);
  // every sum runs over t in increasing order
  TC acc[CB / 4];
#pragma unroll
  for (int u = 0; u < CB / 4; ++u) acc[u] = 0;
  for (int t = 0; t < k; ++t) {
    const TC a = (TC)AJ[i + ldaj * t];
#pragma unroll
    for (int u = 0; u < CB / 4; ++u) acc[u] = fma(a, s_p[t + k * (cg + 4 * u)], acc[u]);
  }
#pragma unroll
  for (int u = 0; u < CB / 4; ++u) {
    const int c = cg + 4 * u;
    if (j0 + c < n) out[i + ldo * (j0 + c)] = (T)acc[u];
  }
}

template <typename T>
__global__ __launch_bounds__(256) void k_error_norms(const T* __restrict__ A, int64_t lda,
                                                     const T* __restrict__ AJ, int64_t ldaj,
                                                     const T* __restrict__ P, int64_t ldp,
                                                     int64_t N, int k, int64_t n,
                                                     double* __restrict__ part /* 4 per block */) {
  constexpr int CB = 32;
  extern __shared__ unsigned char s_raw[];
  double* s_p = reinterpret_cast<double*>(s_raw);  // k x CB
  __shared__ double s_r[4][4];
  const int64_t j0 = (int64_t)blockIdx.y * CB;
  for (int e = threadIdx.x; e < k * CB; e += blockDim.x) {
    const int t = e % k, c = e / k;
    s_p[t + k * c] = (j0 + c < n) ? (double)P[t + ldp * (j0 + c)] : 0.0;
  }
  __syncthreads();
  const int64_t i = blockIdx.x * (int64_t)64 + (threadIdx.x & 63);
  const int cg = threadIdx.x >> 6;
  double se = 0.0, sa = 0.0, mrel = 0.0, mabs = 0.0;
  if (i < N) {
    // each AJ entry is loaded once for the lane's 8 columns (cg, cg + 4,
    // ...); every sum runs over t in increasing order
    double accs[CB / 4];
#pragma unroll
    for (int u = 0; u < CB / 4; ++u) accs[u] = 0.0;
    for (int t = 0; t < k; ++t) {
      const double x = (double)AJ[i + ldaj * t];
#pragma unroll
      for (int u = 0; u < CB / 4; ++u) accs[u] = fma(x, s_p[t + k * (cg + 4 * u)], accs[u]);
    }
#pragma unroll
    for (int u = 0; u < CB / 4; ++u) {
      const int c = cg + 4 * u;
      if (j0 + c >= n) continue;
      const double acc = accs[u];
      const double a = (double)A[i + lda * (j0 + c)];
      const double d = a - acc;
      se = fma(d, d, se);
      sa = fma(a, a, sa);
      const double ad = fabs(d);
      mabs = fmax(mabs, ad);
      if (a != 0.0) mrel = fmax(mrel, ad / fabs(a));
    }
  }
  se = wave_sum(se);
  sa = wave_sum(sa);
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    mrel = fmax(mrel, __shfl_xor(mrel, o, 64));
    mabs = fmax(mabs, __shfl_xor(mabs, o, 64));
  }
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  if (lane == 0) { s_r[wid][0] = se; s_r[wid][1] = sa; s_r[wid][2] = mrel; s_r[wid][3] = mabs; }
  __syncthreads();
  if (threadIdx.x == 0) {
    double a = 0, b = 0, c = 0, d = 0;
    for (int w = 0; w < 4; ++w) {
      a += s_r[w][0]; b += s_r[w][1]; c = fmax(c, s_r[w][2]); d = fmax(d, s_r[w][3]);
    }
    double* o = part + 4 * ((int64_t)blockIdx.y * gridDim.x + blockIdx.x);
    o[0] = a; o[1] = b; o[2] = c; o[3] = d;
  }
}

__global__ void k_reduce_norms(const double* __restrict__ part, int64_t nb, double* __restrict__ out) {
  __shared__ double s[4][256];
  double a = 0, b = 0, c = 0, d = 0;
  for (int64_t e = threadIdx.x; e < nb; e += blockDim.x) {
    a += part[4 * e]; b += part[4 * e + 1];
    c = fmax(c, part[4 * e + 2]); d = fmax(d, part[4 * e + 3]);
  }
  s[0][threadIdx.x] = a; s[1][threadIdx.x] = b; s[2][threadIdx.x] = c; s[3][threadIdx.x] = d;
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int t = 1; t < (int)blockDim.x; ++t) {
      a += s[0][t]; b += s[1][t]; c = fmax(c, s[2][t]); d = fmax(d, s[3][t]);
    }
    out[0] = sqrt(a); out[1] = sqrt(b); out[2] = c; out[3] = d;
  }
}

// Omega as the sketch precision stores it, widened to FP64
template <int PREC>
__global__ void k_omega_values(const float* __restrict__ z, int64_t count, double* __restrict__ out) {
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < count;
       e += (int64_t)gridDim.x * blockDim.x)
    out[e] = (double)gauss_value<PREC>(z[e]);
}

// many value arrays in one launch: job blockIdx.y
template <int PREC>
__global__ void k_omega_values_batch(const OmegaJob* __restrict__ jobs) {
  const OmegaJob jb = jobs[blockIdx.y];
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < jb.count;
       e += (int64_t)gridDim.x * blockDim.x)
    jb.out[e] = (double)gauss_value<PREC>(jb.z[e]);
}

// ---------------------------------------------------------------------------
// explicit instantiations / launchers
// ---------------------------------------------------------------------------
hipError_t launch_fill_gaussian(hipStream_t st, uint64_t seed, uint32_t stream, int64_t major0,
                                int64_t nmajor, int64_t minor0, int64_t nminor, float* out) {
  const int64_t groups = ((minor0 + nminor + 3) >> 2) - (minor0 >> 2);
  const int64_t total = groups * nmajor;
  int64_t blocks = (total + 255) / 256;
  if (blocks < 1) blocks = 1;
  if (blocks > 65535) blocks = 65535;
  hipLaunchKernelGGL(k_fill_gaussian, dim3((unsigned)blocks), dim3(256), 0, st, seed, stream,
                     major0, nmajor, minor0, nminor, out);
  return hipGetLastError();
}

template <int PREC, typename In>
static hipError_t sketch_w_dispatch(hipStream_t st, const In* A, int64_t lda, int64_t n,
                                    const int64_t* rows, int64_t Ns, int lq, uint64_t seed,
                                    int64_t nchunks, double* part) {
  const int64_t chunk = (Ns + nchunks - 1) / nchunks;
  const dim3 grid((unsigned)((n + 63) / 64), (unsigned)nchunks);
  const int lq4 = (lq + 3) / 4;
#define SID_W(RI)                                                                               \
  hipLaunchKernelGGL((k_sketch_w_v1<PREC, In, RI>), grid, dim3(256), 0, st, A, lda, n, rows, Ns, \
                     chunk, lq, seed, part)
  if (lq4 <= 16) SID_W(16);
  else if (lq4 <= 32) SID_W(32);
  else if (lq4 <= 64) SID_W(64);
  else return hipErrorInvalidValue;
#undef SID_W
  return hipGetLastError();
}

template <int PREC, typename In>
static hipError_t sketch_y_dispatch(hipStream_t st, const In* A, int64_t lda, int64_t N,
                                    int64_t n, const float* omega, int l, void* Y) {
  using T = typename std::conditional<PREC == P_F64, double, float>::type;
  const dim3 grid((unsigned)((N + 63) / 64));
  const int l4 = (l + 3) / 4;
#define SID_Y(CJ)                                                                         \
  hipLaunchKernelGGL((k_sketch_y_v1<PREC, In, CJ>), grid, dim3(256), 0, st, A, lda, N, n, \
                     omega, l, (T*)Y)
  if (l4 <= 16) SID_Y(16);
  else if (l4 <= 32) SID_Y(32);
  else if (l4 <= 64) SID_Y(64);
  else return hipErrorInvalidValue;
#undef SID_Y
  return hipGetLastError();
}

hipError_t launch_sketch(hipStream_t st, int prec, bool a_is_f64, const void* A, int64_t lda,
                         int64_t N, int64_t n, const int64_t* rows, int64_t Ns, int lq,
                         uint64_t seed, int64_t nchunks, double* part, double* W,
                         const float* omega, int l, void* Y) {
  hipError_t e = hipSuccess;
#define SID_DISPATCH(P)                                                                         \
  if (a_is_f64) {                                                                               \
    e = sketch_w_dispatch<P, double>(st, (const double*)A, lda, n, rows, Ns, lq, seed, nchunks, \
                                     part);                                                     \
    if (e == hipSuccess && Y) e = sketch_y_dispatch<P, double>(st, (const double*)A, lda, N, n, \
                                                               omega, l, Y);                    \
  } else {                                                                                      \
    e = sketch_w_dispatch<P, float>(st, (const float*)A, lda, n, rows, Ns, lq, seed, nchunks,   \
                                    part);                                                      \
    if (e == hipSuccess && Y) e = sketch_y_dispatch<P, float>(st, (const float*)A, lda, N, n,   \
                                                              omega, l, Y);                     \
  }
  switch (prec) {
    case P_F64: SID_DISPATCH(P_F64); break;
    case P_F32: SID_DISPATCH(P_F32); break;
    case P_BF16: SID_DISPATCH(P_BF16); break;
    case P_BF16X2: SID_DISPATCH(P_BF16X2); break;
    case P_FP8: SID_DISPATCH(P_FP8); break;  // A holds the e4m3 values (launch_fp8_quantize)
    default: return hipErrorInvalidValue;
  }
#undef SID_DISPATCH
  if (e != hipSuccess) return e;
  const int64_t count = (int64_t)lq * n;
  int64_t blocks = (count + 255) / 256;
  if (blocks > 4096) blocks = 4096;
  hipLaunchKernelGGL(k_reduce_partials, dim3((unsigned)blocks), dim3(256), 0, st, part, nchunks,
                     count, W);
  return hipGetLastError();
}

hipError_t launch_cpqr(hipStream_t st, const double* X, int64_t ldx, int m, int nc, int kmax,
                       double rank_tol, double* Wr, double* nrm2, int64_t* piv, double* R,
                       double* Q, int64_t* keff, double* stats, const int64_t* forced) {
  const size_t shm = sizeof(double) * (size_t)m;
  hipLaunchKernelGGL(k_cpqr_l2, dim3(1), dim3(CPQR_THREADS), shm, st, X, ldx, m, nc, kmax,
                     rank_tol, Wr, nrm2, piv, R, Q, keff, stats, forced);
  return hipGetLastError();
}

hipError_t launch_backsolve(hipStream_t st, const double* R, const int64_t* piv,
                            const int64_t* keff, int kcap, int nc, double* Pd, void* P,
                            int64_t ldp, bool p_is_f64) {
  const size_t shm = 0;
  const dim3 grid((unsigned)((nc + 127) / 128));
  if (p_is_f64)
    hipLaunchKernelGGL(k_backsolve<double>, grid, dim3(128), shm, st, R, piv, keff, kcap, nc, Pd,
                       (double*)P, ldp);
  else
    hipLaunchKernelGGL(k_backsolve<float>, grid, dim3(128), shm, st, R, piv, keff, kcap, nc, Pd,
                       (float*)P, ldp);
  return hipGetLastError();
}

hipError_t launch_fit_residual(hipStream_t st, const double* W, int lq, int r0, int q, int nc,
                               const int64_t* piv, const int64_t* keff, const double* Pd, int kcap,
                               const double* mix, double* part, double* out) {
  const int nparts = (q * nc + 255) / 256;
  if (nparts > 0)
    hipLaunchKernelGGL(k_fit_residual_part, dim3((unsigned)nparts), dim3(256), 0, st, W, lq, r0, q,
                       nc, piv, keff, Pd, kcap, mix, part, (const FitJob*)nullptr);
  hipLaunchKernelGGL(k_fit_residual_final, dim3(1), dim3(64), 0, st, part, nparts, q, out,
                     (const FitJob*)nullptr);
  return hipGetLastError();
}

hipError_t launch_fit_residual_batch(hipStream_t st, const FitJob* jobs, int njobs, int max_qn) {
  if (njobs <= 0) return hipSuccess;
  const double* dn = nullptr;
  const int64_t* in = nullptr;
  const int nparts = (max_qn + 255) / 256;
  if (nparts > 0)
    hipLaunchKernelGGL(k_fit_residual_part, dim3((unsigned)nparts, (unsigned)njobs), dim3(256), 0, st,
                       dn, 0, 0, 0, 0, in, in, dn, 0, dn, (double*)nullptr, jobs);
  hipLaunchKernelGGL(k_fit_residual_final, dim3((unsigned)njobs), dim3(64), 0, st, dn, 0, 0,
                     (double*)nullptr, jobs);
  return hipGetLastError();
}

hipError_t launch_ratio_sqrt(hipStream_t st, const double* stats, double* out) {
  hipLaunchKernelGGL(k_ratio_sqrt, dim3(1), dim3(64), 0, st, stats, out, (const RatioJob*)nullptr, 0);
  return hipGetLastError();
}

hipError_t launch_ratio_sqrt_batch(hipStream_t st, const RatioJob* jobs, int njobs) {
  if (njobs <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_ratio_sqrt, dim3((unsigned)((njobs + 63) / 64)), dim3(64), 0, st,
                     (const double*)nullptr, (double*)nullptr, jobs, njobs);
  return hipGetLastError();
}

hipError_t launch_omega_values(hipStream_t st, int prec, const float* z, int64_t count,
                               double* out) {
  int64_t b = (count + 255) / 256;
  if (b > 4096) b = 4096;
  if (b < 1) b = 1;
  switch (prec) {
    case P_F64: hipLaunchKernelGGL(k_omega_values<P_F64>, dim3((unsigned)b), dim3(256), 0, st, z, count, out); break;
    case P_F32: hipLaunchKernelGGL(k_omega_values<P_F32>, dim3((unsigned)b), dim3(256), 0, st, z, count, out); break;
    case P_BF16: hipLaunchKernelGGL(k_omega_values<P_BF16>, dim3((unsigned)b), dim3(256), 0, st, z, count, out); break;
    case P_BF16X2: hipLaunchKernelGGL(k_omega_values<P_BF16X2>, dim3((unsigned)b), dim3(256), 0, st, z, count, out); break;
    case P_FP8: hipLaunchKernelGGL(k_omega_values<P_FP8>, dim3((unsigned)b), dim3(256), 0, st, z, count, out); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_omega_values_batch(hipStream_t st, int prec, const OmegaJob* jobs, int njobs,
                                     int64_t max_count) {
  if (njobs <= 0) return hipSuccess;
  int64_t b = (max_count + 255) / 256;
  if (b > 4096) b = 4096;
  if (b < 1) b = 1;
  const dim3 g((unsigned)b, (unsigned)njobs);
  switch (prec) {
    case P_F64: hipLaunchKernelGGL(k_omega_values_batch<P_F64>, g, dim3(256), 0, st, jobs); break;
    case P_F32: hipLaunchKernelGGL(k_omega_values_batch<P_F32>, g, dim3(256), 0, st, jobs); break;
    case P_BF16: hipLaunchKernelGGL(k_omega_values_batch<P_BF16>, g, dim3(256), 0, st, jobs); break;
    case P_BF16X2: hipLaunchKernelGGL(k_omega_values_batch<P_BF16X2>, g, dim3(256), 0, st, jobs); break;
    case P_FP8: hipLaunchKernelGGL(k_omega_values_batch<P_FP8>, g, dim3(256), 0, st, jobs); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_gemm64_batch(hipStream_t st, const Gemm64Job* jobs, int njobs, int max_m,
                               int max_n) {
  if (njobs <= 0) return hipSuccess;
  const dim3 grid((unsigned)((max_m + 15) / 16), (unsigned)((max_n + 15) / 16), (unsigned)njobs);
  hipLaunchKernelGGL(k_gemm64_batch, grid, dim3(256), 0, st, jobs);
  return hipGetLastError();
}

hipError_t launch_gemm64(hipStream_t st, int M, int Nn, int K, const double* A, int64_t lda,
                         int tA, const double* B, int64_t ldb, int tB, double* C, int64_t ldc) {
  const dim3 grid((unsigned)((M + 15) / 16), (unsigned)((Nn + 15) / 16));
  hipLaunchKernelGGL(k_gemm64, grid, dim3(256), 0, st, M, Nn, K, A, lda, tA, B, ldb, tB, C, ldc,
                     1.0, 0.0);
  return hipGetLastError();
}

hipError_t launch_gemm64_ab(hipStream_t st, int M, int Nn, int K, const double* A, int64_t lda,
                            int tA, const double* B, int64_t ldb, int tB, double alpha, double beta,
                            double* C, int64_t ldc) {
  if (M <= 0 || Nn <= 0) return hipSuccess;
  const dim3 grid((unsigned)((M + 15) / 16), (unsigned)((Nn + 15) / 16));
  hipLaunchKernelGGL(k_gemm64, grid, dim3(256), 0, st, M, Nn, K, A, lda, tA, B, ldb, tB, C, ldc,
                     alpha, beta);
  return hipGetLastError();
}

// y += x elementwise (count entries); vector loads where both are aligned
template <typename T>
__global__ void k_add_inplace(T* __restrict__ y, const T* __restrict__ x, int64_t count) {
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < count;
       e += (int64_t)gridDim.x * blockDim.x)
    y[e] += x[e];
}

// the results a compression hands back, in one launch: J (k pivots), k_eff
// and the two estimates (each skipped when its destination is NULL)
__global__ void k_copy_results(int64_t* __restrict__ J, const int64_t* __restrict__ piv, int k,
                               int64_t* __restrict__ k_eff, const int64_t* __restrict__ keff,
                               double* __restrict__ err, const double* __restrict__ werr) {
  const int t = threadIdx.x;
  if (J)
    for (int i = t; i < k; i += blockDim.x) J[i] = piv[i];
  if (t == 0 && k_eff) *k_eff = *keff;
  if (t < 2 && err) err[t] = werr[t];
}

hipError_t launch_copy_results(hipStream_t st, int64_t* J, const int64_t* piv, int k,
                               int64_t* k_eff, const int64_t* keff, double* err,
                               const double* werr) {
  if (!J && !k_eff && !err) return hipSuccess;
  hipLaunchKernelGGL(k_copy_results, dim3(1), dim3(256), 0, st, J, piv, k, k_eff, keff, err, werr);
  return hipGetLastError();
}

hipError_t launch_add_inplace(hipStream_t st, bool f64, void* y, const void* x, int64_t count,
                              int num_cu) {
  if (count <= 0) return hipSuccess;
  int64_t b = (count + 255) / 256;
  const int64_t cap = (int64_t)num_cu * 16;
  if (b > cap) b = cap;
  if (f64)
    hipLaunchKernelGGL(k_add_inplace<double>, dim3((unsigned)b), dim3(256), 0, st, (double*)y,
                       (const double*)x, count);
  else
    hipLaunchKernelGGL(k_add_inplace<float>, dim3((unsigned)b), dim3(256), 0, st, (float*)y,
                       (const float*)x, count);
  return hipGetLastError();
}

// FP8 data values for the general sketch kernels: one block of 64 threads
// per (64-row tile, column); out = s e4m3(a / s) with the tile's power-of-two
// scale (the same values the streaming pass forms in registers)
template <typename In>
__global__ __launch_bounds__(64) void k_fp8_quantize(const In* __restrict__ A, int64_t lda, int64_t N,
                                                     float* __restrict__ out, int64_t ldo) {
  const int64_t r = (int64_t)blockIdx.x * 64 + threadIdx.x;
  const int64_t j = blockIdx.y;
  const float a = r < N ? (float)A[r + lda * j] : 0.0f;
  float amax = fabsf(a);
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) amax = fmaxf(amax, __shfl_xor(amax, o, 64));
  float inv;
  const float sc = fp8_tile_scale(amax, inv);
  if (r < N) out[r + ldo * j] = e4m3_value(a * inv) * sc;
}

hipError_t launch_fp8_quantize(hipStream_t st, const void* A, bool f64, int64_t lda, int64_t N,
                               int64_t n, float* out, int64_t ldo) {
  const dim3 grid((unsigned)((N + 63) / 64), (unsigned)n);
  if (f64)
    hipLaunchKernelGGL(k_fp8_quantize<double>, grid, dim3(64), 0, st, (const double*)A, lda, N, out, ldo);
  else
    hipLaunchKernelGGL(k_fp8_quantize<float>, grid, dim3(64), 0, st, (const float*)A, lda, N, out, ldo);
  return hipGetLastError();
}

hipError_t launch_gather_cols(hipStream_t st, const void* src, bool src_f64, int64_t lds,
                              int64_t rows, const int64_t* piv, const int64_t* keff, int kcap,
                              void* dst, bool dst_f64, int64_t ldd) {
  int64_t bx = (rows + 255) / 256;
  if (bx > 2048) bx = 2048;
  const dim3 grid((unsigned)bx, (unsigned)kcap);
  if (src_f64 && dst_f64)
    hipLaunchKernelGGL((k_gather_cols<double, double>), grid, dim3(256), 0, st,
                       (const double*)src, lds, rows, piv, keff, kcap, (double*)dst, ldd);
  else if (src_f64)
    hipLaunchKernelGGL((k_gather_cols<double, float>), grid, dim3(256), 0, st,
                       (const double*)src, lds, rows, piv, keff, kcap, (float*)dst, ldd);
  else if (dst_f64)
    hipLaunchKernelGGL((k_gather_cols<float, double>), grid, dim3(256), 0, st,
                       (const float*)src, lds, rows, piv, keff, kcap, (double*)dst, ldd);
  else
    hipLaunchKernelGGL((k_gather_cols<float, float>), grid, dim3(256), 0, st, (const float*)src,
                       lds, rows, piv, keff, kcap, (float*)dst, ldd);
  return hipGetLastError();
}

hipError_t launch_gather_rows(hipStream_t st, const void* A, bool f64, int64_t lda,
                              const int64_t* rows, int64_t Ns, int64_t n, bool to_f32, double* W,
                              int64_t ldw) {
  int64_t b = (Ns * n + 255) / 256;
  if (b > 4096) b = 4096;
  if (f64)
    hipLaunchKernelGGL(k_gather_rows<double>, dim3((unsigned)b), dim3(256), 0, st,
                       (const double*)A, lda, rows, Ns, n, to_f32 ? 1 : 0, W, ldw);
  else
    hipLaunchKernelGGL(k_gather_rows<float>, dim3((unsigned)b), dim3(256), 0, st,
                       (const float*)A, lda, rows, Ns, n, 0, W, ldw);
  return hipGetLastError();
}

hipError_t launch_gather_block(hipStream_t st, const double* W, int lq, int r0, int q,
                               const int64_t* piv, const int64_t* keff, int kcap, double* out) {
  const int total = q * kcap;
  hipLaunchKernelGGL(k_gather_block, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, st, W,
                     lq, r0, q, piv, keff, kcap, out, (const GatherBlockJob*)nullptr);
  return hipGetLastError();
}

hipError_t launch_gather_block_batch(hipStream_t st, const GatherBlockJob* jobs, int njobs,
                                     int max_total) {
  if (njobs <= 0 || max_total <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_gather_block, dim3((unsigned)((max_total + 255) / 256), (unsigned)njobs),
                     dim3(256), 0, st, (const double*)nullptr, 0, 0, 0, (const int64_t*)nullptr,
                     (const int64_t*)nullptr, 0, (double*)nullptr, jobs);
  return hipGetLastError();
}

hipError_t launch_small_backsolve(hipStream_t st, const double* RM, const int64_t* pivM,
                                  const int64_t* rM, int l, const double* Cm, int64_t ldc, int kc,
                                  double* Tm) {
  hipLaunchKernelGGL(k_small_backsolve, dim3((unsigned)((kc + 63) / 64)), dim3(64), 0, st, RM,
                     pivM, rM, l, Cm, ldc, kc, Tm);
  return hipGetLastError();
}

hipError_t launch_apply_t(hipStream_t st, const void* Y, bool y_f64, int64_t N, int l,
                          const double* Tm, int k, void* AJ, bool aj_f64, int64_t ldaj) {
  const dim3 grid((unsigned)((N + 255) / 256), (unsigned)((k + 15) / 16));
  const size_t shm = (y_f64 ? sizeof(double) : sizeof(float)) * (size_t)l * 16;
  if (y_f64 && aj_f64)
    hipLaunchKernelGGL((k_apply_t<double, double>), grid, dim3(256), shm, st, (const double*)Y, N,
                       l, Tm, k, (double*)AJ, ldaj);
  else if (y_f64)
    hipLaunchKernelGGL((k_apply_t<double, float>), grid, dim3(256), shm, st, (const double*)Y, N,
                       l, Tm, k, (float*)AJ, ldaj);
  else if (aj_f64)
    hipLaunchKernelGGL((k_apply_t<float, double>), grid, dim3(256), shm, st, (const float*)Y, N,
                       l, Tm, k, (double*)AJ, ldaj);
  else
    hipLaunchKernelGGL((k_apply_t<float, float>), grid, dim3(256), shm, st, (const float*)Y, N, l,
                       Tm, k, (float*)AJ, ldaj);
  return hipGetLastError();
}

hipError_t launch_reconstruct(hipStream_t st, bool f64, const void* AJ, int64_t ldaj,
                              const void* P, int64_t ldp, int64_t N, int k, int64_t n, void* out,
                              int64_t ldo) {
  const dim3 grid((unsigned)((N + 63) / 64), (unsigned)((n + 31) / 32));
  if (f64) {
    const size_t shm = sizeof(double) * (size_t)k * 32;
    hipLaunchKernelGGL(k_reconstruct<double>, grid, dim3(256), shm, st, (const double*)AJ, ldaj,
                       (const double*)P, ldp, N, k, n, (double*)out, ldo);
  } else {
    const size_t shm = sizeof(float) * (size_t)k * 32;
    hipLaunchKernelGGL(k_reconstruct<float>, grid, dim3(256), shm, st, (const float*)AJ, ldaj,
                       (const float*)P, ldp, N, k, n, (float*)out, ldo);
  }
  return hipGetLastError();
}

hipError_t launch_error_norms(hipStream_t st, bool f64, const void* A, int64_t lda,
                              const void* AJ, int64_t ldaj, const void* P, int64_t ldp, int64_t N,
                              int k, int64_t n, double* part, int64_t part_cap, double* out4) {
  const dim3 grid((unsigned)((N + 63) / 64), (unsigned)((n + 31) / 32));
  const int64_t nb = (int64_t)grid.x * grid.y;
  if (nb > part_cap) return hipErrorInvalidValue;
  const size_t shm = sizeof(double) * (size_t)k * 32;
  if (f64)
    hipLaunchKernelGGL(k_error_norms<double>, grid, dim3(256), shm, st, (const double*)A, lda,
                       (const double*)AJ, ldaj, (const double*)P, ldp, N, k, n, part);
  else
    hipLaunchKernelGGL(k_error_norms<float>, grid, dim3(256), shm, st, (const float*)A, lda,
                       (const float*)AJ, ldaj, (const float*)P, ldp, N, k, n, part);
  hipLaunchKernelGGL(k_reduce_norms, dim3(1), dim3(256), 0, st, part, nb, out4);
  return hipGetLastError();
}

}  // namespace sid
