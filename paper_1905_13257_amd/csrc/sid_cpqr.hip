// sid_cpqr.hip -- the paper's mgsqr (column-pivoted modified Gram-Schmidt,
// Sec. 2.4, Alg. 3-5 step 3) and the ID coefficient solve C = R11^+ R12
// (Alg. 3-5, the step after mgsqr), FP64 on the GPU.
//
// mgsqr is a chain of k dependent steps (argmax of the residual column norms,
// normalize the pivot, project it out of every other column), so its cost is
// latency, not flops.  Here the residual matrix stays in registers, spread
// over G cooperating workgroups (128 columns each with 2 threads per column
// for up to 128 rows, else 64 columns with 4 threads per column), and
// every step crosses exactly one device-wide barrier:
//   1. each workgroup finds its best live column (ties: smallest index),
//   2. publishes (norm^2, index, residual column) into a double-buffered slot,
//   3. barrier (monotonic counter, bounded spin),
//   4. every workgroup reads all G candidates and picks the same winner,
//      normalizes its column into q (LDS) and updates its own columns
//      (R(i, j) = q^T r_j, r_j -= R(i, j) q, new norm^2 of r_j).
// The participating workgroups are spread 8 block indices apart so that, with
// the round-robin workgroup-to-XCD dispatch, they share one XCD's L2.
// Workgroup barriers inside a step wait for LDS traffic only; the published
// candidate data is written and read with device-scope atomics and ordered
// before the barrier arrival by its writers' wait for store completion; the
// stores of R and Q drain in the background.
#include "sid_kernels.hpp"

namespace sid {

constexpr int CQ_THREADS = 256;
// threads per column TPC (template): 2 for m <= 128 (fewer workgroups take
// part in each step's synchronization), else 4; columns per workgroup
// CQ_THREADS / TPC
constexpr int CQ_MINCPW = CQ_THREADS / 4;    // fewest columns per workgroup
constexpr unsigned CQ_SPIN_LIMIT = 1u << 22; // bounded wait (~0.1 s); never reached when co-resident
constexpr int CQ_MSTRIDE = 256;              // published column slot (rows, >= TPC * RPT)

__global__ void k_zero_u32(unsigned int* p, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0u;
}

template <typename T>
__device__ __forceinline__ T ld_agent(const T* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
template <typename T>
__device__ __forceinline__ void st_agent(T* p, T v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
// Wait until this wave's stores are acknowledged.  Device-scope atomic
// stores are acknowledged once they are coherent device-wide, so this orders
// them before a later barrier arrival without the L2 write-back that a
// device-scope release fence performs (measured: 4.4 against 5.0 us per mgsqr
// step at 120 x 500).  The memory clobber keeps the compiler from moving
// memory operations across it.
__device__ __forceinline__ void wait_stores() { asm volatile("s_waitcnt vmcnt(0)" ::: "memory"); }

// (ov, oj) replaces (bv, bj) if it has the larger norm, or the same norm and
// the smaller column index; branch-free
__device__ __forceinline__ void better(double& bv, int& bj, double ov, int oj) {
  const bool take = (ov > bv) | ((ov == bv) & (oj < bj));
  bv = take ? ov : bv;
  bj = take ? oj : bj;
}

// device-wide barrier over G workgroups: counter value after the b-th
// barrier is G*b.  Called by thread 0 after the workgroup's writers have
// fenced their published data and the workgroup has synchronized; spins with
// relaxed loads and acquires once.  Returns false on spin timeout.
__device__ __forceinline__ bool grid_barrier(unsigned int* bar, unsigned target) {
  __hip_atomic_fetch_add(bar, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  unsigned spins = 0;
  bool ok = true;
  while (__hip_atomic_load(bar, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < target) {
    if (++spins > CQ_SPIN_LIMIT) { ok = false; break; }
    __builtin_amdgcn_s_sleep(1);
  }
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
  return ok;
}

template <int TPC, int RPT>
__global__ __launch_bounds__(CQ_THREADS) void k_cpqr_coop(
    const double* __restrict__ X, int64_t ldx, int m, int nc, int kmax, double rank_tol, int G,
    int stride_blk, double* __restrict__ pub_v, int* __restrict__ pub_j,
    double* __restrict__ pub_col, double* __restrict__ red, unsigned int* __restrict__ bar,
    unsigned int* __restrict__ fail, int64_t* __restrict__ piv, double* __restrict__ R,
    double* __restrict__ Q, int64_t* __restrict__ keff, double* __restrict__ stats,
    const int64_t* __restrict__ forced, unsigned int* __restrict__ sticky) {
  static_assert(TPC * RPT <= CQ_MSTRIDE, "published column slot");
  constexpr int CQ_TPC = TPC;
  constexpr int CQ_CPW = CQ_THREADS / TPC;
  if (blockIdx.x % stride_blk) return;
  const int g = blockIdx.x / stride_blk;
  if (g >= G) return;
  __shared__ double s_q[RPT * CQ_TPC];
  __shared__ double s_wv[CQ_THREADS / 64];
  __shared__ int s_wj[CQ_THREADS / 64];
  __shared__ double s_win_v;
  __shared__ int s_win_j, s_win_g, s_failed;
  __shared__ double s_sum[2][CQ_THREADS / 64];

  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int cl = tid / CQ_TPC, seg = tid % CQ_TPC;
  const int j = g * CQ_CPW + cl;
  const bool mine = j < nc;
  // rows m .. of q stay zero, so the update loops need no row guards (the
  // matching entries of w are zero too)
  for (int e = tid; e < RPT * CQ_TPC; e += CQ_THREADS) s_q[e] = 0.0;

  double w[RPT];
  double ps = 0.0;
#pragma unroll
  for (int i = 0; i < RPT; ++i) {
    const int r = seg + CQ_TPC * i;
    w[i] = (mine && r < m) ? X[r + ldx * j] : 0.0;
    ps = fma(w[i], w[i], ps);
  }
  double nrm = ps;
#pragma unroll
  for (int o = 1; o < CQ_TPC; o <<= 1) nrm += __shfl_xor(nrm, o, 64);
  const double tot_local = (seg == 0 && mine) ? nrm : 0.0;
  bool alive = mine;
  bool ok = true;

  double first = -1.0;
  int k = 0, nbar = 0;
  for (; k < kmax; ++k) {
    const int par = k & 1;
    // 1. local argmax (forced order: the given column is the only candidate)
    const bool cand = alive && (!forced || j == forced[k]);
    double bv = cand ? nrm : -1.0;
    int bj = cand ? j : 0x7fffffff;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) better(bv, bj, __shfl_xor(bv, o, 64), __shfl_xor(bj, o, 64));
    if (lane == 0) { s_wv[wv] = bv; s_wj[wv] = bj; }
    lds_barrier();
    bv = s_wv[0];
    bj = s_wj[0];
    for (int u = 1; u < CQ_THREADS / 64; ++u) better(bv, bj, s_wv[u], s_wj[u]);
    // 2. publish the candidate: device-scope atomic stores, and each writer
    //    waits for their completion, so the values are visible device-wide
    //    before its workgroup's barrier arrival is issued
    if (tid == 0) {
      st_agent(&pub_v[par * G + g], bv);
      st_agent(&pub_j[par * G + g], bj);
    }
    if (alive && j == bj) {
      // all RPT rows (zeros past m): no row guards on the critical path
#pragma unroll
      for (int i = 0; i < RPT; ++i)
        st_agent(&pub_col[(int64_t)(par * G + g) * CQ_MSTRIDE + seg + CQ_TPC * i], w[i]);
    }
    wait_stores();
    lds_barrier();
    // 3. barrier
    if (tid == 0) ok = grid_barrier(bar, (unsigned)G * (unsigned)(nbar + 1)) && ok;
    ++nbar;
    lds_barrier();
    // 4. global winner: wave 0 fetches the G candidates in parallel
    if (wv == 0) {
      double v = -1.0;
      int jj = 0x7fffffff, hh = 0x7fffffff;
      if (lane < G) {
        v = ld_agent(&pub_v[par * G + lane]);
        jj = ld_agent(&pub_j[par * G + lane]);
        hh = lane;
      }
#pragma unroll
      for (int o = 32; o > 0; o >>= 1) {
        const double ov = __shfl_xor(v, o, 64);
        const int oj = __shfl_xor(jj, o, 64);
        const int oh = __shfl_xor(hh, o, 64);
        if (ov > v || (ov == v && oj < jj)) { v = ov; jj = oj; hh = oh; }
      }
      if (lane == 0) {
        s_win_v = v;
        s_win_j = jj;
        s_win_g = hh;
      }
    }
    lds_barrier();
    const double vmax = s_win_v;
    const int p = s_win_j;
    const int gp = s_win_g;
    if (!(vmax > 0.0)) break;
    const double nu = sqrt(vmax);
    if (first < 0.0) first = nu;
    else if (rank_tol > 0.0 && nu <= rank_tol * first) break;
    for (int r = tid; r < m; r += CQ_THREADS)
      s_q[r] = ld_agent(&pub_col[(int64_t)(par * G + gp) * CQ_MSTRIDE + r]) / nu;
    lds_barrier();
    if (g == 0) {
      if (tid == 0) piv[k] = p;
      for (int r = tid; r < m; r += CQ_THREADS) Q[r + (int64_t)m * k] = s_q[r];
    }
    // update: R(k, j) = q^T r_j, r_j -= R(k, j) q
    double d = 0.0;
#pragma unroll
    for (int i = 0; i < RPT; ++i) d = fma(s_q[seg + CQ_TPC * i], w[i], d);
#pragma unroll
    for (int o = 1; o < CQ_TPC; o <<= 1) d += __shfl_xor(d, o, 64);
    if (mine && j == p) {
      alive = false;
#pragma unroll
      for (int i = 0; i < RPT; ++i) w[i] = 0.0;
      if (seg == 0) R[(int64_t)k * nc + j] = nu;
    } else if (alive) {
      ps = 0.0;
#pragma unroll
      for (int i = 0; i < RPT; ++i) {
        w[i] = fma(-d, s_q[seg + CQ_TPC * i], w[i]);
        ps = fma(w[i], w[i], ps);
      }
      if (seg == 0) R[(int64_t)k * nc + j] = d;
    } else if (mine) {
      ps = 0.0;
      if (seg == 0) R[(int64_t)k * nc + j] = 0.0;
    }
    nrm = ps;
#pragma unroll
    for (int o = 1; o < CQ_TPC; o <<= 1) nrm += __shfl_xor(nrm, o, 64);
  }

  // statistics: final residual energy of live columns and ||X||_F^2
  double res_local = (seg == 0 && alive) ? nrm : 0.0;
  double a = res_local, b = tot_local;
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    a += __shfl_xor(a, o, 64);
    b += __shfl_xor(b, o, 64);
  }
  if (lane == 0) { s_sum[0][wv] = a; s_sum[1][wv] = b; }
  __syncthreads();
  if (tid == 0) {
    double sa = 0.0, sb = 0.0;
    for (int u = 0; u < CQ_THREADS / 64; ++u) { sa += s_sum[0][u]; sb += s_sum[1][u]; }
    red[2 * g] = sa;
    red[2 * g + 1] = sb;
    // a timed-out wait of this workgroup is recorded before its arrival
    if (!ok) atomicOr(fail, 1u);
    __threadfence();
    const bool okb = grid_barrier(bar, (unsigned)G * (unsigned)(nbar + 1));
    if (!okb) atomicOr(fail, 1u);
    if (g == 0) {
      double ta = 0.0, tb = 0.0;
      for (int h = 0; h < G; ++h) { ta += ld_agent(&red[2 * h]); tb += ld_agent(&red[2 * h + 1]); }
      stats[0] = ta;
      stats[1] = tb;
      s_failed = (!okb || ld_agent(fail) != 0u) ? 1 : 0;
    }
  }
  if (g == 0) {
    __syncthreads();
    for (int i = k + tid; i < kmax; i += CQ_THREADS) piv[i] = -1;
    // keff = -1 marks a timed-out wait (results invalid); the context's
    // sticky flag keeps it until the host reads it (sid_sync)
    if (tid == 0) {
      const bool failed = s_failed != 0;
      *keff = failed ? -1 : k;
      if (failed && sticky) *sticky = 1u;
    }
  }
}

// ---------------------------------------------------------------------------
// mgsqr in one workgroup (the same steps, no device-wide barrier): for
// matrices whose residual fits in the registers of 512 threads (TPC threads
// per column, RPT rows per thread).  Per step: each wave finds its best live
// column, one barrier, every thread reduces the 8 wave candidates, the
// pivot's owners write q into LDS, one barrier, every column is updated.
// The wave candidates and q are double-buffered by step parity, so two
// barriers per step suffice; they wait for LDS traffic only, so the stores of
// R, Q and the pivots drain in the background.
// ---------------------------------------------------------------------------
constexpr int CW_THREADS = 512;
constexpr int CW_WAVES = CW_THREADS / 64;
constexpr int CW_MMAX = 256;

// a batched launch: this workgroup's job replaces the arguments
#define SID_CPQR_TAKE_JOB()                                                       \
  if (jobs) {                                                                     \
    const CpqrJob jb = jobs[blockIdx.x];                                          \
    X_ = jb.X;                                                                    \
    ldx = jb.ldx;                                                                 \
    m = jb.m;                                                                     \
    nc = jb.nc;                                                                   \
    kmax = jb.kmax;                                                               \
    rank_tol = jb.rank_tol;                                                       \
    piv_ = jb.piv;                                                                \
    R_ = jb.R;                                                                    \
    Q_ = jb.Q;                                                                    \
    keff_ = jb.keff;                                                              \
    stats_ = jb.stats;                                                            \
    forced_ = nullptr;                                                            \
  }                                                                               \
  const auto X = to_global(X_);                                                   \
  const auto piv = to_global(piv_);                                               \
  const auto R = to_global(R_);                                                   \
  const auto Q = to_global(Q_);                                                   \
  const auto keff = to_global(keff_);                                             \
  const auto stats = to_global(stats_);                                           \
  const auto forced = to_global(forced_);

template <int TPC, int RPT>
__device__ __forceinline__ void cpqr_wg_body(
    const double* __restrict__ X_, int64_t ldx, int m, int nc, int kmax, double rank_tol,
    int64_t* __restrict__ piv_, double* __restrict__ R_, double* __restrict__ Q_,
    int64_t* __restrict__ keff_, double* __restrict__ stats_, const int64_t* __restrict__ forced_,
    const CpqrJob* __restrict__ jobs) {
  SID_CPQR_TAKE_JOB()
  constexpr int QN = TPC * RPT;  // rows covered by a column's threads
  __shared__ double s_q[2][QN];
  __shared__ double s_wv[2][CW_WAVES];
  __shared__ int s_wj[2][CW_WAVES];
  __shared__ double s_sum[2][CW_WAVES];
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int j = tid / TPC, seg = tid % TPC;
  const bool mine = j < nc;
  // rows m .. of q stay zero, so the loops below need no row guards (the
  // matching entries of w are zero too)
  for (int e = tid; e < 2 * QN; e += CW_THREADS) (&s_q[0][0])[e] = 0.0;

  double w[RPT];
  double ps = 0.0;
#pragma unroll
  for (int i = 0; i < RPT; ++i) {
    const int r = seg + TPC * i;
    w[i] = (mine && r < m) ? X[r + ldx * j] : 0.0;
    ps = fma(w[i], w[i], ps);
  }
  double nrm = ps;
#pragma unroll
  for (int o = 1; o < TPC; o <<= 1) nrm += __shfl_xor(nrm, o, 64);
  const double tot_local = (seg == 0 && mine) ? nrm : 0.0;
  bool alive = mine;
  double first = -1.0;
  int k = 0;
  for (; k < kmax; ++k) {
    const int par = k & 1;
    // 1. this wave's best live column (ties: smallest index; forced order:
    //    the given column is the only candidate)
    const bool cand = alive && (!forced || j == forced[k]);
    double bv = cand ? nrm : -1.0;
    int bj = cand ? j : 0x7fffffff;
#pragma unroll
    for (int o = 32; o >= TPC; o >>= 1) better(bv, bj, __shfl_xor(bv, o, 64), __shfl_xor(bj, o, 64));
    if (lane == 0) { s_wv[par][wv] = bv; s_wj[par][wv] = bj; }
    lds_barrier();
    // 2. the winner, found by every thread from the wave candidates (all
    //    loaded first, then reduced without branches)
    {
      double cv[CW_WAVES];
      int cj[CW_WAVES];
#pragma unroll
      for (int u = 0; u < CW_WAVES; ++u) { cv[u] = s_wv[par][u]; cj[u] = s_wj[par][u]; }
#pragma unroll
      for (int h = CW_WAVES / 2; h > 0; h >>= 1)
#pragma unroll
        for (int u = 0; u < h; ++u) better(cv[u], cj[u], cv[u + h], cj[u + h]);
      bv = cv[0];
      bj = cj[0];
    }
    if (!(bv > 0.0)) break;
    const double nu = sqrt(bv);
    if (first < 0.0) first = nu;
    else if (rank_tol > 0.0 && nu <= rank_tol * first) break;
    const int p = bj;
    // 3. the pivot column, normalized, into LDS (rows >= m write the zeros
    //    their w holds, so the owners need no row guards)
    if (j == p) {
      const double inv = 1.0 / nu;
#pragma unroll
      for (int i = 0; i < RPT; ++i) {
        s_q[par][seg + TPC * i] = w[i] * inv;
        w[i] = 0.0;
      }
      alive = false;
      if (seg == 0) {
        R[(int64_t)k * nc + j] = nu;
        piv[k] = p;
      }
    }
    lds_barrier();
    for (int r = tid; r < m; r += CW_THREADS) Q[r + (int64_t)m * k] = s_q[par][r];
    // 4. R(k, j) = q^T r_j, r_j -= R(k, j) q, new norm of r_j
    const double* qv = &s_q[par][seg];  // q(seg + TPC i) = qv[TPC i]
    double d0 = 0.0, d1 = 0.0;
#pragma unroll
    for (int i = 0; i < RPT; i += 2) {
      d0 = fma(qv[TPC * i], w[i], d0);
      if (i + 1 < RPT) d1 = fma(qv[TPC * (i + 1)], w[i + 1], d1);
    }
    double d = d0 + d1;
#pragma unroll
    for (int o = 1; o < TPC; o <<= 1) d += __shfl_xor(d, o, 64);
    if (alive) {
      double p0 = 0.0, p1 = 0.0;
#pragma unroll
      for (int i = 0; i < RPT; i += 2) {
        w[i] = fma(-d, qv[TPC * i], w[i]);
        p0 = fma(w[i], w[i], p0);
        if (i + 1 < RPT) {
          w[i + 1] = fma(-d, qv[TPC * (i + 1)], w[i + 1]);
          p1 = fma(w[i + 1], w[i + 1], p1);
        }
      }
      ps = p0 + p1;
      if (seg == 0) R[(int64_t)k * nc + j] = d;
    } else {
      ps = 0.0;
      if (mine && j != p && seg == 0) R[(int64_t)k * nc + j] = 0.0;
    }
    nrm = ps;
#pragma unroll
    for (int o = 1; o < TPC; o <<= 1) nrm += __shfl_xor(nrm, o, 64);
  }

  // statistics: final residual energy of live columns and ||X||_F^2
  double a = (seg == 0 && alive) ? nrm : 0.0, b = tot_local;
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    a += __shfl_xor(a, o, 64);
    b += __shfl_xor(b, o, 64);
  }
  if (lane == 0) { s_sum[0][wv] = a; s_sum[1][wv] = b; }
  __syncthreads();
  if (tid == 0) {
    double sa = 0.0, sb = 0.0;
    for (int u = 0; u < CW_WAVES; ++u) { sa += s_sum[0][u]; sb += s_sum[1][u]; }
    stats[0] = sa;
    stats[1] = sb;
    *keff = k;
  }
  for (int i = k + tid; i < kmax; i += CW_THREADS) piv[i] = -1;
}

template <int TPC, int RPT>
__global__ __launch_bounds__(CW_THREADS) void k_cpqr_wg(
    const double* __restrict__ X_, int64_t ldx, int m, int nc, int kmax, double rank_tol,
    int64_t* __restrict__ piv_, double* __restrict__ R_, double* __restrict__ Q_,
    int64_t* __restrict__ keff_, double* __restrict__ stats_, const int64_t* __restrict__ forced_,
    const CpqrJob* __restrict__ jobs) {
  cpqr_wg_body<TPC, RPT>(X_, ldx, m, nc, kmax, rank_tol, piv_, R_, Q_, keff_, stats_, forced_,
                         jobs);
}

// Every job of a batch that the register kernel takes, whatever its
// instance, in one launch: workgroup b runs job b with the instance in
// jobs[b].inst (the arithmetic, and so the bits, of its own launch).  One
// launch keeps the jobs side by side: launches of separate instances on
// separate streams share the few hardware queues and partly serialize.
__global__ __launch_bounds__(CW_THREADS) void k_cpqr_wg_any(const CpqrJob* __restrict__ jobs) {
  const int inst = jobs[blockIdx.x].inst;
#define SID_CWA(TI_, TPC_)                                                                    \
  case 8 * TI_ + 1: cpqr_wg_body<TPC_, 8>(nullptr, 0, 0, 0, 0, 0.0, nullptr, nullptr, nullptr, \
                                          nullptr, nullptr, nullptr, jobs); break;             \
  case 8 * TI_ + 2: cpqr_wg_body<TPC_, 16>(nullptr, 0, 0, 0, 0, 0.0, nullptr, nullptr, nullptr, \
                                           nullptr, nullptr, nullptr, jobs); break;            \
  case 8 * TI_ + 3: cpqr_wg_body<TPC_, 24>(nullptr, 0, 0, 0, 0, 0.0, nullptr, nullptr, nullptr, \
                                           nullptr, nullptr, nullptr, jobs); break;            \
  case 8 * TI_ + 4: cpqr_wg_body<TPC_, 32>(nullptr, 0, 0, 0, 0, 0.0, nullptr, nullptr, nullptr, \
                                           nullptr, nullptr, nullptr, jobs); break;            \
  case 8 * TI_ + 5: cpqr_wg_body<TPC_, 40>(nullptr, 0, 0, 0, 0, 0.0, nullptr, nullptr, nullptr, \
                                           nullptr, nullptr, nullptr, jobs); break;            \
  case 8 * TI_ + 6: cpqr_wg_body<TPC_, 48>(nullptr, 0, 0, 0, 0, 0.0, nullptr, nullptr, nullptr, \
                                           nullptr, nullptr, nullptr, jobs); break;
  switch (inst) {
    SID_CWA(0, 8)
    SID_CWA(1, 4)
    SID_CWA(2, 2)
    SID_CWA(3, 1)
    default: break;
  }
#undef SID_CWA
}

static int cw_tpc(int nc) { return nc <= 64 ? 8 : nc <= 128 ? 4 : nc <= 256 ? 2 : 1; }

bool cpqr_wg_supported(int m, int nc) {
  if (nc < 1 || nc > CW_THREADS || m < 1 || m > CW_MMAX) return false;
  return (m + cw_tpc(nc) - 1) / cw_tpc(nc) <= 48;
}

hipError_t launch_cpqr_wg(hipStream_t st, const double* X, int64_t ldx, int m, int nc, int kmax,
                          double rank_tol, int64_t* piv, double* R, double* Q, int64_t* keff,
                          double* stats, const int64_t* forced) {
  if (!cpqr_wg_supported(m, nc)) return hipErrorInvalidValue;
  const int tpc = cw_tpc(nc);
  const int rpt = (m + tpc - 1) / tpc;
#define SID_CW(TPC_, RPT_)                                                                    \
  hipLaunchKernelGGL((k_cpqr_wg<TPC_, RPT_>), dim3(1), dim3(CW_THREADS), 0, st, X, ldx, m, nc, \
                     kmax, rank_tol, piv, R, Q, keff, stats, forced, (const CpqrJob*)nullptr)
#define SID_CW_R(TPC_)                    \
  if (rpt <= 8) SID_CW(TPC_, 8);          \
  else if (rpt <= 16) SID_CW(TPC_, 16);   \
  else if (rpt <= 24) SID_CW(TPC_, 24);   \
  else if (rpt <= 32) SID_CW(TPC_, 32);   \
  else if (rpt <= 40) SID_CW(TPC_, 40);   \
  else SID_CW(TPC_, 48);
  if (tpc == 8) { SID_CW_R(8) }
  else if (tpc == 4) { SID_CW_R(4) }
  else if (tpc == 2) { SID_CW_R(2) }
  else { SID_CW_R(1) }
#undef SID_CW_R
#undef SID_CW
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// mgsqr in one workgroup for residuals too large for its registers alone
// (e.g. W_sel of 120 x 500 FP64, 480 KB): 512 threads (two waves per SIMD),
// one thread per column (up to 512 columns); each thread keeps the first RR
// rows of its column in registers and the next CL_RL rows in LDS
// (s_w[i][tid]: consecutive threads at consecutive addresses).  The steps are
// those of k_cpqr_wg -- wave candidates, one barrier, every thread reduces
// the 8 candidates, the pivot's thread writes q into LDS, one barrier, every
// column is updated -- with no device-wide barrier and no global memory
// round trip per step.
// ---------------------------------------------------------------------------
constexpr int CL_THREADS = 512;
constexpr int CL_WAVES = CL_THREADS / 64;
constexpr int CL_RL = 38;  // rows per thread in LDS: 38 x 8 B x 512 = 152 KiB

template <int RR>
__global__ __launch_bounds__(CL_THREADS) void k_cpqr_wgl(
    const double* __restrict__ X_, int64_t ldx, int m, int nc, int kmax, double rank_tol,
    int64_t* __restrict__ piv_, double* __restrict__ R_, double* __restrict__ Q_,
    int64_t* __restrict__ keff_, double* __restrict__ stats_, const int64_t* __restrict__ forced_,
    const CpqrJob* __restrict__ jobs) {
  SID_CPQR_TAKE_JOB()
  constexpr int QN = RR + CL_RL;  // rows covered
  __shared__ double s_w[CL_RL][CL_THREADS];
  __shared__ double s_q[2][QN];
  __shared__ double s_wv[2][CL_WAVES];
  __shared__ int s_wj[2][CL_WAVES];
  __shared__ double s_sum[2][CL_WAVES];
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int j = tid;
  const bool mine = j < nc;
  // rows m .. of q stay zero, so the loops below need no row guards (the
  // matching entries of w are zero too)
  for (int e = tid; e < 2 * QN; e += CL_THREADS) (&s_q[0][0])[e] = 0.0;

  double w[RR];
  double p0 = 0.0, p1 = 0.0;
#pragma unroll
  for (int i = 0; i < RR; ++i) {
    w[i] = (mine && i < m) ? X[i + ldx * j] : 0.0;
    if (i & 1) p1 = fma(w[i], w[i], p1);
    else p0 = fma(w[i], w[i], p0);
  }
#pragma unroll 2
  for (int i = 0; i < CL_RL; ++i) {
    const int r = RR + i;
    const double x = (mine && r < m) ? X[r + ldx * j] : 0.0;
    s_w[i][tid] = x;
    if (i & 1) p1 = fma(x, x, p1);
    else p0 = fma(x, x, p0);
  }
  double nrm = p0 + p1;
  const double tot_local = mine ? nrm : 0.0;
  bool alive = mine;
  double first = -1.0;
  int k = 0;
  for (; k < kmax; ++k) {
    const int par = k & 1;
    // 1. this wave's best live column (ties: smallest index; forced order:
    //    the given column is the only candidate)
    const bool cand = alive && (!forced || j == forced[k]);
    double bv = cand ? nrm : -1.0;
    int bj = cand ? j : 0x7fffffff;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) better(bv, bj, __shfl_xor(bv, o, 64), __shfl_xor(bj, o, 64));
    if (lane == 0) { s_wv[par][wv] = bv; s_wj[par][wv] = bj; }
    lds_barrier();
    // 2. the winner, found by every thread from the wave candidates (the
    //    same LDS words for every lane: broadcast reads)
    bv = s_wv[par][0];
    bj = s_wj[par][0];
#pragma unroll
    for (int u = 1; u < CL_WAVES; ++u) better(bv, bj, s_wv[par][u], s_wj[par][u]);
    if (!(bv > 0.0)) break;
    const double nu = sqrt(bv);
    if (first < 0.0) first = nu;
    else if (rank_tol > 0.0 && nu <= rank_tol * first) break;
    const int p = bj;
    // 3. the pivot column, normalized, into LDS
    if (j == p) {
      const double inv = 1.0 / nu;
#pragma unroll
      for (int i = 0; i < RR; ++i) {
        s_q[par][i] = w[i] * inv;
        w[i] = 0.0;
      }
      for (int i = 0; i < CL_RL; ++i) {
        s_q[par][RR + i] = s_w[i][tid] * inv;
        s_w[i][tid] = 0.0;
      }
      alive = false;
      R[(int64_t)k * nc + j] = nu;
      piv[k] = p;
    }
    lds_barrier();
    for (int r = tid; r < m; r += CL_THREADS) Q[r + (int64_t)m * k] = s_q[par][r];
    // 4. R(k, j) = q^T r_j, r_j -= R(k, j) q, new norm of r_j (q: LDS
    //    broadcast reads; the LDS rows are read twice rather than held)
    const double* qv = s_q[par];
    double d0 = 0.0, d1 = 0.0;
#pragma unroll
    for (int i = 0; i < RR; ++i) {
      if (i & 1) d1 = fma(qv[i], w[i], d1);
      else d0 = fma(qv[i], w[i], d0);
    }
#pragma unroll 2
    for (int i = 0; i < CL_RL; ++i) {
      if (i & 1) d1 = fma(qv[RR + i], s_w[i][tid], d1);
      else d0 = fma(qv[RR + i], s_w[i][tid], d0);
    }
    const double d = d0 + d1;
    asm volatile("" ::: "memory");  // q from LDS again below, not held in registers
    if (alive) {
      double a0 = 0.0, a1 = 0.0;
#pragma unroll
      for (int i = 0; i < RR; ++i) {
        w[i] = fma(-d, qv[i], w[i]);
        if (i & 1) a1 = fma(w[i], w[i], a1);
        else a0 = fma(w[i], w[i], a0);
      }
#pragma unroll 2
      for (int i = 0; i < CL_RL; ++i) {
        const double x = fma(-d, qv[RR + i], s_w[i][tid]);
        s_w[i][tid] = x;
        if (i & 1) a1 = fma(x, x, a1);
        else a0 = fma(x, x, a0);
      }
      nrm = a0 + a1;
      R[(int64_t)k * nc + j] = d;
    } else {
      nrm = 0.0;
      if (mine && j != p) R[(int64_t)k * nc + j] = 0.0;
    }
  }

  // statistics: final residual energy of live columns and ||X||_F^2
  double a = alive ? nrm : 0.0, b = tot_local;
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    a += __shfl_xor(a, o, 64);
    b += __shfl_xor(b, o, 64);
  }
  if (lane == 0) { s_sum[0][wv] = a; s_sum[1][wv] = b; }
  __syncthreads();
  if (tid == 0) {
    double sa = 0.0, sb = 0.0;
    for (int u = 0; u < CL_WAVES; ++u) { sa += s_sum[0][u]; sb += s_sum[1][u]; }
    stats[0] = sa;
    stats[1] = sb;
    *keff = k;
  }
  for (int i = k + tid; i < kmax; i += CL_THREADS) piv[i] = -1;
}

constexpr int CL_RR_MAX = 96;

bool cpqr_wgl_supported(int m, int nc) {
  return nc >= 1 && nc <= CL_THREADS && m >= 1 && m <= CL_RR_MAX + CL_RL;
}

hipError_t launch_cpqr_wgl(hipStream_t st, const double* X, int64_t ldx, int m, int nc, int kmax,
                           double rank_tol, int64_t* piv, double* R, double* Q, int64_t* keff,
                           double* stats, const int64_t* forced) {
  if (!cpqr_wgl_supported(m, nc)) return hipErrorInvalidValue;
  const int rr = m - CL_RL;  // register rows per thread (may be <= 0)
#define SID_CL(RR_)                                                                          \
  hipLaunchKernelGGL((k_cpqr_wgl<RR_>), dim3(1), dim3(CL_THREADS), 0, st, X, ldx, m, nc, kmax, \
                     rank_tol, piv, R, Q, keff, stats, forced, (const CpqrJob*)nullptr)
  if (rr <= 26) SID_CL(26);
  else if (rr <= 42) SID_CL(42);
  else if (rr <= 58) SID_CL(58);
  else if (rr <= 74) SID_CL(74);
  else if (rr <= 82) SID_CL(82);
  else SID_CL(96);
#undef SID_CL
  return hipGetLastError();
}

// Instance ids: the register kernel 8 * tpc_index + rpt_index + 1 (the
// choices of launch_cpqr_wg), the LDS kernel -(rr_index + 1) (those of
// launch_cpqr_wgl).
int cpqr_batch_instance(int m, int nc, bool wgl) {
  if (wgl) {
    if (!cpqr_wgl_supported(m, nc)) return 0;
    const int rr = m - CL_RL;
    const int ri = rr <= 26 ? 0 : rr <= 42 ? 1 : rr <= 58 ? 2 : rr <= 74 ? 3 : rr <= 82 ? 4 : 5;
    return -(ri + 1);
  }
  if (!cpqr_wg_supported(m, nc)) return 0;
  const int tpc = cw_tpc(nc);
  const int rpt = (m + tpc - 1) / tpc;
  const int ti = tpc == 8 ? 0 : tpc == 4 ? 1 : tpc == 2 ? 2 : 3;
  const int ri = rpt <= 8 ? 0 : rpt <= 16 ? 1 : rpt <= 24 ? 2 : rpt <= 32 ? 3 : rpt <= 40 ? 4 : 5;
  return 8 * ti + ri + 1;
}

hipError_t launch_cpqr_batch(hipStream_t st, int instance, const CpqrJob* jobs, int njobs) {
  if (njobs <= 0) return hipSuccess;
  if (!jobs || instance == 0) return hipErrorInvalidValue;
  const dim3 g((unsigned)njobs);
  if (instance == CPQR_BATCH_ANY_WG) {
    hipLaunchKernelGGL(k_cpqr_wg_any, g, dim3(CW_THREADS), 0, st, jobs);
    return hipGetLastError();
  }
  const double* X0 = nullptr;
  int64_t* pnull = nullptr;
  double* dnull = nullptr;
#define SID_CWB(TPC_, RPT_)                                                                   \
  hipLaunchKernelGGL((k_cpqr_wg<TPC_, RPT_>), g, dim3(CW_THREADS), 0, st, X0, (int64_t)0, 0, 0, \
                     0, 0.0, pnull, dnull, dnull, pnull, dnull, (const int64_t*)nullptr, jobs)
#define SID_CWB_R(TPC_, RI_)             \
  if (RI_ == 0) SID_CWB(TPC_, 8);        \
  else if (RI_ == 1) SID_CWB(TPC_, 16);  \
  else if (RI_ == 2) SID_CWB(TPC_, 24);  \
  else if (RI_ == 3) SID_CWB(TPC_, 32);  \
  else if (RI_ == 4) SID_CWB(TPC_, 40);  \
  else SID_CWB(TPC_, 48);
#define SID_CLB(RR_)                                                                         \
  hipLaunchKernelGGL((k_cpqr_wgl<RR_>), g, dim3(CL_THREADS), 0, st, X0, (int64_t)0, 0, 0, 0, \
                     0.0, pnull, dnull, dnull, pnull, dnull, (const int64_t*)nullptr, jobs)
  if (instance > 0) {
    const int ti = (instance - 1) / 8, ri = (instance - 1) % 8;
    if (ri > 5 || ti > 3) return hipErrorInvalidValue;
    if (ti == 0) { SID_CWB_R(8, ri) }
    else if (ti == 1) { SID_CWB_R(4, ri) }
    else if (ti == 2) { SID_CWB_R(2, ri) }
    else { SID_CWB_R(1, ri) }
  } else {
    const int ri = -instance - 1;
    if (ri == 0) SID_CLB(26);
    else if (ri == 1) SID_CLB(42);
    else if (ri == 2) SID_CLB(58);
    else if (ri == 3) SID_CLB(74);
    else if (ri == 4) SID_CLB(82);
    else if (ri == 5) SID_CLB(96);
    else return hipErrorInvalidValue;
  }
#undef SID_CLB
#undef SID_CWB_R
#undef SID_CWB
  return hipGetLastError();
}

bool cpqr_coop_supported(int m, int nc) { return m <= 256 && nc <= 64 * CQ_MINCPW && nc >= 1; }

static int coop_tpc(int m, int nc) {
  const int cpw2 = CQ_THREADS / 2;
  return (m <= 128 && (nc + cpw2 - 1) / cpw2 <= 64) ? 2 : 4;
}

size_t cpqr_coop_scratch_bytes(int m, int nc) {
  const int G = (nc + CQ_MINCPW - 1) / CQ_MINCPW;  // the most workgroups either layout uses
  return sizeof(double) * (size_t)(2 * G + 2 * G * CQ_MSTRIDE + 2 * G) +
         sizeof(int) * (size_t)(2 * G) + 64;
}

hipError_t launch_cpqr_coop(hipStream_t st, const double* X, int64_t ldx, int m, int nc, int kmax,
                            double rank_tol, void* scratch, unsigned int* sync2, int64_t* piv,
                            double* R, double* Q, int64_t* keff, double* stats,
                            bool cooperative, unsigned int* sticky, const int64_t* forced) {
  const int tpc = coop_tpc(m, nc);
  const int cpw = CQ_THREADS / tpc;
  const int G = (nc + cpw - 1) / cpw;
  double* pub_v = (double*)scratch;
  double* pub_col = pub_v + 2 * G;
  double* red = pub_col + (size_t)2 * G * CQ_MSTRIDE;
  int* pub_j = (int*)(red + 2 * G);
  unsigned int* bar = sync2;
  unsigned int* fail = sync2 + 1;
  hipLaunchKernelGGL(k_zero_u32, dim3(1), dim3(64), 0, st, sync2, 2);
  const int stride = (G <= 32) ? 8 : 1;
  const dim3 grid((unsigned)(G * stride)), block(CQ_THREADS);
  void* args[] = {(void*)&X, (void*)&ldx, (void*)&m, (void*)&nc, (void*)&kmax, (void*)&rank_tol,
                  (void*)&G, (void*)&stride, (void*)&pub_v, (void*)&pub_j, (void*)&pub_col,
                  (void*)&red, (void*)&bar, (void*)&fail, (void*)&piv, (void*)&R, (void*)&Q,
                  (void*)&keff, (void*)&stats, (void*)&forced, (void*)&sticky};
  const int rpt = (m + tpc - 1) / tpc;
  const void* kern =
      tpc == 2 ? (rpt <= 8    ? (const void*)k_cpqr_coop<2, 8>
                  : rpt <= 16 ? (const void*)k_cpqr_coop<2, 16>
                  : rpt <= 32 ? (const void*)k_cpqr_coop<2, 32>
                  : rpt <= 48 ? (const void*)k_cpqr_coop<2, 48>
                              : (const void*)k_cpqr_coop<2, 64>)
               : (rpt <= 8    ? (const void*)k_cpqr_coop<4, 8>
                  : rpt <= 16 ? (const void*)k_cpqr_coop<4, 16>
                  : rpt <= 32 ? (const void*)k_cpqr_coop<4, 32>
                  : rpt <= 48 ? (const void*)k_cpqr_coop<4, 48>
                              : (const void*)k_cpqr_coop<4, 64>);
  // The G workgroups must be resident together.  A plain launch (the
  // default) is checked against the device's occupancy for this kernel
  // first: the whole grid must fit at once; if other work keeps some
  // workgroups waiting for longer than the bounded spin, the wait gives up
  // (keff = -1 and the context's sticky flag, which sid_sync reports)
  // instead of hanging.  A cooperative launch (opt-in) guarantees
  // co-residency but waits for the device's other work to drain first,
  // which serialized it with the side stream's small solves (0.4 ms per
  // step on a non-default stream); it cannot be recorded into a graph.
  if (!cooperative) {
    int dev = 0, ncu = 0, per_cu = 0;
    hipError_t qe = hipGetDevice(&dev);
    if (qe == hipSuccess) qe = hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev);
    if (qe == hipSuccess) qe = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kern, CQ_THREADS, 0);
    if (qe != hipSuccess) return qe;
    if ((int64_t)per_cu * ncu < (int64_t)grid.x) return hipErrorCooperativeLaunchTooLarge;
  }
  const hipError_t e = cooperative
                           ? hipLaunchCooperativeKernel(kern, grid, block, args, 0, st)
                           : hipLaunchKernel(kern, grid, block, args, 0, st);
  return e;
}

// ---------------------------------------------------------------------------
// Upper-triangular solves with many right-hand sides.
// R11 (r x r, row-major ld r, r = *keff) gathered from the pivoted columns of
// mgsqr's R: R11(a, b) = R(a, piv[b]).
// ---------------------------------------------------------------------------
__global__ void k_gather_r11(const double* __restrict__ R_, int64_t ldr /* = nc */,
                             const int64_t* __restrict__ piv_, const int64_t* __restrict__ keff_,
                             int kcap, double* __restrict__ R11_,
                             const GatherR11Job* __restrict__ jobs) {
  if (jobs) {  // a batched launch: job blockIdx.y
    const GatherR11Job jb = jobs[blockIdx.y];
    R_ = jb.R;
    ldr = jb.ldr;
    piv_ = jb.piv;
    keff_ = jb.keff;
    kcap = jb.kcap;
    R11_ = jb.R11;
  }
  const auto R = to_global(R_);
  const auto piv = to_global(piv_);
  const auto keff_p = to_global(keff_);
  const auto R11 = to_global(R11_);
  const int keff = (int)*keff_p;
  for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < kcap * kcap; e += gridDim.x * blockDim.x) {
    const int a = e / kcap, b = e - a * kcap;
    R11[e] = (a < keff && b < keff && b >= a) ? R[(int64_t)a * ldr + piv[b]] : 0.0;
  }
}

// Solve R11 x = rhs_j for the columns j of a right-hand side.
//  mode 0 (ID coefficients): rhs_j = R(0:keff, j) (R row-major ld nc); pivot
//    columns get e_i; output Pd(:, j) (ld kcap) and P(:, j) (ld ldp, OutT).
//  mode 1 (single-pass T): rhs_j = C(0:keff, j) (column-major ld ldc); x is
//    scattered to T(piv[a], j) (ld ldt), other rows zero.
// One thread per right-hand side; x in LDS (column of this thread).
template <typename OutT, int MODE>
__global__ __launch_bounds__(64) void k_trsv_multi(
    const double* __restrict__ R11, int kcap, const int64_t* __restrict__ keff_p,
    const int64_t* __restrict__ piv, const double* __restrict__ rhs, int64_t ldrhs, int ncols,
    double* __restrict__ out64, int64_t ldo64, OutT* __restrict__ out, int64_t ldo) {
  extern __shared__ double s_x[];  // kcap x 64
  const int keff = (int)*keff_p;
  const int t = threadIdx.x;
  const int j = blockIdx.x * 64 + t;
  if (j >= ncols) return;
  int pos = -1;
  if (MODE == 0)
    for (int b = 0; b < keff; ++b)
      if (piv[b] == j) pos = b;
  if (pos < 0) {
    for (int a = keff - 1; a >= 0; --a) {
      double acc = (MODE == 0) ? rhs[(int64_t)a * ldrhs + j] : rhs[a + ldrhs * (int64_t)j];
      const double* Ra = R11 + (int64_t)a * kcap;
      for (int b = a + 1; b < keff; ++b) acc = fma(-Ra[b], s_x[b * 64 + t], acc);
      s_x[a * 64 + t] = acc / Ra[a];
    }
  }
  if (MODE == 0) {
    const auto x = out64 + ldo64 * j;
    for (int a = 0; a < kcap; ++a) {
      const double v = (pos >= 0) ? (a == pos ? 1.0 : 0.0) : (a < keff ? s_x[a * 64 + t] : 0.0);
      x[a] = v;
      if (out) out[a + ldo * j] = (OutT)v;
    }
  } else {
    const auto x = out64 + ldo64 * j;
    for (int a = 0; a < kcap; ++a) x[a] = 0.0;
    for (int a = 0; a < keff; ++a) x[piv[a]] = s_x[a * 64 + t];
  }
}

// The same solves with one wave per right-hand side (column-oriented back
// substitution: x_a = rhs_a / R11(a, a), then rhs_b -= R11(b, a) x_a for
// b < a in parallel over the lanes), R11 staged transposed in LDS.  NV = 2:
// kcap <= 128 (two rows per lane), R11 as a full kcap x kcap array; NV = 3:
// kcap <= TW_KMAX3 (three rows per lane), only the upper triangle, column a
// (rows 0..a) at a (a + 1) / 2, so that it fits the LDS.  The same
// operations in the same order either way.
constexpr int TW_WAVES = 8;
constexpr int TW_KMAX3 = 184;

__host__ __device__ constexpr int trsv_wave_rt(int nv, int kcap) {
  return nv == 2 ? kcap * kcap + 128 : kcap * (kcap + 1) / 2 + 192;
}

template <typename OutT, int MODE, int NV = 2>
__global__ __launch_bounds__(64 * TW_WAVES) void k_trsv_wave(
    const double* __restrict__ R11_, int kcap, const int64_t* __restrict__ keff_,
    const int64_t* __restrict__ piv_, const double* __restrict__ rhs_, int64_t ldrhs, int ncols,
    double* __restrict__ out64_, int64_t ldo64, OutT* __restrict__ out_, int64_t ldo,
    const TrsvJob* __restrict__ jobs) {
  if (jobs) {  // a batched launch: job blockIdx.y, out64 only
    const TrsvJob jb = jobs[blockIdx.y];
    R11_ = jb.R11;
    kcap = jb.kcap;
    keff_ = jb.keff;
    piv_ = jb.piv;
    rhs_ = jb.rhs;
    ldrhs = jb.ldrhs;
    ncols = jb.ncols;
    out64_ = jb.out64;
    ldo64 = jb.ldo64;
    out_ = nullptr;
  }
  const auto R11 = to_global(R11_);
  const auto keff_p = to_global(keff_);
  const auto piv = to_global(piv_);
  const auto rhs = to_global(rhs_);
  const auto out64 = to_global(out64_);
  const auto out = to_global(out_);
  extern __shared__ double s_tw[];
  double* s_rt = s_tw;                              // R11 transposed (see above; padded)
  double* s_dinv = s_rt + trsv_wave_rt(NV, kcap);   // 1 / R11(a, a)
  double* s_x = s_dinv + kcap;                      // [wave][a]
  int* s_inv = (int*)(s_x + TW_WAVES * kcap);       // inverse pivot permutation (mode 1)
  const int keff = (int)*keff_p;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  if constexpr (NV == 2) {
    for (int e = tid; e < kcap * kcap + 128; e += 64 * TW_WAVES) {
      const int a = e / kcap, b = e - a * kcap;
      s_rt[e] = (a < keff && b < keff) ? R11[(int64_t)b * kcap + a] : 0.0;
    }
  } else {
    for (int a = w; a < kcap; a += TW_WAVES)
      for (int b = lane; b <= a; b += 64)
        s_rt[a * (a + 1) / 2 + b] = (a < keff && b < keff) ? R11[(int64_t)b * kcap + a] : 0.0;
    for (int e = tid; e < 192; e += 64 * TW_WAVES) s_rt[kcap * (kcap + 1) / 2 + e] = 0.0;
  }
  for (int a = tid; a < kcap; a += 64 * TW_WAVES) {
    s_dinv[a] = a < keff ? 1.0 / R11[(int64_t)a * kcap + a] : 0.0;
    s_inv[a] = -1;
  }
  __syncthreads();
  if (MODE == 1)
    for (int a = tid; a < keff; a += 64 * TW_WAVES) s_inv[piv[a]] = a;
  __syncthreads();
  const int j = blockIdx.x * TW_WAVES + w;
  if (j >= ncols) return;
  const int b0 = lane, b1 = lane + 64, b2 = lane + 128;
  auto rhs_at = [&](int a) -> double {
    return MODE == 0 ? rhs[(int64_t)a * ldrhs + j] : rhs[a + ldrhs * (int64_t)j];
  };
  double v0 = b0 < keff ? rhs_at(b0) : 0.0;
  double v1 = b1 < keff ? rhs_at(b1) : 0.0;
  double v2 = (NV == 3 && b2 < keff) ? rhs_at(b2) : 0.0;
  int pos = -1;
  if (MODE == 0) {
    const bool hit0 = b0 < keff && piv[b0] == j, hit1 = b1 < keff && piv[b1] == j;
    const uint64_t m0 = __ballot(hit0), m1 = __ballot(hit1);
    pos = m0 ? __ffsll((unsigned long long)m0) - 1 : m1 ? 64 + __ffsll((unsigned long long)m1) - 1 : -1;
    if constexpr (NV == 3) {
      const uint64_t m2 = __ballot(b2 < keff && piv[b2] == j);
      if (pos < 0 && m2) pos = 128 + __ffsll((unsigned long long)m2) - 1;
    }
  }
  if (pos < 0) {
    for (int a = keff - 1; a >= 0; --a) {
      // rhs_a (already reduced) from lane a & 63, as two 32-bit halves
      const double va = NV == 3 ? (a < 64 ? v0 : a < 128 ? v1 : v2) : (a < 64 ? v0 : v1);
      const long long bits = __double_as_longlong(va);
      const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)bits, a & 63);
      const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(bits >> 32), a & 63);
      const double xa = __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo)) * s_dinv[a];
      // (entries past row a of the column are read but not used)
      const double* col = s_rt + (NV == 2 ? a * kcap : a * (a + 1) / 2);
      const double u0 = fma(-col[b0], xa, v0), u1 = fma(-col[b1], xa, v1);
      v0 = b0 < a ? u0 : (b0 == a ? xa : v0);
      v1 = b1 < a ? u1 : (b1 == a ? xa : v1);
      if constexpr (NV == 3) {
        const double u2 = fma(-col[b2], xa, v2);
        v2 = b2 < a ? u2 : (b2 == a ? xa : v2);
      }
    }
  }
  if (MODE == 0) {
    const auto x = out64 + ldo64 * j;
#pragma unroll
    for (int h = 0; h < NV; ++h) {
      const int a = h == 0 ? b0 : h == 1 ? b1 : b2;
      if (a >= kcap) continue;
      const double vh = h == 0 ? v0 : h == 1 ? v1 : v2;
      const double v = pos >= 0 ? (a == pos ? 1.0 : 0.0) : (a < keff ? vh : 0.0);
      x[a] = v;
      if (out) out[a + ldo * j] = (OutT)v;
    }
  } else {
    if (b0 < keff) s_x[w * kcap + b0] = v0;
    if (b1 < keff) s_x[w * kcap + b1] = v1;
    if (NV == 3 && b2 < keff) s_x[w * kcap + b2] = v2;
    __builtin_amdgcn_s_waitcnt(0xc07f);  // lgkmcnt(0): this wave's LDS writes done
    __builtin_amdgcn_wave_barrier();
    const auto x = out64 + ldo64 * j;
    for (int r = lane; r < kcap; r += 64) {
      const int a = s_inv[r];
      x[r] = a >= 0 ? s_x[w * kcap + a] : 0.0;
    }
  }
}

template <typename OutT, int MODE, int NV = 2>
static hipError_t trsv_wave_launch(hipStream_t st, const double* R11, int kcap, const int64_t* keff,
                                   const int64_t* piv, const double* rhs, int64_t ldrhs, int ncols,
                                   double* out64, int64_t ldo64, OutT* out, int64_t ldo) {
  const size_t shm =
      sizeof(double) * ((size_t)trsv_wave_rt(NV, kcap) + kcap + (size_t)TW_WAVES * kcap) +
      sizeof(int) * (size_t)kcap;
  auto kern = k_trsv_wave<OutT, MODE, NV>;
  if (shm > 65536)
    (void)hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)shm);
  hipLaunchKernelGGL(kern, dim3((unsigned)((ncols + TW_WAVES - 1) / TW_WAVES)), dim3(64 * TW_WAVES),
                     shm, st, R11, kcap, keff, piv, rhs, ldrhs, ncols, out64, ldo64, out, ldo,
                     (const TrsvJob*)nullptr);
  return hipGetLastError();
}

hipError_t launch_trsv_batch(hipStream_t st, int mode, const TrsvJob* jobs, int njobs,
                             int max_kcap, int max_ncols) {
  if (njobs <= 0) return hipSuccess;
  if (!jobs || max_kcap < 1 || max_kcap > 128 || max_ncols < 1) return hipErrorInvalidValue;
  const size_t shm =
      sizeof(double) * ((size_t)max_kcap * max_kcap + 128 + max_kcap + (size_t)TW_WAVES * max_kcap) +
      sizeof(int) * (size_t)max_kcap;
  auto kern = mode == 0 ? k_trsv_wave<double, 0> : k_trsv_wave<double, 1>;
  if (shm > 65536)
    (void)hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)shm);
  const double* dn = nullptr;
  const int64_t* in = nullptr;
  hipLaunchKernelGGL(kern, dim3((unsigned)((max_ncols + TW_WAVES - 1) / TW_WAVES), (unsigned)njobs),
                     dim3(64 * TW_WAVES), shm, st, dn, 0, in, in, dn, (int64_t)0, 0, (double*)nullptr,
                     (int64_t)0, (double*)nullptr, (int64_t)0, jobs);
  return hipGetLastError();
}

template <typename OutT, int MODE>
static hipError_t trsv_launch(hipStream_t st, const double* R11, int kcap, const int64_t* keff,
                              const int64_t* piv, const double* rhs, int64_t ldrhs, int ncols,
                              double* out64, int64_t ldo64, OutT* out, int64_t ldo) {
  const size_t shm = sizeof(double) * (size_t)kcap * 64;
  auto kern = k_trsv_multi<OutT, MODE>;
  if (shm > 65536)
    (void)hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)shm);
  hipLaunchKernelGGL(kern, dim3((unsigned)((ncols + 63) / 64)), dim3(64), shm, st, R11, kcap, keff,
                     piv, rhs, ldrhs, ncols, out64, ldo64, out, ldo);
  return hipGetLastError();
}

hipError_t launch_gather_r11(hipStream_t st, const double* R, int nc, const int64_t* piv,
                             const int64_t* keff, int kcap, double* R11) {
  hipLaunchKernelGGL(k_gather_r11, dim3(64), dim3(256), 0, st, R, (int64_t)nc, piv, keff, kcap, R11,
                     (const GatherR11Job*)nullptr);
  return hipGetLastError();
}

hipError_t launch_gather_r11_batch(hipStream_t st, const GatherR11Job* jobs, int njobs) {
  if (njobs <= 0) return hipSuccess;
  const double* dn = nullptr;
  const int64_t* in = nullptr;
  hipLaunchKernelGGL(k_gather_r11, dim3(64, (unsigned)njobs), dim3(256), 0, st, dn, (int64_t)0, in,
                     in, 0, (double*)nullptr, jobs);
  return hipGetLastError();
}

hipError_t launch_id_coefficients(hipStream_t st, const double* R, int nc, const int64_t* piv,
                                  const int64_t* keff, int kcap, double* R11, double* Pd,
                                  void* P, int64_t ldp, bool p_is_f64) {
  hipLaunchKernelGGL(k_gather_r11, dim3(64), dim3(256), 0, st, R, (int64_t)nc, piv, keff, kcap, R11,
                     (const GatherR11Job*)nullptr);
  if (kcap <= 128) {
    if (p_is_f64)
      return trsv_wave_launch<double, 0>(st, R11, kcap, keff, piv, R, nc, nc, Pd, kcap, (double*)P, ldp);
    return trsv_wave_launch<float, 0>(st, R11, kcap, keff, piv, R, nc, nc, Pd, kcap, (float*)P, ldp);
  }
  if (kcap <= TW_KMAX3) {
    if (p_is_f64)
      return trsv_wave_launch<double, 0, 3>(st, R11, kcap, keff, piv, R, nc, nc, Pd, kcap, (double*)P,
                                            ldp);
    return trsv_wave_launch<float, 0, 3>(st, R11, kcap, keff, piv, R, nc, nc, Pd, kcap, (float*)P,
                                         ldp);
  }
  if (p_is_f64)
    return trsv_launch<double, 0>(st, R11, kcap, keff, piv, R, nc, nc, Pd, kcap, (double*)P, ldp);
  return trsv_launch<float, 0>(st, R11, kcap, keff, piv, R, nc, nc, Pd, kcap, (float*)P, ldp);
}

hipError_t launch_small_solve(hipStream_t st, const double* RM, int l, const int64_t* pivM,
                              const int64_t* rM, double* R11, const double* C, int64_t ldc, int kc,
                              double* T) {
  hipLaunchKernelGGL(k_gather_r11, dim3(64), dim3(256), 0, st, RM, (int64_t)l, pivM, rM, l, R11,
                     (const GatherR11Job*)nullptr);
  if (l <= 128)
    return trsv_wave_launch<double, 1>(st, R11, l, rM, pivM, C, ldc, kc, T, l, (double*)nullptr, 0);
  if (l <= TW_KMAX3)
    return trsv_wave_launch<double, 1, 3>(st, R11, l, rM, pivM, C, ldc, kc, T, l, (double*)nullptr, 0);
  return trsv_launch<double, 1>(st, R11, l, rM, pivM, C, ldc, kc, T, l, (double*)nullptr, 0);
}

}  // namespace sid
