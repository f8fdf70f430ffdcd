// sid_api.hip -- host runtime behind include/sid.h: argument validation,
// grow-only device workspace, and the launch sequence of a compression on
// the context's stream.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "../../include/sid.h"

#include "sid_adaptive.hpp"
#include "sid_apply.hpp"
#include "sid_sketch_f64.hpp"
#include "sid_svd.hpp"
#include "sid_interp.hpp"
#include "sid_kernels.hpp"

// ---------------------------------------------------------------------------
// Allocation-free sketch (sid_sketch_noalloc): the pass's scratch (Omega's
// values, Omega^T in bfloat16, the per-workgroup-pair W partials) lives in
// this file-scope device array.  Host code never passes the array's name to
// a kernel: its device address is taken once per device at set-up
// (hipGetSymbolAddress in sid_create) and kept in noalloc_ptr[device].
// ---------------------------------------------------------------------------
#define SID_NOALLOC_SCRATCH_BYTES (80u << 20)
static __device__ __align__(256) unsigned char scratch[SID_NOALLOC_SCRATCH_BYTES];

namespace {

constexpr int kMaxDevices = 64;
std::mutex noalloc_mu;
void* noalloc_ptr[kMaxDevices] = {};

// the device address of `scratch` on the current device (set-up only: the
// device must be current); nullptr on failure
void* noalloc_scratch_init(int device) {
  if (device < 0 || device >= kMaxDevices) return nullptr;
  std::lock_guard<std::mutex> g(noalloc_mu);
  if (!noalloc_ptr[device]) {
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess) {
      (void)hipGetLastError();
      return nullptr;
    }
    noalloc_ptr[device] = p;
  }
  return noalloc_ptr[device];
}

enum Slot {
  WS_OMEGA, WS_PART, WS_W, WS_WR, WS_NRM, WS_PIV, WS_R, WS_Q, WS_KEFF, WS_STATS, WS_PD,
  WS_ERR, WS_Y, WS_M, WS_MPR, WS_WJ, WS_PIVM, WS_RM, WS_QM, WS_RKM, WS_C, WS_T, WS_MIX,
  WS_STATSM, WS_NORMPART, WS_NORMOUT, WS_OM64, WS_PARTF, WS_OMT, WS_COOP, WS_SYNC, WS_R11, WS_R11M, WS_FITPART, WS_YTMP, WS_REF_W, WS_REF_WJ, WS_OMP, WS_A8, WS_PSIIMG, WS_IACJT, WS_IPB, WS_IB, WS_IPART, WS_AZ, WS_AE2, WS_APART, WS_SV_H, WS_SV_B, WS_SV_Q, WS_SV_OM32,
  WS_SV_OM, WS_SV_SMALL, WS_SV_WP, WS_SV_TSP, WS_PROBE, WS_COUNT
};

struct Buf {
  void* p = nullptr;
  size_t bytes = 0;
};

// What the batched sketch pass reads of one problem (its plan is reused
// only for exactly the same values)
struct BatchSig {
  const void* A;
  int64_t N, n, lda, lq, l, lz, k;
  uint64_t seed;
  double rank_tol, rcond;  // the mgsqr jobs' stopping tolerances
  double probe_tol;        // adaptive rank (> 0) keeps the per-problem tail
  bool operator==(const BatchSig& o) const {
    return A == o.A && N == o.N && n == o.n && lda == o.lda && lq == o.lq && l == o.l &&
           lz == o.lz && k == o.k && seed == o.seed && rank_tol == o.rank_tol &&
           rcond == o.rcond && probe_tol == o.probe_tol;
  }
};

// One problem's factorization results that the batched mgsqr launches write
// (W's mgsqr; in single pass also M = W(0:lz, :) Omega, Mpr and M's mgsqr)
struct BatchFactor {
  bool pre = false;  // its mgsqr runs in the batched launches
  int64_t *piv = nullptr, *keff = nullptr, *pivM = nullptr, *rkM = nullptr;
  double *R = nullptr, *Q = nullptr, *stats = nullptr, *om64 = nullptr, *M = nullptr,
         *Mpr = nullptr, *RM = nullptr, *QM = nullptr, *statsM = nullptr;
  // the steps after mgsqr, when the whole batch runs them as batched
  // launches (BatchPlan::tail)
  double *R11 = nullptr, *Pd = nullptr, *WJ = nullptr, *C = nullptr, *T = nullptr,
         *R11M = nullptr, *mix = nullptr, *fitpart = nullptr, *err = nullptr;
};

// Device state of one batch of problems for the persistent sketch pass: the
// queue table, the counter and every problem's partials, W and (single pass)
// Omega, Omega^T and Y, in one allocation owned by the context.  A graph
// that captured a batched call reads these buffers at every replay.
struct BatchPlan {
  std::vector<BatchSig> sig;
  int dmode = 0;
  bool wanty = false;
  void* dev = nullptr;
  size_t bytes = 0;
  sid::FbBatchEntry* d_tab = nullptr;
  unsigned int* d_queue = nullptr;          // one counter per layout class
  std::vector<sid::FbBatchClass> classes;  // the table's layout classes, in order
  int64_t max_lqn = 0;
  int max_n = 0;
  std::vector<double*> W;       // by problem index
  std::vector<float*> Y, omega;
  std::vector<BatchFactor> fac;  // by problem index
  // the batched mgsqr launches: jobs grouped by kernel instance
  sid::CpqrJob* d_jobs = nullptr;
  std::vector<std::array<int, 3>> job_groups;  // (instance, first job, count)
  // single pass: the products before M's mgsqr, in two launches
  sid::OmegaJob* d_om_jobs = nullptr;
  sid::Gemm64Job* d_mm_jobs = nullptr;
  int n_om_jobs = 0, n_mm_jobs = 0, mm_max_m = 0, mm_max_n = 0;
  int64_t om_max_count = 0;
  // single pass, every problem batched and no adaptive rank: the steps after
  // mgsqr as batched launches too (job tables below, one job per problem),
  // then per problem only P's conversion, AJ = Y T and the result copies
  bool tail = false;
  sid::GatherR11Job* d_gr11 = nullptr;  // [count] W's R11, then [count] M's
  sid::TrsvJob *d_trsv0 = nullptr, *d_trsv1 = nullptr;
  sid::RatioJob* d_ratio = nullptr;
  sid::GatherBlockJob* d_gblock = nullptr;
  sid::Gemm64Job *d_gemm_c = nullptr, *d_gemm_mix = nullptr;
  sid::FitJob* d_fit = nullptr;
  // AJ = Y T of every problem with an output in one launch: the device job
  // table and the host copy it was last uploaded from (the outputs are the
  // caller's and may change from call to call)
  sid::ApplyJob* d_apply = nullptr;
  std::vector<sid::ApplyJob> apply_host;
  int n_gemm_mix = 0, t_max_k = 0, t_max_n = 0, t_max_l = 0, t_max_gblock = 0, t_max_q = 0,
      t_max_qn = 0;
};

}  // namespace

struct sid_ctx {
  int device = 0;
  int num_cu = 1;
  // cooperative launch of the multi-workgroup pivoted QR outside graph
  // capture (SID_COOPERATIVE=1 turns it on; by default a plain launch
  // checked against the device's occupancy)
  bool cooperative = false;
  // sticky device flag: a device-wide wait of the pivoted QR timed out
  // (set by the kernels, read and cleared by sid_sync)
  unsigned int* fail_flag = nullptr;
  // SID_SKETCH_PAIRS=1: the bfloat16 sketch forms take the workgroup-pair
  // pass also where the one-workgroup-per-row-range pass applies (for
  // comparison; by default the pair pass serves the shapes the other one
  // does not take: l > 128 or l + e + q > 160)
  bool sketch_pairs = false;
  hipStream_t stream = nullptr;
  bool own_stream = false;
  std::string err;
  Buf ws[WS_COUNT];
  size_t limit = 0;
  // batched calls: child contexts (own stream and workspace each) and the
  // events that order them after and before this context's stream
  std::vector<sid_ctx*> children;
  std::vector<hipEvent_t> child_done;
  hipEvent_t fork = nullptr;
  // single pass: the factorization of M (independent of the pivots of W)
  // runs on a side stream while mgsqr of W runs on the main one
  hipStream_t side = nullptr;
  hipEvent_t side_fork = nullptr, side_join = nullptr;
  // batched calls on the persistent sketch pass: the plans of the last few
  // problem sets (newest last) and the number of child streams of the
  // factorization phase (set by the autotuner)
  std::vector<BatchPlan*> plans;
  int batch_streams = 4;
  std::vector<std::pair<std::string, int>> tuned;  // autotuner cache: key -> streams
};

struct sid_rowset {
  sid_ctx* ctx = nullptr;
  int64_t* d_rows = nullptr;
  int64_t count = 0;
  int64_t N = 0;
};

// Streaming state: the sketches of the columns seen so far, owned by the
// stream (not by the context's workspace, which other calls reuse).
struct sid_stream {
  sid_ctx* ctx = nullptr;
  sid_params p{};
  sid_dtype dtype = SID_F32;
  int64_t N = 0, n_max = 0;
  int64_t lq = 0, l = 0;
  bool single = false;
  int64_t cols = 0;         // columns already sketched
  int64_t staged = 0;       // columns copied into the stage, not yet sketched
  int64_t stage_cols = 0;   // stage capacity (columns)
  int64_t ld_stage = 0;     // stage leading dimension (multiple of 4)
  void* stage = nullptr;    // N x stage_cols (data type), allocated on first use
  __bf16* psi_img = nullptr;  // Psi images of the workgroup-pair pass (formed once)
  double* W = nullptr;      // lq x n_max, column-major
  void* Y = nullptr;        // N x l row-major (single pass), FP64 for F64 sketches else FP32
  bool y_init = false;
  // SBR-SVD streams (sid_svd_stream_begin): the ID fields above run the pass
  // forming G = W^T (two-pass mode, l selection rows); every sketched block
  // also updates H += A_blk G_blk
  bool svd = false;
  sid_svd_params sp{};
  double* H = nullptr;      // N x l, column-major
  double* Wp = nullptr;     // one block of W with its leading dimension rounded up to 16
};

namespace {

sid_status fail(sid_ctx* ctx, sid_status st, const std::string& msg) {
  if (ctx) ctx->err = msg;
  return st;
}

sid_status hip_fail(sid_ctx* ctx, hipError_t e, const char* where) {
  std::string m = std::string(where) + ": " + hipGetErrorString(e);
  return fail(ctx, SID_EDEVICE, m);
}

size_t held_bytes(const sid_ctx* c) {
  size_t s = 0;
  for (const Buf& b : c->ws) s += b.bytes;
  return s;
}

// grow-only workspace slot; returns nullptr (and sets the error) on failure
void* ws(sid_ctx* c, Slot s, size_t bytes) {
  if (bytes == 0) bytes = 16;
  Buf& b = c->ws[s];
  if (b.bytes >= bytes) return b.p;
  // growing synchronizes, frees and allocates: none of that may happen while
  // the stream is being captured into a graph
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  if (hipStreamIsCapturing(c->stream, &cs) == hipSuccess && cs != hipStreamCaptureStatusNone) {
    c->err = "the workspace would have to grow while the stream is being captured; call "
             "sid_reserve with the same shape and parameters before capture";
    return nullptr;
  }
  const size_t want = bytes + bytes / 8;
  if (c->limit && held_bytes(c) - b.bytes + want > c->limit) {
    c->err = "workspace limit exceeded";
    return nullptr;
  }
  if (b.p) {
    (void)hipStreamSynchronize(c->stream);
    (void)hipFree(b.p);
    b.p = nullptr;
    b.bytes = 0;
  }
  void* p = nullptr;
  if (hipMalloc(&p, want) != hipSuccess) {
    (void)hipGetLastError();
    c->err = "device allocation of " + std::to_string(want) + " bytes failed";
    return nullptr;
  }
  b.p = p;
  b.bytes = want;
  return p;
}

struct Shape {
  int64_t N, n, k, l, q, lz, lq, Ns, nchunks;
  bool single;
  int prec;
};

// which mgsqr kernel an (m x nc) factorization uses.  0: one workgroup,
// residual in registers; 3: one workgroup, part of it in LDS (up to 96 rows:
// beyond, its LDS traffic per step costs more than the cooperative kernel's
// device-wide barrier; measured at 120 x 500); 1: several workgroups; 2: the
// general kernel.  (The cooperative and the general kernels use context
// scratch, so two of the same kind must not run at once.)
int mgsqr_kind(int m, int nc) {
  return sid::cpqr_wg_supported(m, nc)                 ? 0
         : (m <= 96 && sid::cpqr_wgl_supported(m, nc)) ? 3
         : sid::cpqr_coop_supported(m, nc)             ? 1
                                                       : 2;
}

double default_rcond(int prec) {
  switch (prec) {
    case SID_SK_F64: return 1e-13;
    case SID_SK_F32: return 1e-6;
    case SID_SK_BF16X2: return 1e-5;
    case SID_SK_FP8E4M3: return 1e-2;
    default: return 1e-3;
  }
}

// row chunks of the generic sketch kernels (partials per chunk)
int64_t nchunks_for(int64_t Ns, int64_t n) {
  const int64_t ntiles = (n + 63) / 64;
  int64_t nch = (Ns + 1023) / 1024;
  int64_t cap = 2048 / ntiles;
  if (cap < 1) cap = 1;
  if (nch > cap) nch = cap;
  if (nch < 1) nch = 1;
  return nch;
}

sid_status validate(sid_ctx* ctx, int64_t N, int64_t n, const sid_params* p, Shape* sh) {
  if (!p) return fail(ctx, SID_EINVAL, "params is NULL");
  if (N <= 0 || n <= 0) return fail(ctx, SID_EINVAL, "N and n must be positive");
  if (p->k < 1) return fail(ctx, SID_EINVAL, "k must be >= 1");
  if (p->oversample < 0) return fail(ctx, SID_EINVAL, "oversample must be >= 0");
  if (p->probe_rows < 0) return fail(ctx, SID_EINVAL, "probe_rows must be >= 0");
  if (p->k > n) return fail(ctx, SID_EINVAL, "k must not exceed the number of columns n");
  if (p->mode != SID_TWO_PASS && p->mode != SID_SINGLE_PASS && p->mode != SID_COARSE_SKELETON)
    return fail(ctx, SID_EINVAL, "unknown mode");
  if (p->mode == SID_COARSE_SKELETON && !p->coarse)
    return fail(ctx, SID_EINVAL, "the coarse-skeleton mode needs a coarse row set");
  if (p->prec < SID_SK_F64 || p->prec > SID_SK_FP8E4M3)
    return fail(ctx, SID_EINVAL, "unknown sketch precision");
  if (!(p->rank_tol >= 0.0) || !(p->sp_rcond >= 0.0))
    return fail(ctx, SID_EINVAL, "rank_tol and sp_rcond must be >= 0");
  if (p->refine != 0 && p->refine != 1) return fail(ctx, SID_EINVAL, "refine must be 0 or 1");
  if (p->refine && (p->refine_prec < SID_SK_F64 || p->refine_prec > SID_SK_FP8E4M3))
    return fail(ctx, SID_EINVAL, "unknown refinement precision");
  if (p->select != SID_SEL_GAUSS && p->select != SID_SEL_ROWS_LITERAL)
    return fail(ctx, SID_EINVAL, "unknown select");
  if (!(p->probe_tol >= 0.0) || !std::isfinite(p->probe_tol))
    return fail(ctx, SID_EINVAL, "probe_tol must be finite and >= 0");
  if (p->probe_tol > 0.0 && (p->probe_rows < 1 || p->select != SID_SEL_GAUSS))
    return fail(ctx, SID_EINVAL, "an adaptive rank (probe_tol > 0) needs probe rows");
  if (p->select == SID_SEL_ROWS_LITERAL) {
    if (!p->coarse) return fail(ctx, SID_EINVAL, "literal selection needs a coarse row set");
    if (p->mode == SID_SINGLE_PASS)
      return fail(ctx, SID_EINVAL, "literal selection has no single-pass form");
    if (p->prec != SID_SK_F64 && p->prec != SID_SK_F32)
      return fail(ctx, SID_EINVAL, "literal selection reads the data in F64 or F32");
    if (p->refine) return fail(ctx, SID_EINVAL, "literal selection has no refinement pass");
    if (p->coarse->ctx != ctx) return fail(ctx, SID_EINVAL, "row set belongs to another context");
    if (p->coarse->N != N) return fail(ctx, SID_EINVAL, "row set was built for a different N");
    const int64_t Ns = p->coarse->count;
    if (Ns > 4096) return fail(ctx, SID_EINVAL, "literal selection takes at most 4096 coarse rows");
    if (Ns <= p->k) return fail(ctx, SID_EINVAL, "coarse row count must exceed k");
    sh->N = N;
    sh->n = n;
    sh->k = p->k;
    sh->l = sh->lz = sh->lq = Ns;
    sh->q = 0;
    sh->Ns = Ns;
    sh->nchunks = 1;
    sh->single = false;
    sh->prec = p->prec;
    return SID_OK;
  }
  const int64_t l = p->k + p->oversample;
  const bool single = p->mode == SID_SINGLE_PASS;
  const int64_t e = single ? (p->corange_rows < 0 ? p->oversample : p->corange_rows) : 0;
  const int64_t lz = l + e;
  const int64_t lq = lz + p->probe_rows;
  if (lq > 256) return fail(ctx, SID_EINVAL, "sketch rows (l + co-range + probe) must be <= 256");
  int64_t Ns = N;
  if (p->coarse) {
    if (p->coarse->ctx != ctx) return fail(ctx, SID_EINVAL, "row set belongs to another context");
    if (p->coarse->N != N) return fail(ctx, SID_EINVAL, "row set was built for a different N");
    Ns = p->coarse->count;
    if (Ns <= p->k) return fail(ctx, SID_EINVAL, "coarse row count must exceed k");
  }
  sh->N = N;
  sh->n = n;
  sh->k = p->k;
  sh->l = l;
  sh->q = p->probe_rows;
  sh->lz = lz;
  sh->lq = lq;
  sh->Ns = Ns;
  sh->nchunks = nchunks_for(Ns, n);
  sh->single = p->mode == SID_SINGLE_PASS;
  sh->prec = p->prec;
  return SID_OK;
}

// rows of the skeleton output AJ: |S| for the coarse skeleton (Alg. 6), else N
int64_t skeleton_rows(const sid_params* p, int64_t N) {
  return (p->mode == SID_COARSE_SKELETON && p->coarse) ? p->coarse->count : N;
}

struct Work {
  double *az, *ae2, *apart;  // adaptive rank: Z (q x k), prefix errors (k + 1), partials
  float* omega;
  double *part, *W, *Wr, *nrm, *R, *Q, *stats, *Pd, *err;
  int64_t *piv, *keff;
  void* Y;
  double *M, *Mpr, *WJ, *RM, *QM, *C, *T, *mix, *statsM, *om64;
  int64_t *pivM, *rkM;
  void* coop;
  unsigned int* sync2;
  double* R11;
  double* R11M;  // single pass: the triangular factor of M's solve (beside R11's use)
  double* fitpart;
};

// sketch_bufs = false: the caller brings Omega, W and Y (the batched pass);
// only the factorization's buffers are reserved
sid_status reserve(sid_ctx* c, const Shape& s, Work* w, bool sketch_bufs = true) {
  const size_t d = sizeof(double);
  const int64_t mx = s.n > s.lz ? s.n : s.lz;
  static double dummy_d;
  static float dummy_f;
  w->omega = sketch_bufs ? (float*)ws(c, WS_OMEGA, sizeof(float) * (size_t)(s.n * s.l)) : &dummy_f;
  w->part = sketch_bufs ? (double*)ws(c, WS_PART, d * (size_t)(s.nchunks * s.lq * s.n)) : &dummy_d;
  w->W = sketch_bufs ? (double*)ws(c, WS_W, d * (size_t)(s.lq * s.n)) : &dummy_d;
  w->Wr = (double*)ws(c, WS_WR, d * (size_t)(s.lz * s.l > s.l * s.n ? s.lz * s.l : s.l * s.n));
  w->nrm = (double*)ws(c, WS_NRM, d * (size_t)mx);
  w->piv = (int64_t*)ws(c, WS_PIV, sizeof(int64_t) * (size_t)s.k);
  w->R = (double*)ws(c, WS_R, d * (size_t)(s.k * s.n));
  w->Q = (double*)ws(c, WS_Q, d * (size_t)(s.l * s.k));
  w->keff = (int64_t*)ws(c, WS_KEFF, sizeof(int64_t));
  w->stats = (double*)ws(c, WS_STATS, d * 2);
  w->Pd = (double*)ws(c, WS_PD, d * (size_t)(s.k * s.n));
  w->err = (double*)ws(c, WS_ERR, d * 2);
  {
    // the probe rows, or (adaptive rank) the selection rows at the chosen rank
    const int64_t fr = s.q > s.l ? s.q : s.l;
    w->fitpart = (double*)ws(c, WS_FITPART, d * (size_t)(2 * ((fr * s.n + 255) / 256) + 2));
  }
  if (!w->fitpart) return SID_ENOMEM;
  {
    const int mmax = (int)s.lz;
    const int ncmax = (int)(s.n > s.l ? s.n : s.l);
    w->coop = ws(c, WS_COOP, sid::cpqr_coop_scratch_bytes(mmax, ncmax));
    w->sync2 = (unsigned int*)ws(c, WS_SYNC, 64);
    const int64_t kk = s.k > s.l ? s.k : s.l;
    w->R11 = (double*)ws(c, WS_R11, d * (size_t)(kk * kk));
    if (!w->coop || !w->sync2 || !w->R11) return SID_ENOMEM;
  }
  if (!w->omega || !w->part || !w->W || !w->Wr || !w->nrm || !w->piv || !w->R || !w->Q ||
      !w->keff || !w->stats || !w->Pd || !w->err)
    return SID_ENOMEM;
  w->az = (double*)ws(c, WS_AZ, d * (size_t)((s.q > 0 ? s.q : 1) * s.k));
  w->ae2 = (double*)ws(c, WS_AE2, d * (size_t)(s.k + 1));
  w->apart = (double*)ws(c, WS_APART, d * (size_t)(sid::probe_adapt_blocks((int)(s.q > 0 ? s.q : 1),
                                                                           (int)s.n) * (s.k + 1)));
  if (!w->az || !w->ae2 || !w->apart) return SID_ENOMEM;
  w->Y = nullptr;
  if (s.single) {
    const size_t ye = (s.prec == SID_SK_F64) ? d : sizeof(float);
    w->Y = sketch_bufs ? ws(c, WS_Y, ye * (size_t)(s.N * s.l)) : (void*)&dummy_f;
    w->M = (double*)ws(c, WS_M, d * (size_t)(s.lz * s.l));
    w->Mpr = (double*)ws(c, WS_MPR, d * (size_t)((s.q > 0 ? s.q : 1) * s.l));
    w->WJ = (double*)ws(c, WS_WJ, d * (size_t)(s.lz * s.k));
    w->RM = (double*)ws(c, WS_RM, d * (size_t)(s.l * s.l));
    w->QM = (double*)ws(c, WS_QM, d * (size_t)(s.lz * s.l));
    w->C = (double*)ws(c, WS_C, d * (size_t)(s.l * s.k));
    w->T = (double*)ws(c, WS_T, d * (size_t)(s.l * s.k));
    w->mix = (double*)ws(c, WS_MIX, d * (size_t)((s.q > 0 ? s.q : 1) * s.k));
    w->statsM = (double*)ws(c, WS_STATSM, d * 2);
    w->pivM = (int64_t*)ws(c, WS_PIVM, sizeof(int64_t) * (size_t)s.l);
    w->rkM = (int64_t*)ws(c, WS_RKM, sizeof(int64_t));
    w->om64 = (double*)ws(c, WS_OM64, d * (size_t)(s.n * s.l));
    w->R11M = (double*)ws(c, WS_R11M, d * (size_t)(s.l * s.l));
    if (!w->om64 || !w->Y || !w->M || !w->Mpr || !w->WJ || !w->RM || !w->QM || !w->C || !w->T || !w->mix ||
        !w->statsM || !w->pivM || !w->rkM || !w->R11M)
      return SID_ENOMEM;
  }
  return SID_OK;
}

// Which kernels a sketch pass of this shape takes (run_sketch) and what it
// needs in the workspace (sid_reserve, which assumes FP32 data with a
// 16-byte aligned base and lda % 4 == 0).
enum class SketchPath { PAIR_BF16, FUSED_BF16, FUSED_F32, FP8_GENERAL, F64_TILED, GENERAL };

SketchPath plan_sketch(const sid_ctx* ctx, sid_dtype dtype, int64_t lda, const void* A, int prec,
                       const Shape& sh, bool has_rows, bool want_y) {
  const bool bf = prec == SID_SK_BF16 || prec == SID_SK_BF16X2 || prec == SID_SK_FP8E4M3;
  const int64_t slab = sh.n < 512 ? sh.n : 512;
  // a coarse row list runs on the streaming pass for the bf16 forms of the
  // two-pass (W only) sketch
  const bool rows_ok = !has_rows || (!want_y && (prec == SID_SK_BF16 || prec == SID_SK_BF16X2));
  const bool fused_ok = dtype == SID_F32 && rows_ok &&
                        sid::fused_bf16_supported(slab, (int)sh.lq, (int)sh.l, lda, A, has_rows);
  if (bf && fused_ok && !ctx->sketch_pairs) return SketchPath::FUSED_BF16;
  // the workgroup-pair pass (all rows, FP32 data, column slabs of up to
  // sketch_v2_slab columns; Y's offsets fit 32 bits): l up to 256 and
  // l + e + q up to 256, e.g. k = 150, p = 30
  if (bf && !has_rows && dtype == SID_F32 &&
      (!want_y || (uint64_t)sh.N * (uint64_t)sh.l * 4u < (1ull << 32))) {
    const int vslab = sid::sketch_v2_slab((int)sh.lq, (int)sh.l, want_y);
    if (vslab > 0) {
      const int64_t vs = sh.n < vslab ? sh.n : vslab;
      if (sid::sketch_v2_supported(vs, (int)sh.lq, (int)sh.l, want_y, lda, A))
        return SketchPath::PAIR_BF16;
    }
  }
  if (bf && fused_ok) return SketchPath::FUSED_BF16;
  if (prec == SID_SK_FP8E4M3) return SketchPath::FP8_GENERAL;
  if (prec == SID_SK_F32 && fused_ok) return SketchPath::FUSED_F32;
  if (prec == SID_SK_F64 && !has_rows) return SketchPath::F64_TILED;
  return SketchPath::GENERAL;
}

// whether run_sketch can add this pass's part of Y in the kernel (y_add):
// the workgroup-pair pass does
bool sketch_adds_y(const sid_ctx* ctx, sid_dtype dtype, int64_t lda, const void* A,
                   const Shape& sh) {
  return plan_sketch(ctx, dtype, lda, A, sh.prec, sh, false, true) == SketchPath::PAIR_BF16;
}

// reserve what run_sketch takes beyond reserve(): the matrix-core pass's
// partials and Omega^T, the slab sum of Y (the one-workgroup pass), the FP8
// data copy
sid_status reserve_sketch(sid_ctx* ctx, const Shape& sh, int prec, bool has_rows,
                                 bool want_y) {
  const SketchPath path = plan_sketch(ctx, SID_F32, 4, nullptr, prec, sh, has_rows, want_y);
  const int64_t slab = sh.n < 512 ? sh.n : 512;
  if (path == SketchPath::PAIR_BF16) {
    const int vslab = sid::sketch_v2_slab((int)sh.lq, (int)sh.l, want_y);
    const int64_t vs = sh.n < vslab ? sh.n : vslab;
    int64_t rpp = 0;
    const int64_t pairs = sid::sketch_v2_pairs(sh.N, ctx->num_cu, &rpp);
    if (!ws(ctx, WS_PARTF, sizeof(float) * (size_t)(pairs * sh.lq * vs)) ||
        !ws(ctx, WS_OMT, sizeof(uint16_t) * sid::sketch_v2_omt_elems((int)sh.l, (int)vs)))
      return SID_ENOMEM;
    const size_t img_bytes = sid::sketch_v2_psi_image_bytes(sh.N, (int)sh.lq);
    if (sh.n > vs && img_bytes > 0 && !ws(ctx, WS_PSIIMG, img_bytes)) return SID_ENOMEM;
  } else if (path == SketchPath::FUSED_BF16 || path == SketchPath::FUSED_F32) {
    int64_t rpw = 0;
    const int64_t grid = sid::fused_bf16_grid(sh.N, ctx->num_cu, &rpw);  // N >= Ns: the larger
    const bool bf = path == SketchPath::FUSED_BF16;
    if (!ws(ctx, WS_PARTF, sizeof(float) * (size_t)(grid * sh.lq * slab)) ||
        !ws(ctx, bf ? WS_OMT : WS_OMP, bf ? sizeof(uint16_t) * 128 * 512 : sizeof(float) * 128 * 512))
      return SID_ENOMEM;
    if (want_y && sh.n > slab && !ws(ctx, WS_YTMP, sizeof(float) * (size_t)(sh.N * sh.l)))
      return SID_ENOMEM;
  } else if (path == SketchPath::FP8_GENERAL) {
    if (!ws(ctx, WS_A8, sizeof(float) * (size_t)(sh.N * sh.n))) return SID_ENOMEM;
  }
  return SID_OK;
}

#define SID_NEED_DEVICE(ctx)                                                        \
  do {                                                                              \
    if ((ctx)->device < 0)                                                          \
      return fail((ctx), SID_ESTATE, "validation-only context (created with device -1)"); \
  } while (0)

#define SID_CHECK(expr, where)                        \
  do {                                                \
    hipError_t e_ = (expr);                           \
    if (e_ != hipSuccess) return hip_fail(ctx, e_, where); \
  } while (0)

}  // namespace

extern "C" {

void sid_params_init(sid_params* p, int64_t k) {
  if (!p) return;
  std::memset(p, 0, sizeof(*p));
  p->k = k;
  p->oversample = 10;
  p->seed = 0;
  p->coarse = nullptr;
  p->mode = SID_TWO_PASS;
  p->prec = SID_SK_F32;
  p->probe_rows = 10;
  p->corange_rows = -1;
  p->rank_tol = 0.0;
  p->sp_rcond = 0.0;
  p->refine = 0;
  p->refine_prec = SID_SK_BF16X2;
  p->select = SID_SEL_GAUSS;
  p->probe_tol = 0.0;
}

sid_status sid_create(sid_ctx** out, int device, void* hip_stream) {
  if (!out) return SID_EINVAL;
  *out = nullptr;
  if (device == -1) {  // validation-only context: checks arguments, launches nothing
    sid_ctx* c = new (std::nothrow) sid_ctx();
    if (!c) return SID_ENOMEM;
    c->device = -1;
    *out = c;
    return SID_OK;
  }
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || ndev <= 0) {
    (void)hipGetLastError();
    return SID_EDEVICE;
  }
  if (device < 0 || device >= ndev) return SID_EINVAL;
  if (hipSetDevice(device) != hipSuccess) return SID_EDEVICE;
  sid_ctx* c = new (std::nothrow) sid_ctx();
  if (!c) return SID_ENOMEM;
  c->device = device;
  {
    const char* env = std::getenv("SID_COOPERATIVE");
    c->cooperative = env && env[0] == '1';
    const char* vp = std::getenv("SID_SKETCH_PAIRS");
    c->sketch_pairs = vp && vp[0] == '1';
  }
  int ncu = 0;
  if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, device) == hipSuccess &&
      ncu > 0)
    c->num_cu = ncu;
  if (!noalloc_scratch_init(device)) {
    delete c;
    return SID_EDEVICE;
  }
  if (hipMalloc(&c->fail_flag, 64) != hipSuccess || hipMemset(c->fail_flag, 0, 64) != hipSuccess) {
    (void)hipGetLastError();
    if (c->fail_flag) (void)hipFree(c->fail_flag);
    delete c;
    return SID_ENOMEM;
  }
  if (hip_stream) {
    c->stream = (hipStream_t)hip_stream;
  } else {
    if (hipStreamCreate(&c->stream) != hipSuccess) {
      delete c;
      return SID_EDEVICE;
    }
    c->own_stream = true;
  }
  *out = c;
  return SID_OK;
}

sid_status sid_destroy(sid_ctx* ctx) {
  if (!ctx) return SID_EINVAL;
  if (ctx->device < 0) {
    delete ctx;
    return SID_OK;
  }
  (void)hipSetDevice(ctx->device);
  (void)hipStreamSynchronize(ctx->stream);
  for (sid_ctx* c : ctx->children) (void)sid_destroy(c);
  if (ctx->side) (void)hipStreamDestroy(ctx->side);
  if (ctx->side_fork) (void)hipEventDestroy(ctx->side_fork);
  if (ctx->side_join) (void)hipEventDestroy(ctx->side_join);
  for (hipEvent_t e : ctx->child_done) (void)hipEventDestroy(e);
  for (BatchPlan* pl : ctx->plans) {
    if (pl->dev) (void)hipFree(pl->dev);
    delete pl;
  }
  if (ctx->fork) (void)hipEventDestroy(ctx->fork);
  for (Buf& b : ctx->ws)
    if (b.p) (void)hipFree(b.p);
  if (ctx->fail_flag) (void)hipFree(ctx->fail_flag);
  if (ctx->own_stream) (void)hipStreamDestroy(ctx->stream);
  delete ctx;
  return SID_OK;
}

const char* sid_last_error(const sid_ctx* ctx) {
  if (!ctx) return "null context";
  return ctx->err.c_str();
}

size_t sid_workspace_bytes(const sid_ctx* ctx) { return ctx ? held_bytes(ctx) : 0; }

sid_status sid_sync(sid_ctx* ctx) {
  if (!ctx) return SID_EINVAL;
  if (ctx->device < 0) return SID_OK;
  SID_CHECK(hipSetDevice(ctx->device), "hipSetDevice");
  SID_CHECK(hipStreamSynchronize(ctx->stream), "synchronize");
  bool failed = false;
  std::vector<sid_ctx*> all{ctx};
  for (sid_ctx* c : ctx->children) all.push_back(c);
  for (sid_ctx* c : all) {
    if (c != ctx) SID_CHECK(hipStreamSynchronize(c->stream), "synchronize");
    unsigned int f = 0;
    SID_CHECK(hipMemcpy(&f, c->fail_flag, sizeof(f), hipMemcpyDeviceToHost), "read failure flag");
    if (f) {
      failed = true;
      SID_CHECK(hipMemset(c->fail_flag, 0, sizeof(f)), "clear failure flag");
    }
  }
  if (failed)
    return fail(ctx, SID_EDEVICE,
                "a device-wide wait of the pivoted QR timed out (its workgroups were not resident "
                "together); the affected results have k_eff = -1 and are invalid");
  return SID_OK;
}

sid_status sid_set_workspace_limit(sid_ctx* ctx, size_t bytes) {
  if (!ctx) return SID_EINVAL;
  ctx->limit = bytes;
  return SID_OK;
}

sid_status sid_rowset_create(sid_ctx* ctx, const int64_t* host_rows, int64_t count, int64_t N,
                             sid_rowset** out) {
  if (!ctx || !out) return fail(ctx, SID_EINVAL, "null argument");
  *out = nullptr;
  if (!host_rows || count <= 0 || N <= 0) return fail(ctx, SID_EINVAL, "empty row set");
  if (count > N) return fail(ctx, SID_EINVAL, "more coarse rows than rows");
  for (int64_t i = 0; i < count; ++i) {
    if (host_rows[i] < 0 || host_rows[i] >= N)
      return fail(ctx, SID_EINVAL, "coarse row index out of range");
    if (i > 0 && host_rows[i] <= host_rows[i - 1])
      return fail(ctx, SID_EINVAL, "coarse rows must be strictly increasing");
  }
  SID_NEED_DEVICE(ctx);
  SID_CHECK(hipSetDevice(ctx->device), "hipSetDevice");
  sid_rowset* rs = new (std::nothrow) sid_rowset();
  if (!rs) return fail(ctx, SID_ENOMEM, "host allocation failed");
  if (hipMalloc(&rs->d_rows, sizeof(int64_t) * (size_t)count) != hipSuccess) {
    (void)hipGetLastError();
    delete rs;
    return fail(ctx, SID_ENOMEM, "device allocation failed");
  }
  hipError_t e = hipMemcpy(rs->d_rows, host_rows, sizeof(int64_t) * (size_t)count,
                           hipMemcpyHostToDevice);
  if (e != hipSuccess) {
    (void)hipFree(rs->d_rows);
    delete rs;
    return hip_fail(ctx, e, "row set upload");
  }
  rs->ctx = ctx;
  rs->count = count;
  rs->N = N;
  *out = rs;
  return SID_OK;
}

sid_status sid_rowset_destroy(sid_rowset* rs) {
  if (!rs) return SID_EINVAL;
  if (rs->d_rows) {
    (void)hipSetDevice(rs->ctx->device);
    (void)hipStreamSynchronize(rs->ctx->stream);
    (void)hipFree(rs->d_rows);
  }
  delete rs;
  return SID_OK;
}

sid_status sid_reserve(sid_ctx* ctx, int64_t N, int64_t n, const sid_params* p) {
  if (!ctx) return SID_EINVAL;
  Shape sh;
  sid_status st = validate(ctx, N, n, p, &sh);
  if (st != SID_OK) return st;
  SID_NEED_DEVICE(ctx);
  SID_CHECK(hipSetDevice(ctx->device), "hipSetDevice");
  Work w;
  if (reserve(ctx, sh, &w) != SID_OK) return SID_ENOMEM;
  // everything else a compress call of this shape would allocate or create
  // (for FP32 data with a 16-byte aligned base and lda % 4 == 0): the
  // sketch kernels' buffers for the sketch precision and, with refine, for
  // the refinement precision; the refinement buffers; the single-pass side
  // stream
  const bool has_rows = p->coarse != nullptr;
  if (p->select == SID_SEL_GAUSS && reserve_sketch(ctx, sh, sh.prec, has_rows, sh.single) != SID_OK)
    return SID_ENOMEM;
  if (p->refine) {
    const size_t d = sizeof(double);
    if (!ws(ctx, WS_REF_W, d * (size_t)(sh.l * sh.n)) ||
        !ws(ctx, WS_REF_WJ, sizeof(int64_t) * (size_t)(sh.k + 1)))
      return SID_ENOMEM;
    Shape shr = sh;
    shr.prec = p->refine_prec;
    shr.single = false;
    shr.q = 0;
    shr.lz = shr.lq = sh.l;
    if (reserve_sketch(ctx, shr, p->refine_prec, has_rows, false) != SID_OK) return SID_ENOMEM;
  }
  if (sh.single && !ctx->side) {
    SID_CHECK(hipStreamCreate(&ctx->side), "side stream");
    SID_CHECK(hipEventCreateWithFlags(&ctx->side_fork, hipEventDisableTiming), "side event");
    SID_CHECK(hipEventCreateWithFlags(&ctx->side_join, hipEventDisableTiming), "side event");
  }
  return SID_OK;
}

static sid_status factor(sid_ctx* ctx, const sid_params* p, const Shape& sh, const Work& w,
                         sid_dtype dtype, const void* A, int64_t lda, int64_t* J, void* P,
                         int64_t ldp, void* AJ, int64_t ldaj, double* err, int64_t* k_eff,
                         bool prefactored = false);
static sid_status refine_pass(sid_ctx* ctx, const void* A, sid_dtype dtype, int64_t lda,
                              const sid_params* p, const Shape& sh, const Work& w, int64_t* J,
                              void* P, int64_t ldp, double* err, int64_t* k_eff);

// The sketch pass over the columns col0 .. col0 + sh.n - 1 of the matrix
// (A points at column col0): W (lq x sh.n) and, if Y is given, Y = A Omega
// with Omega's rows col0 .. col0 + sh.n - 1 (y_add: Y += A Omega; only the
// workgroup-pair pass takes it, see sketch_adds_y).
static sid_status run_sketch(sid_ctx* ctx, const void* A, sid_dtype dtype, int64_t lda,
                             const sid_params* p, const Shape& sh, const Work& w, double* W,
                             void* Y, int64_t col0 = 0, bool y_add = false,
                             const __bf16* psi_img = nullptr) {
  hipStream_t st = ctx->stream;
  if (Y) {
    SID_CHECK(sid::launch_fill_gaussian(st, p->seed, 0u, col0, sh.n, 0, sh.l, w.omega),
              "omega generation");
  }
  const int64_t* rows = p->coarse ? p->coarse->d_rows : nullptr;
  // the streaming pass takes up to 512 columns per launch; wider matrices
  // go through it in column slabs (W's columns are independent, Y sums the
  // slabs' contributions)
  const int64_t slab = sh.n < 512 ? sh.n : 512;
  const SketchPath path =
      plan_sketch(ctx, dtype, lda, A, sh.prec, sh, rows != nullptr, Y != nullptr);
  if (path == SketchPath::PAIR_BF16) {
    // the workgroup-pair pass, in column slabs (W's columns are independent,
    // Y sums the slabs' contributions)
    const int vslab = sid::sketch_v2_slab((int)sh.lq, (int)sh.l, Y != nullptr);
    const int64_t vs = sh.n < vslab ? sh.n : vslab;
    int64_t rpp = 0;
    const int64_t pairs = sid::sketch_v2_pairs(sh.N, ctx->num_cu, &rpp);
    float* partf = (float*)ws(ctx, WS_PARTF, sizeof(float) * (size_t)(pairs * sh.lq * vs));
    __bf16* omT = (__bf16*)ws(ctx, WS_OMT, sizeof(uint16_t) * sid::sketch_v2_omt_elems((int)sh.l, (int)vs));
    if (!partf || !omT) return SID_ENOMEM;
    const int dmode = sh.prec == SID_SK_BF16X2   ? sid::FB_BF16X2
                      : sh.prec == SID_SK_FP8E4M3 ? sid::FB_FP8
                                                  : sid::FB_BF16;
    // over several slabs, Psi is formed once as images that every slab's
    // launch reads (the values the launches would generate)
    const size_t img_bytes = sid::sketch_v2_psi_image_bytes(sh.N, (int)sh.lq);
    if (!psi_img && sh.n > vs && img_bytes > 0) {
      __bf16* img = (__bf16*)ws(ctx, WS_PSIIMG, img_bytes);
      if (!img) return SID_ENOMEM;
      SID_CHECK(sid::launch_sketch_v2_psi_image(st, dmode, p->seed, sh.N, (int)sh.lq, img),
                "Psi images");
      psi_img = img;
    }
    // every slab after the first adds its part of Y in the kernel
    for (int64_t c0 = 0; c0 < sh.n; c0 += vs) {
      const int64_t nb = sh.n - c0 < vs ? sh.n - c0 : vs;
      int64_t nparts = 0;
      SID_CHECK(sid::launch_sketch_v2(st, dmode, (const float*)A + c0 * lda, lda, sh.N, (int)nb,
                                      (int)sh.lq, (int)sh.l, p->seed, w.omega + c0 * sh.l, omT,
                                      ctx->num_cu, partf, W + c0 * sh.lq, (float*)Y, &nparts,
                                      c0 > 0 || y_add, psi_img),
                "sketch pass (workgroup pairs)");
    }
    return SID_OK;
  }
  if (y_add) return fail(ctx, SID_EINVAL, "internal: Y accumulation on a path without it");
  if (path == SketchPath::FP8_GENERAL) {
    // general kernels: the e4m3 data values are formed first (one more pass
    // over A and an N x n FP32 copy in the workspace)
    float* a8 = (float*)ws(ctx, WS_A8, sizeof(float) * (size_t)(sh.N * sh.n));
    if (!a8) return SID_ENOMEM;
    SID_CHECK(sid::launch_fp8_quantize(st, A, dtype == SID_F64, lda, sh.N, sh.n, a8, sh.N),
              "FP8 data values");
    SID_CHECK(sid::launch_sketch(st, sh.prec, false, a8, sh.N, sh.N, sh.n, rows, sh.Ns, (int)sh.lq,
                                 p->seed, sh.nchunks, w.part, W, w.omega, (int)sh.l, Y),
              "sketch pass");
    return SID_OK;
  }
  const bool f32mfma = path == SketchPath::FUSED_F32;
  if (path == SketchPath::FUSED_BF16 || path == SketchPath::FUSED_F32) {
    // one streaming pass on the matrix cores (W partials per workgroup, FP32)
    int64_t rpw = 0;
    const int64_t grid = sid::fused_bf16_grid(sh.Ns, ctx->num_cu, &rpw);
    float* partf = (float*)ws(ctx, WS_PARTF, sizeof(float) * (size_t)(grid * sh.lq * slab));
    __bf16* omT = nullptr;
    float* omP = nullptr;
    if (f32mfma) omP = (float*)ws(ctx, WS_OMP, sizeof(float) * 128 * 512);
    else omT = (__bf16*)ws(ctx, WS_OMT, sizeof(uint16_t) * 128 * 512);
    if (!partf || (!omT && !omP)) return SID_ENOMEM;
    float* ytmp = nullptr;
    if (Y && sh.n > slab) {
      ytmp = (float*)ws(ctx, WS_YTMP, sizeof(float) * (size_t)(sh.N * sh.l));
      if (!ytmp) return SID_ENOMEM;
    }
    const int dmode = sh.prec == SID_SK_BF16X2   ? sid::FB_BF16X2
                      : sh.prec == SID_SK_FP8E4M3 ? sid::FB_FP8
                                                  : sid::FB_BF16;
    for (int64_t c0 = 0; c0 < sh.n; c0 += slab) {
      const int64_t nb = sh.n - c0 < slab ? sh.n - c0 : slab;
      float* yd = Y ? (c0 == 0 ? (float*)Y : ytmp) : nullptr;
      int64_t nparts = 0;
      if (f32mfma)
        SID_CHECK(sid::launch_sketch_fused_f32(st, (const float*)A + c0 * lda, lda, sh.N, (int)nb,
                                               (int)sh.lq, (int)sh.l, p->seed,
                                               w.omega + c0 * sh.l, omP, ctx->num_cu, partf,
                                               W + c0 * sh.lq, yd),
                  "fused FP32 sketch pass");
      else
        SID_CHECK(sid::launch_sketch_fused_bf16(st, dmode, (const float*)A + c0 * lda, lda, sh.Ns,
                                                (int)nb, (int)sh.lq, (int)sh.l, p->seed,
                                                w.omega + c0 * sh.l, omT, ctx->num_cu, partf,
                                                W + c0 * sh.lq, yd, &nparts, rows),
                  "fused sketch pass");
      if (Y && c0 > 0)
        SID_CHECK(sid::launch_add_inplace(st, false, Y, ytmp, sh.N * sh.l, ctx->num_cu),
                  "Y slab sum");
    }
    return SID_OK;
  }
  if (path == SketchPath::F64_TILED) {
    // all rows: the register-tiled FP64 passes (the same bits as the general
    // kernels)
    SID_CHECK(sid::launch_sketch_w_f64(st, A, dtype == SID_F64, lda, sh.N, sh.n, (int)sh.lq,
                                       p->seed, sh.nchunks, w.part, W),
              "FP64 sketch pass (W)");
    if (Y)
      SID_CHECK(sid::launch_sketch_y_f64(st, A, dtype == SID_F64, lda, sh.N, sh.n, w.omega,
                                         (int)sh.l, (double*)Y),
                "FP64 sketch pass (Y)");
    return SID_OK;
  }
  SID_CHECK(sid::launch_sketch(st, sh.prec, dtype == SID_F64, A, lda, sh.N, sh.n, rows, sh.Ns,
                               (int)sh.lq, p->seed, sh.nchunks, w.part, W, w.omega, (int)sh.l,
                               Y),
            "sketch pass");
  return SID_OK;
}

sid_status sid_sketch(sid_ctx* ctx, const void* A, sid_dtype dtype, int64_t N, int64_t n,
                      int64_t lda, const sid_params* p, double* W, void* Y) {
  if (!ctx) return SID_EINVAL;
  if (!A || !W) return fail(ctx, SID_EINVAL, "A and W must be non-NULL");
  if (dtype != SID_F32 && dtype != SID_F64) return fail(ctx, SID_EINVAL, "unknown dtype");
  if (lda < N) return fail(ctx, SID_EINVAL, "lda < N");
  Shape sh;
  sid_status s = validate(ctx, N, n, p, &sh);
  if (s != SID_OK) return s;
  SID_NEED_DEVICE(ctx);
  SID_CHECK(hipSetDevice(ctx->device), "hipSetDevice");
  Shape sh2 = sh;
  sh2.single = false;
  Work w;
  if (reserve(ctx, sh2, &w) != SID_OK) return SID_ENOMEM;
  return run_sketch(ctx, A, dtype, lda, p, sh, w, W, Y);
}

sid_status sid_sketch_noalloc(sid_ctx* ctx, const void* A, sid_dtype dtype, int64_t N, int64_t n,
                              int64_t lda, const sid_params* p, double* W, void* Y) {
  if (!ctx) return SID_EINVAL;
  if (!A || !W) return fail(ctx, SID_EINVAL, "A and W must be non-NULL");
  if (dtype != SID_F32) return fail(ctx, SID_EINVAL, "the allocation-free sketch reads FP32 data");
  if (lda < N) return fail(ctx, SID_EINVAL, "lda < N");
  Shape sh;
  sid_status s = validate(ctx, N, n, p, &sh);
  if (s != SID_OK) return s;
  if (p->coarse) return fail(ctx, SID_EINVAL, "the allocation-free sketch reads all rows");
  if (p->select != SID_SEL_GAUSS) return fail(ctx, SID_EINVAL, "literal selection has no sketch");
  if (sh.prec != SID_SK_BF16 && sh.prec != SID_SK_BF16X2 && sh.prec != SID_SK_FP8E4M3)
    return fail(ctx, SID_EINVAL, "the allocation-free sketch runs the bf16 / bf16x2 / fp8 forms");
  const bool want_y = Y != nullptr;
  // the same kernels as sid_sketch takes for this input, in one launch
  const SketchPath path = plan_sketch(ctx, dtype, lda, A, sh.prec, sh, false, want_y);
  const bool pairs_path = path == SketchPath::PAIR_BF16;
  if ((path != SketchPath::FUSED_BF16 && !pairs_path) ||
      sh.n > (pairs_path ? sid::sketch_v2_slab((int)sh.lq, (int)sh.l, want_y) : 512))
    return fail(ctx, SID_EINVAL,
                "the allocation-free sketch needs a 16-byte aligned A, lda % 4 == 0 and a shape "
                "the matrix-core passes take in one launch");
  // the scratch this call needs, carved in 256-byte aligned pieces: Omega's
  // values, Omega^T in bfloat16, the per-workgroup (pair) W partials
  int64_t rows = 0;
  const int64_t nparts = pairs_path ? sid::sketch_v2_pairs(sh.N, ctx->num_cu, &rows)
                                    : sid::fused_bf16_grid(sh.N, ctx->num_cu, &rows);
  auto up = [](size_t b) { return (b + 255) / 256 * 256; };
  const size_t omt_elems =
      pairs_path ? sid::sketch_v2_omt_elems((int)sh.l, (int)sh.n) : (size_t)128 * 512;
  const size_t b_om = want_y ? up(sizeof(float) * (size_t)(sh.n * sh.l)) : 0;
  const size_t b_omt = want_y ? up(sizeof(uint16_t) * omt_elems) : 0;
  const size_t b_part = up(sizeof(float) * (size_t)(nparts * sh.lq * sh.n));
  const size_t need = b_om + b_omt + b_part;
  if (need > SID_NOALLOC_SCRATCH_BYTES)
    return fail(ctx, SID_EINVAL,
                "input too large for the allocation-free sketch: it needs " + std::to_string(need) +
                    " bytes of scratch, the static scratch holds " +
                    std::to_string((size_t)SID_NOALLOC_SCRATCH_BYTES));
  SID_NEED_DEVICE(ctx);
  SID_CHECK(hipSetDevice(ctx->device), "hipSetDevice");
  unsigned char* base = (unsigned char*)noalloc_ptr[ctx->device];
  if (!base) return fail(ctx, SID_ESTATE, "no scratch address for this device");
  float* om = want_y ? (float*)base : nullptr;
  __bf16* omt = want_y ? (__bf16*)(base + b_om) : nullptr;
  float* part = (float*)(base + b_om + b_omt);
  hipStream_t st = ctx->stream;
  if (want_y)
    SID_CHECK(sid::launch_fill_gaussian(st, p->seed, 0u, 0, sh.n, 0, sh.l, om), "omega generation");
  const int dmode = sh.prec == SID_SK_BF16X2   ? sid::FB_BF16X2
                    : sh.prec == SID_SK_FP8E4M3 ? sid::FB_FP8
                                                : sid::FB_BF16;
  int64_t np = 0;
  if (pairs_path)
    SID_CHECK(sid::launch_sketch_v2(st, dmode, (const float*)A, lda, sh.N, (int)sh.n, (int)sh.lq,
                                    (int)sh.l, p->seed, om, omt, ctx->num_cu, part, W, (float*)Y,
                                    &np),
              "sketch pass (allocation-free)");
  else
    SID_CHECK(sid::launch_sketch_fused_bf16(st, dmode, (const float*)A, lda, sh.N, (int)sh.n,
                                            (int)sh.lq, (int)sh.l, p->seed, om, omt, ctx->num_cu,
                                            part, W, (float*)Y, &np, nullptr),
              "sketch pass (allocation-free)");
  return SID_OK;
}

sid_status sid_probe(sid_ctx* ctx, int kind, void* buf, int64_t N, int64_t n) {
  if (!ctx) return SID_EINVAL;
  if (kind < 0 || kind > 4) return fail(ctx, SID_EINVAL, "unknown probe");
  if (kind <= 2) {
    if (!buf || N < 1 || n < 1 || ((uintptr_t)buf % 16) != 0 || (N * n) % 4 != 0)
      return fail(ctx, SID_EINVAL, "probe buffer: non-NULL, 16-byte aligned, N n a multiple of 4");
    if (kind == 1 && N % 64 != 0) return fail(ctx, SID_EINVAL, "column-store probe: N % 64 == 0");
  } else if (N < 1 || N > (1 << 30)) {
    return fail(ctx, SID_EINVAL, "matrix-instruction probe: 1 <= rounds <= 2^30");
  }
  SID_NEED_DEVICE(ctx);
  SID_CHECK(hipSetDevice(ctx->device), "hipSetDevice");
  float* sink = (float*)ws(ctx, WS_PROBE, sizeof(float) * 8 * (size_t)ctx->num_cu);
  if (!sink) return SID_ENOMEM;
  SID_CHECK(sid::launch_probe(ctx->stream, kind, buf, N, n, ctx->num_cu, sink), "probe");
  return SID_OK;
}

sid_status sid_compress(sid_ctx* ctx, const void* A, sid_dtype dtype, int64_t N, int64_t n,
                        int64_t lda, const sid_params* p, int64_t* J, void* P, int64_t ldp,
                        void* AJ, int64_t ldaj, double* err, int64_t* k_eff) {
  if (!ctx) return SID_EINVAL;
  if (!A) return fail(ctx, SID_EINVAL, "A is NULL");
  if (dtype != SID_F32 && dtype != SID_F64) return fail(ctx, SID_EINVAL, "unknown dtype");
  if (lda < N) return fail(ctx, SID_EINVAL, "lda < N");
  Shape sh;
  sid_status s = validate(ctx, N, n, p, &sh);
  if (s != SID_OK) return s;
  if (P && ldp < p->k) return fail(ctx, SID_EINVAL, "ldp < k");
  if (AJ && ldaj < skeleton_rows(p, N))
    return fail(ctx, SID_EINVAL, "ldaj < rows of the skeleton (N, or |S| for the coarse skeleton)");
  SID_NEED_DEVICE(ctx);
  SID_CHECK(hipSetDevice(ctx->device), "hipSetDevice");
  Work w;
  if (reserve(ctx, sh, &w) != SID_OK) return SID_ENOMEM;
  if (p->select == SID_SEL_ROWS_LITERAL) {
    // (1) Alg. 5 as written: mgsqr runs on the coarse rows themselves
    SID_CHECK(sid::launch_gather_rows(ctx->stream, A, dtype == SID_F64, lda, p->coarse->d_rows,
                                      sh.Ns, sh.n, p->prec == SID_SK_F32, w.W, sh.Ns),
              "A(S, :)");
  } else {
    // (1) sketch pass: W = Psi(:, S) A(S, :) and, single pass, Y = A Omega
    s = run_sketch(ctx, A, dtype, lda, p, sh, w, w.W, sh.single ? w.Y : nullptr);
    if (s != SID_OK) return s;
  }
  s = factor(ctx, p, sh, w, dtype, A, lda, J, P, ldp, AJ, ldaj, err, k_eff);
  if (s != SID_OK || !p->refine) return s;
  return refine_pass(ctx, A, dtype, lda, p, sh, w, J, P, ldp, err, k_eff);
}

// Refinement of P on a second sketch W' = Psi(0:l, S) A(S, :) taken in
// refine_prec: with the pivots J of the first sketch fixed, P1 is the
// least-squares solution of min ||W'(:, J) X - W'||, formed by mgsqr of W'
// with the pivot order forced to J (the projections of every other column
// onto the pivots' Q are those of modified Gram-Schmidt on the augmented
// matrix) and the usual back substitution P1 = R11'^-1 R12'.  The estimates
// are then re-fitted with P1.  The first factorization's R, Q and R11 are no
// longer needed here and are reused.
static sid_status refine_pass(sid_ctx* ctx, const void* A, sid_dtype dtype, int64_t lda,
                              const sid_params* p, const Shape& sh, const Work& w, int64_t* J,
                              void* P, int64_t ldp, double* err, int64_t* k_eff) {
  hipStream_t st = ctx->stream;
  const int k = (int)sh.k, l = (int)sh.l, n_ = (int)sh.n;
  sid_params pr = *p;
  pr.prec = p->refine_prec;
  pr.mode = SID_TWO_PASS;
  pr.probe_rows = 0;
  pr.refine = 0;
  Shape shr = sh;
  shr.prec = p->refine_prec;
  shr.single = false;
  shr.q = 0;
  shr.lz = sh.l;
  shr.lq = sh.l;
  const size_t d = sizeof(double);
  double* Wp = (double*)ws(ctx, WS_REF_W, d * (size_t)(l * n_));
  int64_t* Jf = (int64_t*)ws(ctx, WS_REF_WJ, sizeof(int64_t) * (size_t)(k + 1));
  if (!Wp || !Jf) return SID_ENOMEM;
  sid_status s = run_sketch(ctx, A, dtype, lda, &pr, shr, w, Wp, nullptr);
  if (s != SID_OK) return s;
  // the forced order: J as the first mgsqr left it (-1 past its k_eff)
  SID_CHECK(hipMemcpyAsync(Jf, w.piv, sizeof(int64_t) * (size_t)k, hipMemcpyDeviceToDevice, st),
            "J");
  bool coop_launch = ctx->cooperative;
  {
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(st, &cs) == hipSuccess && cs != hipStreamCaptureStatusNone)
      coop_launch = false;
  }
  if (l <= 96 && sid::cpqr_wgl_supported(l, n_) && !sid::cpqr_wg_supported(l, n_))
    SID_CHECK(sid::launch_cpqr_wgl(st, Wp, l, l, n_, k, 0.0, w.piv, w.R, w.Q, w.keff, w.stats, Jf),
              "mgsqr of W' in the order J");
  else if (sid::cpqr_wg_supported(l, n_))
    SID_CHECK(sid::launch_cpqr_wg(st, Wp, l, l, n_, k, 0.0, w.piv, w.R, w.Q, w.keff, w.stats, Jf),
              "mgsqr of W' in the order J");
  else if (sid::cpqr_coop_supported(l, n_))
    SID_CHECK(sid::launch_cpqr_coop(st, Wp, l, l, n_, k, 0.0, w.coop, w.sync2, w.piv, w.R, w.Q,
                                    w.keff, w.stats, coop_launch, ctx->fail_flag, Jf),
              "mgsqr of W' in the order J");
  else
    SID_CHECK(sid::launch_cpqr(st, Wp, l, l, n_, k, 0.0, w.Wr, w.nrm, w.piv, w.R, w.Q, w.keff,
                               w.stats, Jf),
              "mgsqr of W' in the order J");
  SID_CHECK(sid::launch_id_coefficients(st, w.R, n_, w.piv, w.keff, k, w.R11, w.Pd, P, ldp,
                                        dtype == SID_F64),
            "refined coefficients");
  // the estimates describe the P handed back: the probe rows and the
  // selection rows of the first sketch are fitted again with P1 (w.Pd)
  SID_CHECK(sid::launch_fit_residual(st, w.W, sh.lq, sh.lz, (int)sh.q, n_, w.piv, w.keff, w.Pd,
                                     k, (sh.single && sh.q > 0) ? w.mix : nullptr, w.fitpart,
                                     w.err),
            "probe residual (refined P)");
  SID_CHECK(sid::launch_fit_residual(st, w.W, sh.lq, 0, l, n_, w.piv, w.keff, w.Pd, k, nullptr,
                                     w.fitpart, w.err + 1),
            "sketch residual (refined P)");
  // a pivot whose column W' reproduces from the earlier ones ends the forced
  // factorization early: J and k_eff are copied again
  SID_CHECK(sid::launch_copy_results(st, J, w.piv, k, k_eff, w.keff, err, w.err), "results");
  return SID_OK;
}

// Everything after the sketch pass, from W (w.W, lq x n), single pass also
// Y (w.Y) and Omega's values (w.omega, n x l): mgsqr, coefficients,
// estimates and the skeleton.  A is read only by the two-pass gather.
// single pass: AJ = Y T (N x k, ld ldaj, FP64 when f64) on the kernel the
// shape and the sketch form take
static sid_status apply_skeleton(sid_ctx* ctx, hipStream_t st, const Shape& sh, const void* Y,
                                 const double* T, void* AJ, int64_t ldaj, bool f64) {
  const int k = (int)sh.k, l = (int)sh.l;
  const bool yf64 = sh.prec == SID_SK_F64;
  const bool ybf = sh.prec == SID_SK_BF16 || sh.prec == SID_SK_BF16X2 || sh.prec == SID_SK_FP8E4M3;
  if (ybf && !f64 && sid::apply_t_bf16_runs_supported(k, l))
    SID_CHECK(sid::launch_apply_t_bf16_runs(st, (const float*)Y, sh.N, l, T, k, (float*)AJ, ldaj,
                                            ctx->num_cu),
              "AJ = Y T");
  else if (ybf && sid::apply_t_bf16_supported(k, l))
    SID_CHECK(sid::launch_apply_t_bf16(st, (const float*)Y, sh.N, l, T, k, AJ, f64, ldaj,
                                       ctx->num_cu),
              "AJ = Y T");
  else if (sid::apply_t_mfma_supported(k, l, yf64))
    SID_CHECK(sid::launch_apply_t_mfma(st, Y, yf64, sh.N, l, T, k, AJ, f64, ldaj, ctx->num_cu),
              "AJ = Y T");
  else
    SID_CHECK(sid::launch_apply_t(st, Y, yf64, sh.N, l, T, k, AJ, f64, ldaj), "AJ = Y T");
  return SID_OK;
}

// prefactored (the batched path): mgsqr of W_sel and, in single pass, M,
// Mpr, Omega's FP64 values and mgsqr of M are already in w (steps 5a and 2
// are skipped).
static sid_status factor(sid_ctx* ctx, const sid_params* p, const Shape& sh, const Work& w,
                         sid_dtype dtype, const void* A, int64_t lda, int64_t* J, void* P,
                         int64_t ldp, void* AJ, int64_t ldaj, double* err, int64_t* k_eff,
                         bool prefactored) {
  hipStream_t st = ctx->stream;
  const bool f64 = dtype == SID_F64;
  const int k = (int)sh.k, l = (int)sh.l, q = (int)sh.q, lz = (int)sh.lz, lq = (int)sh.lq,
            n_ = (int)sh.n;
  const int w_kind = mgsqr_kind(l, n_);
  // a cooperative launch cannot be recorded into a graph: under capture the
  // multi-workgroup QR is a plain launch (its bounded waits report through
  // the sticky flag)
  bool coop_launch = ctx->cooperative;
  {
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(st, &cs) == hipSuccess && cs != hipStreamCaptureStatusNone)
      coop_launch = false;
  }
  const int m_kind = sh.single ? mgsqr_kind(lz, l) : 0;
  const bool overlap = sh.single && !(m_kind == w_kind && (m_kind == 1 || m_kind == 2));
  if (overlap && !ctx->side) {
    SID_CHECK(hipStreamCreate(&ctx->side), "side stream");
    SID_CHECK(hipEventCreateWithFlags(&ctx->side_fork, hipEventDisableTiming), "side event");
    SID_CHECK(hipEventCreateWithFlags(&ctx->side_join, hipEventDisableTiming), "side event");
  }
  const double rcond = p->sp_rcond > 0.0 ? p->sp_rcond : default_rcond(sh.prec);
  if (sh.single && !prefactored) {
    // (5a) single pass, independent of the pivots: M = W(0:lz, :) Omega,
    // Mpr = W_pr Omega and mgsqr of M, on a side stream when they can
    // overlap mgsqr of W (step 2)
    hipStream_t ms = st;
    if (overlap) {
      SID_CHECK(hipEventRecord(ctx->side_fork, st), "side fork");
      SID_CHECK(hipStreamWaitEvent(ctx->side, ctx->side_fork, 0), "side fork wait");
      ms = ctx->side;
    }
    SID_CHECK(sid::launch_omega_values(ms, sh.prec, w.omega, sh.n * sh.l, w.om64), "omega values");
    SID_CHECK(sid::launch_gemm64(ms, lz, l, n_, w.W, lq, 0, w.om64, l, 1, w.M, lz), "M = W Omega");
    if (q > 0)
      SID_CHECK(sid::launch_gemm64(ms, q, l, n_, w.W + lz, lq, 0, w.om64, l, 1, w.Mpr, q),
                "Mpr = Wpr Omega");
    if (m_kind == 3)
      SID_CHECK(sid::launch_cpqr_wgl(ms, w.M, lz, lz, l, l, rcond, w.pivM, w.RM, w.QM, w.rkM,
                                     w.statsM),
                "pivoted QR of M");
    else if (m_kind == 0)
      SID_CHECK(sid::launch_cpqr_wg(ms, w.M, lz, lz, l, l, rcond, w.pivM, w.RM, w.QM, w.rkM,
                                    w.statsM),
                "pivoted QR of M");
    else if (m_kind == 1)
      SID_CHECK(sid::launch_cpqr_coop(ms, w.M, lz, lz, l, l, rcond, w.coop, w.sync2, w.pivM, w.RM,
                                      w.QM, w.rkM, w.statsM, coop_launch, ctx->fail_flag),
                "pivoted QR of M");
    else
      SID_CHECK(sid::launch_cpqr(ms, w.M, lz, lz, l, l, rcond, w.Wr, w.nrm, w.pivM, w.RM, w.QM,
                                 w.rkM, w.statsM),
                "pivoted QR of M");
    if (overlap) SID_CHECK(hipEventRecord(ctx->side_join, ctx->side), "side join");
  }
  // (2) mgsqr on the selection rows of W
  if (prefactored) {
    // (run by the batched launches)
  } else if (w_kind == 3)
    SID_CHECK(sid::launch_cpqr_wgl(st, w.W, lq, l, n_, k, p->rank_tol, w.piv, w.R, w.Q, w.keff,
                                   w.stats),
              "pivoted QR");
  else if (w_kind == 0)
    SID_CHECK(sid::launch_cpqr_wg(st, w.W, lq, l, n_, k, p->rank_tol, w.piv, w.R, w.Q, w.keff,
                                  w.stats),
              "pivoted QR");
  else if (w_kind == 1)
    SID_CHECK(sid::launch_cpqr_coop(st, w.W, lq, l, n_, k, p->rank_tol, w.coop, w.sync2, w.piv,
                                    w.R, w.Q, w.keff, w.stats, coop_launch, ctx->fail_flag),
              "pivoted QR");
  else
    SID_CHECK(sid::launch_cpqr(st, w.W, lq, l, n_, k, p->rank_tol, w.Wr, w.nrm, w.piv, w.R, w.Q,
                               w.keff, w.stats),
              "pivoted QR");
  // (2b) adaptive rank: the smallest prefix of the pivots whose probe fit
  // meets probe_tol (Remark 2.2 with the probe estimator)
  const bool adaptive = p->probe_tol > 0.0;
  if (adaptive)
    SID_CHECK(sid::launch_probe_adapt(st, w.W, lq, lz, q, n_, w.piv, w.keff, w.R, k, w.R11, w.az,
                                      w.apart, w.ae2, p->probe_tol),
              "adaptive rank");
  // (3) coefficients P = R11^{-1} R(:, j) on the non-pivot columns, and
  // (4) the estimates: err[1] sketch fit (final residual of mgsqr, or at an
  // adaptive rank the fit of the selection rows), err[0] probe rows.  In
  // single pass with the side stream, P and err[1] are formed there while
  // the main stream goes on to T and AJ (they do not depend on P).
  const bool p_side = sh.single && overlap && AJ && !adaptive;
  hipStream_t ps = st;
  if (p_side) {
    SID_CHECK(hipEventRecord(ctx->side_fork, st), "side fork");
    SID_CHECK(hipStreamWaitEvent(ctx->side, ctx->side_fork, 0), "side fork wait");
    ps = ctx->side;
  }
  SID_CHECK(sid::launch_id_coefficients(ps, w.R, n_, w.piv, w.keff, k, w.R11, w.Pd, P, ldp, f64),
            "coefficients");
  if (adaptive)
    SID_CHECK(sid::launch_fit_residual(st, w.W, lq, 0, l, n_, w.piv, w.keff, w.Pd, k, nullptr,
                                       w.fitpart, w.err + 1),
              "sketch residual");
  else
    SID_CHECK(sid::launch_ratio_sqrt(ps, w.stats, w.err + 1), "sketch residual");
  if (!sh.single) {
    SID_CHECK(sid::launch_fit_residual(st, w.W, lq, l, q, n_, w.piv, w.keff, w.Pd, k, nullptr,
                                       w.fitpart, w.err),
              "probe residual");
    if (AJ && p->mode == SID_COARSE_SKELETON)
      // Alg. 6: keep the coarse skeleton A(S, J); no fine row is read
      SID_CHECK(sid::launch_gather_coarse_skeleton(st, A, f64, lda, p->coarse->d_rows, sh.Ns,
                                                   w.piv, w.keff, k, AJ, ldaj),
                "coarse skeleton gather");
    else if (AJ)
      SID_CHECK(sid::launch_gather_cols(st, A, f64, lda, sh.N, w.piv, w.keff, k, AJ, f64, ldaj),
                "skeleton gather");
  } else {
    // (5b) single pass.  Psi Y = Psi A Omega = W Omega, so the small matrix
    // M = W(0:lz, :) Omega plays the role of Z = Psi Q (up to the triangular
    // factor of Y), and the minimum-residual solve of the two-sided sketch
    // (Halko et al. Sec. 5.5 item (4)) becomes T = M^+ W(0:lz, J), AJ = Y T.
    // lz = l + e: the e extra co-range rows make M tall (the square form is
    // the ill-conditioned case the paper warns about in Sec. 2.3).  M^+ is
    // applied through mgsqr of M (step 5a) truncated at sp_rcond (least
    // squares on the pivoted columns).
    // (the join recorded after M's mgsqr: the coefficients queued on the
    // side stream since are not waited for here)
    if (overlap && !prefactored)
      SID_CHECK(hipStreamWaitEvent(st, ctx->side_join, 0), "side join wait");
    SID_CHECK(sid::launch_gather_block(st, w.W, lq, 0, lz, w.piv, w.keff, k, w.WJ), "W(:, J)");
    SID_CHECK(sid::launch_gemm64(st, l, k, lz, w.QM, lz, 1, w.WJ, lz, 0, w.C, l), "QM^T W(:, J)");
    SID_CHECK(sid::launch_small_solve(st, w.RM, l, w.pivM, w.rkM, w.R11M, w.C, l, k, w.T), "T");
    // the probe estimate needs T but not AJ: on the side stream it runs
    // during AJ = Y T (and the err / J copies below wait for it)
    hipStream_t es = st;
    if (overlap && AJ) {
      SID_CHECK(hipEventRecord(ctx->side_fork, st), "side fork");
      SID_CHECK(hipStreamWaitEvent(ctx->side, ctx->side_fork, 0), "side fork wait");
      es = ctx->side;
    }
    if (q > 0)
      SID_CHECK(sid::launch_gemm64(es, q, k, l, w.Mpr, q, 0, w.T, l, 0, w.mix, q), "Mpr T");
    SID_CHECK(sid::launch_fit_residual(es, w.W, lq, lz, q, n_, w.piv, w.keff, w.Pd, k,
                                       q > 0 ? w.mix : nullptr, w.fitpart, w.err),
              "probe residual");
    if (es != st) SID_CHECK(hipEventRecord(ctx->side_join, es), "side join");
    if (AJ) {
      const sid_status as = apply_skeleton(ctx, st, sh, w.Y, w.T, AJ, ldaj, f64);
      if (as != SID_OK) return as;
    }
    if (es != st) SID_CHECK(hipStreamWaitEvent(st, ctx->side_join, 0), "side join wait");
  }
  SID_CHECK(sid::launch_copy_results(st, J, w.piv, k, k_eff, w.keff, err, w.err), "results");
  return SID_OK;
}

sid_status sid_reconstruct(sid_ctx* ctx, const void* AJ, int64_t ldaj, const void* P, int64_t ldp,
                           sid_dtype dtype, int64_t N, int64_t k, int64_t n, void* Ahat,
                           int64_t ldo) {
  if (!ctx) return SID_EINVAL;
  if (!AJ || !P || !Ahat) return fail(ctx, SID_EINVAL, "null pointer");
  if (dtype != SID_F32 && dtype != SID_F64) return fail(ctx, SID_EINVAL, "unknown dtype");
  if (N <= 0 || n <= 0 || k <= 0) return fail(ctx, SID_EINVAL, "N, n, k must be positive");
  if (ldaj < N || ldo < N || ldp < k) return fail(ctx, SID_EINVAL, "leading dimension too small");
  if (k > 256) return fail(ctx, SID_EINVAL, "k must be <= 256");
  SID_NEED_DEVICE(ctx);
  SID_CHECK(hipSetDevice(ctx->device), "hipSetDevice");
  if (dtype == SID_F32 && k <= 128) {
    // the matrix-core kernel: AJ read in place, P packed as bfloat16 hi/lo
    // operand tiles
    const int kp = (int)((k + 15) / 16 * 16);
    void* pb = ws(ctx, WS_IPB, sid::interp_pb_bytes(n, kp));
    if (!pb) return SID_ENOMEM;
    SID_CHECK(sid::launch_pack_p(ctx->stream, (const float*)P, ldp, (int)k, kp, n, pb), "pack P");
    SID_CHECK(sid::launch_id_mfma(ctx->stream, (const float*)AJ, ldaj, N, (int)k, kp, pb, n,
                                  (float*)Ahat, ldo, nullptr, 0, nullptr, 0, nullptr),
              "reconstruct");
    return SID_OK;
  }
  SID_CHECK(sid::launch_reconstruct(ctx->stream, dtype == SID_F64, AJ, ldaj, P, ldp, N, (int)k, n,
                                    Ahat, ldo),
            "reconstruct");
  return SID_OK;
}

sid_status sid_error_norms(sid_ctx* ctx, const void* A, int64_t lda, const void* AJ, int64_t ldaj,
                           const void* P, int64_t ldp, sid_dtype dtype, int64_t N, int64_t k,
                           int64_t n, double* out4) {
  if (!ctx) return SID_EINVAL;
  if (!A || !AJ || !P || !out4) return fail(ctx, SID_EINVAL, "null pointer");
  if (dtype != SID_F32 && dtype != SID_F64) return fail(ctx, SID_EINVAL, "unknown dtype");
  if (N <= 0 || n <= 0 || k <= 0) return fail(ctx, SID_EINVAL, "N, n, k must be positive");
  if (lda < N || ldaj < N || ldp < k) return fail(ctx, SID_EINVAL, "leading dimension too small");
  if (k > 256) return fail(ctx, SID_EINVAL, "k must be <= 256");
  SID_NEED_DEVICE(ctx);
  SID_CHECK(hipSetDevice(ctx->device), "hipSetDevice");
  const int64_t nb = ((N + 63) / 64) * ((n + 31) / 32);
  double* part = (double*)ws(ctx, WS_NORMPART, sizeof(double) * 4 * (size_t)nb);
  double* dout = (double*)ws(ctx, WS_NORMOUT, sizeof(double) * 4);
  if (!part || !dout) return SID_ENOMEM;
  SID_CHECK(sid::launch_error_norms(ctx->stream, dtype == SID_F64, A, lda, AJ, ldaj, P, ldp, N,
                                    (int)k, n, part, nb, dout),
            "error norms");
  SID_CHECK(hipMemcpyAsync(out4, dout, 4 * sizeof(double), hipMemcpyDeviceToHost, ctx->stream),
            "copy norms");
  SID_CHECK(hipStreamSynchronize(ctx->stream), "synchronize");
  return SID_OK;
}

sid_status sid_fill_gaussian(sid_ctx* ctx, uint64_t seed, int stream, int64_t major0,
                             int64_t nmajor, int64_t minor0, int64_t nminor, float* out) {
  if (!ctx) return SID_EINVAL;
  if (!out) return fail(ctx, SID_EINVAL, "out is NULL");
  if (stream < 0 || major0 < 0 || nmajor < 0 || minor0 < 0 || nminor < 0)
    return fail(ctx, SID_EINVAL, "negative argument");
  if (minor0 + nminor > ((int64_t)1 << 34)) return fail(ctx, SID_EINVAL, "minor index too large");
  if (nmajor == 0 || nminor == 0) return SID_OK;
  SID_NEED_DEVICE(ctx);
  SID_CHECK(hipSetDevice(ctx->device), "hipSetDevice");
  SID_CHECK(sid::launch_fill_gaussian(ctx->stream, seed, (uint32_t)stream, major0, nmajor, minor0,
                                      nminor, out),
            "fill gaussian");
  return SID_OK;
}

// ---------------------------------------------------------------------------
// Streaming: columns arrive in blocks; W's columns are independent of each
// other and Y = A Omega is a sum over column blocks, so the sketches of the
// blocks seen so far are exactly the sketches of the matrix so far.  Small
// blocks are gathered into a stage of up to 512 columns before a sketch
// pass (one pass per 512 columns instead of one per block: Y is read and
// written once per pass).
// ---------------------------------------------------------------------------
namespace {

size_t elem_size(sid_dtype d) { return d == SID_F64 ? sizeof(double) : sizeof(float); }

size_t y_elem_size(const sid_stream* s) {
  return s->p.prec == SID_SK_F64 ? sizeof(double) : sizeof(float);
}

void stream_free(sid_stream* s) {
  if (!s) return;
  if (s->ctx && s->ctx->device >= 0) {
    (void)hipSetDevice(s->ctx->device);
    (void)hipStreamSynchronize(s->ctx->stream);
    if (s->stage) (void)hipFree(s->stage);
    if (s->psi_img) (void)hipFree(s->psi_img);
    if (s->W) (void)hipFree(s->W);
    if (s->Y) (void)hipFree(s->Y);
    if (s->H) (void)hipFree(s->H);
    if (s->Wp) (void)hipFree(s->Wp);
  }
  delete s;
}

sid_status stream_alloc(sid_ctx* ctx, sid_stream* s) {
  const size_t wb = sizeof(double) * (size_t)(s->lq * s->n_max);
  if (hipMalloc((void**)&s->W, wb) != hipSuccess) {
    (void)hipGetLastError();
    return fail(ctx, SID_ENOMEM, "stream: device allocation of W failed");
  }
  if (s->single) {
    if (hipMalloc(&s->Y, y_elem_size(s) * (size_t)(s->N * s->l)) != hipSuccess) {
      (void)hipGetLastError();
      return fail(ctx, SID_ENOMEM, "stream: device allocation of Y failed");
    }
  }
  return SID_OK;
}

sid_status svd_h_update(sid_ctx* ctx, const void* A, sid_dtype dtype, int64_t lda, int64_t N,
                        int64_t ncols, const double* W, int64_t l, double* wp, double* H,
                        bool accumulate);

// sketch columns cols .. cols + ncols - 1 from src (leading dimension ld);
// an SBR-SVD stream then adds them to H while they are resident
sid_status stream_flush(sid_stream* s, const void* src, int64_t ld, int64_t ncols) {
  sid_ctx* ctx = s->ctx;
  if (ncols <= 0) return SID_OK;
  Shape sh;
  sid_status st = validate(ctx, s->N, s->n_max, &s->p, &sh);
  if (st != SID_OK) return st;
  // row chunks of the general kernels as for the resident call over n_max
  // columns (validate set sh.nchunks from n_max), so a stream's W is that
  // call's W bit for bit
  sh.n = ncols;
  Work w;
  if (reserve(ctx, sh, &w) != SID_OK) return SID_ENOMEM;
  // Y accumulates over the flushes: in the kernel on the workgroup-pair
  // pass, else through the workspace's Y and an add pass (the same sums)
  const bool kadd = s->single && s->y_init && sketch_adds_y(ctx, s->dtype, ld, src, sh);
  void* ydst = nullptr;
  if (s->single) ydst = (s->y_init && !kadd) ? w.Y : s->Y;
  // on the workgroup-pair pass, a stream of more columns than one stage
  // forms Psi once as images (stream-owned) that every flush reads
  if (!s->psi_img && s->n_max > s->stage_cols && s->dtype == SID_F32 &&
      plan_sketch(ctx, s->dtype, ld, src, sh.prec, sh, s->p.coarse != nullptr, s->single) ==
          SketchPath::PAIR_BF16) {
    const size_t ib = sid::sketch_v2_psi_image_bytes(s->N, (int)sh.lq);
    if (ib > 0) {
      if (hipMalloc((void**)&s->psi_img, ib) != hipSuccess) {
        (void)hipGetLastError();
        s->psi_img = nullptr;
        return fail(ctx, SID_ENOMEM, "stream: device allocation of the Psi images failed");
      }
      const int dmode = sh.prec == SID_SK_BF16X2   ? sid::FB_BF16X2
                        : sh.prec == SID_SK_FP8E4M3 ? sid::FB_FP8
                                                    : sid::FB_BF16;
      SID_CHECK(sid::launch_sketch_v2_psi_image(ctx->stream, dmode, s->p.seed, s->N, (int)sh.lq,
                                                s->psi_img),
                "stream: Psi images");
    }
  }
  st = run_sketch(ctx, src, s->dtype, ld, &s->p, sh, w, s->W + s->lq * s->cols, ydst, s->cols,
                  kadd, s->psi_img);
  if (st != SID_OK) return st;
  if (s->single && s->y_init && !kadd)
    SID_CHECK(sid::launch_add_inplace(ctx->stream, s->p.prec == SID_SK_F64, s->Y, w.Y,
                                      s->N * s->l, ctx->num_cu),
              "stream: Y accumulation");
  if (s->svd) {
    st = svd_h_update(ctx, src, s->dtype, ld, s->N, ncols, s->W + s->lq * s->cols, s->lq, s->Wp,
                      s->H, s->cols > 0);
    if (st != SID_OK) return st;
  }
  s->y_init = s->single;
  s->cols += ncols;
  return SID_OK;
}

sid_status stream_flush_stage(sid_stream* s) {
  if (s->staged == 0) return SID_OK;
  const int64_t n = s->staged;
  s->staged = 0;
  return stream_flush(s, s->stage, s->ld_stage, n);
}

struct StreamHeader {
  char magic[8];
  int64_t version, N, n_max, cols, dtype, y_init;
  int64_t k, oversample, mode, prec, probe_rows, corange_rows;
  uint64_t seed;
  double rank_tol, sp_rcond, probe_tol;
};

const char kStreamMagic[8] = {'S', 'I', 'D', 'S', 'T', 'R', 'M', '1'};

sid_status stream_make(sid_ctx* ctx, sid_dtype dtype, int64_t N, int64_t n_max,
                       const sid_params* p, sid_stream** out) {
  Shape sh;
  sid_status st = validate(ctx, N, n_max, p, &sh);
  if (st != SID_OK) return st;
  sid_stream* s = new (std::nothrow) sid_stream();
  if (!s) return fail(ctx, SID_ENOMEM, "host allocation failed");
  s->ctx = ctx;
  s->p = *p;
  s->dtype = dtype;
  s->N = N;
  s->n_max = n_max;
  s->lq = sh.lq;
  s->l = sh.l;
  s->single = sh.single;
  s->stage_cols = n_max < 512 ? n_max : 512;
  {
    // on the workgroup-pair pass a flush of whole column slabs (e.g. 384 at
    // l = 180) avoids a narrow slab per flush
    Shape fs = sh;
    fs.n = s->stage_cols;
    if (plan_sketch(ctx, SID_F32, 4, nullptr, p->prec, fs, false, sh.single) == SketchPath::PAIR_BF16) {
      const int vslab = sid::sketch_v2_slab((int)sh.lq, (int)sh.l, sh.single);
      if (vslab > 0 && vslab <= 512) {
        const int64_t w = (512 / vslab) * vslab;
        s->stage_cols = n_max < w ? n_max : w;
      }
    }
  }
  s->ld_stage = (N + 3) / 4 * 4;
  st = stream_alloc(ctx, s);
  if (st != SID_OK) {
    stream_free(s);
    return st;
  }
  *out = s;
  return SID_OK;
}

}  // namespace

sid_status sid_stream_begin(sid_ctx* ctx, sid_dtype dtype, int64_t N, int64_t n_max,
                            const sid_params* p, sid_stream** out) {
  if (!ctx) return SID_EINVAL;
  if (!out) return fail(ctx, SID_EINVAL, "out is NULL");
  *out = nullptr;
  if (dtype != SID_F32 && dtype != SID_F64) return fail(ctx, SID_EINVAL, "unknown dtype");
  Shape sh;
  const sid_status vs = validate(ctx, N, n_max, p, &sh);
  if (vs != SID_OK) return vs;
  if (p->refine)
    return fail(ctx, SID_EINVAL, "refinement re-reads A; a stream keeps no columns");
  if (p->select != SID_SEL_GAUSS)
    return fail(ctx, SID_EINVAL, "a stream sketches its blocks; literal selection needs all rows");
  if (p->mode == SID_COARSE_SKELETON)
    return fail(ctx, SID_EINVAL, "the coarse-skeleton mode is not streamed (a stream keeps no rows)");
  SID_NEED_DEVICE(ctx);
  SID_CHECK(hipSetDevice(ctx->device), "hipSetDevice");
  return stream_make(ctx, dtype, N, n_max, p, out);
}

sid_status sid_stream_push(sid_stream* s, const void* A_blk, int64_t ncols, int64_t ld) {
  if (!s) return SID_EINVAL;
  sid_ctx* ctx = s->ctx;
  if (ncols < 0) return fail(ctx, SID_EINVAL, "ncols < 0");
  if (ncols == 0) return SID_OK;
  if (!A_blk) return fail(ctx, SID_EINVAL, "A_blk is NULL");
  if (ld < s->N) return fail(ctx, SID_EINVAL, "ld < N");
  if (s->cols + s->staged + ncols > s->n_max)
    return fail(ctx, SID_EINVAL, "more columns pushed than n_max");
  SID_CHECK(hipSetDevice(ctx->device), "hipSetDevice");
  const size_t esz = elem_size(s->dtype);
  const char* src = (const char*)A_blk;
  const bool aligned = (ld % 4) == 0 && ((uintptr_t)A_blk % 16) == 0;
  int64_t done = 0;
  while (done < ncols) {
    const int64_t left = ncols - done;
    if (s->staged == 0 && left >= s->stage_cols && aligned) {
      // a whole pass straight from the caller's memory
      sid_status st = stream_flush(s, src + (size_t)done * (size_t)ld * esz, ld, s->stage_cols);
      if (st != SID_OK) return st;
      done += s->stage_cols;
      continue;
    }
    if (!s->stage) {
      if (hipMalloc(&s->stage, esz * (size_t)(s->ld_stage * s->stage_cols)) != hipSuccess) {
        (void)hipGetLastError();
        return fail(ctx, SID_ENOMEM, "stream: device allocation of the stage failed");
      }
    }
    const int64_t take = left < s->stage_cols - s->staged ? left : s->stage_cols - s->staged;
    SID_CHECK(hipMemcpy2DAsync((char*)s->stage + (size_t)s->staged * (size_t)s->ld_stage * esz,
                               (size_t)s->ld_stage * esz, src + (size_t)done * (size_t)ld * esz,
                               (size_t)ld * esz, (size_t)s->N * esz, (size_t)take,
                               hipMemcpyDeviceToDevice, ctx->stream),
              "stream: stage copy");
    s->staged += take;
    done += take;
    if (s->staged == s->stage_cols) {
      sid_status st = stream_flush_stage(s);
      if (st != SID_OK) return st;
    }
  }
  return SID_OK;
}

sid_status sid_stream_finish(sid_stream* s, int64_t* J, void* P, int64_t ldp, void* AJ,
                             int64_t ldaj, double* err, int64_t* k_eff) {
  if (!s) return SID_EINVAL;
  sid_ctx* ctx = s->ctx;
  if (s->svd) return fail(ctx, SID_EINVAL, "an SBR-SVD stream ends with sid_svd_stream_finish");
  sid_status st = SID_OK;
  do {
    if (hipSetDevice(ctx->device) != hipSuccess) {
      st = fail(ctx, SID_EDEVICE, "hipSetDevice");
      break;
    }
    if (!s->single && AJ) {
      st = fail(ctx, SID_EINVAL,
                "two-pass stream: AJ must be NULL (the stream keeps no columns; copy A(:, J) "
                "from the caller's data)");
      break;
    }
    st = stream_flush_stage(s);
    if (st != SID_OK) break;
    Shape sh;
    st = validate(ctx, s->N, s->cols, &s->p, &sh);
    if (st != SID_OK) break;
    if (P && ldp < s->p.k) {
      st = fail(ctx, SID_EINVAL, "ldp < k");
      break;
    }
    if (AJ && ldaj < s->N) {
      st = fail(ctx, SID_EINVAL, "ldaj < N");
      break;
    }
    Work w;
    if (reserve(ctx, sh, &w) != SID_OK) {
      st = SID_ENOMEM;
      break;
    }
    w.W = s->W;
    if (s->single) {
      w.Y = s->Y;
      hipError_t e = sid::launch_fill_gaussian(ctx->stream, s->p.seed, 0u, 0, sh.n, 0, sh.l,
                                               w.omega);
      if (e != hipSuccess) {
        st = hip_fail(ctx, e, "omega generation");
        break;
      }
    }
    st = factor(ctx, &s->p, sh, w, s->dtype, nullptr, 0, J, P, ldp, AJ, ldaj, err, k_eff);
  } while (false);
  stream_free(s);
  return st;
}

sid_status sid_stream_info(const sid_stream* s, int64_t* N, int64_t* cols, int64_t* k,
                           int* dtype, int* mode) {
  if (!s) return SID_EINVAL;
  if (N) *N = s->N;
  if (cols) *cols = s->cols + s->staged;
  if (k) *k = s->p.k;
  if (dtype) *dtype = (int)s->dtype;
  if (mode) *mode = (int)s->p.mode;
  return SID_OK;
}

sid_status sid_stream_abort(sid_stream* s) {
  if (!s) return SID_EINVAL;
  stream_free(s);
  return SID_OK;
}

sid_status sid_stream_save(sid_stream* s, void* host_buf, size_t* bytes) {
  if (!s) return SID_EINVAL;
  sid_ctx* ctx = s->ctx;
  if (s->svd) return fail(ctx, SID_EINVAL, "SBR-SVD streams cannot be saved");
  if (!bytes) return fail(ctx, SID_EINVAL, "bytes is NULL");
  if (s->p.coarse)
    return fail(ctx, SID_EINVAL, "a stream over a coarse row set cannot be saved");
  SID_CHECK(hipSetDevice(ctx->device), "hipSetDevice");
  sid_status st = stream_flush_stage(s);
  if (st != SID_OK) return st;
  const size_t wb = sizeof(double) * (size_t)(s->lq * s->cols);
  const size_t yb = s->y_init ? y_elem_size(s) * (size_t)(s->N * s->l) : 0;
  const size_t need = sizeof(StreamHeader) + wb + yb;
  if (!host_buf) {
    *bytes = need;
    return SID_OK;
  }
  if (*bytes < need) {
    *bytes = need;
    return fail(ctx, SID_EINVAL, "buffer too small for the stream state");
  }
  StreamHeader h;
  std::memset(&h, 0, sizeof(h));
  std::memcpy(h.magic, kStreamMagic, 8);
  h.version = 2;
  h.N = s->N;
  h.n_max = s->n_max;
  h.cols = s->cols;
  h.dtype = s->dtype;
  h.y_init = s->y_init ? 1 : 0;
  h.k = s->p.k;
  h.oversample = s->p.oversample;
  h.mode = s->p.mode;
  h.prec = s->p.prec;
  h.probe_rows = s->p.probe_rows;
  h.corange_rows = s->p.corange_rows;
  h.seed = s->p.seed;
  h.rank_tol = s->p.rank_tol;
  h.sp_rcond = s->p.sp_rcond;
  h.probe_tol = s->p.probe_tol;
  char* out = (char*)host_buf;
  std::memcpy(out, &h, sizeof(h));
  if (wb) SID_CHECK(hipMemcpyAsync(out + sizeof(h), s->W, wb, hipMemcpyDeviceToHost, ctx->stream),
                    "stream save: W");
  if (yb)
    SID_CHECK(hipMemcpyAsync(out + sizeof(h) + wb, s->Y, yb, hipMemcpyDeviceToHost, ctx->stream),
              "stream save: Y");
  SID_CHECK(hipStreamSynchronize(ctx->stream), "stream save: synchronize");
  *bytes = need;
  return SID_OK;
}

sid_status sid_stream_restore(sid_ctx* ctx, const void* host_buf, size_t bytes, sid_stream** out) {
  if (!ctx) return SID_EINVAL;
  if (!out || !host_buf) return fail(ctx, SID_EINVAL, "null argument");
  *out = nullptr;
  if (bytes < sizeof(StreamHeader)) return fail(ctx, SID_EINVAL, "stream state too short");
  StreamHeader h;
  std::memcpy(&h, host_buf, sizeof(h));
  if (std::memcmp(h.magic, kStreamMagic, 8) != 0 || h.version != 2)
    return fail(ctx, SID_EINVAL, "not a saved stream state");
  if (h.dtype != SID_F32 && h.dtype != SID_F64) return fail(ctx, SID_EINVAL, "bad dtype in state");
  SID_NEED_DEVICE(ctx);
  SID_CHECK(hipSetDevice(ctx->device), "hipSetDevice");
  sid_params p;
  sid_params_init(&p, h.k);
  p.oversample = h.oversample;
  p.mode = (sid_mode)h.mode;
  p.prec = (sid_sketch_prec)h.prec;
  p.probe_rows = (int32_t)h.probe_rows;
  p.corange_rows = (int32_t)h.corange_rows;
  p.seed = h.seed;
  p.rank_tol = h.rank_tol;
  p.sp_rcond = h.sp_rcond;
  p.probe_tol = h.probe_tol;
  sid_stream* s = nullptr;
  sid_status st = stream_make(ctx, (sid_dtype)h.dtype, h.N, h.n_max, &p, &s);
  if (st != SID_OK) return st;
  if (h.cols < 0 || h.cols > h.n_max || (h.y_init != 0) != (s->single && h.cols > 0)) {
    stream_free(s);
    return fail(ctx, SID_EINVAL, "inconsistent stream state");
  }
  const size_t wb = sizeof(double) * (size_t)(s->lq * h.cols);
  const size_t yb = h.y_init ? y_elem_size(s) * (size_t)(s->N * s->l) : 0;
  if (bytes < sizeof(h) + wb + yb) {
    stream_free(s);
    return fail(ctx, SID_EINVAL, "stream state truncated");
  }
  const char* in = (const char*)host_buf;
  hipError_t e = hipSuccess;
  if (wb) e = hipMemcpyAsync(s->W, in + sizeof(h), wb, hipMemcpyHostToDevice, ctx->stream);
  if (e == hipSuccess && yb)
    e = hipMemcpyAsync(s->Y, in + sizeof(h) + wb, yb, hipMemcpyHostToDevice, ctx->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
  if (e != hipSuccess) {
    stream_free(s);
    return hip_fail(ctx, e, "stream restore: upload");
  }
  s->cols = h.cols;
  s->y_init = h.y_init != 0;
  *out = s;
  return SID_OK;
}

// ---------------------------------------------------------------------------
// Batched compression: independent problems (Sec. 3 compresses each flow
// variable / dataset separately; Sec. 3.3 compresses a long record block by
// block).
//
// Persistent path (FP32 data, one bfloat16 sketch form and one mode for all
// problems, shapes of the one-workgroup-per-row-range matrix-core pass, no
// coarse rows or refinement): one launch sketches every problem -- a work
// queue of all problems' row shares, the problems with the most work per
// share first -- then one launch sums every problem's partials into its W.
// Each share is a row range the single-matrix launch would give one
// workgroup, so W and Y are bit for bit those of per-problem calls.  The
// latency-bound factorizations then run per problem on child streams (own
// workspace each).  Nothing is allocated once the batch's plan exists
// (sid_reserve_batched, or an earlier call with the same problems), so the
// whole call can be captured in a HIP graph.
// Other batches: each problem's sid_compress on the child streams.
// The children start after the work already queued on the context's stream
// and the context's stream waits for all of them.
// ---------------------------------------------------------------------------
// (C++ linkage: these helpers pass std::string and std::vector)
extern "C++" {
namespace {
constexpr int SID_BATCH_STREAMS_MAX = 8;
constexpr size_t SID_BATCH_PLANS = 8;

bool capturing(hipStream_t st) {
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  return hipStreamIsCapturing(st, &cs) == hipSuccess && cs != hipStreamCaptureStatusNone;
}

sid_status ensure_children(sid_ctx* ctx, int want) {
  if ((!ctx->fork || (int)ctx->children.size() < want) && capturing(ctx->stream))
    return fail(ctx, SID_ESTATE,
                "batched call under graph capture: create its child streams first "
                "(sid_reserve_batched, or an eager call with as many problems)");
  if (!ctx->fork) {
    if (hipEventCreateWithFlags(&ctx->fork, hipEventDisableTiming) != hipSuccess) {
      (void)hipGetLastError();
      return fail(ctx, SID_EDEVICE, "event creation failed");
    }
  }
  while ((int)ctx->children.size() < want) {
    sid_ctx* c = nullptr;
    const sid_status st = sid_create(&c, ctx->device, nullptr);
    if (st != SID_OK) return fail(ctx, st, "child context creation failed");
    c->limit = ctx->limit;
    c->cooperative = ctx->cooperative;
    hipEvent_t e = nullptr;
    if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) {
      (void)hipGetLastError();
      (void)sid_destroy(c);
      return fail(ctx, SID_EDEVICE, "event creation failed");
    }
    ctx->children.push_back(c);
    ctx->child_done.push_back(e);
  }
  return SID_OK;
}

// every problem validated; shapes into sh
sid_status validate_batch(sid_ctx* ctx, const sid_problem* probs, int64_t count, sid_dtype dtype,
                          std::vector<Shape>* sh) {
  if (count < 0) return fail(ctx, SID_EINVAL, "count < 0");
  if (count > 0 && !probs) return fail(ctx, SID_EINVAL, "probs is NULL");
  if (dtype != SID_F32 && dtype != SID_F64) return fail(ctx, SID_EINVAL, "unknown dtype");
  sh->assign((size_t)count, Shape{});
  for (int64_t b = 0; b < count; ++b) {
    const sid_problem& q = probs[b];
    const std::string at = "problem " + std::to_string(b) + ": ";
    if (!q.A) return fail(ctx, SID_EINVAL, at + "A is NULL");
    if (q.lda < q.N) return fail(ctx, SID_EINVAL, at + "lda < N");
    const sid_status vs = validate(ctx, q.N, q.n, &q.params, &(*sh)[(size_t)b]);
    if (vs != SID_OK) return fail(ctx, vs, at + ctx->err);
    if (q.P && q.ldp < q.params.k) return fail(ctx, SID_EINVAL, at + "ldp < k");
    if (q.AJ && q.ldaj < skeleton_rows(&q.params, q.N))
      return fail(ctx, SID_EINVAL, at + "ldaj < rows of the skeleton");
    if (q.params.coarse && q.params.coarse->ctx != ctx)
      return fail(ctx, SID_EINVAL, at + "row set belongs to another context");
  }
  return SID_OK;
}

bool batch_persistent_ok(const sid_ctx* ctx, const sid_problem* probs, int64_t count,
                         sid_dtype dtype, const std::vector<Shape>& sh) {
  // (the batched launches put up to 2 count jobs in one grid dimension)
  if (dtype != SID_F32 || count < 1 || count > 16384 || ctx->sketch_pairs) return false;
  const int prec = probs[0].params.prec;
  if (prec != SID_SK_BF16 && prec != SID_SK_BF16X2 && prec != SID_SK_FP8E4M3) return false;
  const bool single = sh[0].single;
  for (int64_t b = 0; b < count; ++b) {
    const sid_problem& q = probs[b];
    const Shape& s = sh[(size_t)b];
    if (q.params.prec != prec || s.single != single || q.params.coarse ||
        q.params.select != SID_SEL_GAUSS || q.params.refine || q.params.mode == SID_COARSE_SKELETON)
      return false;
    if (!sid::fused_bf16_batch_supported(s.n, (int)s.lq, (int)s.l, q.lda, q.A)) return false;
    // the single-matrix call takes the same pass, so the bits agree
    if (plan_sketch(ctx, dtype, q.lda, q.A, prec, s, false, single) != SketchPath::FUSED_BF16)
      return false;
  }
  return true;
}

// the plan of this batch: found among the context's plans, or built (not
// under graph capture: it allocates)
sid_status batch_plan(sid_ctx* ctx, const sid_problem* probs, int64_t count,
                      const std::vector<Shape>& sh, BatchPlan** out) {
  const int prec = probs[0].params.prec;
  const int dmode = prec == SID_SK_BF16X2 ? sid::FB_BF16X2 : prec == SID_SK_FP8E4M3 ? sid::FB_FP8
                                                                                  : sid::FB_BF16;
  const bool wanty = sh[0].single;
  std::vector<BatchSig> sig((size_t)count);
  for (int64_t b = 0; b < count; ++b) {
    const Shape& s = sh[(size_t)b];
    const sid_params& q = probs[b].params;
    sig[(size_t)b] = BatchSig{probs[b].A, s.N, s.n, probs[b].lda, s.lq, s.l, s.lz, s.k, q.seed,
                              q.rank_tol, q.sp_rcond > 0.0 ? q.sp_rcond : default_rcond(s.prec),
                              q.probe_tol};
  }
  for (size_t i = 0; i < ctx->plans.size(); ++i) {
    BatchPlan* pl = ctx->plans[i];
    if (pl->dmode == dmode && pl->wanty == wanty && pl->sig == sig) {
      ctx->plans.erase(ctx->plans.begin() + (long)i);
      ctx->plans.push_back(pl);
      *out = pl;
      return SID_OK;
    }
  }
  if (capturing(ctx->stream))
    return fail(ctx, SID_ESTATE,
                "batched call under graph capture: build its plan first (sid_reserve_batched, or "
                "an eager call with the same problems)");
  // queue order: by layout class, then the most work per share first
  std::vector<int64_t> rpw((size_t)count), nsh((size_t)count);
  std::vector<int> order((size_t)count), cls((size_t)count);
  for (int64_t b = 0; b < count; ++b) {
    nsh[(size_t)b] = sid::fused_bf16_grid(sh[(size_t)b].N, ctx->num_cu, &rpw[(size_t)b]);
    order[(size_t)b] = (int)b;
    cls[(size_t)b] = sid::fused_bf16_batch_class((int)sh[(size_t)b].lq, (int)sh[(size_t)b].l, wanty);
  }
  std::stable_sort(order.begin(), order.end(), [&](int x, int y) {
    if (cls[(size_t)x] != cls[(size_t)y]) return cls[(size_t)x] < cls[(size_t)y];
    return rpw[(size_t)x] * sh[(size_t)x].n > rpw[(size_t)y] * sh[(size_t)y].n;
  });
  auto up = [](size_t v) { return (v + 255) / 256 * 256; };
  // the problems whose mgsqr runs in the batched launches: the one-workgroup
  // kernels take W_sel (and, single pass, M)
  auto batchable = [](int m, int nc) {
    const int kd = mgsqr_kind(m, nc);
    return kd == 0 || kd == 3;
  };
  std::vector<char> pre((size_t)count);
  for (int64_t b = 0; b < count; ++b) {
    const Shape& s = sh[(size_t)b];
    pre[(size_t)b] = batchable((int)s.l, (int)s.n) && (!wanty || batchable((int)s.lz, (int)s.l));
  }
  const size_t d = sizeof(double), i8 = sizeof(int64_t);
  auto fac_bytes = [&](const Shape& s) {
    size_t v = up(i8 * (size_t)s.k) + up(d * (size_t)(s.k * s.n)) + up(d * (size_t)(s.l * s.k)) +
               up(i8) + up(2 * d);
    if (wanty)
      v += up(d * (size_t)(s.n * s.l)) + up(d * (size_t)(s.lz * s.l)) +
           up(d * (size_t)((s.q > 0 ? s.q : 1) * s.l)) + up(i8 * (size_t)s.l) +
           up(d * (size_t)(s.l * s.l)) + up(d * (size_t)(s.lz * s.l)) + up(i8) + up(2 * d);
    return v;
  };
  bool tail = wanty;
  for (int64_t b = 0; b < count; ++b) {
    const Shape& s = sh[(size_t)b];
    tail = tail && pre[(size_t)b] && sig[(size_t)b].probe_tol <= 0.0 && s.k <= 128 && s.l <= 128;
  }
  auto tail_bytes = [&](const Shape& s) {
    const int64_t qq = s.q > 0 ? s.q : 1;
    return up(d * (size_t)(s.k * s.k)) + up(d * (size_t)(s.k * s.n)) + up(d * (size_t)(s.lz * s.k)) +
           up(d * (size_t)(s.l * s.k)) + up(d * (size_t)(s.l * s.k)) + up(d * (size_t)(s.l * s.l)) +
           up(d * (size_t)(qq * s.k)) + up(d * (size_t)(2 * ((qq * s.n + 255) / 256) + 2)) +
           up(2 * d);
  };
  size_t bytes = up(sizeof(sid::FbBatchEntry) * (size_t)count) + 256 +
                 up(sizeof(sid::CpqrJob) * (size_t)(2 * count)) +
                 up(sizeof(sid::OmegaJob) * (size_t)count) +
                 up(sizeof(sid::Gemm64Job) * (size_t)(2 * count));
  if (tail)
    bytes += up(sizeof(sid::GatherR11Job) * (size_t)(2 * count)) +
             2 * up(sizeof(sid::TrsvJob) * (size_t)count) + up(sizeof(sid::RatioJob) * (size_t)count) +
             up(sizeof(sid::GatherBlockJob) * (size_t)count) +
             2 * up(sizeof(sid::Gemm64Job) * (size_t)count) + up(sizeof(sid::FitJob) * (size_t)count) +
             up(sizeof(sid::ApplyJob) * (size_t)count);
  for (int64_t b = 0; b < count; ++b) {
    const Shape& s = sh[(size_t)b];
    bytes += up(sizeof(float) * (size_t)(nsh[(size_t)b] * s.lq * s.n)) +
             up(sizeof(double) * (size_t)(s.lq * s.n));
    if (wanty)
      bytes += up(sizeof(float) * (size_t)(s.n * s.l)) + up(sizeof(uint16_t) * 128 * 512) +
               up(sizeof(float) * (size_t)(s.N * s.l));
    if (pre[(size_t)b]) bytes += fac_bytes(s);
    if (tail) bytes += tail_bytes(s);
  }
  if (ctx->plans.size() >= SID_BATCH_PLANS) {
    // the oldest plan goes; nothing queued may still read it
    SID_CHECK(hipStreamSynchronize(ctx->stream), "batched: plan eviction");
    for (sid_ctx* c : ctx->children) SID_CHECK(hipStreamSynchronize(c->stream), "batched: plan eviction");
    BatchPlan* old = ctx->plans.front();
    ctx->plans.erase(ctx->plans.begin());
    if (old->dev) (void)hipFree(old->dev);
    delete old;
  }
  BatchPlan* pl = new (std::nothrow) BatchPlan();
  if (!pl) return fail(ctx, SID_ENOMEM, "batched: plan");
  if (hipMalloc(&pl->dev, bytes) != hipSuccess) {
    (void)hipGetLastError();
    delete pl;
    return fail(ctx, SID_ENOMEM, "batched: device memory for the batch (" + std::to_string(bytes) +
                                     " bytes)");
  }
  pl->bytes = bytes;
  pl->sig = sig;
  pl->dmode = dmode;
  pl->wanty = wanty;
  unsigned char* cur = (unsigned char*)pl->dev;
  auto take = [&](size_t b) {
    unsigned char* r = cur;
    cur += up(b);
    return r;
  };
  pl->d_tab = (sid::FbBatchEntry*)take(sizeof(sid::FbBatchEntry) * (size_t)count);
  pl->d_queue = (unsigned int*)take(256);
  pl->d_jobs = (sid::CpqrJob*)take(sizeof(sid::CpqrJob) * (size_t)(2 * count));
  pl->d_om_jobs = (sid::OmegaJob*)take(sizeof(sid::OmegaJob) * (size_t)count);
  pl->d_mm_jobs = (sid::Gemm64Job*)take(sizeof(sid::Gemm64Job) * (size_t)(2 * count));
  pl->tail = tail;
  if (tail) {
    pl->d_gr11 = (sid::GatherR11Job*)take(sizeof(sid::GatherR11Job) * (size_t)(2 * count));
    pl->d_trsv0 = (sid::TrsvJob*)take(sizeof(sid::TrsvJob) * (size_t)count);
    pl->d_trsv1 = (sid::TrsvJob*)take(sizeof(sid::TrsvJob) * (size_t)count);
    pl->d_ratio = (sid::RatioJob*)take(sizeof(sid::RatioJob) * (size_t)count);
    pl->d_gblock = (sid::GatherBlockJob*)take(sizeof(sid::GatherBlockJob) * (size_t)count);
    pl->d_gemm_c = (sid::Gemm64Job*)take(sizeof(sid::Gemm64Job) * (size_t)count);
    pl->d_gemm_mix = (sid::Gemm64Job*)take(sizeof(sid::Gemm64Job) * (size_t)count);
    pl->d_fit = (sid::FitJob*)take(sizeof(sid::FitJob) * (size_t)count);
    pl->d_apply = (sid::ApplyJob*)take(sizeof(sid::ApplyJob) * (size_t)count);
  }
  pl->W.assign((size_t)count, nullptr);
  pl->Y.assign((size_t)count, nullptr);
  pl->omega.assign((size_t)count, nullptr);
  pl->fac.assign((size_t)count, BatchFactor{});
  std::vector<sid::FbBatchEntry> tab((size_t)count);
  int64_t share0 = 0;
  pl->classes.clear();
  for (int64_t qpos = 0; qpos < count; ++qpos) {
    const int b = order[(size_t)qpos];
    const Shape& s = sh[(size_t)b];
    if (pl->classes.empty() || pl->classes.back().cls != cls[(size_t)b]) {
      // a new class: its own queue, shares numbered from 0
      pl->classes.push_back(sid::FbBatchClass{cls[(size_t)b], (int)qpos, 0, 0});
      share0 = 0;
    }
    ++pl->classes.back().count;
    sid::FbBatchEntry& e = tab[(size_t)qpos];
    e.A = (const float*)probs[b].A;
    e.lda = probs[b].lda;
    e.N = s.N;
    e.n = (int)s.n;
    e.lq = (int)s.lq;
    e.l = (int)s.l;
    e.cls = cls[(size_t)b];
    e.seed = probs[b].params.seed;
    e.rows_per_wg = rpw[(size_t)b];
    e.share0 = share0;
    e.nshares = nsh[(size_t)b];
    share0 += e.nshares;
    pl->classes.back().nshares = share0;
    e.part = (float*)take(sizeof(float) * (size_t)(e.nshares * s.lq * s.n));
    e.W = (double*)take(sizeof(double) * (size_t)(s.lq * s.n));
    e.omega = nullptr;
    e.omT = nullptr;
    e.Y = nullptr;
    if (wanty) {
      e.omega = (float*)take(sizeof(float) * (size_t)(s.n * s.l));
      e.omT = (__bf16*)take(sizeof(uint16_t) * 128 * 512);
      e.Y = (float*)take(sizeof(float) * (size_t)(s.N * s.l));
    }
    pl->W[(size_t)b] = e.W;
    pl->Y[(size_t)b] = e.Y;
    pl->omega[(size_t)b] = e.omega;
    if (s.n > pl->max_n) pl->max_n = (int)s.n;
    if (s.lq * s.n > pl->max_lqn) pl->max_lqn = s.lq * s.n;
  }
  // the factorization buffers and the mgsqr jobs (W_sel's, then M's),
  // grouped by kernel instance
  std::vector<std::pair<int, sid::CpqrJob>> jobs;
  std::vector<sid::OmegaJob> omj;
  std::vector<sid::Gemm64Job> mmj, gemmc, gemmmix;
  std::vector<sid::GatherR11Job> gr11w, gr11m;
  std::vector<sid::TrsvJob> trsv0, trsv1;
  std::vector<sid::RatioJob> ratio;
  std::vector<sid::GatherBlockJob> gblock;
  std::vector<sid::FitJob> fit;
  for (int64_t b = 0; b < count; ++b) {
    if (!pre[(size_t)b]) continue;
    const Shape& s = sh[(size_t)b];
    const BatchSig& g = sig[(size_t)b];
    BatchFactor& f = pl->fac[(size_t)b];
    f.pre = true;
    f.piv = (int64_t*)take(i8 * (size_t)s.k);
    f.R = (double*)take(d * (size_t)(s.k * s.n));
    f.Q = (double*)take(d * (size_t)(s.l * s.k));
    f.keff = (int64_t*)take(i8);
    f.stats = (double*)take(2 * d);
    const bool wl = mgsqr_kind((int)s.l, (int)s.n) == 3;
    const int wi = sid::cpqr_batch_instance((int)s.l, (int)s.n, wl);
    jobs.push_back({wi, sid::CpqrJob{pl->W[(size_t)b], s.lq, (int)s.l, (int)s.n, (int)s.k, wi,
                                     g.rank_tol, f.piv, f.R, f.Q, f.keff, f.stats}});
    if (wanty) {
      f.om64 = (double*)take(d * (size_t)(s.n * s.l));
      f.M = (double*)take(d * (size_t)(s.lz * s.l));
      f.Mpr = (double*)take(d * (size_t)((s.q > 0 ? s.q : 1) * s.l));
      f.pivM = (int64_t*)take(i8 * (size_t)s.l);
      f.RM = (double*)take(d * (size_t)(s.l * s.l));
      f.QM = (double*)take(d * (size_t)(s.lz * s.l));
      f.rkM = (int64_t*)take(i8);
      f.statsM = (double*)take(2 * d);
      const bool ml = mgsqr_kind((int)s.lz, (int)s.l) == 3;
      const int mi = sid::cpqr_batch_instance((int)s.lz, (int)s.l, ml);
      jobs.push_back({mi, sid::CpqrJob{f.M, s.lz, (int)s.lz, (int)s.l, (int)s.l, mi, g.rcond,
                                       f.pivM, f.RM, f.QM, f.rkM, f.statsM}});
      // Omega's values, M = W(0:lz, :) Omega and Mpr = W_pr Omega, the
      // launches of the single call's step 5a
      omj.push_back(sid::OmegaJob{pl->omega[(size_t)b], s.n * s.l, f.om64});
      pl->om_max_count = std::max(pl->om_max_count, s.n * s.l);
      const double* Wb = pl->W[(size_t)b];
      mmj.push_back(sid::Gemm64Job{(int)s.lz, (int)s.l, (int)s.n, 0, 1, 0, Wb, s.lq, f.om64, s.l,
                                   f.M, s.lz, 1.0, 0.0});
      if (s.q > 0)
        mmj.push_back(sid::Gemm64Job{(int)s.q, (int)s.l, (int)s.n, 0, 1, 0, Wb + s.lz, s.lq, f.om64,
                                     s.l, f.Mpr, s.q, 1.0, 0.0});
      pl->mm_max_m = std::max(pl->mm_max_m, (int)s.lz);
      pl->mm_max_n = std::max(pl->mm_max_n, (int)s.l);
    }
    if (tail) {
      // the single call's steps 3, 4, 5b after mgsqr (factor()), on the
      // plan's buffers
      const int k = (int)s.k, l = (int)s.l, lz = (int)s.lz, q = (int)s.q, n_ = (int)s.n;
      const int qq = q > 0 ? q : 1;
      f.R11 = (double*)take(d * (size_t)(k * k));
      f.Pd = (double*)take(d * (size_t)(k * n_));
      f.WJ = (double*)take(d * (size_t)(lz * k));
      f.C = (double*)take(d * (size_t)(l * k));
      f.T = (double*)take(d * (size_t)(l * k));
      f.R11M = (double*)take(d * (size_t)(l * l));
      f.mix = (double*)take(d * (size_t)(qq * k));
      f.fitpart = (double*)take(d * (size_t)(2 * ((qq * n_ + 255) / 256) + 2));
      f.err = (double*)take(2 * d);
      const double* Wb = pl->W[(size_t)b];
      gr11w.push_back(sid::GatherR11Job{f.R, n_, f.piv, f.keff, k, 0, f.R11});
      gr11m.push_back(sid::GatherR11Job{f.RM, l, f.pivM, f.rkM, l, 0, f.R11M});
      trsv0.push_back(sid::TrsvJob{f.R11, k, n_, f.keff, f.piv, f.R, n_, f.Pd, k});
      trsv1.push_back(sid::TrsvJob{f.R11M, l, k, f.rkM, f.pivM, f.C, l, f.T, l});
      ratio.push_back(sid::RatioJob{f.stats, f.err + 1});
      gblock.push_back(sid::GatherBlockJob{Wb, (int)s.lq, 0, lz, k, f.piv, f.keff, f.WJ});
      gemmc.push_back(sid::Gemm64Job{l, k, lz, 1, 0, 0, f.QM, lz, f.WJ, lz, f.C, l, 1.0, 0.0});
      if (q > 0)
        gemmmix.push_back(sid::Gemm64Job{q, k, l, 0, 0, 0, f.Mpr, q, f.T, l, f.mix, q, 1.0, 0.0});
      fit.push_back(sid::FitJob{Wb, (int)s.lq, lz, q, n_, k, 0, f.piv, f.keff, f.Pd,
                                q > 0 ? f.mix : nullptr, f.fitpart, f.err});
      pl->t_max_k = std::max(pl->t_max_k, k);
      pl->t_max_n = std::max(pl->t_max_n, n_);
      pl->t_max_l = std::max(pl->t_max_l, l);
      pl->t_max_gblock = std::max(pl->t_max_gblock, lz * k);
      pl->t_max_q = std::max(pl->t_max_q, q);
      pl->t_max_qn = std::max(pl->t_max_qn, q * n_);
    }
  }
  pl->n_om_jobs = (int)omj.size();
  pl->n_mm_jobs = (int)mmj.size();
  pl->n_gemm_mix = (int)gemmmix.size();
  std::stable_sort(jobs.begin(), jobs.end(),
                   [](const std::pair<int, sid::CpqrJob>& x, const std::pair<int, sid::CpqrJob>& y) {
                     return x.first < y.first;
                   });
  // one group per LDS-kernel instance (those come first), then every
  // register-kernel job in one group of its own launch
  std::vector<sid::CpqrJob> jtab;
  for (size_t i = 0; i < jobs.size(); ++i) {
    const int gi = jobs[i].first > 0 ? sid::CPQR_BATCH_ANY_WG : jobs[i].first;
    if (pl->job_groups.empty() || pl->job_groups.back()[0] != gi)
      pl->job_groups.push_back({gi, (int)i, 0});
    ++pl->job_groups.back()[2];
    jtab.push_back(jobs[i].second);
  }
  hipError_t e = hipMemcpyAsync(pl->d_tab, tab.data(), sizeof(sid::FbBatchEntry) * (size_t)count,
                                hipMemcpyHostToDevice, ctx->stream);
  if (e == hipSuccess && !jtab.empty())
    e = hipMemcpyAsync(pl->d_jobs, jtab.data(), sizeof(sid::CpqrJob) * jtab.size(),
                       hipMemcpyHostToDevice, ctx->stream);
  if (e == hipSuccess && !omj.empty())
    e = hipMemcpyAsync(pl->d_om_jobs, omj.data(), sizeof(sid::OmegaJob) * omj.size(),
                       hipMemcpyHostToDevice, ctx->stream);
  if (e == hipSuccess && !mmj.empty())
    e = hipMemcpyAsync(pl->d_mm_jobs, mmj.data(), sizeof(sid::Gemm64Job) * mmj.size(),
                       hipMemcpyHostToDevice, ctx->stream);
  if (tail) {
    // the M jobs of the R11 gather follow the W jobs
    gr11w.insert(gr11w.end(), gr11m.begin(), gr11m.end());
    auto upl = [&](void* dst, const void* src, size_t nb) {
      if (e == hipSuccess && nb > 0)
        e = hipMemcpyAsync(dst, src, nb, hipMemcpyHostToDevice, ctx->stream);
    };
    upl(pl->d_gr11, gr11w.data(), sizeof(sid::GatherR11Job) * gr11w.size());
    upl(pl->d_trsv0, trsv0.data(), sizeof(sid::TrsvJob) * trsv0.size());
    upl(pl->d_trsv1, trsv1.data(), sizeof(sid::TrsvJob) * trsv1.size());
    upl(pl->d_ratio, ratio.data(), sizeof(sid::RatioJob) * ratio.size());
    upl(pl->d_gblock, gblock.data(), sizeof(sid::GatherBlockJob) * gblock.size());
    upl(pl->d_gemm_c, gemmc.data(), sizeof(sid::Gemm64Job) * gemmc.size());
    upl(pl->d_gemm_mix, gemmmix.data(), sizeof(sid::Gemm64Job) * gemmmix.size());
    upl(pl->d_fit, fit.data(), sizeof(sid::FitJob) * fit.size());
  }
  if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
  if (e != hipSuccess) {
    (void)hipFree(pl->dev);
    delete pl;
    return hip_fail(ctx, e, "batched: table upload");
  }
  ctx->plans.push_back(pl);
  *out = pl;
  return SID_OK;
}

sid_status compress_batch(sid_ctx* ctx, const sid_problem* probs, int64_t count, sid_dtype dtype,
                          const std::vector<Shape>& sh, int nstreams_want) {
  const bool persistent = batch_persistent_ok(ctx, probs, count, dtype, sh);
  BatchPlan* plan = nullptr;
  if (persistent) {
    const sid_status ps = batch_plan(ctx, probs, count, sh, &plan);
    if (ps != SID_OK) return ps;
  }
  const int nstreams = count < nstreams_want ? (int)count : nstreams_want;
  const int ncls = persistent ? (int)plan->classes.size() : 0;
  sid_status st = ensure_children(ctx, std::max(nstreams, ncls - 1));
  if (st != SID_OK) return st;
  if (persistent) {
    // the setup, then one persistent launch per layout class: the first on
    // the context's stream, the others beside it on child streams, joined
    // before the sums of the partials
    SID_CHECK(sid::launch_sketch_batch_setup(ctx->stream, plan->dmode, plan->wanty, plan->d_tab,
                                             (int)count, plan->max_n, plan->d_queue),
              "batched sketch: setup");
    if (ncls > 1) SID_CHECK(hipEventRecord(ctx->fork, ctx->stream), "batched sketch: fork event");
    for (int c = 0; c < ncls; ++c) {
      hipStream_t cs = c == 0 ? ctx->stream : ctx->children[(size_t)(c - 1)]->stream;
      if (c > 0) SID_CHECK(hipStreamWaitEvent(cs, ctx->fork, 0), "batched sketch: fork wait");
      SID_CHECK(sid::launch_sketch_batch_class(cs, plan->dmode, plan->wanty, plan->d_tab,
                                               plan->classes[(size_t)c], plan->d_queue, ctx->num_cu),
                "batched sketch pass");
    }
    for (int c = 1; c < ncls; ++c) {
      const size_t ci = (size_t)(c - 1);
      SID_CHECK(hipEventRecord(ctx->child_done[ci], ctx->children[ci]->stream),
                "batched sketch: join event");
      SID_CHECK(hipStreamWaitEvent(ctx->stream, ctx->child_done[ci], 0), "batched sketch: join wait");
    }
    SID_CHECK(sid::launch_reduce_partials_batch(ctx->stream, plan->d_tab, (int)count, plan->max_lqn),
              "batched sketch: sums of the partials");
  }
  SID_CHECK(hipEventRecord(ctx->fork, ctx->stream), "batched: fork event");
  for (int c = 0; c < nstreams; ++c)
    SID_CHECK(hipStreamWaitEvent(ctx->children[c]->stream, ctx->fork, 0), "batched: fork wait");
  // The mgsqr runs of all problems whose shapes the one-workgroup kernels
  // take go into a few launches (one for all register-kernel jobs, one per
  // LDS-kernel instance, side by side), after the small products they need (single pass:
  // Omega's FP64 values, M and Mpr, two launches for the whole batch); every
  // job gets the bits of the single call.
  bool any_pre = false;
  if (persistent)
    for (const BatchFactor& f : plan->fac) any_pre = any_pre || f.pre;
  if (any_pre) {
    SID_CHECK(sid::launch_omega_values_batch(ctx->stream, sh[0].prec, plan->d_om_jobs,
                                             plan->n_om_jobs, plan->om_max_count),
              "batched: omega values");
    SID_CHECK(sid::launch_gemm64_batch(ctx->stream, plan->d_mm_jobs, plan->n_mm_jobs,
                                       plan->mm_max_m, plan->mm_max_n),
              "batched: M = W Omega, Mpr");
    // the groups side by side: the first on the context's stream, the
    // others on the child streams
    SID_CHECK(hipEventRecord(ctx->fork, ctx->stream), "batched: fork event");
    const int ng = (int)plan->job_groups.size();
    for (int i = 0; i < ng; ++i) {
      const auto& g = plan->job_groups[(size_t)i];
      hipStream_t cs = i == 0 ? ctx->stream : ctx->children[(size_t)((i - 1) % nstreams)]->stream;
      if (i > 0 && i - 1 < nstreams)
        SID_CHECK(hipStreamWaitEvent(cs, ctx->fork, 0), "batched: fork wait");
      SID_CHECK(sid::launch_cpqr_batch(cs, g[0], plan->d_jobs + g[1], g[2]), "batched: pivoted QR");
    }
    for (int c = 0; c < nstreams && c < ng - 1; ++c) {
      SID_CHECK(hipEventRecord(ctx->child_done[c], ctx->children[c]->stream), "batched: join event");
      SID_CHECK(hipStreamWaitEvent(ctx->stream, ctx->child_done[c], 0), "batched: join wait");
    }
    if (plan->tail) {
      // the steps after mgsqr, each one launch for the batch (the single
      // call's kernels on the plan's buffers): R11, P's solve into Pd, the
      // sketch-fit estimate, W(:, J), C = QM^T W(:, J), M's R11, T, Mpr T,
      // the probe estimate
      const int cnt = (int)count;
      SID_CHECK(sid::launch_gather_r11_batch(ctx->stream, plan->d_gr11, 2 * cnt), "batched: R11");
      SID_CHECK(sid::launch_trsv_batch(ctx->stream, 0, plan->d_trsv0, cnt, plan->t_max_k,
                                       plan->t_max_n),
                "batched: coefficients");
      SID_CHECK(sid::launch_ratio_sqrt_batch(ctx->stream, plan->d_ratio, cnt), "batched: sketch fit");
      SID_CHECK(sid::launch_gather_block_batch(ctx->stream, plan->d_gblock, cnt, plan->t_max_gblock),
                "batched: W(:, J)");
      SID_CHECK(sid::launch_gemm64_batch(ctx->stream, plan->d_gemm_c, cnt, plan->t_max_l,
                                         plan->t_max_k),
                "batched: QM^T W(:, J)");
      SID_CHECK(sid::launch_trsv_batch(ctx->stream, 1, plan->d_trsv1, cnt, plan->t_max_l,
                                       plan->t_max_k),
                "batched: T");
      SID_CHECK(sid::launch_gemm64_batch(ctx->stream, plan->d_gemm_mix, plan->n_gemm_mix,
                                         plan->t_max_q, plan->t_max_k),
                "batched: Mpr T");
      SID_CHECK(sid::launch_fit_residual_batch(ctx->stream, plan->d_fit, cnt, plan->t_max_qn),
                "batched: probe residual");
    }
    SID_CHECK(hipEventRecord(ctx->fork, ctx->stream), "batched: fork event");
    for (int c = 0; c < nstreams; ++c)
      SID_CHECK(hipStreamWaitEvent(ctx->children[c]->stream, ctx->fork, 0), "batched: fork wait");
  }
  sid_status result = SID_OK;
  const bool tail = any_pre && plan->tail;
  if (tail) {
    // AJ = Y T of every problem with an output: one launch on the context's
    // stream (the one-problem kernel's arithmetic, so the single call's
    // bits); per problem on the child streams: P from Pd in the caller's
    // type and layout (the values the single call's solve writes) and the
    // result copies
    const bool f64 = dtype == SID_F64;
    std::vector<sid::ApplyJob> aj;
    int max_nwg = 0, kmax = 0;
    for (int64_t b = 0; b < count; ++b) {
      const sid_problem& q = probs[b];
      const Shape& s = sh[(size_t)b];
      if (!q.AJ || f64 || !sid::apply_t_bf16_runs_supported((int)s.k, (int)s.l)) continue;
      sid::ApplyJob j{};
      j.Y = plan->Y[(size_t)b];
      j.T = plan->fac[(size_t)b].T;
      j.AJ = (float*)q.AJ;
      j.N = s.N;
      j.ldaj = q.ldaj;
      j.l = (int)s.l;
      j.k = (int)s.k;
      j.al = s.l % 4 == 0;
      j.vec = q.ldaj % 4 == 0 && (uintptr_t)q.AJ % 16 == 0;
      j.nwg = sid::apply_batch_workgroups(s.N, ctx->num_cu);
      aj.push_back(j);
      max_nwg = std::max(max_nwg, j.nwg);
      kmax = std::max(kmax, (int)s.k);
    }
    if (!aj.empty()) {
      if (aj.size() != plan->apply_host.size() ||
          std::memcmp(aj.data(), plan->apply_host.data(), sizeof(sid::ApplyJob) * aj.size()) != 0) {
        SID_CHECK(hipMemcpyAsync(plan->d_apply, aj.data(), sizeof(sid::ApplyJob) * aj.size(),
                                 hipMemcpyHostToDevice, ctx->stream),
                  "batched: AJ job table");
        plan->apply_host = aj;
      }
      SID_CHECK(sid::launch_apply_t_bf16_runs_batch(ctx->stream, plan->d_apply, (int)aj.size(),
                                                    max_nwg, kmax),
                "batched: AJ = Y T");
    }
    for (int64_t b = 0; b < count && result == SID_OK; ++b) {
      const sid_problem& q = probs[b];
      const Shape& s = sh[(size_t)b];
      const BatchFactor& f = plan->fac[(size_t)b];
      hipStream_t cs = ctx->children[(size_t)(b % nstreams)]->stream;
      hipError_t he = hipSuccess;
      if (q.P) he = sid::launch_convert(cs, f.Pd, true, s.k, s.n, s.k, q.P, f64, q.ldp);
      if (he == hipSuccess && q.AJ &&
          (f64 || !sid::apply_t_bf16_runs_supported((int)s.k, (int)s.l)))
        result = apply_skeleton(ctx, cs, s, plan->Y[(size_t)b], f.T, q.AJ, q.ldaj, f64);
      if (he == hipSuccess && result == SID_OK)
        he = sid::launch_copy_results(cs, q.J, f.piv, (int)s.k, q.k_eff, f.keff, q.err, f.err);
      if (he != hipSuccess) result = hip_fail(ctx, he, "batched: per-problem results");
    }
  }
  for (int64_t b = 0; !tail && b < count && result == SID_OK; ++b) {
    const sid_problem& q = probs[b];
    sid_ctx* c = ctx->children[(size_t)(b % nstreams)];
    if (persistent) {
      Work w;
      result = reserve(c, sh[(size_t)b], &w, false);
      if (result != SID_OK) {
        fail(ctx, result, "problem " + std::to_string(b) + ": workspace");
        break;
      }
      w.W = plan->W[(size_t)b];
      w.Y = plan->Y[(size_t)b];
      w.omega = plan->omega[(size_t)b];
      const BatchFactor& f = plan->fac[(size_t)b];
      if (f.pre) {
        w.piv = f.piv;
        w.R = f.R;
        w.Q = f.Q;
        w.keff = f.keff;
        w.stats = f.stats;
        if (sh[(size_t)b].single) {
          w.om64 = f.om64;
          w.M = f.M;
          w.Mpr = f.Mpr;
          w.pivM = f.pivM;
          w.RM = f.RM;
          w.QM = f.QM;
          w.rkM = f.rkM;
          w.statsM = f.statsM;
        }
      }
      result = factor(c, &q.params, sh[(size_t)b], w, dtype, q.A, q.lda, q.J, q.P, q.ldp, q.AJ,
                      q.ldaj, q.err, q.k_eff, f.pre);
    } else {
      // row sets are bound to the parent context; the child reads the same
      // device array
      sid_params pr = q.params;
      sid_rowset tmp;
      if (pr.coarse) {
        tmp = *pr.coarse;
        tmp.ctx = c;
        pr.coarse = &tmp;
      }
      result = sid_compress(c, q.A, dtype, q.N, q.n, q.lda, &pr, q.J, q.P, q.ldp, q.AJ, q.ldaj,
                            q.err, q.k_eff);
    }
    if (result != SID_OK) fail(ctx, result, "problem " + std::to_string(b) + ": " + c->err);
  }
  // join (also after a failure, so the context's stream never runs ahead)
  for (int c = 0; c < nstreams; ++c) {
    SID_CHECK(hipEventRecord(ctx->child_done[c], ctx->children[c]->stream), "batched: join event");
    SID_CHECK(hipStreamWaitEvent(ctx->stream, ctx->child_done[c], 0), "batched: join wait");
  }
  return result;
}

// autotuner cache key: architecture, sketch form, mode, batch size and the
// widest problem (chunks of 128 columns), bucketed
std::string tune_key(const sid_ctx* ctx, const sid_problem* probs, int64_t count,
                     const std::vector<Shape>& sh) {
  hipDeviceProp_t prop{};
  std::string arch = "unknown";
  if (hipGetDeviceProperties(&prop, ctx->device) == hipSuccess) arch = prop.gcnArchName;
  const size_t colon = arch.find(':');
  if (colon != std::string::npos) arch = arch.substr(0, colon);
  int64_t maxn = 0;
  for (const Shape& s : sh) maxn = s.n > maxn ? s.n : maxn;
  int cb = 0;
  while ((int64_t)1 << (cb + 1) <= count) ++cb;
  return arch + " prec=" + std::to_string(probs[0].params.prec) +
         " single=" + std::to_string(sh[0].single ? 1 : 0) + " count=2^" + std::to_string(cb) +
         " nch=" + std::to_string((maxn + 127) / 128);
}

// the cache file (SID_TUNE_CACHE): one "key<TAB>streams" line per entry
int tune_lookup(sid_ctx* ctx, const std::string& key) {
  for (const auto& kv : ctx->tuned)
    if (kv.first == key) return kv.second;
  const char* path = std::getenv("SID_TUNE_CACHE");
  if (!path || !path[0]) return 0;
  FILE* f = std::fopen(path, "r");
  if (!f) return 0;
  char line[512];
  int found = 0;
  while (std::fgets(line, sizeof line, f)) {
    std::string ln(line);
    const size_t tab = ln.find('\t');
    if (tab == std::string::npos) continue;
    if (ln.substr(0, tab) == key) found = std::atoi(ln.c_str() + tab + 1);
  }
  std::fclose(f);
  if (found >= 1 && found <= SID_BATCH_STREAMS_MAX) {
    ctx->tuned.emplace_back(key, found);
    return found;
  }
  return 0;
}
}  // namespace
}  // extern "C++"

sid_status sid_compress_batched(sid_ctx* ctx, const sid_problem* probs, int64_t count,
                                sid_dtype dtype) {
  if (!ctx) return SID_EINVAL;
  std::vector<Shape> sh;
  const sid_status vs = validate_batch(ctx, probs, count, dtype, &sh);
  if (vs != SID_OK) return vs;
  if (count == 0) return SID_OK;
  SID_NEED_DEVICE(ctx);
  SID_CHECK(hipSetDevice(ctx->device), "hipSetDevice");
  // A captured batched call (the persistent launch plus per-problem work on
  // the child streams, each with a side stream) ended the process inside the
  // runtime's end of capture, for eight problems as for 64, while single
  // sid_compress captures replay correctly; no mistake in this sequence has
  // been found, so batched calls are refused under capture.
  if (capturing(ctx->stream))
    return fail(ctx, SID_ESTATE, "sid_compress_batched cannot be captured in a HIP graph");
  return compress_batch(ctx, probs, count, dtype, sh, ctx->batch_streams);
}

sid_status sid_reserve_batched(sid_ctx* ctx, const sid_problem* probs, int64_t count,
                               sid_dtype dtype, int tune) {
  if (!ctx) return SID_EINVAL;
  std::vector<Shape> sh;
  const sid_status vs = validate_batch(ctx, probs, count, dtype, &sh);
  if (vs != SID_OK) return vs;
  if (count == 0) return SID_OK;
  SID_NEED_DEVICE(ctx);
  SID_CHECK(hipSetDevice(ctx->device), "hipSetDevice");
  if (capturing(ctx->stream)) return fail(ctx, SID_ESTATE, "sid_reserve_batched under graph capture");
  const bool persistent = batch_persistent_ok(ctx, probs, count, dtype, sh);
  if (persistent) {
    BatchPlan* plan = nullptr;
    const sid_status ps = batch_plan(ctx, probs, count, sh, &plan);
    if (ps != SID_OK) return ps;
  }
  sid_status st = ensure_children(ctx, SID_BATCH_STREAMS_MAX);
  if (st != SID_OK) return st;
  // every child may take any problem (the stream count can change)
  for (sid_ctx* c : ctx->children)
    for (int64_t b = 0; b < count; ++b) {
      const sid_problem& q = probs[b];
      if (persistent) {
        Work w;
        if (reserve(c, sh[(size_t)b], &w, false) != SID_OK) return fail(ctx, SID_ENOMEM, "batched: workspace");
        if (sh[(size_t)b].single && !c->side) {
          SID_CHECK(hipStreamCreate(&c->side), "side stream");
          SID_CHECK(hipEventCreateWithFlags(&c->side_fork, hipEventDisableTiming), "side event");
          SID_CHECK(hipEventCreateWithFlags(&c->side_join, hipEventDisableTiming), "side event");
        }
      } else {
        sid_params pr = q.params;
        sid_rowset tmp;
        if (pr.coarse) {
          tmp = *pr.coarse;
          tmp.ctx = c;
          pr.coarse = &tmp;
        }
        const sid_status rs = sid_reserve(c, q.N, q.n, &pr);
        if (rs != SID_OK) return fail(ctx, rs, "problem " + std::to_string(b) + ": " + c->err);
      }
    }
  // the autotuner: the number of child streams of the factorization phase,
  // per (architecture, sketch form, mode, batch size, width) bucket -- from
  // the context's cache, the cache file, or (tune != 0) timed here on the
  // batch itself (every candidate computes the same results)
  const std::string key = tune_key(ctx, probs, count, sh);
  int best = tune ? 0 : tune_lookup(ctx, key);
  if (tune) {
    hipEvent_t t0 = nullptr, t1 = nullptr;
    SID_CHECK(hipEventCreate(&t0), "autotune event");
    SID_CHECK(hipEventCreate(&t1), "autotune event");
    float best_ms = 0.0f;
    const int cands[] = {1, 2, 4, 8};
    sid_status rs = SID_OK;
    for (int rep = 0; rep < 2 && rs == SID_OK; ++rep)
      for (int cs : cands) {
        if (hipEventRecord(t0, ctx->stream) != hipSuccess) { rs = SID_EDEVICE; break; }
        rs = compress_batch(ctx, probs, count, dtype, sh, cs);
        if (rs != SID_OK) break;
        float ms = 0.0f;
        if (hipEventRecord(t1, ctx->stream) != hipSuccess || hipEventSynchronize(t1) != hipSuccess ||
            hipEventElapsedTime(&ms, t0, t1) != hipSuccess) {
          rs = SID_EDEVICE;
          break;
        }
        if (rep == 1 && (best == 0 || ms < best_ms)) {  // the first round warms up
          best = cs;
          best_ms = ms;
        }
      }
    (void)hipEventDestroy(t0);
    (void)hipEventDestroy(t1);
    if (rs != SID_OK) return rs == SID_EDEVICE ? fail(ctx, rs, "autotune timing failed") : rs;
    bool have = false;
    for (auto& kv : ctx->tuned)
      if (kv.first == key) { kv.second = best; have = true; }
    if (!have) ctx->tuned.emplace_back(key, best);
    const char* path = std::getenv("SID_TUNE_CACHE");
    if (path && path[0]) {
      FILE* f = std::fopen(path, "a");
      if (f) {
        std::fprintf(f, "%s\t%d\n", key.c_str(), best);
        std::fclose(f);
      }
    }
  }
  if (best >= 1) ctx->batch_streams = best;
  return SID_OK;
}

int sid_batch_streams(const sid_ctx* ctx) { return ctx ? ctx->batch_streams : -1; }

// ---------------------------------------------------------------------------
// Single-pass ID with interpolation (Alg. 6): the structured mesh, its
// coarse row set and the coarse-to-fine reconstruction.
// ---------------------------------------------------------------------------
struct sid_interp {
  sid_ctx* ctx = nullptr;
  sid::InterpDev dev{};
  void* d_tables = nullptr;
  sid_rowset* rs = nullptr;
  int64_t N = 0, Nc = 0;
};

namespace {

// One dimension of the operator: for every fine index the element of coarse
// nodes it lies in (the first element whose closed interval contains it; the
// end elements continued outside a bounded dimension, the element from the
// last node to the first one shifted by the period closing a periodic one)
// and the local coordinate in it, the weight of the element's second node.
bool build_dim(int64_t n, const double* coord, const int64_t* coarse, int64_t m, double period,
               int32_t* lo, int32_t* hi, double* w, std::string* why) {
  auto xc = [&](int64_t i) { return coord ? coord[i] : (double)i; };
  for (int64_t i = 1; i < n; ++i)
    if (!(xc(i) > xc(i - 1))) {
      *why = "coordinates must be strictly increasing";
      return false;
    }
  for (int64_t a = 0; a < m; ++a) {
    if (coarse[a] < 0 || coarse[a] >= n || (a > 0 && coarse[a] <= coarse[a - 1])) {
      *why = "coarse indices must be strictly increasing and within the dimension";
      return false;
    }
  }
  if (!(period >= 0.0) || !std::isfinite(period)) {
    *why = "period must be finite and >= 0";
    return false;
  }
  const double X0 = xc(coarse[0]), Xl = xc(coarse[m - 1]);
  if (period > 0.0 && !(Xl - X0 < period)) {
    *why = "the coarse nodes of a periodic dimension must span less than its period";
    return false;
  }
  for (int64_t i = 0; i < n; ++i) {
    if (m == 1) {
      lo[i] = hi[i] = 0;
      w[i] = 0.0;
      continue;
    }
    double x = xc(i);
    int64_t a = -1;
    double xa = 0.0, xb = 0.0;
    int64_t b = 0;
    if (period > 0.0) {
      x = X0 + std::fmod(x - X0, period);
      if (x < X0) x += period;
      for (int64_t e = 0; e < m && a < 0; ++e) {
        const double l = xc(coarse[e]);
        const double r = (e + 1 < m) ? xc(coarse[e + 1]) : X0 + period;
        if (l <= x && x <= r) {
          a = e;
          b = (e + 1 < m) ? e + 1 : 0;
          xa = l;
          xb = r;
        }
      }
      if (a < 0) {  // rounding at the top of the period: the closing element's end
        a = m - 1;
        b = 0;
        xa = Xl;
        xb = X0 + period;
        x = xb;
      }
    } else {
      if (x < X0) {
        a = 0;
      } else if (x > Xl) {
        a = m - 2;
      } else {
        for (int64_t e = 0; e + 1 < m && a < 0; ++e)
          if (xc(coarse[e]) <= x && x <= xc(coarse[e + 1])) a = e;
      }
      b = a + 1;
      xa = xc(coarse[a]);
      xb = xc(coarse[b]);
    }
    lo[i] = (int32_t)a;
    hi[i] = (int32_t)b;
    w[i] = (x - xa) / (xb - xa);
  }
  return true;
}

}  // namespace

sid_status sid_interp_create(sid_ctx* ctx, const sid_mesh* mesh, sid_interp** out) {
  if (!ctx) return SID_EINVAL;
  if (!mesh || !out) return fail(ctx, SID_EINVAL, "null argument");
  *out = nullptr;
  if (mesh->ncomp < 1 || mesh->reserved != 0)
    return fail(ctx, SID_EINVAL, "ncomp must be >= 1 and reserved 0");
  int64_t N = mesh->ncomp, Nc = mesh->ncomp, ntot = 0;
  for (int d = 0; d < 3; ++d) {
    if (mesh->n[d] < 1 || mesh->ncoarse[d] < 1 || mesh->ncoarse[d] > mesh->n[d] ||
        !mesh->coarse[d])
      return fail(ctx, SID_EINVAL, "every dimension needs n >= ncoarse >= 1 and a coarse list");
    if (mesh->n[d] > ((int64_t)1 << 31) || N > ((int64_t)1 << 31))
      return fail(ctx, SID_EINVAL, "the grid must have fewer than 2^31 points");
    N *= mesh->n[d];
    Nc *= mesh->ncoarse[d];
    ntot += mesh->n[d];
  }
  if (N >= ((int64_t)1 << 31)) return fail(ctx, SID_EINVAL, "the grid must have fewer than 2^31 points");
  std::vector<int32_t> lo((size_t)ntot), hi((size_t)ntot);
  std::vector<double> w64((size_t)ntot);
  int64_t off = 0;
  for (int d = 0; d < 3; ++d) {
    std::string why;
    if (!build_dim(mesh->n[d], mesh->coord[d], mesh->coarse[d], mesh->ncoarse[d],
                   mesh->period[d], lo.data() + off, hi.data() + off, w64.data() + off, &why))
      return fail(ctx, SID_EINVAL, "dimension " + std::to_string(d) + ": " + why);
    off += mesh->n[d];
  }
  std::vector<float> w32((size_t)ntot);
  for (int64_t i = 0; i < ntot; ++i) w32[(size_t)i] = (float)w64[(size_t)i];
  // coarse rows: the tensor product of the coarse lists, component-major
  std::vector<int64_t> rows((size_t)Nc);
  {
    const int64_t* cx = mesh->coarse[0];
    const int64_t* cy = mesh->coarse[1];
    const int64_t* cz = mesh->coarse[2];
    size_t e = 0;
    for (int64_t c = 0; c < mesh->ncomp; ++c)
      for (int64_t a = 0; a < mesh->ncoarse[0]; ++a)
        for (int64_t b = 0; b < mesh->ncoarse[1]; ++b)
          for (int64_t z = 0; z < mesh->ncoarse[2]; ++z)
            rows[e++] = ((c * mesh->n[0] + cx[a]) * mesh->n[1] + cy[b]) * mesh->n[2] + cz[z];
  }
  SID_NEED_DEVICE(ctx);
  sid_interp* ip = new (std::nothrow) sid_interp();
  if (!ip) return fail(ctx, SID_ENOMEM, "host allocation failed");
  sid_status st = sid_rowset_create(ctx, rows.data(), Nc, N, &ip->rs);
  if (st != SID_OK) {
    delete ip;
    return st;
  }
  const size_t bi = sizeof(int32_t) * (size_t)ntot, bf = sizeof(float) * (size_t)ntot,
               bd = sizeof(double) * (size_t)ntot;
  // layout: w64 | lo | hi | w32 (the doubles first keep every part aligned)
  std::vector<unsigned char> host(bd + 2 * bi + bf);
  std::memcpy(host.data(), w64.data(), bd);
  std::memcpy(host.data() + bd, lo.data(), bi);
  std::memcpy(host.data() + bd + bi, hi.data(), bi);
  std::memcpy(host.data() + bd + 2 * bi, w32.data(), bf);
  if (hipMalloc(&ip->d_tables, host.size()) != hipSuccess) {
    (void)hipGetLastError();
    sid_rowset_destroy(ip->rs);
    delete ip;
    return fail(ctx, SID_ENOMEM, "device allocation failed");
  }
  hipError_t e = hipMemcpy(ip->d_tables, host.data(), host.size(), hipMemcpyHostToDevice);
  if (e != hipSuccess) {
    (void)hipFree(ip->d_tables);
    sid_rowset_destroy(ip->rs);
    delete ip;
    return hip_fail(ctx, e, "interpolation table upload");
  }
  unsigned char* base = (unsigned char*)ip->d_tables;
  ip->ctx = ctx;
  ip->N = N;
  ip->Nc = Nc;
  sid::InterpDev& t = ip->dev;
  t.w64 = (const double*)base;
  t.lo = (const int32_t*)(base + bd);
  t.hi = (const int32_t*)(base + bd + bi);
  t.w32 = (const float*)(base + bd + 2 * bi);
  t.nx = (int32_t)mesh->n[0];
  t.ny = (int32_t)mesh->n[1];
  t.nz = (int32_t)mesh->n[2];
  t.mx = (int32_t)mesh->ncoarse[0];
  t.my = (int32_t)mesh->ncoarse[1];
  t.mz = (int32_t)mesh->ncoarse[2];
  t.ncomp = mesh->ncomp;
  t.N = N;
  t.Nc = Nc;
  *out = ip;
  return SID_OK;
}

sid_status sid_interp_destroy(sid_interp* ip) {
  if (!ip) return SID_EINVAL;
  if (ip->d_tables) {
    (void)hipSetDevice(ip->ctx->device);
    (void)hipStreamSynchronize(ip->ctx->stream);
    (void)hipFree(ip->d_tables);
  }
  if (ip->rs) (void)sid_rowset_destroy(ip->rs);
  delete ip;
  return SID_OK;
}

const sid_rowset* sid_interp_rowset(const sid_interp* ip) { return ip ? ip->rs : nullptr; }

sid_status sid_interp_info(const sid_interp* ip, int64_t* N, int64_t* Nc) {
  if (!ip) return SID_EINVAL;
  if (N) *N = ip->N;
  if (Nc) *Nc = ip->Nc;
  return SID_OK;
}

namespace {

sid_status interp_check(sid_ctx* ctx, const sid_interp* ip, const void* ACJ, int64_t ldacj,
                        const void* P, int64_t ldp, sid_dtype dtype, int64_t k, int64_t n) {
  if (!ip) return fail(ctx, SID_EINVAL, "interp is NULL");
  if (ip->ctx != ctx) return fail(ctx, SID_EINVAL, "interp belongs to another context");
  if (!ACJ || !P) return fail(ctx, SID_EINVAL, "null pointer");
  if (dtype != SID_F32 && dtype != SID_F64) return fail(ctx, SID_EINVAL, "unknown dtype");
  if (k < 1 || n < 1) return fail(ctx, SID_EINVAL, "k and n must be positive");
  if (k > 256) return fail(ctx, SID_EINVAL, "k must be <= 256");
  if (ldacj < ip->Nc || ldp < k) return fail(ctx, SID_EINVAL, "leading dimension too small");
  return SID_OK;
}

// FP32 with k <= 128 takes the matrix-core path: pack ACJ row-major and P
// as bfloat16 hi/lo operands.  Returns kp (0: FMA path).
sid_status interp_prepare(sid_ctx* ctx, const sid_interp* ip, const void* ACJ, int64_t ldacj,
                          const void* P, int64_t ldp, sid_dtype dtype, int64_t k, int64_t n,
                          int* kp_out, float** acjt, void** pb) {
  *kp_out = 0;
  if (dtype != SID_F32 || k > 128) return SID_OK;
  const int kp = (int)((k + 15) / 16 * 16);
  *acjt = (float*)ws(ctx, WS_IACJT, sizeof(float) * (size_t)ip->Nc * (size_t)kp);
  *pb = ws(ctx, WS_IPB, sid::interp_pb_bytes(n, kp));
  if (!*acjt || !*pb) return SID_ENOMEM;
  SID_CHECK(sid::launch_interp_pack(ctx->stream, (const float*)ACJ, ldacj, ip->Nc, (int)k, kp,
                                    *acjt, (const float*)P, ldp, n, *pb),
            "interpolation operands");
  *kp_out = kp;
  return SID_OK;
}

}  // namespace

sid_status sid_interp_reconstruct(sid_ctx* ctx, const sid_interp* ip, const void* ACJ,
                                  int64_t ldacj, const void* P, int64_t ldp, sid_dtype dtype,
                                  int64_t k, int64_t n, void* Ahat, int64_t ldo) {
  if (!ctx) return SID_EINVAL;
  sid_status s = interp_check(ctx, ip, ACJ, ldacj, P, ldp, dtype, k, n);
  if (s != SID_OK) return s;
  if (!Ahat) return fail(ctx, SID_EINVAL, "Ahat is NULL");
  if (ldo < ip->N) return fail(ctx, SID_EINVAL, "ldo < N");
  SID_NEED_DEVICE(ctx);
  SID_CHECK(hipSetDevice(ctx->device), "hipSetDevice");
  int kp = 0;
  float* acjt = nullptr;
  void* pb = nullptr;
  s = interp_prepare(ctx, ip, ACJ, ldacj, P, ldp, dtype, k, n, &kp, &acjt, &pb);
  if (s != SID_OK) return s;
  if (kp) {
    SID_CHECK(sid::launch_interp_mfma(ctx->stream, ip->dev, kp, acjt, pb, n, (float*)Ahat, ldo,
                                      nullptr, 0, nullptr, 0, nullptr),
              "interpolated reconstruction");
    return SID_OK;
  }
  const size_t es = dtype == SID_F64 ? sizeof(double) : sizeof(float);
  void* B = ws(ctx, WS_IB, es * (size_t)ip->N * (size_t)k);
  if (!B) return SID_ENOMEM;
  SID_CHECK(sid::launch_interp_apply(ctx->stream, ip->dev, dtype == SID_F64, ACJ, ldacj, (int)k, B,
                                     ip->N),
            "Mf ACJ");
  SID_CHECK(sid::launch_reconstruct(ctx->stream, dtype == SID_F64, B, ip->N, P, ldp, ip->N,
                                    (int)k, n, Ahat, ldo),
            "reconstruct");
  return SID_OK;
}

sid_status sid_interp_error_norms(sid_ctx* ctx, const sid_interp* ip, const void* A,
                                  int64_t lda, const void* ACJ, int64_t ldacj, const void* P,
                                  int64_t ldp, sid_dtype dtype, int64_t k, int64_t n,
                                  double* out4) {
  if (!ctx) return SID_EINVAL;
  sid_status s = interp_check(ctx, ip, ACJ, ldacj, P, ldp, dtype, k, n);
  if (s != SID_OK) return s;
  if (!A || !out4) return fail(ctx, SID_EINVAL, "null pointer");
  if (lda < ip->N) return fail(ctx, SID_EINVAL, "lda < N");
  SID_NEED_DEVICE(ctx);
  SID_CHECK(hipSetDevice(ctx->device), "hipSetDevice");
  double* dout = (double*)ws(ctx, WS_NORMOUT, sizeof(double) * 4);
  if (!dout) return SID_ENOMEM;
  int kp = 0;
  float* acjt = nullptr;
  void* pb = nullptr;
  s = interp_prepare(ctx, ip, ACJ, ldacj, P, ldp, dtype, k, n, &kp, &acjt, &pb);
  if (s != SID_OK) return s;
  if (kp) {
    const int64_t nb = sid::interp_mfma_blocks(ip->N);
    double* part = (double*)ws(ctx, WS_IPART, sizeof(double) * 4 * (size_t)nb);
    if (!part) return SID_ENOMEM;
    SID_CHECK(sid::launch_interp_mfma(ctx->stream, ip->dev, kp, acjt, pb, n, nullptr, 0,
                                      (const float*)A, lda, part, nb, dout),
              "interpolated error norms");
  } else {
    const size_t es = dtype == SID_F64 ? sizeof(double) : sizeof(float);
    void* B = ws(ctx, WS_IB, es * (size_t)ip->N * (size_t)k);
    const int64_t nb = ((ip->N + 63) / 64) * ((n + 31) / 32);
    double* part = (double*)ws(ctx, WS_NORMPART, sizeof(double) * 4 * (size_t)nb);
    if (!B || !part) return SID_ENOMEM;
    SID_CHECK(sid::launch_interp_apply(ctx->stream, ip->dev, dtype == SID_F64, ACJ, ldacj, (int)k,
                                       B, ip->N),
              "Mf ACJ");
    SID_CHECK(sid::launch_error_norms(ctx->stream, dtype == SID_F64, A, lda, B, ip->N, P, ldp,
                                      ip->N, (int)k, n, part, nb, dout),
              "error norms");
  }
  SID_CHECK(hipMemcpyAsync(out4, dout, 4 * sizeof(double), hipMemcpyDeviceToHost, ctx->stream),
            "copy norms");
  SID_CHECK(hipStreamSynchronize(ctx->stream), "synchronize");
  return SID_OK;
}


// ---------------------------------------------------------------------------
// SBR-SVD (Alg. 2)
// ---------------------------------------------------------------------------
void sid_svd_params_init(sid_svd_params* p, int64_t k) {
  if (!p) return;
  std::memset(p, 0, sizeof(*p));
  p->k = k;
  p->oversample = 10;
  p->block = 10;
  p->seed = 0;
  p->prec = SID_SK_F64;
}

}  // extern "C"

namespace {

// Parameters of SBR-SVD on an N x n matrix (n: snapshots; for a stream, its
// n_max), and the ID parameters of the pass forming G (l selection rows).
sid_status svd_check(sid_ctx* ctx, const sid_svd_params* sp, int64_t N, int64_t n,
                     sid_params* gp) {
  const int64_t k = sp->k, b = sp->block, l = sp->k + sp->oversample;
  if (k < 1 || sp->oversample < 0 || b < 1 || b > 64)
    return fail(ctx, SID_EINVAL, "need k >= 1, oversample >= 0, 1 <= block <= 64");
  if (l % b != 0) return fail(ctx, SID_EINVAL, "k + oversample must be a multiple of block");
  if (l > 256 || l > n || l > N)
    return fail(ctx, SID_EINVAL, "k + oversample must be <= min(n, N, 256)");
  if (sp->prec < SID_SK_F64 || sp->prec > SID_SK_FP8E4M3)
    return fail(ctx, SID_EINVAL, "unknown sketch precision");
  sid_params_init(gp, l);
  gp->oversample = 0;
  gp->seed = sp->seed;
  gp->mode = SID_TWO_PASS;
  gp->prec = sp->prec;
  gp->probe_rows = 0;
  Shape sh;
  return validate(ctx, N, n, gp, &sh);
}

// H (ld N) = A W^T, or H += A W^T (accumulate), for the ncols columns of A
// (ld lda) and of W (l x ncols, ld l); W is copied with its leading dimension
// rounded up to 16 into wp (that many times ncols doubles).
sid_status svd_h_update(sid_ctx* ctx, const void* A, sid_dtype dtype, int64_t lda, int64_t N,
                        int64_t ncols, const double* W, int64_t l, double* wp, double* H,
                        bool accumulate) {
  hipStream_t hs = ctx->stream;
  const int64_t lp = (l + 15) / 16 * 16;
  SID_CHECK(sid::launch_convert(hs, W, true, l, ncols, l, wp, true, lp), "W padded");
  SID_CHECK(sid::launch_h_gemm(hs, A, dtype == SID_F64, lda, N, (int)ncols, wp, lp, (int)l, H, N,
                               accumulate),
            "H = A W^T");
  return SID_OK;
}

// The block loop and the SVD of B (Alg. 2 after the pass) from W = Psi A
// (l x n, ld l: G = W^T) and H = A G (N x l, ld N; overwritten).
sid_status svd_blocks(sid_ctx* ctx, const sid_svd_params* sp, sid_dtype dtype, int64_t N,
                      int64_t n, const double* W, double* H, double* S, void* U, int64_t ldu,
                      void* V, int64_t ldv, int64_t* rank) {
  const int64_t k = sp->k, b = sp->block, l = sp->k + sp->oversample;
  hipStream_t hs = ctx->stream;
  const size_t d = sizeof(double);
  double* Bt = (double*)ws(ctx, WS_SV_B, d * (size_t)N * (size_t)l);
  double* Q = (double*)ws(ctx, WS_SV_Q, d * (size_t)n * (size_t)l);
  float* om32 = (float*)ws(ctx, WS_SV_OM32, sizeof(float) * (size_t)N * (size_t)b);
  double* om = (double*)ws(ctx, WS_SV_OM, d * (size_t)N * (size_t)b);
  // partials of the tall-skinny products (blocks of at most 128 x 128)
  int64_t rpb = 0;
  const int64_t nbt = sid::tsmm_blocks(N, ctx->num_cu, &rpb);
  // (at least 2 x 128 x 128: it also holds (U~ S^-1)^T, up to 256 x 128)
  double* tsp = (double*)ws(ctx, WS_SV_TSP, d * (size_t)(nbt < 2 ? 2 : nbt) * 128 * 128);
  // small buffers: Y0, Y (n x b), C, Z (l x b), R, Rt (b x b), Gram, Vj (l x l),
  // Us, Uv (l x k), mindiag (+ Jacobi's sweep count), Uout (n x k), Jacobi
  // work (l' x l', l' = l rounded up to even) and rotation records
  const size_t le = (size_t)(l + (l & 1));
  const size_t nsmall = 2 * (size_t)(n * b) + 2 * (size_t)(l * b) + 2 * (size_t)(b * b) +
                        2 * (size_t)(l * l) + 2 * (size_t)(l * k) + 4 + (size_t)(n * k) + le * le +
                        sid::jacobi_rot_doubles((int)l) + 2;
  double* sm = (double*)ws(ctx, WS_SV_SMALL, d * nsmall);
  if (!Bt || !Q || !om32 || !om || !tsp || !sm) return SID_ENOMEM;
  double* Y0 = sm;
  double* Y = Y0 + n * b;
  double* C = Y + n * b;
  double* Z = C + l * b;
  double* R = Z + l * b;
  double* Rt = R + b * b;
  double* Gm = Rt + b * b;
  double* Vj = Gm + l * l;
  double* Us = Vj + l * l;
  double* Uv = Us + l * k;
  double* mind = Uv + l * k;
  double* Uo = mind + 4;
  double* Jw = Uo + n * k;  // Jacobi's working matrix when l > 128
  double* Jrot = Jw + le * le;  // Jacobi's rotation records
  // the stop test's state on the device: basis columns so far, stopped flag
  int64_t* jstate = (int64_t*)(Jrot + sid::jacobi_rot_doubles((int)l));
  // X^T Y over the N rows in blocks of at most 128 x 128 (the product
  // kernel's limit); C gets alpha X^T Y + beta C
  auto tsmm = [&](const double* X, int p, const double* Y, int64_t ysr, int64_t ysc, int q,
                  double alpha, double beta, double* C, int64_t ldc) -> hipError_t {
    for (int a0 = 0; a0 < p; a0 += 128)
      for (int c0 = 0; c0 < q; c0 += 128) {
        const hipError_t e = sid::launch_tsmm(hs, X + (int64_t)N * a0, N, Y + ysc * c0, ysr, ysc, N,
                                              p - a0 < 128 ? p - a0 : 128,
                                              q - c0 < 128 ? q - c0 : 128, alpha, beta,
                                              C + a0 + ldc * c0, ldc, tsp, ctx->num_cu);
        if (e != hipSuccess) return e;
      }
    return hipSuccess;
  };
  // ||G||_F^2 for the stop test
  SID_CHECK(sid::launch_sumsq(hs, W, l * n, mind + 3), "||G||^2");
  // (2) the blocks.  The stop test runs on the device (in k_trmul), so the
  // blocks are queued without waiting for it: after a rank-deficient block
  // the remaining blocks only write basis columns past the stop, which the
  // steps after the loop never read; one read of the column count follows
  // the loop.  j counts the columns the queued blocks assume.
  int64_t j = 0;
  const int64_t s = l / b;
  for (int64_t i = 0; i < s; ++i) {
    // Omega_i = Psi(i b .. i b + b, :)^T, rounded as the sketch read it,
    // stored b x N (ld b): row r of Omega_i is b contiguous values
    SID_CHECK(sid::launch_fill_gaussian(hs, sp->seed, 1u, 0, N, i * b, b, om32), "Omega_i");
    SID_CHECK(sid::launch_omega_values(hs, sp->prec, om32, N * b, om), "Omega_i values");
    // Y_i = G_i - Q (B Omega_i), G_i = W(i b .. i b + b, :)^T
    SID_CHECK(sid::launch_transpose64(hs, W + i * b, b, n, l, Y0, n), "G_i");
    if (j > 0) {
      SID_CHECK(tsmm(Bt, (int)j, om, b, 1, (int)b, 1.0, 0.0, C, l), "B Omega_i");
      SID_CHECK(sid::launch_gemm64_ab(hs, (int)n, (int)b, (int)j, Q, n, 0, C, l, 0, -1.0, 1.0, Y0,
                                      n),
                "G_i - Q B Omega_i");
    }
    // (Q_i, R_i) = qr(Y_i), then against Q once more: (Q_i, R~_i)
    SID_CHECK(hipMemcpyAsync(Y, Y0, d * (size_t)(n * b), hipMemcpyDeviceToDevice, hs), "copy Y");
    SID_CHECK(sid::launch_small_qr(hs, Y, (int)n, (int)b, R), "qr(Y_i)");
    if (j > 0) {
      SID_CHECK(sid::launch_gemm64_ab(hs, (int)j, (int)b, (int)n, Q, n, 1, Y, n, 0, 1.0, 0.0, Z, l),
                "Q^T Q_i");
      SID_CHECK(sid::launch_gemm64_ab(hs, (int)n, (int)b, (int)j, Q, n, 0, Z, l, 0, -1.0, 1.0, Y, n),
                "Q_i - Q Q^T Q_i");
    }
    SID_CHECK(sid::launch_small_qr(hs, Y, (int)n, (int)b, Rt), "qr again");
    SID_CHECK(sid::launch_trmul(hs, Rt, R, (int)b, mind, mind + 3, i, jstate),
              "R_i = R~_i R_i and the stop test");
    // B_i^T = (H_i - B^T (Q^T Y_i + B Omega_i)) R_i^-1 into the next b columns
    // of B^T, one pass over the rows
    double* Bi = Bt + j * N;
    if (j > 0)
      SID_CHECK(sid::launch_gemm64_ab(hs, (int)j, (int)b, (int)n, Q, n, 1, Y0, n, 0, 1.0, 1.0, C, l),
                "Q^T Y_i + B Omega_i");
    SID_CHECK(sid::launch_block_update(hs, Bt, N, (int)j, H + i * b * N, C, l, R, (int)b, Bi),
              "B_i^T = (H_i - B^T M_i) R_i^-1");
    SID_CHECK(hipMemcpyAsync(Q + j * n, Y, d * (size_t)(n * b), hipMemcpyDeviceToDevice, hs),
              "Q_i");
    j += b;
  }
  {
    int64_t jd = 0;
    SID_CHECK(hipMemcpyAsync(&jd, jstate, sizeof(int64_t), hipMemcpyDeviceToHost, hs),
              "basis column count");
    SID_CHECK(hipStreamSynchronize(hs), "synchronize");
    j = jd;
  }
  if (rank) *rank = j;
  if (j == 0) {
    SID_CHECK(hipMemsetAsync(S, 0, d * (size_t)k, hs), "S");
    const size_t es = dtype == SID_F64 ? d : sizeof(float);
    SID_CHECK(hipMemset2DAsync(U, es * (size_t)ldu, 0, es * (size_t)n, (size_t)k, hs), "U");
    SID_CHECK(hipMemset2DAsync(V, es * (size_t)ldv, 0, es * (size_t)N, (size_t)k, hs), "V");
    SID_CHECK(hipStreamSynchronize(hs), "synchronize");
    return SID_OK;
  }
  // (3) B = U~ S V^T from B B^T = U~ S^2 U~^T (Jacobi); V_k = B^T U~_k S_k^-1,
  // U_k = Q U~_k
  SID_CHECK(tsmm(Bt, (int)j, Bt, 1, N, (int)j, 1.0, 0.0, Gm, j), "B B^T");
  SID_CHECK(sid::launch_jacobi(hs, Gm, (int)j, Vj, Jw, Jrot, (int*)(mind + 2)),
            "eigen-decomposition of B B^T");
  SID_CHECK(sid::launch_eig_sort(hs, Gm, (int)j, Vj, (int)k, S, Us, Uv), "sort");
  // (columns of Us, Uv past j are zero); V in the output type, in slabs of
  // at most 128 columns
  for (int64_t c0 = 0; c0 < k; c0 += 128) {
    const int kc = (int)(k - c0 < 128 ? k - c0 : 128);
    const size_t es = dtype == SID_F64 ? d : sizeof(float);
    // this slab of U~ S^-1 row by row (stride 128) in the products' scratch
    SID_CHECK(sid::launch_transpose64(hs, Us + j * c0, j, kc, j, tsp, 128), "(U~ S^-1)^T");
    SID_CHECK(sid::launch_tall_mul(hs, Bt, N, N, (int)j, tsp, 128, kc,
                                   (unsigned char*)V + es * (size_t)(ldv * c0), dtype == SID_F64,
                                   ldv),
              "V = B^T U~ S^-1");
  }
  SID_CHECK(sid::launch_gemm64_ab(hs, (int)n, (int)k, (int)j, Q, n, 0, Uv, j, 0, 1.0, 0.0, Uo, n),
            "U = Q U~");
  SID_CHECK(sid::launch_convert(hs, Uo, true, n, k, n, U, dtype == SID_F64, ldu), "U out");
  SID_CHECK(hipStreamSynchronize(hs), "synchronize");
  return SID_OK;
}


}  // namespace

extern "C" {

sid_status sid_sbr_svd(sid_ctx* ctx, const void* A, sid_dtype dtype, int64_t N, int64_t n,
                       int64_t lda, const sid_svd_params* sp, double* S, void* U, int64_t ldu,
                       void* V, int64_t ldv, int64_t* rank) {
  if (!ctx) return SID_EINVAL;
  if (!sp || !A || !S || !U || !V) return fail(ctx, SID_EINVAL, "null argument");
  if (dtype != SID_F32 && dtype != SID_F64) return fail(ctx, SID_EINVAL, "unknown dtype");
  sid_params gp;
  sid_status st = svd_check(ctx, sp, N, n, &gp);
  if (st != SID_OK) return st;
  if (lda < N || ldu < n || ldv < N) return fail(ctx, SID_EINVAL, "leading dimension too small");
  const int64_t l = sp->k + sp->oversample;
  Shape sh;
  st = validate(ctx, N, n, &gp, &sh);
  if (st != SID_OK) return st;
  SID_NEED_DEVICE(ctx);
  SID_CHECK(hipSetDevice(ctx->device), "hipSetDevice");
  Work w;
  if (reserve(ctx, sh, &w) != SID_OK) return SID_ENOMEM;
  const size_t d = sizeof(double);
  double* H = (double*)ws(ctx, WS_SV_H, d * (size_t)N * (size_t)l);
  double* wp = (double*)ws(ctx, WS_SV_WP, d * (size_t)((l + 15) / 16 * 16) * (size_t)n);
  if (!H || !wp) return SID_ENOMEM;
  // (1) the pass over A: G = W^T from the ID's sketch with l selection rows
  // (W = Psi A, l x n, ld l), then H = A G in FP64 (FP32 data promoted exactly)
  st = run_sketch(ctx, A, dtype, lda, &gp, sh, w, w.W, nullptr);
  if (st != SID_OK) return st;
  st = svd_h_update(ctx, A, dtype, lda, N, n, w.W, l, wp, H, false);
  if (st != SID_OK) return st;
  // (2) the blocks and the SVD of B
  return svd_blocks(ctx, sp, dtype, N, n, w.W, H, S, U, ldu, V, ldv, rank);
}

sid_status sid_svd_stream_begin(sid_ctx* ctx, sid_dtype dtype, int64_t N, int64_t n_max,
                                const sid_svd_params* sp, sid_stream** out) {
  if (!ctx) return SID_EINVAL;
  if (!out) return fail(ctx, SID_EINVAL, "out is NULL");
  *out = nullptr;
  if (!sp) return fail(ctx, SID_EINVAL, "null argument");
  if (dtype != SID_F32 && dtype != SID_F64) return fail(ctx, SID_EINVAL, "unknown dtype");
  sid_params gp;
  sid_status st = svd_check(ctx, sp, N, n_max, &gp);
  if (st != SID_OK) return st;
  SID_NEED_DEVICE(ctx);
  SID_CHECK(hipSetDevice(ctx->device), "hipSetDevice");
  sid_stream* s = nullptr;
  st = stream_make(ctx, dtype, N, n_max, &gp, &s);
  if (st != SID_OK) return st;
  const int64_t l = sp->k + sp->oversample;
  if (s->lq != l) {
    stream_free(s);
    return fail(ctx, SID_EINVAL, "internal: G's sketch rows differ from k + oversample");
  }
  s->svd = true;
  s->sp = *sp;
  const size_t d = sizeof(double);
  const int64_t lp = (l + 15) / 16 * 16;
  if (hipMalloc((void**)&s->H, d * (size_t)N * (size_t)l) != hipSuccess ||
      hipMalloc((void**)&s->Wp, d * (size_t)lp * (size_t)s->stage_cols) != hipSuccess) {
    (void)hipGetLastError();
    stream_free(s);
    return fail(ctx, SID_ENOMEM, "stream: device allocation of H failed");
  }
  *out = s;
  return SID_OK;
}

sid_status sid_svd_stream_finish(sid_stream* s, double* S, void* U, int64_t ldu, void* V,
                                 int64_t ldv, int64_t* rank) {
  if (!s) return SID_EINVAL;
  sid_ctx* ctx = s->ctx;
  if (!s->svd) return fail(ctx, SID_EINVAL, "not an SBR-SVD stream (sid_stream_finish ends it)");
  sid_status st = SID_OK;
  do {
    if (!S || !U || !V) {
      st = fail(ctx, SID_EINVAL, "null argument");
      break;
    }
    if (hipSetDevice(ctx->device) != hipSuccess) {
      st = fail(ctx, SID_EDEVICE, "hipSetDevice");
      break;
    }
    st = stream_flush_stage(s);
    if (st != SID_OK) break;
    const int64_t n = s->cols;
    sid_params gp;
    st = svd_check(ctx, &s->sp, s->N, n, &gp);
    if (st != SID_OK) break;
    if (ldu < n || ldv < s->N) {
      st = fail(ctx, SID_EINVAL, "leading dimension too small");
      break;
    }
    st = svd_blocks(ctx, &s->sp, s->dtype, s->N, n, s->W, s->H, S, U, ldu, V, ldv, rank);
  } while (false);
  stream_free(s);
  return st;
}

}  // extern "C"
