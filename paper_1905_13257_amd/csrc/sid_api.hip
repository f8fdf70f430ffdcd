// sid_api.hip -- host runtime behind include/sid.h: argument validation,
// grow-only device workspace, and the launch sequence of a compression on
// the context's stream.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/sid.h"
#include "sid_kernels.hpp"

namespace {

enum Slot {
  WS_OMEGA, WS_PART, WS_W, WS_WR, WS_NRM, WS_PIV, WS_R, WS_Q, WS_KEFF, WS_STATS, WS_PD,
  WS_ERR, WS_Y, WS_M, WS_MPR, WS_WJ, WS_PIVM, WS_RM, WS_QM, WS_RKM, WS_C, WS_T, WS_MIX,
  WS_STATSM, WS_NORMPART, WS_NORMOUT, WS_OM64, WS_PARTF, WS_OMT, WS_COOP, WS_SYNC, WS_R11, WS_FITPART, WS_COUNT
};

struct Buf {
  void* p = nullptr;
  size_t bytes = 0;
};

}  // namespace

struct sid_ctx {
  int device = 0;
  int num_cu = 1;
  bool cooperative = false;  // SID_COOPERATIVE=1: cooperative launch of the pivoted QR
  hipStream_t stream = nullptr;
  bool own_stream = false;
  std::string err;
  Buf ws[WS_COUNT];
  size_t limit = 0;
};

struct sid_rowset {
  sid_ctx* ctx = nullptr;
  int64_t* d_rows = nullptr;
  int64_t count = 0;
  int64_t N = 0;
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

double default_rcond(int prec) {
  switch (prec) {
    case SID_SK_F64: return 1e-13;
    case SID_SK_F32: return 1e-6;
    case SID_SK_BF16X2: return 1e-5;
    case SID_SK_FP8E4M3: return 1e-2;
    default: return 1e-3;
  }
}

sid_status validate(sid_ctx* ctx, int64_t N, int64_t n, const sid_params* p, Shape* sh) {
  if (!p) return fail(ctx, SID_EINVAL, "params is NULL");
  if (N <= 0 || n <= 0) return fail(ctx, SID_EINVAL, "N and n must be positive");
  if (p->k < 1) return fail(ctx, SID_EINVAL, "k must be >= 1");
  if (p->oversample < 0) return fail(ctx, SID_EINVAL, "oversample must be >= 0");
  if (p->probe_rows < 0) return fail(ctx, SID_EINVAL, "probe_rows must be >= 0");
  if (p->k > n) return fail(ctx, SID_EINVAL, "k must not exceed the number of columns n");
  if (p->mode != SID_TWO_PASS && p->mode != SID_SINGLE_PASS)
    return fail(ctx, SID_EINVAL, "unknown mode");
  if (p->prec < SID_SK_F64 || p->prec > SID_SK_FP8E4M3)
    return fail(ctx, SID_EINVAL, "unknown sketch precision");
  if (!(p->rank_tol >= 0.0) || !(p->sp_rcond >= 0.0))
    return fail(ctx, SID_EINVAL, "rank_tol and sp_rcond must be >= 0");
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
  const int64_t ntiles = (n + 63) / 64;
  int64_t nch = (Ns + 1023) / 1024;
  int64_t cap = 2048 / ntiles;
  if (cap < 1) cap = 1;
  if (nch > cap) nch = cap;
  if (nch < 1) nch = 1;
  sh->nchunks = nch;
  sh->single = p->mode == SID_SINGLE_PASS;
  sh->prec = p->prec;
  return SID_OK;
}

struct Work {
  float* omega;
  double *part, *W, *Wr, *nrm, *R, *Q, *stats, *Pd, *err;
  int64_t *piv, *keff;
  void* Y;
  double *M, *Mpr, *WJ, *RM, *QM, *C, *T, *mix, *statsM, *om64;
  int64_t *pivM, *rkM;
  void* coop;
  unsigned int* sync2;
  double* R11;
  double* fitpart;
};

sid_status reserve(sid_ctx* c, const Shape& s, Work* w) {
  const size_t d = sizeof(double);
  const int64_t mx = s.n > s.lz ? s.n : s.lz;
  w->omega = (float*)ws(c, WS_OMEGA, sizeof(float) * (size_t)(s.n * s.l));
  w->part = (double*)ws(c, WS_PART, d * (size_t)(s.nchunks * s.lq * s.n));
  w->W = (double*)ws(c, WS_W, d * (size_t)(s.lq * s.n));
  w->Wr = (double*)ws(c, WS_WR, d * (size_t)(s.lz * s.l > s.l * s.n ? s.lz * s.l : s.l * s.n));
  w->nrm = (double*)ws(c, WS_NRM, d * (size_t)mx);
  w->piv = (int64_t*)ws(c, WS_PIV, sizeof(int64_t) * (size_t)s.k);
  w->R = (double*)ws(c, WS_R, d * (size_t)(s.k * s.n));
  w->Q = (double*)ws(c, WS_Q, d * (size_t)(s.l * s.k));
  w->keff = (int64_t*)ws(c, WS_KEFF, sizeof(int64_t));
  w->stats = (double*)ws(c, WS_STATS, d * 2);
  w->Pd = (double*)ws(c, WS_PD, d * (size_t)(s.k * s.n));
  w->err = (double*)ws(c, WS_ERR, d * 2);
  w->fitpart = (double*)ws(c, WS_FITPART, d * (size_t)(2 * ((s.q * s.n + 255) / 256) + 2));
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
  w->Y = nullptr;
  if (s.single) {
    const size_t ye = (s.prec == SID_SK_F64) ? d : sizeof(float);
    w->Y = ws(c, WS_Y, ye * (size_t)(s.N * s.l));
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
    if (!w->om64 || !w->Y || !w->M || !w->Mpr || !w->WJ || !w->RM || !w->QM || !w->C || !w->T || !w->mix ||
        !w->statsM || !w->pivM || !w->rkM)
      return SID_ENOMEM;
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
  }
  int ncu = 0;
  if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, device) == hipSuccess &&
      ncu > 0)
    c->num_cu = ncu;
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
  for (Buf& b : ctx->ws)
    if (b.p) (void)hipFree(b.p);
  if (ctx->own_stream) (void)hipStreamDestroy(ctx->stream);
  delete ctx;
  return SID_OK;
}

const char* sid_last_error(const sid_ctx* ctx) {
  if (!ctx) return "null context";
  return ctx->err.c_str();
}

size_t sid_workspace_bytes(const sid_ctx* ctx) { return ctx ? held_bytes(ctx) : 0; }

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
  return reserve(ctx, sh, &w);
}

static sid_status run_sketch(sid_ctx* ctx, const void* A, sid_dtype dtype, int64_t lda,
                             const sid_params* p, const Shape& sh, const Work& w, double* W,
                             void* Y) {
  hipStream_t st = ctx->stream;
  if (Y) {
    SID_CHECK(sid::launch_fill_gaussian(st, p->seed, 0u, 0, sh.n, 0, sh.l, w.omega),
              "omega generation");
  }
  const int64_t* rows = p->coarse ? p->coarse->d_rows : nullptr;
  const bool bf = sh.prec == SID_SK_BF16 || sh.prec == SID_SK_BF16X2 ||
                  sh.prec == SID_SK_FP8E4M3;
  const bool fused_ok =
      dtype == SID_F32 &&
      sid::fused_bf16_supported(sh.n, (int)sh.lq, (int)sh.l, lda, A, rows != nullptr);
  if (sh.prec == SID_SK_FP8E4M3 && !fused_ok)
    return fail(ctx, SID_EINVAL,
                "the FP8 sketch needs FP32 data with 16-byte aligned columns (lda % 4 == 0), all "
                "rows (no coarse set), n <= 512, l <= 128 and l + co-range + probe <= 160");
  if (bf && fused_ok) {
    // one streaming pass on the matrix cores (W partials per workgroup, FP32)
    int64_t rpw = 0;
    const int64_t grid = sid::fused_bf16_grid(sh.N, ctx->num_cu, &rpw);
    float* partf = (float*)ws(ctx, WS_PARTF, sizeof(float) * (size_t)(grid * sh.lq * sh.n));
    __bf16* omT = (__bf16*)ws(ctx, WS_OMT, sizeof(uint16_t) * 128 * 512);
    if (!partf || !omT) return SID_ENOMEM;
    int64_t nparts = 0;
    const int dmode = sh.prec == SID_SK_BF16X2   ? sid::FB_BF16X2
                      : sh.prec == SID_SK_FP8E4M3 ? sid::FB_FP8
                                                  : sid::FB_BF16;
    SID_CHECK(sid::launch_sketch_fused_bf16(st, dmode, (const float*)A, lda,
                                            sh.N, (int)sh.n, (int)sh.lq, (int)sh.l, p->seed,
                                            w.omega, omT, ctx->num_cu, partf, W, (float*)Y,
                                            &nparts),
              "fused sketch pass");
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
  if (AJ && ldaj < N) return fail(ctx, SID_EINVAL, "ldaj < N");
  SID_NEED_DEVICE(ctx);
  SID_CHECK(hipSetDevice(ctx->device), "hipSetDevice");
  Work w;
  if (reserve(ctx, sh, &w) != SID_OK) return SID_ENOMEM;
  hipStream_t st = ctx->stream;
  const bool f64 = dtype == SID_F64;
  const int k = (int)sh.k, l = (int)sh.l, q = (int)sh.q, lz = (int)sh.lz, lq = (int)sh.lq,
            n_ = (int)sh.n;

  // (1) sketch pass: W = Psi(:, S) A(S, :) and, single pass, Y = A Omega
  s = run_sketch(ctx, A, dtype, lda, p, sh, w, w.W, sh.single ? w.Y : nullptr);
  if (s != SID_OK) return s;
  // (2) mgsqr on the selection rows of W
  if (sid::cpqr_wg_supported(l, n_))
    SID_CHECK(sid::launch_cpqr_wg(st, w.W, lq, l, n_, k, p->rank_tol, w.piv, w.R, w.Q, w.keff,
                                  w.stats),
              "pivoted QR");
  else if (sid::cpqr_coop_supported(l, n_))
    SID_CHECK(sid::launch_cpqr_coop(st, w.W, lq, l, n_, k, p->rank_tol, w.coop, w.sync2, w.piv,
                                    w.R, w.Q, w.keff, w.stats, ctx->cooperative),
              "pivoted QR");
  else
    SID_CHECK(sid::launch_cpqr(st, w.W, lq, l, n_, k, p->rank_tol, w.Wr, w.nrm, w.piv, w.R, w.Q,
                               w.keff, w.stats),
              "pivoted QR");
  // (3) coefficients P = R11^{-1} R(:, j) on the non-pivot columns
  SID_CHECK(sid::launch_id_coefficients(st, w.R, n_, w.piv, w.keff, k, w.R11, w.Pd, P, ldp, f64),
            "coefficients");
  // (4) estimates: err[1] sketch fit (final residual of mgsqr), err[0] probe rows
  SID_CHECK(sid::launch_ratio_sqrt(st, w.stats, w.err + 1), "sketch residual");
  if (!sh.single) {
    SID_CHECK(sid::launch_fit_residual(st, w.W, lq, l, q, n_, w.piv, w.keff, w.Pd, k, nullptr,
                                       w.fitpart, w.err),
              "probe residual");
    if (AJ)
      SID_CHECK(sid::launch_gather_cols(st, A, f64, lda, sh.N, w.piv, w.keff, k, AJ, f64, ldaj),
                "skeleton gather");
  } else {
    // (5) single pass.  Psi Y = Psi A Omega = W Omega, so the small matrix
    // M = W(0:lz, :) Omega plays the role of Z = Psi Q (up to the triangular
    // factor of Y), and the minimum-residual solve of the two-sided sketch
    // (Halko et al. Sec. 5.5 item (4)) becomes T = M^+ W(0:lz, J), AJ = Y T.
    // lz = l + e: the e extra co-range rows make M tall (the square form is
    // the ill-conditioned case the paper warns about in Sec. 2.3).  M^+ is
    // applied through mgsqr of M truncated at sp_rcond (least squares on the
    // pivoted columns).
    const double rcond = p->sp_rcond > 0.0 ? p->sp_rcond : default_rcond(sh.prec);
    SID_CHECK(sid::launch_omega_values(st, sh.prec, w.omega, sh.n * sh.l, w.om64), "omega values");
    SID_CHECK(sid::launch_gemm64(st, lz, l, n_, w.W, lq, 0, w.om64, l, 1, w.M, lz), "M = W Omega");
    if (q > 0)
      SID_CHECK(sid::launch_gemm64(st, q, l, n_, w.W + lz, lq, 0, w.om64, l, 1, w.Mpr, q),
                "Mpr = Wpr Omega");
    if (sid::cpqr_wg_supported(lz, l))
      SID_CHECK(sid::launch_cpqr_wg(st, w.M, lz, lz, l, l, rcond, w.pivM, w.RM, w.QM, w.rkM,
                                    w.statsM),
                "pivoted QR of M");
    else if (sid::cpqr_coop_supported(lz, l))
      SID_CHECK(sid::launch_cpqr_coop(st, w.M, lz, lz, l, l, rcond, w.coop, w.sync2, w.pivM, w.RM,
                                      w.QM, w.rkM, w.statsM, ctx->cooperative),
                "pivoted QR of M");
    else
      SID_CHECK(sid::launch_cpqr(st, w.M, lz, lz, l, l, rcond, w.Wr, w.nrm, w.pivM, w.RM, w.QM,
                                 w.rkM, w.statsM),
                "pivoted QR of M");
    SID_CHECK(sid::launch_gather_block(st, w.W, lq, 0, lz, w.piv, w.keff, k, w.WJ), "W(:, J)");
    SID_CHECK(sid::launch_gemm64(st, l, k, lz, w.QM, lz, 1, w.WJ, lz, 0, w.C, l), "QM^T W(:, J)");
    SID_CHECK(sid::launch_small_solve(st, w.RM, l, w.pivM, w.rkM, w.R11, w.C, l, k, w.T), "T");
    if (AJ) {
      const bool yf64 = sh.prec == SID_SK_F64;
      const bool ybf = sh.prec == SID_SK_BF16 || sh.prec == SID_SK_BF16X2 ||
                       sh.prec == SID_SK_FP8E4M3;
      if (ybf && sid::apply_t_bf16_supported(k, l))
        SID_CHECK(sid::launch_apply_t_bf16(st, (const float*)w.Y, sh.N, l, w.T, k, AJ, f64, ldaj,
                                           ctx->num_cu),
                  "AJ = Y T");
      else if (sid::apply_t_mfma_supported(k, l, yf64))
        SID_CHECK(sid::launch_apply_t_mfma(st, w.Y, yf64, sh.N, l, w.T, k, AJ, f64, ldaj),
                  "AJ = Y T");
      else
        SID_CHECK(sid::launch_apply_t(st, w.Y, yf64, sh.N, l, w.T, k, AJ, f64, ldaj), "AJ = Y T");
    }
    if (q > 0)
      SID_CHECK(sid::launch_gemm64(st, q, k, l, w.Mpr, q, 0, w.T, l, 0, w.mix, q), "Mpr T");
    SID_CHECK(sid::launch_fit_residual(st, w.W, lq, lz, q, n_, w.piv, w.keff, w.Pd, k,
                                       q > 0 ? w.mix : nullptr, w.fitpart, w.err),
              "probe residual");
  }
  if (J) SID_CHECK(hipMemcpyAsync(J, w.piv, sizeof(int64_t) * (size_t)k, hipMemcpyDeviceToDevice, st),
                   "copy J");
  if (k_eff)
    SID_CHECK(hipMemcpyAsync(k_eff, w.keff, sizeof(int64_t), hipMemcpyDeviceToDevice, st),
              "copy k_eff");
  if (err)
    SID_CHECK(hipMemcpyAsync(err, w.err, 2 * sizeof(double), hipMemcpyDeviceToDevice, st),
              "copy err");
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
  if (k > 4096) return fail(ctx, SID_EINVAL, "k too large");
  SID_NEED_DEVICE(ctx);
  SID_CHECK(hipSetDevice(ctx->device), "hipSetDevice");
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
  if (k > 1024) return fail(ctx, SID_EINVAL, "k too large");
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

}  // extern "C"
