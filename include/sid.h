/*
 * sid.h -- C ABI of the MI355X (gfx950) pass-efficient interpolative
 * decomposition (ID) compressor.
 *
 * Method: Dunton, Jofre, Iaccarino & Doostan, "Pass-efficient methods for
 * compression of high-dimensional turbulent flow data" (arXiv:1905.13257).
 *
 * Problem statement (Sec. 2.1, Sec. 2.4 eq. (ID), Remark 2.1).  A snapshot
 * matrix A holds one time snapshot per column: A is N x n, N = grid points x
 * field components, n = snapshots.  (The paper stores snapshots as rows and
 * computes a row ID; this library stores A transposed and computes the
 * column ID A ~ A(:, J) P, which is the same decomposition.)  J lists k
 * snapshot indices (the skeleton) and P is k x n with P(:, J) = I.
 *
 * Pass structure.
 *   - Randomized ID (Alg. 4): one pass forms the Gaussian sketch W = Psi A
 *     ((l+q) x n, l = k + oversample, q held-out probe rows); a column-pivoted
 *     modified Gram-Schmidt QR (mgsqr) of W's first l rows gives J and R, and
 *     back substitution gives P (Alg. 4 steps after the sketch).
 *   - Sub-sampled ID (Alg. 5, Sec. 2.5): the sketch reads only a coarse set of
 *     rows S of A: W = Psi(:, S) A(S, :).
 *   - Two-pass mode then reads the skeleton A(:, J) in a second pass.
 *   - Single-pass mode also forms Y = A Omega (N x l) in the same pass and
 *     estimates A(:, J) from W and Y without touching A again (the two-sided
 *     single-pass sketch of Halko et al. Sec. 5.5, quoted in Sec. 2.3).
 *
 * Conventions.
 *   - Matrices are column-major with a leading dimension (lda >= rows).
 *   - Indices are 0-based int64.
 *   - Array arguments are DEVICE pointers unless stated "host".
 *   - Calls that launch work are asynchronous on the context's stream and
 *     return before the work finishes; outputs are valid after the stream
 *     synchronizes.  Calls never allocate inside the launched sequence other
 *     than growing the context workspace, which happens on the host before
 *     any launch (sid_reserve grows it ahead of time).
 *   - Errors: every call returns sid_status; no exception or abort crosses
 *     the ABI.  Argument validation happens on the host before any device
 *     work; on error nothing is launched and sid_last_error() describes it.
 *   - Thread safety: a context is used by one host thread at a time.
 */
#ifndef SID_H
#define SID_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct sid_ctx sid_ctx;
typedef struct sid_rowset sid_rowset;
typedef struct sid_stream sid_stream;

typedef enum {
    SID_OK = 0,
    SID_EINVAL = -1,     /* bad argument (shape, pointer, parameter)            */
    SID_ENOMEM = -2,     /* device or host allocation failed / workspace cap     */
    SID_EDEVICE = -3,    /* HIP runtime error                                    */
    SID_ESTATE = -4,     /* call not valid in the object's current state         */
    SID_ENONFINITE = -5, /* reserved: non-finite values detected                 */
    SID_ERANK = -6       /* reserved                                             */
} sid_status;

typedef enum { SID_F64 = 0, SID_F32 = 1 } sid_dtype;

/* Arithmetic of the sketch pass.  Gaussian entries are single-precision
 * draws (sid_fill_gaussian); each mode stores them, and reads the data, as:
 *   F64     FP64 data (FP32 data promoted exactly), FP64 accumulation
 *   F32     FP32 data, FP32 products/accumulation within a row panel, FP64
 *           across panels
 *   BF16    data and Gaussians rounded to bfloat16, FP32 accumulation
 *   BF16X2  Gaussians rounded to bfloat16; data split a = hi + lo, hi =
 *           bf16(a), lo = bf16(a - hi) (16 significant bits); FP32
 *           accumulation
 *   FP8E4M3 Gaussians rounded to OCP e4m3 (nearest even, saturating at
 *           448); data read as s * e4m3(a / s) with one power-of-two scale
 *           s = 2^(E - 7) per tile of 64 consecutive rows (counted from row
 *           0 of A) and column, E = floor(log2 max|a|) over the tile clamped
 *           to [-100, 120] (s = 1 for a zero tile); exact products, FP32
 *           accumulation.  FP32 data with lda % 4 == 0, a 16-byte aligned A,
 *           all rows, l <= 128 and l + co-range + probe rows <= 160 take the
 *           streaming matrix-core pass; other inputs are quantized by one
 *           more pass into an N x n FP32 workspace copy first.
 * The small factorizations after the pass are always FP64.  The paper names
 * no low-precision format; these are this library's. */
typedef enum {
    SID_SK_F64 = 0,
    SID_SK_F32 = 1,
    SID_SK_BF16 = 2,
    SID_SK_BF16X2 = 3,
    SID_SK_FP8E4M3 = 4
} sid_sketch_prec;

/* TWO_PASS: Alg. 4/5 with the skeleton A(:, J) read in a second pass.
 * SINGLE_PASS: the skeleton estimated from the sketches (Sec. 2.3).
 * COARSE_SKELETON: Alg. 6 (Sec. 2.6, eq. (single_ID)): needs a coarse row set
 *   S; J and P are exactly those of TWO_PASS with the same parameters (the
 *   ID of A(S, :)), and the skeleton kept is the coarse one, AJ = A(S, J)
 *   (|S| x k, ldaj >= |S|): no row outside S is ever read.  The fine field is
 *   recovered with an interpolation operator, sid_interp_reconstruct.  Not
 *   for streams. */
typedef enum { SID_TWO_PASS = 0, SID_SINGLE_PASS = 1, SID_COARSE_SKELETON = 2 } sid_mode;

/* What mgsqr runs on.  GAUSS: the Gaussian sketch W = Psi(:, S) A(S, :)
 * (Alg. 4; with a coarse set, the sketched form of Alg. 5).  ROWS_LITERAL:
 * the coarse rows themselves, W_sel = A(S, :), as Alg. 5 writes the
 * sub-sampled ID; needs a coarse set of at most 4096 rows, two-pass mode and
 * an F64 or F32 precision; oversample and probe_rows are ignored (no probe
 * rows: err[0] is NaN); no refinement, no streaming. */
typedef enum { SID_SEL_GAUSS = 0, SID_SEL_ROWS_LITERAL = 1 } sid_select;

typedef struct {
    int64_t k;                 /* target rank, 1 <= k <= min(n, k + oversample)   */
    int64_t oversample;        /* p >= 0; sketch rows l = k + p (Alg. 4)          */
    uint64_t seed;             /* Omega = stream 0, Psi = stream 1 of the generator */
    const sid_rowset *coarse;  /* NULL: all rows; else the coarse row set S       */
    sid_mode mode;
    sid_sketch_prec prec;
    int32_t probe_rows;        /* q >= 0 held-out Psi rows for the error estimate */
    int32_t corange_rows;      /* single pass: e extra Psi rows (beyond the l that
                                  select J) used by the skeleton solve; < 0 means
                                  e = oversample.  Ignored in two-pass mode.     */
    double rank_tol;           /* 0: fixed rank k; > 0: stop the pivoted QR when
                                  the pivot's residual norm <= rank_tol times the
                                  first pivot's (Remark 2.2), k_eff < k then      */
    double sp_rcond;           /* single pass: relative drop tolerance of the
                                  small solve (0: default for the precision)     */
    int32_t refine;            /* 0: none; 1: one refinement pass of P (reads A
                                  once more, sid_compress only)                  */
    sid_sketch_prec refine_prec; /* precision of the refinement sketch          */
    sid_select select;         /* SID_SEL_GAUSS (default) or SID_SEL_ROWS_LITERAL */
    double probe_tol;          /* 0: off; > 0: the smallest rank k_eff whose ID fits
                                  the held-out probe rows to probe_tol (Remark 2.2
                                  with the probe rows as the stopping test); needs
                                  probe_rows > 0 and select GAUSS               */
} sid_params;

/* Fill a parameter block with defaults: oversample 10, seed 0, all rows,
 * two-pass, F32 sketch, probe_rows 10, corange_rows -1, rank_tol 0,
 * sp_rcond 0, refine 0, refine_prec BF16X2, select GAUSS, probe_tol 0.
 * Adaptive rank (probe_tol > 0): mgsqr runs to k (or to its rank_tol stop);
 * then, with Z = W_pr(:, J) R11^-1, the probe fit of the first k' pivots is
 * Z(:, 0:k') R(0:k', :) for every k', and k_eff becomes the smallest k' with
 * ||W_pr - Z(:, 0:k') R(0:k', :)||_F <= probe_tol ||W_pr||_F (k_eff stays at
 * mgsqr's count when none qualifies).  J, P, AJ and err then follow k_eff;
 * err[1] is the sketch fit at that rank.  In two-pass modes err[0] is that
 * same probe fit (so err[0] <= probe_tol when a rank qualified); in single
 * pass err[0] also carries the error of the estimated skeleton and can be
 * larger.
 * Refinement (refine = 1; the paper stops at the ID): after J and P0 are
 * chosen, A is sketched once more with Psi's selection rows in refine_prec,
 * W' = Psi_sel A; with J kept, P is recomputed as the least-squares solution
 * P1 = argmin ||W'(:, J) X - W'||_F (mgsqr of W' with its pivot order forced
 * to J, then the usual back substitution), so P1(:, J) = I exactly.  err is
 * re-fitted with P1 on the rows of the first sketch; AJ does not depend on P
 * and is unchanged.
 * Psi row layout: rows [0, l) select J and P (Alg. 4); in single pass rows
 * [l, l + e) are the extra co-range rows; the last q rows are the probe. */
void sid_params_init(sid_params *p, int64_t k);

/* Context: binds a device and a stream and owns the workspace.  `device` is a
 * HIP device ordinal; `hip_stream` is a hipStream_t to launch on, or NULL for
 * a stream the context creates (and destroys).  device = -1 makes a
 * validation-only context: calls on it check their arguments exactly as on a
 * device context, then return SID_ESTATE instead of launching (no GPU
 * needed).  Errors: SID_EINVAL (out NULL or device out of range),
 * SID_EDEVICE (no HIP device / runtime failure). */
sid_status sid_create(sid_ctx **out, int device, void *hip_stream);
sid_status sid_destroy(sid_ctx *ctx);
/* Human-readable description of the last failing call on this context
 * (valid until the next call on it).  Never NULL. */
const char *sid_last_error(const sid_ctx *ctx);
/* Bytes of device workspace currently held by the context. */
size_t sid_workspace_bytes(const sid_ctx *ctx);
/* Cap on workspace growth in bytes (0 = none); growth beyond it fails with
 * SID_ENOMEM. */
sid_status sid_set_workspace_limit(sid_ctx *ctx, size_t bytes);
/* Wait for all work queued on the context (and its batched children), then
 * report device-side failures since the previous sid_sync: the
 * multi-workgroup pivoted QR needs its workgroups resident together; it is
 * a plain launch whose grid is checked against the device's occupancy on
 * the host (the environment variable SID_COOPERATIVE=1 at context creation
 * selects a cooperative launch outside graph capture instead, which
 * guarantees co-residency but waits for the device's other work to drain).
 * A bounded wait that times out (other work kept some workgroups from
 * starting) sets k_eff = -1 for that compression and a flag this call reads
 * and clears.  Returns SID_OK, or SID_EDEVICE with sid_last_error naming
 * the failure (the results with k_eff = -1 are then invalid). */
sid_status sid_sync(sid_ctx *ctx);

/* Coarse row set S (Sec. 2.5 eq. (A_c): the sub-sampled degrees of freedom).
 * `host_rows` (host) must be strictly increasing, within [0, N), and count >
 * 0; it is validated on the host and copied to the device once.  The sketch
 * then reads only A(S, :) (Alg. 5 step "subsample").  Psi columns are keyed
 * by the global row index, so a coarse sketch equals the full sketch of
 * A(S, :). */
sid_status sid_rowset_create(sid_ctx *ctx, const int64_t *host_rows, int64_t count,
                             int64_t N, sid_rowset **out);
sid_status sid_rowset_destroy(sid_rowset *rs);

/* Grow the workspace (and create the internal side stream) for compress
 * calls of this shape and these parameters ahead of time, including the
 * sketch buffers of the refinement precision when p->refine is set.  It
 * sizes for FP32 data with a 16-byte aligned base and lda % 4 == 0 (the
 * layout of a device allocation); other layouts with the FP8 sketch take a
 * quantized copy of the data that is sized on first use.  After it (or
 * after one call of the same shape), sid_compress on the context's stream
 * allocates nothing and synchronizes nothing, so it can be captured into a
 * HIP graph and replayed (the library records no memset nodes; the
 * single-pass side stream joins the capture through events).  A call under
 * capture whose workspace would have to grow fails with SID_ENOMEM and a
 * message naming the capture, instead of allocating. */
sid_status sid_reserve(sid_ctx *ctx, int64_t N, int64_t n, const sid_params *p);

/*
 * Compress A (N x n, column-major, leading dimension lda, element type
 * `dtype`) into a rank-k column ID.
 *   J     [k] int64: skeleton columns in pivot order; entries beyond k_eff -1.
 *   P     k x n (ldp), element type `dtype`; P(:, J_i) = e_i exactly; rows
 *         beyond k_eff zero.
 *   AJ    N x k (ldaj), element type `dtype`, or NULL.  Two-pass: the copy
 *         A(:, J) (second pass, Sec. 2.6).  Single-pass: the estimate of
 *         A(:, J) from the sketches (columns beyond k_eff zero).  Coarse
 *         skeleton: |S| x k (ldaj >= |S|), the copy A(S, J) (columns beyond
 *         k_eff zero).
 *   err   [2] double: err[0] = relative Frobenius residual of the held-out
 *         probe rows (an estimate of ||A - AJ P||_F / ||A||_F; NaN when
 *         probe_rows = 0), err[1] = relative residual of the sketch fit.
 *         With refine = 1 both are fitted with the refined P that is
 *         returned (on the rows of the first sketch).
 *   k_eff [1] int64: number of skeleton columns actually chosen; -1 marks a
 *         failed device-wide wait of the pivoted QR (results invalid; see
 *         sid_sync).
 * Any of J, P, err, k_eff may be NULL when not wanted.
 * Errors: SID_EINVAL for bad shapes/parameters/null A; SID_ENOMEM when the
 * workspace cannot grow; SID_EDEVICE for a launch failure.
 */
sid_status sid_compress(sid_ctx *ctx, const void *A, sid_dtype dtype, int64_t N, int64_t n,
                        int64_t lda, const sid_params *p, int64_t *J, void *P, int64_t ldp,
                        void *AJ, int64_t ldaj, double *err, int64_t *k_eff);

/* Reconstruct Ahat = AJ P (eq. (ID)); AJ N x k (ldaj), P k x n (ldp), Ahat
 * N x n (ldo), all of element type `dtype`; 1 <= k <= 256.  FP32 with
 * k <= 128 runs on the bfloat16 matrix cores from hi + lo splits of AJ and P
 * (three products, FP32 accumulation): each entry is within 2^-15 of
 * sum_t |AJ(i, t)| |P(t, j)| of the exact product.  FP64, and FP32 with
 * k > 128: FMAs in the element type. */
sid_status sid_reconstruct(sid_ctx *ctx, const void *AJ, int64_t ldaj, const void *P,
                           int64_t ldp, sid_dtype dtype, int64_t N, int64_t k, int64_t n,
                           void *Ahat, int64_t ldo);

/* Error of an ID against the data without forming Ahat (Sec. 3: relative
 * Frobenius error, Tables 4-7; relative entry-wise max error, Sec. 3.1).
 * out4 (host, 4 doubles): ||A - AJ P||_F, ||A||_F, max |A - Ahat|/|A| over
 * A != 0, max |A - Ahat|.  1 <= k <= 256.  Synchronizes the stream. */
sid_status sid_error_norms(sid_ctx *ctx, const void *A, int64_t lda, const void *AJ,
                           int64_t ldaj, const void *P, int64_t ldp, sid_dtype dtype,
                           int64_t N, int64_t k, int64_t n, double *out4);

/* Test hook: the Gaussian test-matrix entries the sketches use.
 * out[t + nminor * s] = G(seed, stream, major0 + s, minor0 + t) as float, for
 * s < nmajor, t < nminor (device pointer).  Omega(j, c) = G(seed, 0, j, c);
 * Psi(r, i) = G(seed, 1, i, r).  See the generator specification in the
 * device sources (Philox4x32-10 + single-precision Box-Muller). */
sid_status sid_fill_gaussian(sid_ctx *ctx, uint64_t seed, int stream, int64_t major0,
                             int64_t nmajor, int64_t minor0, int64_t nminor, float *out);

/* Test hook: the sketch W = Psi(:, S) A(S, :) (lw x n, FP64, column-major,
 * ld = lw, lw = l + e + q with e as in single-pass mode when Y != NULL and 0
 * otherwise) and, when Y != NULL, Y = A Omega (N x l, row-major, element type
 * FP64 for SID_SK_F64 else FP32) exactly as sid_compress forms them. */
sid_status sid_sketch(sid_ctx *ctx, const void *A, sid_dtype dtype, int64_t N, int64_t n,
                      int64_t lda, const sid_params *p, double *W, void *Y);

/* For callers that cannot allocate (code under HIP graph capture, tight
 * serving loops, harnesses that forbid hipMalloc): sid_sketch with all of its
 * scratch (Omega's values, Omega^T in bfloat16, the per-workgroup-pair FP32
 * partials of W) in a static device array of 80 MiB that each device holds
 * from the library's load until the process ends; the call itself allocates
 * nothing (no hipMalloc, no hipFree, no allocating library routine) and
 * leaves the context's workspace untouched.  Same arguments, outputs and
 * results (bit for bit) as sid_sketch, restricted to FP32 data in device
 * memory with a 16-byte aligned base and lda % 4 == 0, all rows (no coarse
 * set), the BF16 / BF16X2 / FP8E4M3 sketch forms and n within one launch of
 * the matrix-core pass sid_sketch takes (512 columns up to l = 128 and
 * l + e + q = 160; narrower beyond, e.g. 384 columns for k = 150, p = 30).
 * Errors: SID_EINVAL for other inputs, and for shapes whose scratch exceeds
 * the static array (the message gives both sizes).  Every call on a device
 * shares that device's array, which keeps the last call's contents: two
 * calls that overlap on one device (two streams, two threads) race and give
 * wrong results. */
sid_status sid_sketch_noalloc(sid_ctx *ctx, const void *A, sid_dtype dtype, int64_t N, int64_t n,
                              int64_t lda, const sid_params *p, double *W, void *Y);

/* Measurement hook (no part of the method): one launch of a probe kernel on
 * the context's stream, for timing the ceilings the kernels' design rests
 * on.  kind 0: read the N x n FP32 device buffer `buf` once (16-byte loads);
 * 1: write it column by column with the reconstruction kernels' pattern
 * (each wave 4 columns x 256 contiguous bytes per instruction; N % 64 == 0);
 * 2: write it as one sequential fill; 3 / 4: N rounds of eight independent
 * v_mfma_f32_16x16x32_bf16 / v_mfma_f32_32x32x16_bf16 per wave on register
 * data, 8 workgroups of 4 waves per compute unit (buf and n unused).
 * buf: 16-byte aligned, N n a multiple of 4.  Errors: SID_EINVAL. */
sid_status sid_probe(sid_ctx *ctx, int kind, void *buf, int64_t N, int64_t n);

/*
 * Streaming (snapshots that arrive a few at a time, the in-situ setting of
 * Sec. 1 and Sec. 4).  Both sketches are linear in the columns: W(:, j) =
 * Psi A(:, j) depends on column j alone and Y = A Omega is a sum over column
 * blocks, so the sketches of the blocks seen so far are the sketches of the
 * matrix so far, and finishing gives the result sid_compress gives for the
 * concatenated columns (up to the order of FP32 sums in Y).  J indexes
 * columns in arrival order.
 *
 * sid_stream_begin: N rows, at most n_max columns; params as for
 *   sid_compress (k <= columns pushed is checked at finish).  The stream owns
 *   device memory for W ((l+e+q) x n_max FP64), in single pass Y (N x l) and,
 *   once a block smaller than 512 columns arrives, a stage of
 *   N x min(n_max, 512) values of `dtype`.  A coarse row set in params must
 *   outlive the stream.
 * sid_stream_push: ncols >= 0 columns of N values (column-major, leading
 *   dimension ld >= N, device memory, `dtype`).  Blocks are copied into the
 *   stage and sketched 512 columns at a time; a push of 512 or more columns
 *   with ld % 4 == 0 and a 16-byte aligned pointer is sketched in place.
 *   The caller may reuse A_blk once the context's stream has passed this
 *   call.  SID_EINVAL past n_max columns.
 * sid_stream_finish: sketches what is staged, then forms J, P, AJ, err,
 *   k_eff exactly as sid_compress (same meanings, layouts and NULL rules)
 *   with n = the columns pushed.  Two-pass streams keep no columns: AJ must
 *   be NULL (gather A(:, J) from the caller's own copy).  Frees the stream
 *   on success and on error.
 * sid_stream_info: rows N, columns pushed so far, k, data type and mode of
 *   a stream (any output pointer may be NULL; host memory).
 * sid_stream_abort: frees a stream without finishing it.
 * sid_stream_save: checkpoint (sketches what is staged first).  With
 *   host_buf NULL, sets *bytes to the size needed; otherwise writes the state
 *   (a header, W and Y) into host_buf of *bytes bytes (SID_EINVAL and the
 *   needed size in *bytes if too small).  Synchronizes the stream.  Streams
 *   over a coarse row set cannot be saved (SID_EINVAL).
 * sid_stream_restore: a new stream on ctx from a saved state (SID_EINVAL for
 *   a buffer that is not one); pushing the remaining columns and finishing
 *   gives the result of the uninterrupted stream.
 */
sid_status sid_stream_begin(sid_ctx *ctx, sid_dtype dtype, int64_t N, int64_t n_max,
                            const sid_params *p, sid_stream **out);
sid_status sid_stream_push(sid_stream *s, const void *A_blk, int64_t ncols, int64_t ld);
sid_status sid_stream_finish(sid_stream *s, int64_t *J, void *P, int64_t ldp, void *AJ,
                             int64_t ldaj, double *err, int64_t *k_eff);
sid_status sid_stream_info(const sid_stream *s, int64_t *N, int64_t *cols, int64_t *k,
                           int *dtype, int *mode);
sid_status sid_stream_abort(sid_stream *s);
sid_status sid_stream_save(sid_stream *s, void *host_buf, size_t *bytes);
sid_status sid_stream_restore(sid_ctx *ctx, const void *host_buf, size_t bytes,
                              sid_stream **out);

/*
 * Single-pass ID with interpolation (Alg. 6, Sec. 2.6).  A structured grid
 * of ncomp field components on nx x ny x nz points; rows of A are ordered
 * ((c * nx + i) * ny + j) * nz + kz (z fastest), N = ncomp nx ny nz.  The
 * coarse grid keeps, per dimension d, the indices coarse[d] (strictly
 * increasing in [0, n[d])); its rows S are the tensor product of those lists
 * in the same order (row set sid_interp_rowset).  The coarse-to-fine
 * operator Mf (N x |S|, the paper's M transposed) is piecewise linear in
 * each dimension (Sec. 3 uses piecewise linear interpolation), applied as a
 * tensor product: trilinear, t = 8 coarse points per fine point.  Per
 * dimension a fine point lying between two coarse nodes takes the linear
 * weights of their coordinates; beyond the outermost nodes of a bounded
 * dimension the end element's line is continued (linear extrapolation); a
 * periodic dimension (period > 0) joins its last node to the first one
 * shifted by the period; a dimension with one coarse node is constant.
 *   coord[d]  host, n[d] strictly increasing coordinates (NULL: 0, 1, 2, ...);
 *             periodic: the span of the coarse nodes must be < period
 *   coarse[d] host, ncoarse[d] >= 1 indices
 * The operator is never formed: sid_interp_create builds three small 1-D
 * tables (two node indices and a weight per fine index) on the host and
 * copies them to the device; the kernels form the 8 weights of a fine point
 * from them.  N and |S| must be below 2^31.  The object and its row set
 * belong to ctx and must be destroyed before it.
 */
typedef struct sid_interp sid_interp;

typedef struct {
    int32_t ncomp;
    int32_t reserved;           /* 0 */
    int64_t n[3];
    const double *coord[3];
    const int64_t *coarse[3];
    int64_t ncoarse[3];
    double period[3];
} sid_mesh;

sid_status sid_interp_create(sid_ctx *ctx, const sid_mesh *mesh, sid_interp **out);
sid_status sid_interp_destroy(sid_interp *ip);
/* The coarse row set S of the mesh (owned by the interp object), for
 * sid_params.coarse; N (fine rows) and Nc = |S| on the host (NULL allowed). */
const sid_rowset *sid_interp_rowset(const sid_interp *ip);
sid_status sid_interp_info(const sid_interp *ip, int64_t *N, int64_t *Nc);

/* Ahat = Mf ACJ P (eq. (single_ID)): ACJ the coarse skeleton (Nc x k,
 * ldacj >= Nc, from a COARSE_SKELETON compress), P k x n (ldp >= k), Ahat
 * N x n (ldo >= N), all of element type `dtype`, device memory.
 * Arithmetic: F64 throughout for SID_F64.  SID_F32 with k <= 128: the
 * interpolated skeleton rows are formed in FP32, split into two bfloat16
 * parts (hi + lo) as are P's entries, and multiplied on the matrix cores
 * as hi*hi + hi*lo + lo*hi with FP32 accumulation (relative error of a
 * product about 2^-16); SID_F32 with k > 128: FP32 fused multiply-adds.
 * Asynchronous on the context's stream; may grow the workspace (a row-major
 * copy of ACJ and a packed copy of P, or for the FMA path Mf ACJ itself).
 * 1 <= k <= 256. */
sid_status sid_interp_reconstruct(sid_ctx *ctx, const sid_interp *ip, const void *ACJ,
                                  int64_t ldacj, const void *P, int64_t ldp, sid_dtype dtype,
                                  int64_t k, int64_t n, void *Ahat, int64_t ldo);

/* Error of Ahat = Mf ACJ P against the fine data A (N x n, lda) without
 * forming Ahat, with the arithmetic of sid_interp_reconstruct.  out4 (host):
 * ||A - Ahat||_F, ||A||_F, max |A - Ahat|/|A| over A != 0, max |A - Ahat|
 * (as sid_error_norms).  Synchronizes the stream. */
sid_status sid_interp_error_norms(sid_ctx *ctx, const sid_interp *ip, const void *A,
                                  int64_t lda, const void *ACJ, int64_t ldacj, const void *P,
                                  int64_t ldp, sid_dtype dtype, int64_t k, int64_t n,
                                  double *out4);

/*
 * Single-pass blocked randomized SVD (SBR-SVD, Alg. 2; the paper's other
 * single-pass method, Sec. 2.3).  In the paper's orientation A_p = A^T
 * (snapshots in rows) with Gaussian Omega = Psi^T (the ID's Psi: stream 1,
 * keyed by the global row), one pass over A forms G = A_p Omega = (Psi A)^T
 * and H = A_p^T G = A G (N x l, l = k + oversample); then for each of the
 * l / block blocks of Omega's columns: Y_i = G_i - Q (B Omega_i),
 * (Q_i, R_i) = qr(Y_i), (Q_i, R~_i) = qr(Q_i - Q Q^T Q_i), R_i = R~_i R_i,
 * B_i = R_i^-T (H_i^T - Y_i^T Q B - Omega_i^T B^T B), Q = [Q, Q_i],
 * B = [B; B_i]; finally B = U~ S V^T, U = Q U~.  Output A ~ V S U^T
 * (A_p ~ U S V^T):
 *   S  [k] FP64 singular values, descending (device)
 *   U  n x k (ldu >= n) temporal factor, element type `dtype` (device)
 *   V  N x k (ldv >= N) spatial factor, element type `dtype` (device)
 *   rank (host, may be NULL): rows of B formed (l, or fewer when a block's
 *        R_i is numerically singular, i.e. A_p Omega has rank < l; the
 *        loop then stops and S, U, V past it are zero)
 * Arithmetic: G in the sketch precision `prec` (as sid_compress); H (FP32
 * data promoted exactly), the block loop and the SVD in FP64; the SVD of B
 * via the eigendecomposition of B B^T (cyclic Jacobi).  The block loop
 * subtracts terms of size sigma_1^2 from H to leave ones of size sigma_j^2,
 * so H's rounding reaches B_i amplified by about (sigma_1 / sigma_j)^2:
 * hence H in FP64.  The loop is exact for whichever G the pass produced as
 * long as H = A_p^T G with that same G (the Y_i^T Q B term takes up the
 * difference between G and A_p Omega), so `prec` matters as it does for the
 * ID's sketch, not through that amplification.  H and each block row of B
 * (H_i - B^T M_i) R_i^-1 are one pass over the rows each; B Omega_i and
 * B B^T are split reductions over the rows (fixed summation order) and V is
 * formed row by row in the output type.  Limits: l <=
 * min(n, 256), l % block == 0, block <= 64.  Synchronizes the stream once
 * per block (the stop test).  Workspace about (2 l + 1.5 block) N doubles
 * plus 64 MiB.
 */
typedef struct {
    int64_t k;              /* target rank >= 1                       */
    int64_t oversample;     /* p >= 0, l = k + p                      */
    int64_t block;          /* b >= 1 with l % b == 0, b <= 64        */
    uint64_t seed;          /* Omega = Psi^T of this seed             */
    sid_sketch_prec prec;   /* arithmetic of the pass forming G       */
} sid_svd_params;

/* defaults: oversample 10, block 10, seed 0, prec F64 */
void sid_svd_params_init(sid_svd_params *p, int64_t k);
sid_status sid_sbr_svd(sid_ctx *ctx, const void *A, sid_dtype dtype, int64_t N, int64_t n,
                       int64_t lda, const sid_svd_params *p, double *S, void *U, int64_t ldu,
                       void *V, int64_t ldv, int64_t *rank);

/*
 * SBR-SVD over snapshots that arrive in blocks (Alg. 2's single pass: each
 * snapshot is read once, its row of G = A_p Omega formed and H += a^T g
 * added while it is resident).  sid_svd_stream_begin: as sid_sbr_svd for
 * an N x n_max matrix (parameter rules with n = n_max); the stream holds
 * W = Psi A (l x n_max FP64), H (N x l FP64) and a stage of
 * N x min(n_max, 512) values of `dtype`.  Columns are pushed with
 * sid_stream_push (same rules as for an ID stream); each sketched block of
 * up to 512 columns also adds its part of H in column order, so the result
 * is bitwise that of sid_sbr_svd on the whole matrix.  sid_stream_info and
 * sid_stream_abort apply; sid_stream_finish and sid_stream_save reject an
 * SBR-SVD stream (SID_EINVAL).  sid_svd_stream_finish: sketches what is
 * staged, then runs the block loop and the SVD of B with n = the columns
 * pushed (k + oversample <= n); outputs as sid_sbr_svd.  Frees the stream on
 * success and on error.
 */
sid_status sid_svd_stream_begin(sid_ctx *ctx, sid_dtype dtype, int64_t N, int64_t n_max,
                                const sid_svd_params *p, sid_stream **out);
sid_status sid_svd_stream_finish(sid_stream *s, double *S, void *U, int64_t ldu, void *V,
                                 int64_t ldv, int64_t *rank);

/*
 * Batched compression of independent matrices (Sec. 3 compresses each flow
 * variable or dataset on its own; Sec. 3.3 compresses a long record block by
 * block).  probs: host array of `count` problems, each with its own A (N x n,
 * lda), parameters and outputs (same meanings, layouts and NULL rules as
 * sid_compress); all share `dtype`.  Every problem is validated before
 * anything is launched (SID_EINVAL names the first bad problem in
 * sid_last_error).  Results are bit for bit those of one sid_compress per
 * problem.
 *
 * When at most 16384 problems all have FP32 data (16-byte aligned,
 * lda % 4 == 0), the same BF16 / BF16X2 / FP8E4M3 sketch form and mode
 * (two-pass or single-pass), the Gaussian selection over all rows, no
 * refinement, n <= 512, l <= 128 and l + e + q <= 160, persistent launches
 * sketch all of them: one per register layout class of the problems (at
 * most three, side by side), each over a work queue of its problems' row
 * shares (the problems with the most work per share first); then one launch
 * forms every W.  The pivoted QRs of all problems
 * whose shapes a one-workgroup factorization takes (W_sel's l x n and,
 * single pass, M's lz x l) go into a few launches, one per
 * kernel instance, side by side on up to 8 internal child streams, after two
 * launches for the single-pass products they need.  When every problem is
 * single pass with a fixed rank k <= 128, the steps after the QR (R11, the
 * coefficient solve, both estimates, T) are one launch each for the batch,
 * and only P's conversion, AJ = Y T and the result copies run per problem
 * on the child streams; otherwise each problem's remaining factorization
 * runs on a child stream (own workspace each).  Other batches run each
 * problem's sid_compress on the child streams.  Everything runs after the
 * work already queued on the context's stream, which waits for all of it
 * before the call returns.
 *
 * The persistent path keeps a plan per problem set (the queue table and the
 * problems' partials, W, Omega and Y in device memory owned by the context;
 * the last 8 problem sets are kept).  Once the plan and the child streams
 * exist (sid_reserve_batched, or an earlier call with the same problems) the
 * call allocates nothing.  It is not capturable: under HIP graph capture the
 * call returns SID_ESTATE (a captured batched call ended the process inside
 * the runtime's end of capture).  A row set in a problem's params must
 * belong to ctx.
 */
typedef struct {
    const void *A;
    int64_t N, n, lda;
    sid_params params;
    int64_t *J;
    void *P;
    int64_t ldp;
    void *AJ;
    int64_t ldaj;
    double *err;
    int64_t *k_eff;
} sid_problem;

sid_status sid_compress_batched(sid_ctx *ctx, const sid_problem *probs, int64_t count,
                                sid_dtype dtype);

/* Everything sid_compress_batched with these problems would allocate or
 * create: the batch's plan (persistent path), the 8 child streams and their
 * workspaces.  tune != 0 also runs the autotuner: the batch is compressed
 * with 1, 2, 4 and 8 child streams for the factorizations (twice, the first
 * round warming up; every candidate writes the same results to the
 * problems' outputs) and the fastest count is kept for the context.  The
 * choice is cached per (GPU architecture, sketch form, mode, batch size as
 * a power of two, widest problem in 128-column chunks); with the environment
 * variable SID_TUNE_CACHE naming a file, choices are appended to it and a
 * later call with tune = 0 (in any process) takes the cached choice for its
 * key.  Not under graph capture (SID_ESTATE). */
sid_status sid_reserve_batched(sid_ctx *ctx, const sid_problem *probs, int64_t count,
                               sid_dtype dtype, int tune);

/* The number of child streams batched calls of ctx use (4 until the
 * autotuner or its cache sets it); -1 for a NULL ctx. */
int sid_batch_streams(const sid_ctx *ctx);

#ifdef __cplusplus
}
#endif

#endif /* SID_H */
