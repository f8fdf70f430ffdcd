/*
 * oracle_core.c -- TEST INFRASTRUCTURE ONLY.
 *
 * Plain, slow, obviously-correct CPU reference for the pass-efficient
 * interpolative decomposition (ID) of Dunton, Jofre, Iaccarino & Doostan,
 * "Pass-efficient methods for compression of high-dimensional turbulent flow
 * data" (arXiv:1905.13257).  Only tests/, the smoke check and the benchmark's
 * CPU-baseline leg may load this library.  It shares no code, header, table or
 * constant generator with the HIP product path.
 *
 * Contents
 *   1. Philox4x32-10 (Salmon, Moraes, Dror & Shaw, SC'11), the counter-based
 *      generator the sketches draw from.
 *   2. The Gaussian transform of the generator's output (Box & Muller 1958),
 *      evaluated with a fixed sequence of IEEE single-precision operations so
 *      that any correct implementation of the same specification is
 *      bit-identical.  The paper draws i.i.d. Gaussian test matrices
 *      (Sec. 2.2, eq. for the sketch A*Omega; Alg. 4 step "Generate Omega").
 *   3. The sketches W = Psi(:,S) A(S,:) and Y = A Omega in FP64, summed in
 *      plain sequential order (Sec. 2.4, Alg. 4 "Y <- A Omega"; the two-sided
 *      single-pass sketch of Halko et al. Sec. 5.5 restated in Sec. 2.3).
 *   4. Plain elementwise reductions used by the tests (Frobenius norms of
 *      A - A_J P, relative max error of Sec. 3.1).
 *
 * Orientation: the paper stores snapshots as rows (A_p is m x n, m = time);
 * this library stores them as columns, A = A_p^T (N x n, column-major,
 * n = number of snapshots).  A column ID A ~ A(:,J) P is then the paper's row
 * ID (eq. of Sec. 2.4) transposed, see Remark 2.1.
 *
 * Build: gcc -O2 -fopenmp -ffp-contract=off -shared -fPIC (no fast-math: the
 * Gaussian specification relies on IEEE rounding of every operation).
 */
#include <stdint.h>
#include <string.h>
#include <math.h>
#include <stdlib.h>

/* ------------------------------------------------------------------------ */
/* 1. Philox4x32-10                                                          */
/* ------------------------------------------------------------------------ */

/* Round constants of Philox4x32 as published (multipliers and Weyl key
 * increments). */
#define OR_PHILOX_MUL_A 0xD2511F53u
#define OR_PHILOX_MUL_B 0xCD9E8D57u
#define OR_PHILOX_KEY_A 0x9E3779B9u
#define OR_PHILOX_KEY_B 0xBB67AE85u

/* Ten rounds of the Philox S-P network on a 128-bit counter under a 64-bit
 * key.  Round r uses key + r * (KEY_A, KEY_B). */
void oracle_philox4x32_10(const uint32_t ctr_in[4], const uint32_t key_in[2],
                          uint32_t out[4])
{
    uint32_t x0 = ctr_in[0], x1 = ctr_in[1], x2 = ctr_in[2], x3 = ctr_in[3];
    uint32_t k0 = key_in[0], k1 = key_in[1];
    for (int round = 0; round < 10; ++round) {
        uint64_t prod_a = (uint64_t)OR_PHILOX_MUL_A * (uint64_t)x0;
        uint64_t prod_b = (uint64_t)OR_PHILOX_MUL_B * (uint64_t)x2;
        uint32_t hi_a = (uint32_t)(prod_a >> 32), lo_a = (uint32_t)prod_a;
        uint32_t hi_b = (uint32_t)(prod_b >> 32), lo_b = (uint32_t)prod_b;
        uint32_t y0 = hi_b ^ x1 ^ k0;
        uint32_t y1 = lo_b;
        uint32_t y2 = hi_a ^ x3 ^ k1;
        uint32_t y3 = lo_a;
        x0 = y0; x1 = y1; x2 = y2; x3 = y3;
        k0 += OR_PHILOX_KEY_A;
        k1 += OR_PHILOX_KEY_B;
    }
    out[0] = x0; out[1] = x1; out[2] = x2; out[3] = x3;
}

/* ------------------------------------------------------------------------ */
/* 2. Gaussian specification (single precision Box-Muller)                   */
/* ------------------------------------------------------------------------ */
/*
 * Entry (major, minor) of random stream `stream` under `seed`:
 *   counter = (major mod 2^32, minor / 4, stream, major / 2^32),
 *   key     = (seed mod 2^32, seed / 2^32),
 *   (x0,x1,x2,x3) = Philox4x32-10(counter, key);
 *   minor % 4 in {0,1} takes the Box-Muller pair of (x0,x1), {2,3} of (x2,x3);
 *   even minor -> r*cos(theta), odd minor -> r*sin(theta).
 * Pair (a, b) of 32-bit words:
 *   u     = ((a >> 8) + 1) * 2^-24                 in (0, 1], exact
 *   L     = ln(u) by the reduction/series below    (single precision)
 *   r     = sqrtf(-2 L)
 *   quad  = b >> 30,  f = (b >> 7) & (2^23 - 1)
 *   t     = (2 f + 1) * 2^-24                      in (0, 1), exact
 *   phi   = t * HALF_PI                            in (0, pi/2)
 *   (c,s) = Taylor polynomials of cos/sin in phi (Horner in phi^2, fmaf)
 *   (cos theta, sin theta) = (c,s), (-s,c), (-c,-s), (s,-c) for quad 0..3
 * ln(u): u = m 2^e with m in [1,2); if m >= SQRT2 then m /= 2, e += 1;
 *   s = (m - 1)/(m + 1); ln m = s (2 + s^2 (2/3 + s^2 (2/5 + s^2 (2/7 +
 *   s^2 (2/9 + s^2 2/11))))); ln u = fmaf(e, LN2, ln m).
 * All constants are the single-precision roundings (to nearest) of the
 * exact values; every operation is one IEEE single operation, no contraction
 * other than the explicit fmaf calls.
 */
static inline float or_from_bits(uint32_t b) { float f; memcpy(&f, &b, 4); return f; }
static inline uint32_t or_to_bits(float f) { uint32_t b; memcpy(&b, &f, 4); return b; }

static float or_ln_spec(float u)
{
    const float SQRT2 = or_from_bits(0x3FB504F3u);
    const float LN2   = or_from_bits(0x3F317218u);
    const float T3    = or_from_bits(0x3F2AAAABu);   /* 2/3  */
    const float T5    = or_from_bits(0x3ECCCCCDu);   /* 2/5  */
    const float T7    = or_from_bits(0x3E924925u);   /* 2/7  */
    const float T9    = or_from_bits(0x3E638E39u);   /* 2/9  */
    const float T11   = or_from_bits(0x3E3A2E8Cu);   /* 2/11 */
    uint32_t bits = or_to_bits(u);
    int expo = (int)((bits >> 23) & 0xFFu) - 127;
    float m = or_from_bits((bits & 0x007FFFFFu) | 0x3F800000u);
    if (m >= SQRT2) { m = m * 0.5f; expo += 1; }
    float s  = (m - 1.0f) / (m + 1.0f);
    float s2 = s * s;
    float poly = fmaf(s2, T11, T9);
    poly = fmaf(s2, poly, T7);
    poly = fmaf(s2, poly, T5);
    poly = fmaf(s2, poly, T3);
    poly = fmaf(s2, poly, 2.0f);
    float ln_m = s * poly;
    return fmaf((float)expo, LN2, ln_m);
}

static void or_sincos_quarter(float phi, float *c_out, float *s_out)
{
    /* sin: odd Taylor terms through phi^13; cos: even terms through phi^14 */
    const float S3  = or_from_bits(0xBE2AAAABu);
    const float S5  = or_from_bits(0x3C088889u);
    const float S7  = or_from_bits(0xB9500D01u);
    const float S9  = or_from_bits(0x3638EF1Du);
    const float S11 = or_from_bits(0xB2D7322Bu);
    const float S13 = or_from_bits(0x2F309231u);
    const float C2  = or_from_bits(0xBF000000u);
    const float C4  = or_from_bits(0x3D2AAAABu);
    const float C6  = or_from_bits(0xBAB60B61u);
    const float C8  = or_from_bits(0x37D00D01u);
    const float C10 = or_from_bits(0xB493F27Eu);
    const float C12 = or_from_bits(0x310F76C7u);
    const float C14 = or_from_bits(0xAD49CBA5u);
    float p2 = phi * phi;
    float sp = fmaf(p2, S13, S11);
    sp = fmaf(p2, sp, S9);
    sp = fmaf(p2, sp, S7);
    sp = fmaf(p2, sp, S5);
    sp = fmaf(p2, sp, S3);
    sp = fmaf(p2, sp, 1.0f);
    float cp = fmaf(p2, C14, C12);
    cp = fmaf(p2, cp, C10);
    cp = fmaf(p2, cp, C8);
    cp = fmaf(p2, cp, C6);
    cp = fmaf(p2, cp, C4);
    cp = fmaf(p2, cp, C2);
    cp = fmaf(p2, cp, 1.0f);
    *s_out = phi * sp;
    *c_out = cp;
}

static void or_box_muller(uint32_t a, uint32_t b, float *z_cos, float *z_sin)
{
    const float HALF_PI = or_from_bits(0x3FC90FDBu);
    const float TWO_M24 = or_from_bits(0x33800000u);   /* 2^-24 */
    float u = (float)((a >> 8) + 1u) * TWO_M24;
    float L = or_ln_spec(u);
    float r = sqrtf(-2.0f * L);
    uint32_t quad = b >> 30;
    uint32_t frac = (b >> 7) & 0x007FFFFFu;
    float t = (float)(2u * frac + 1u) * TWO_M24;
    float phi = t * HALF_PI;
    float c, s;
    or_sincos_quarter(phi, &c, &s);
    float ct, st;
    switch (quad) {
        case 0:  ct =  c; st =  s; break;
        case 1:  ct = -s; st =  c; break;
        case 2:  ct = -c; st = -s; break;
        default: ct =  s; st = -c; break;
    }
    *z_cos = r * ct;
    *z_sin = r * st;
}

/* Four consecutive Gaussian entries minor = 4g .. 4g+3 of (major, stream). */
static void or_gauss4(uint64_t seed, uint32_t stream, uint64_t major,
                      uint32_t group, float z[4])
{
    uint32_t ctr[4] = { (uint32_t)major, group, stream, (uint32_t)(major >> 32) };
    uint32_t key[2] = { (uint32_t)seed, (uint32_t)(seed >> 32) };
    uint32_t x[4];
    oracle_philox4x32_10(ctr, key, x);
    or_box_muller(x[0], x[1], &z[0], &z[1]);
    or_box_muller(x[2], x[3], &z[2], &z[3]);
}

/* One Gaussian entry G(seed, stream, major, minor). */
float oracle_gauss(uint64_t seed, uint32_t stream, uint64_t major, uint64_t minor)
{
    float z[4];
    or_gauss4(seed, stream, major, (uint32_t)(minor >> 2), z);
    return z[minor & 3u];
}

/* out[t + nminor * s] = G(seed, stream, majors[s], minor0 + t)  (minor fastest)
 * majors == NULL means majors[s] = major0 + s. */
void oracle_fill_gaussian(uint64_t seed, uint32_t stream,
                          const int64_t *majors, int64_t major0, int64_t nmajor,
                          int64_t minor0, int64_t nminor, float *out)
{
    #pragma omp parallel for schedule(static)
    for (int64_t s = 0; s < nmajor; ++s) {
        uint64_t major = majors ? (uint64_t)majors[s] : (uint64_t)(major0 + s);
        for (int64_t t = 0; t < nminor; ++t)
            out[t + nminor * s] = oracle_gauss(seed, stream, major, (uint64_t)(minor0 + t));
    }
}

/* ------------------------------------------------------------------------ */
/* 3. Sketches in FP64                                                       */
/* ------------------------------------------------------------------------ */
/*
 * W(r, j) = sum_{s=0}^{Ns-1} Psi(r, s) * A(rows[s], j),   r < lq, j < n
 *   Psi(r, s) = value of G(seed, 1, rows[s], r) in the sketch precision
 *   (supplied by the caller through psi_round: 0 = keep the single value,
 *   otherwise already-rounded values are produced by oracle_round_* below).
 * The sum over s is taken in increasing s, one FP64 product and one FP64
 * addition per term.  A is column-major (lda), given in FP64 (exact copies of
 * FP32 data where the data are FP32).
 *
 * The Gaussian block Psi(:, s0:s1) is generated inside the loop so that Psi
 * never has to be stored whole; blocks are visited in increasing s, so the
 * summation order per entry is unchanged.
 */
typedef double (*or_round_fn)(double);

static double or_round_none(double x) { return x; }

/* round-to-nearest-even to bfloat16 (8 significant bits), via FP32 */
static double or_round_bf16(double x)
{
    float f = (float)x;                       /* data here are FP32-exact */
    uint32_t b = or_to_bits(f);
    if ((b & 0x7F800000u) == 0x7F800000u) return x;   /* inf / nan */
    uint32_t lsb = (b >> 16) & 1u;
    b = (b + 0x7FFFu + lsb) & 0xFFFF0000u;
    return (double)or_from_bits(b);
}

/* round-to-nearest-even to OCP FP8 e4m3fn (3 fraction bits, bias 7,
 * max 448, subnormal step 2^-9), saturating at +-448 */
static double or_round_e4m3(double x)
{
    double ax = fabs(x);
    if (ax == 0.0) return x;
    if (ax >= 448.0) return x < 0 ? -448.0 : 448.0;
    int e;
    (void)frexp(ax, &e);          /* ax = f * 2^e, f in [0.5, 1) */
    int ex = e - 1;               /* ax in [2^ex, 2^(ex+1)) */
    if (ex < -6) ex = -6;         /* subnormal range shares the 2^-9 step */
    double step = ldexp(1.0, ex - 3);
    double q = ax / step;         /* exact: power-of-two scaling */
    double fl = floor(q);
    double rem = q - fl;
    if (rem > 0.5 || (rem == 0.5 && fmod(fl, 2.0) != 0.0)) fl += 1.0;
    double r = fl * step;
    if (r > 448.0) r = 448.0;
    return x < 0 ? -r : r;
}

double oracle_round_bf16(double x) { return or_round_bf16(x); }
double oracle_round_e4m3(double x) { return or_round_e4m3(x); }

void oracle_round_e4m3_array(double *x, int64_t count)
{
    for (int64_t i = 0; i < count; ++i) x[i] = or_round_e4m3(x[i]);
}

static or_round_fn or_pick_round(int mode)
{
    /* 0: FP32 single value as is; 1: bfloat16; 2: e4m3 */
    if (mode == 1) return or_round_bf16;
    if (mode == 2) return or_round_e4m3;
    return or_round_none;
}

void oracle_sketch_w(uint64_t seed, int psi_round,
                     const double *A, int64_t lda, int64_t n,
                     const int64_t *rows, int64_t Ns, int64_t lq,
                     double *W /* lq x n, column-major, overwritten */)
{
    or_round_fn rnd = or_pick_round(psi_round);
    const int64_t BLK = 2048;
    double *psi = (double *)malloc(sizeof(double) * (size_t)(lq * BLK));
    float *tmp = (float *)malloc(sizeof(float) * (size_t)(lq * BLK));
    memset(W, 0, sizeof(double) * (size_t)(lq * n));
    for (int64_t s0 = 0; s0 < Ns; s0 += BLK) {
        int64_t nb = (Ns - s0 < BLK) ? (Ns - s0) : BLK;
        oracle_fill_gaussian(seed, 1u, rows + s0, 0, nb, 0, lq, tmp);
        for (int64_t t = 0; t < lq * nb; ++t) psi[t] = rnd((double)tmp[t]);
        #pragma omp parallel for schedule(static)
        for (int64_t j = 0; j < n; ++j) {
            double *wj = W + lq * j;
            for (int64_t s = 0; s < nb; ++s) {
                double a = A[rows[s0 + s] + lda * j];
                const double *ps = psi + lq * s;
                for (int64_t r = 0; r < lq; ++r) {
                    double prod = ps[r] * a;
                    wj[r] = wj[r] + prod;
                }
            }
        }
    }
    free(tmp);
    free(psi);
}

/*
 * Y(i, c) = sum_{j=0}^{n-1} A(i, j) * Omega(j, c),  i < N, c < l
 * Omega is row-major n x l (Omega(j, c) at j*l + c); Y is row-major N x l.
 * The sum over j is taken in increasing j.
 */
void oracle_sketch_y(const double *A, int64_t lda, int64_t N, int64_t n,
                     const double *Omega, int64_t l, double *Y)
{
    const int64_t RB = 64;
    #pragma omp parallel for schedule(static)
    for (int64_t i0 = 0; i0 < N; i0 += RB) {
        int64_t i1 = (i0 + RB < N) ? i0 + RB : N;
        for (int64_t i = i0; i < i1; ++i)
            for (int64_t c = 0; c < l; ++c) Y[i * l + c] = 0.0;
        for (int64_t j = 0; j < n; ++j) {
            const double *om = Omega + l * j;
            for (int64_t i = i0; i < i1; ++i) {
                double a = A[i + lda * j];
                double *yi = Y + i * l;
                for (int64_t c = 0; c < l; ++c) {
                    double prod = a * om[c];
                    yi[c] = yi[c] + prod;
                }
            }
        }
    }
}

/* ------------------------------------------------------------------------ */
/* 4. Error norms of a column ID, evaluated entry by entry                   */
/* ------------------------------------------------------------------------ */
/*
 * Ahat(i, j) = sum_{t<k} AJ(i, t) P(t, j)  (AJ column-major N x k, P k x n).
 * out[0] = sum (A - Ahat)^2, out[1] = sum A^2,
 * out[2] = max |A - Ahat| / |A| over A != 0 (relative max error of Sec. 3.1),
 * out[3] = max |A - Ahat|.
 */
void oracle_error_norms(const double *A, int64_t lda, const double *AJ, int64_t ldaj,
                        const double *P, int64_t ldp, int64_t N, int64_t k, int64_t n,
                        double out[4])
{
    double se = 0.0, sa = 0.0, mrel = 0.0, mabs = 0.0;
    #pragma omp parallel for schedule(static) reduction(+:se,sa) reduction(max:mrel,mabs)
    for (int64_t j = 0; j < n; ++j) {
        for (int64_t i = 0; i < N; ++i) {
            double ah = 0.0;
            for (int64_t t = 0; t < k; ++t) ah = ah + AJ[i + ldaj * t] * P[t + ldp * j];
            double a = A[i + lda * j];
            double d = a - ah;
            se += d * d;
            sa += a * a;
            double ad = fabs(d);
            if (ad > mabs) mabs = ad;
            if (a != 0.0) {
                double rel = ad / fabs(a);
                if (rel > mrel) mrel = rel;
            }
        }
    }
    out[0] = se; out[1] = sa; out[2] = mrel; out[3] = mabs;
}
