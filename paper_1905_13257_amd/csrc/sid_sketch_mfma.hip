// sid_sketch_mfma.hip -- the sketch pass as one streaming read of A on the
// gfx950 matrix cores (bfloat16 MFMA, FP32 accumulation).
//
// One pass over A forms both sketches of the single-pass ID:
//   W = Psi A   ((lq x n), the Gaussian sketch whose first l rows select the
//               skeleton, Alg. 4 "Y <- A Omega" in the paper's row orientation)
//   Y = A Omega (N x l, the range sketch of the two-sided single-pass sketch,
//               Halko et al. Sec. 5.5 items (1)-(2), quoted in Sec. 2.3).
//
// Layout of the work.  One persistent 512-thread workgroup per CU (two waves
// per SIMD, 256 registers each, so that one wave's matrix products overlap
// the other's loads, conversions and Gaussian generation) owns a contiguous
// range of rows of A and walks it in panels of 64 rows.  A panel is consumed
// in chunks of 128 columns; wave w owns columns 16w .. 16w+15 of every chunk.
//   * Loads: each lane fetches 16 FP32 values of one column: four 64-byte
//     runs per column, 256 contiguous bytes per column and chunk.  The loads
//     of chunk c+1 are issued as soon as chunk c has been split into bf16,
//     so they are in flight during chunk c's matrix products.
//   * W(:, chunk) += Psi(:, panel) A(panel, chunk): the B operand comes
//     straight from registers (hi and, in the split form, lo bf16 parts).
//     The W partial of the whole row range stays on chip: W rows 0..127 in
//     accumulators (8 tiles x 4 chunks x 4 = 128 registers per lane), rows
//     128..lq-1 in an LDS array to which each chunk's product is added.
//   * The same bf16 values are written transposed into a row-major chunk
//     buffer in LDS; after a barrier each wave forms Y(panel, its tiles) +=
//     A(panel, chunk) Omega(chunk, :) with Omega^T (bf16) read through L2.
//     The Y accumulators cover the panel and are stored after its last chunk.
//   * Psi(:, next panel) is generated (Philox + Box-Muller, bf16) into the
//     other half of a double-buffered LDS array, one slice per chunk.
// The W partial of each workgroup is written once at the end (FP32) and the
// partials are summed in a fixed order in FP64 by k_reduce_partials_f32.
//
// MFMA operand layouts used (v_mfma_f32_16x16x32_bf16, wave64):
//   A (16 x 32): lane l holds row l%16, k = 8*(l/16) .. +7
//   B (32 x 16): lane l holds col l%16, k = 8*(l/16) .. +7
//   C (16 x 16): lane l holds col l%16, rows 4*(l/16) .. +3
// The contraction of W runs over panel rows in a permuted order: within a
// 32-row step, operand slot 8g+i (g = l/16) holds row 4g+i for i < 4 and row
// 16+4g+(i-4) for i >= 4, which makes every load instruction read 64
// contiguous bytes per column.  Psi is stored in LDS in the same slot order,
// so the products pair up as in the plain order.
#include <type_traits>

#include "sid_kernels.hpp"

namespace sid {

typedef __bf16 bf16x8_t __attribute__((ext_vector_type(8)));
typedef float f32x4_t __attribute__((ext_vector_type(4)));

constexpr int FB_WAVES = 8;                  // two waves per SIMD
constexpr int FB_THREADS = 64 * FB_WAVES;
constexpr int FB_PR = 64;                    // rows per panel (two K steps of 32)
constexpr int FB_CHUNK = 16 * FB_WAVES;      // columns per chunk
constexpr int FB_NCH = 4;                    // max chunks
constexpr int FB_NPAD = FB_CHUNK * FB_NCH;   // 512: max columns
constexpr int FB_KS = FB_CHUNK / 32;         // K steps of the Y product per chunk
constexpr int FB_CROW = FB_CHUNK + 8;        // LDS row stride of a chunk (bf16)
constexpr int FB_PROW = FB_PR + 8;           // LDS row stride of Psi (bf16)
constexpr int FB_MTR = 8;                    // W row tiles kept in registers

__device__ __forceinline__ __bf16 to_bf16(float f) { return (__bf16)f; }

__global__ void k_zero_queue(unsigned int* q) {
  if (threadIdx.x < FB_NCLASS) q[threadIdx.x] = 0u;
}

// panel row of operand slot (ks, g, i)
__device__ __forceinline__ int slot_row(int ks, int g, int i) {
  return 32 * ks + (i < 4 ? 4 * g + i : 16 + 4 * g + (i - 4));
}
// operand slot of panel row r
__device__ __forceinline__ int row_slot(int r) {
  const int q = r & 31;
  return (r & ~31) + 8 * ((q & 15) >> 2) + (q & 3) + 4 * (q >> 4);
}

// Chunk loads of one wave: lane (col lr, group lg) gets slots 0..15 of its
// column (K steps 0 and 1).  pc = A + (first row of the panel); col is this
// lane's column.  Columns at or beyond n read column n-1; the caller zeroes
// them when it converts (a select here would wait for the load at once).
__device__ __forceinline__ const float* chunk_col(const float* pc, int64_t lda, int n, int col,
                                                  int lg) {
  int colc = col < n ? col : n - 1;
  // opaque: the 64-bit column offsets would otherwise be hoisted out of the
  // panel loop (two registers per chunk); recomputing one is two
  // multiply-adds
  asm volatile("" : "+v"(colc));
  return pc + (int64_t)colc * lda + 4 * lg;
}

// full panel: four 16-byte loads per lane, slot 4h+t = row 16h + 4lg + t
__device__ __forceinline__ void load_chunk(const float* __restrict__ pc, int64_t lda, int n, int col,
                                           int lg, float (&v)[16]) {
  typedef const __attribute__((address_space(1))) f32x4_t* gptr4;
  const float* base = chunk_col(pc, lda, n, col, lg);
#pragma unroll
  for (int h = 0; h < 4; ++h) {
    const f32x4_t a = __builtin_nontemporal_load((gptr4)(base + 16 * h));
#pragma unroll
    for (int t = 0; t < 4; ++t) v[4 * h + t] = a[t];
  }
}

// ragged tail panel (rows_left < 64 rows exist): rows past the end read the
// last row and are zeroed
__device__ __forceinline__ void load_chunk_tail(const float* __restrict__ pc, int64_t lda, int n,
                                                int col, int rows_left, int lg, float (&v)[16]) {
  typedef const __attribute__((address_space(1))) float* gptr;
  const gptr base = (gptr)(chunk_col(pc, lda, n, col, lg) - 4 * lg);
#pragma unroll
  for (int h = 0; h < 4; ++h)
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      const int r = 16 * h + 4 * lg + t;
      const bool ok = r < rows_left;
      const float x = base[ok ? r : rows_left - 1];
      v[4 * h + t] = ok ? x : 0.0f;
    }
}

// Chunk loads through a row list (coarse rows S, Alg. 5): slot 4h + t of the
// lane is row sr[16h + 4lg + t] of A; rows at or past rows_left read the last
// listed row and are zeroed.
__device__ __forceinline__ void load_chunk_rows(const float* __restrict__ A, int64_t lda, int n,
                                                int col, const int64_t* sr, int rows_left, int lg,
                                                float (&v)[16]) {
  typedef const __attribute__((address_space(1))) float* gptr;
  int colc = col < n ? col : n - 1;
  asm volatile("" : "+v"(colc));
  const gptr base = (gptr)(A + (int64_t)colc * lda);
#pragma unroll
  for (int h = 0; h < 4; ++h)
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      const int r = 16 * h + 4 * lg + t;
      const bool ok = r < rows_left;
      const float x = base[sr[ok ? r : rows_left - 1]];
      v[4 * h + t] = ok ? x : 0.0f;
    }
}

// Items [i0, i1) of Psi(0:lq, panel p0): item w covers panel row w % 64 and
// rows 4*(w/64) .. +3 of Psi.  Written in operand-slot order.
template <bool FP8>
__device__ __forceinline__ void gen_psi(__bf16* __restrict__ s_psi, uint64_t seed, int64_t p0,
                                        int64_t r1, int lq, int i0, int i1, int tid,
                                        const int64_t* sr = nullptr) {
  // opaque thread index: the start items of the slices would otherwise be
  // hoisted out of the panel loop and pin registers
  asm volatile("" : "+v"(tid));
#pragma unroll 1
  for (int w = i0 + tid; w < i1; w += FB_THREADS) {
    const int kk = w & (FB_PR - 1), g = w / FB_PR;
    float z[4] = {0.f, 0.f, 0.f, 0.f};
    // Psi is keyed by the global row of A (the coarse row list when given)
    if (p0 + kk < r1) gauss4(seed, 1u, (uint64_t)(sr ? sr[kk] : p0 + kk), (uint32_t)g, z);
    const int pos = row_slot(kk);
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int m = 4 * g + e;
      if (m < lq) s_psi[m * FB_PROW + pos] = to_bf16(FP8 ? e4m3_value(z[e]) : z[e]);
    }
  }
}

// DM: how the data enter the products (FB_BF16: bf16(a); FB_BF16X2: hi + lo;
// FB_FP8: the e4m3 value of a scaled by its tile's power of two, which is a
// bfloat16 value, so the bf16 products are exact).
// MT: 16-row tiles of W (lq <= 16*MT); LT: 16-column tiles of Y (l <= 16*LT);
// NCH: chunks of 128 columns per panel (n <= 128*NCH); WANTY: form Y.
// Every count that shapes the register state is a template argument, so the
// chunk loop unrolls into straight-line code with no merges of accumulators.
// ROWS: W = Psi(:, S) A(S, :) over the coarse row list `rows` (N = |S|; two
// pass only, no Y); the list of each panel is staged in LDS.
//
// fused_tile: one workgroup's share, rows [r0, r1) of A, whose W partial
// (FP32, column-major lq x n) goes to dst.  nch (<= NCH) chunks are
// processed: chunks past the last column are skipped whole, so the template
// counts only bound the register state and the results do not depend on
// them.  The single-matrix kernel runs one share per workgroup; the batched
// kernel runs shares of many matrices from a work queue.
template <int DM, bool WANTY, int MT, int LT, int NCH, bool ROWS, bool GUARDS = false>
__device__ __forceinline__ void fused_tile(
    const float* __restrict__ A, int64_t lda, int64_t N, int n, int lq, int l, uint64_t seed,
    const __bf16* __restrict__ omT /* LT*16 x FB_NPAD, k contiguous, zero padded */,
    const int64_t r0, int64_t r1, const int nch, float* __restrict__ dst, float* __restrict__ Y,
    const int64_t* __restrict__ rows) {
  static_assert(!(ROWS && WANTY), "a row list sketches W only");
  static_assert(FB_WAVES % LT == 0 || LT % FB_WAVES == 0, "Y tiles split evenly over the waves");
  static_assert(4 * LT >= FB_WAVES && NCH <= FB_NCH, "tile counts");
  // Y tiles of a panel: 4 row tiles x LT column tiles; wave w owns column
  // tile w % LT and YR row tiles from rt0 = (w / LT) YR
  constexpr int YR = 4 * LT / FB_WAVES;
  constexpr bool SPLIT = DM == FB_BF16X2;
  constexpr bool FP8 = DM == FB_FP8;
  constexpr int NH = SPLIT ? 2 : 1;               // bf16 terms per value
  constexpr int MTR = MT < FB_MTR ? MT : FB_MTR;  // W row tiles in registers
  constexpr int MTX = MT - MTR;                   // W row tiles accumulated in LDS
  __shared__ __attribute__((aligned(16))) __bf16 s_psi[2][MT * 16 * FB_PROW];
  __shared__ __attribute__((aligned(16))) __bf16 s_chk[NH][FB_PR * FB_CROW];
  // W rows 16 MTR .. 16 MT - 1, in C-fragment order: [mtx][chunk][wave][lane][4]
  __shared__ __attribute__((aligned(16))) float s_wx[MTX > 0 ? MTX * NCH * FB_THREADS * 4 : 4];
  __shared__ int64_t s_rows[2][ROWS ? FB_PR : 1];  // row lists of this and the next panel

  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int lr = lane & 15, lg = lane >> 4;  // MFMA lane coordinates
  const int lq4 = (lq + 3) >> 2;
  // GUARDS (the batched kernel: a smaller matrix on the largest layout):
  // row tiles of W past the rows below lq only feed rows that are never
  // stored, and are skipped
  const int mt_live = GUARDS ? (lq + 15) >> 4 : MT;
  const int gen_items = FB_PR * lq4;
  // wave 0 stages the row list of the panel starting at q0 (clamped to r1)
  auto stage_rows = [&](int64_t q0, int buf) {
    if constexpr (ROWS) {
      if (tid < FB_PR && q0 < r1) {
        const int64_t q = q0 + tid < r1 ? q0 + tid : r1 - 1;
        s_rows[buf][tid] = rows[q];
      }
    }
  };

  // Psi rows >= lq stay zero for the whole kernel; the LDS part of W starts
  // at zero
  for (int e = tid; e < 2 * MT * 16 * FB_PROW; e += FB_THREADS) (&s_psi[0][0])[e] = to_bf16(0.0f);
  if constexpr (MTX > 0)
    for (int e = tid; e < MTX * NCH * FB_THREADS * 4; e += FB_THREADS) s_wx[e] = 0.0f;

  f32x4_t wacc[MTR][NCH];
#pragma unroll
  for (int mt = 0; mt < MTR; ++mt)
#pragma unroll
    for (int j = 0; j < NCH; ++j) wacc[mt][j] = f32x4_t{0.f, 0.f, 0.f, 0.f};
  f32x4_t yacc[YR];
#pragma unroll
  for (int r = 0; r < YR; ++r) yacc[r] = f32x4_t{0.f, 0.f, 0.f, 0.f};
  const int yc = wave % LT, rt0 = (wave / LT) * YR;
  const bool y_live = true;  // (a Y guard as well spilled registers)

  // full panels end at r1f; a ragged tail panel [r1f, r1) is handled last
  const int64_t r1f = r0 + ((r1 - r0) / FB_PR) * FB_PR;
  const int col_w = 16 * wave + lr;  // this lane's column within a chunk
  float v[16];                       // this wave's slice of the chunk in flight
  if constexpr (ROWS) {
    stage_rows(r0, 0);
    lds_barrier();  // zeroed Psi and the first row list visible
    if (r0 < r1f) load_chunk_rows(A, lda, n, col_w, s_rows[0], FB_PR, lg, v);
    if (r0 < r1) gen_psi<FP8>(s_psi[0], seed, r0, r1, lq, 0, gen_items, tid, s_rows[0]);
  } else {
    if (r0 < r1f) load_chunk(A + r0, lda, n, col_w, lg, v);
    lds_barrier();  // zeroed Psi visible
    if (r0 < r1) gen_psi<FP8>(s_psi[0], seed, r0, r1, lq, 0, gen_items, tid);
  }

  // per-lane offset of this lane's Omega^T fragments (bf16 elements)
  const uint32_t om_lane = (uint32_t)((yc * 16 + lr) * FB_NPAD + 8 * lg);
  typedef const __attribute__((address_space(1))) __bf16* gbf16p;
  typedef const __attribute__((address_space(1))) bf16x8_t* gbf16x8p;

  // One panel of FB_PR rows starting at p0 (Psi in buffer pb).  TAIL: the
  // ragged last panel with `rows` < FB_PR rows; its chunks are loaded on the
  // spot and nothing is prefetched.  Otherwise v holds chunk 0 on entry and
  // the first chunk of the next full panel on exit.
  auto panel = [&](auto tail_tag, int64_t p0, int pb) {
    constexpr bool TAIL = decltype(tail_tag)::value;
    const int64_t pn = p0 + FB_PR;
    const int rows = TAIL ? (int)(r1 - p0) : FB_PR;
    const __bf16* psi = s_psi[pb];
#pragma unroll
    for (int j = 0; j < NCH; ++j) {
      if (j >= nch) break;  // uniform over the workgroup
      const bool col_ok = col_w + FB_CHUNK * j < n;
      if constexpr (TAIL) {
        if constexpr (ROWS) load_chunk_rows(A, lda, n, col_w + FB_CHUNK * j, s_rows[pb], rows, lg, v);
        else load_chunk_tail(A + p0, lda, n, col_w + FB_CHUNK * j, rows, lg, v);
      }
      // the next panel's row list goes into the other buffer, whose last
      // readers (the loads of this panel's chunks) finished before the
      // previous panel's last barrier
      if (!TAIL && j == 0) stage_rows(pn, pb ^ 1);
      // the previous chunk's Y reads are done (and, at the start of a
      // panel, its Psi is complete)
      lds_barrier();
      // (1) Omega^T fragments of this chunk.  They are issued before the
      //     next chunk's loads, so that waiting for them never waits for
      //     those (vmcnt counts in issue order).  Omega^T is the same for
      //     every panel; the opaque copy of its address keeps the compiler
      //     from hoisting the fragments of all chunks out of the loop.
      bf16x8_t of[FB_KS];
      if (WANTY && y_live) {
        uintptr_t om_addr = (uintptr_t)omT;
        asm volatile("" : "+s"(om_addr));
        const gbf16p om = (gbf16p)om_addr;
#pragma unroll
        for (int ks = 0; ks < FB_KS; ++ks)
          of[ks] = *(gbf16x8p)(om + (om_lane + (uint32_t)(FB_CHUNK * j + 32 * ks)));
      }
      // (2) split into bf16 hi (+ lo) B operands and the transposed copy
      //     (FP8: the column's 64-row tile scale from the four lanes that
      //     hold it)
      float fs = 1.0f, fsi = 1.0f;
      if constexpr (FP8) {
        float amax = 0.0f;
#pragma unroll
        for (int i = 0; i < 16; ++i) amax = fmaxf(amax, fabsf(v[i]));
        amax = fmaxf(amax, __shfl_xor(amax, 16, 64));
        amax = fmaxf(amax, __shfl_xor(amax, 32, 64));
        fs = fp8_tile_scale(amax, fsi);
      }
      bf16x8_t bh[2], bl[2];
#pragma unroll
      for (int ks = 0; ks < 2; ++ks)
#pragma unroll
        for (int i = 0; i < 8; ++i) {
          float x = col_ok ? v[8 * ks + i] : 0.0f;
          if constexpr (FP8) x = e4m3_value(x * fsi) * fs;
          const __bf16 h = to_bf16(x);
          bh[ks][i] = h;
          const int ci = slot_row(ks, lg, i) * FB_CROW + col_w;
          if constexpr (WANTY) s_chk[0][ci] = h;
          if constexpr (SPLIT) {
            const __bf16 lo = to_bf16(x - (float)h);
            bl[ks][i] = lo;
            if constexpr (WANTY) s_chk[NH - 1][ci] = lo;
          }
        }
      // (3) the next chunk's loads: in flight during the products, the Psi
      //     slice and the Y product below
      __builtin_amdgcn_sched_barrier(0);
      if constexpr (!TAIL) {
        if constexpr (ROWS) {
          if (j + 1 < nch)
            load_chunk_rows(A, lda, n, col_w + FB_CHUNK * (j + 1), s_rows[pb], FB_PR, lg, v);
          else if (pn < r1f)
            load_chunk_rows(A, lda, n, col_w, s_rows[pb ^ 1], FB_PR, lg, v);
        } else {
          if (j + 1 < nch) {
            load_chunk(A + p0, lda, n, col_w + FB_CHUNK * (j + 1), lg, v);
          } else if (pn < r1f) {
            load_chunk(A + pn, lda, n, col_w, lg, v);
          }
        }
      }
      __builtin_amdgcn_sched_barrier(0);
      // (4) W(:, chunk) += Psi(:, panel) A(panel, chunk)
#pragma unroll
      for (int ks = 0; ks < 2; ++ks)
#pragma unroll
        for (int mt = 0; mt < MTR; ++mt) {
          if (mt >= mt_live) continue;
          const bf16x8_t af =
              *reinterpret_cast<const bf16x8_t*>(&psi[(mt * 16 + lr) * FB_PROW + 32 * ks + 8 * lg]);
          wacc[mt][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af, bh[ks], wacc[mt][j], 0, 0, 0);
          if constexpr (SPLIT)
            wacc[mt][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af, bl[ks], wacc[mt][j], 0, 0, 0);
        }
      if (MTX > 0 && mt_live > MTR) {
#pragma unroll
        for (int mx = 0; mx < MTX; ++mx) {
          f32x4_t* wx = reinterpret_cast<f32x4_t*>(&s_wx[(((mx * NCH + j) * FB_WAVES + wave) * 64 + lane) * 4]);
          f32x4_t acc = f32x4_t{0.f, 0.f, 0.f, 0.f};
#pragma unroll
          for (int ks = 0; ks < 2; ++ks) {
            const bf16x8_t af = *reinterpret_cast<const bf16x8_t*>(
                &psi[((MTR + mx) * 16 + lr) * FB_PROW + 32 * ks + 8 * lg]);
            acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af, bh[ks], acc, 0, 0, 0);
            if constexpr (SPLIT) acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af, bl[ks], acc, 0, 0, 0);
          }
          *wx += acc;
        }
      }
      // (5) slice j of Psi(:, next panel) (the buffer the previous panel used)
      if (!TAIL && pn < r1)
        gen_psi<FP8>(s_psi[pb ^ 1], seed, pn, r1, lq, gen_items * j / nch, gen_items * (j + 1) / nch,
                     tid, ROWS ? s_rows[pb ^ 1] : nullptr);
      lds_barrier();  // chunk buffer complete
      // (6) Y(panel, this wave's tiles) += A(panel, chunk) Omega(chunk, :)
      if (WANTY && y_live) {
#pragma unroll
        for (int ks = 0; ks < FB_KS; ++ks) {
#pragma unroll
          for (int r = 0; r < YR; ++r) {
            const int ci = ((rt0 + r) * 16 + lr) * FB_CROW + 32 * ks + 8 * lg;
            const bf16x8_t ah = *reinterpret_cast<const bf16x8_t*>(&s_chk[0][ci]);
            yacc[r] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, of[ks], yacc[r], 0, 0, 0);
            if constexpr (SPLIT) {
              const bf16x8_t al = *reinterpret_cast<const bf16x8_t*>(&s_chk[NH - 1][ci]);
              yacc[r] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al, of[ks], yacc[r], 0, 0, 0);
            }
          }
        }
      }
    }
    // Y(panel, this wave's tiles)
    if constexpr (WANTY) {
      // opaque 4lg: keeps the 64-bit row offsets from being hoisted out of
      // the panel loop
      int lg4 = 4 * lg;
      asm volatile("" : "+v"(lg4));
      // global (not flat) stores: the batched kernel's pointers come from
      // its table, and flat stores would also count in the LDS counter
      typedef __attribute__((address_space(1))) float* gfp;
      const gfp yp = (gfp)(Y + p0 * (int64_t)l);
      const int c = yc * 16 + lr;
#pragma unroll
      for (int r = 0; r < YR; ++r) {
#pragma unroll
        for (int t = 0; t < 4; ++t) {
          const int rr = (rt0 + r) * 16 + lg4 + t;
          if (c < l && (!TAIL || rr < rows)) yp[rr * l + c] = yacc[r][t];
        }
        yacc[r] = f32x4_t{0.f, 0.f, 0.f, 0.f};
      }
    }
  };

  int pb = 0;  // Psi buffer of the current panel
  int64_t p0 = r0;
  for (; p0 < r1f; p0 += FB_PR, pb ^= 1) panel(std::false_type{}, p0, pb);
  if (p0 < r1) panel(std::true_type{}, p0, pb);

  // W partial of this share (FP32, column-major lq x n)
#pragma unroll
  for (int j = 0; j < NCH; ++j) {
    const int col = FB_CHUNK * j + col_w;
    if (col >= n) continue;
#pragma unroll
    for (int mt = 0; mt < MT; ++mt) {
      f32x4_t w4;
      if (mt < MTR) {
        w4 = wacc[mt < MTR ? mt : 0][j];
      } else {
        w4 = *reinterpret_cast<const f32x4_t*>(
            &s_wx[((((mt - MTR) * NCH + j) * FB_WAVES + wave) * 64 + lane) * 4]);
      }
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        const int m = mt * 16 + 4 * lg + t;
        if (m < lq) ((__attribute__((address_space(1))) float*)dst)[m + (int64_t)lq * col] = w4[t];
      }
    }
  }
}

template <int DM, bool WANTY, int MT, int LT, int NCH, bool ROWS = false>
__global__ __launch_bounds__(FB_THREADS) void k_sketch_fused_bf16(
    const float* __restrict__ A, int64_t lda, int64_t N, int n, int lq, int l, uint64_t seed,
    const __bf16* __restrict__ omT, int64_t rows_per_wg, float* __restrict__ part /* grid x lq x n */,
    float* __restrict__ Y, const int64_t* __restrict__ rows = nullptr) {
  const int64_t r0 = (int64_t)blockIdx.x * rows_per_wg;
  const int64_t r1 = r0 + rows_per_wg < N ? r0 + rows_per_wg : N;
  fused_tile<DM, WANTY, MT, LT, NCH, ROWS>(A, lda, N, n, lq, l, seed, omT, r0, r1,
                                           (n + FB_CHUNK - 1) / FB_CHUNK,
                                           part + (int64_t)blockIdx.x * lq * n, Y, rows);
}

// ---------------------------------------------------------------------------
// Batched sketch pass: many independent matrices in one persistent launch.
// The shares of all matrices (each matrix cut into the row ranges the
// single-matrix launch gives its workgroups, so every partial, and with the
// same fixed-order sum W and Y, is bit for bit that of a single-matrix call)
// form one work queue, in the order of the table (the host puts the
// matrices with the most work per share first), one queue per layout class:
// the matrices whose W rows and Y columns fit a smaller register layout
// (fused_bf16_batch_class) run in their own launch, beside the others on
// another stream.  A workgroup takes the next share of its class with one
// atomic increment and runs it with the class's layout (MT, LT) and NCH =
// 4; a share of a smaller matrix skips the chunks past its columns, and the
// row tiles of W and column tiles of Y past its sizes only compute zeros
// that are never stored.  Every workgroup leaves when its queue is empty.
// ---------------------------------------------------------------------------
template <int DM, bool WANTY, int MT, int LT>
__global__ __launch_bounds__(FB_THREADS) void k_sketch_fused_bf16_batch(
    const FbBatchEntry* __restrict__ tab, int count, int64_t nshares,
    unsigned int* __restrict__ queue) {
  __shared__ int64_t s_share;
  for (;;) {
    lds_barrier();  // the previous share is done with the LDS (and s_share)
    if (threadIdx.x == 0) s_share = (int64_t)atomicAdd(queue, 1u);
    lds_barrier();
    const int64_t t = s_share;
    if (t >= nshares) break;
    // the matrix: the last entry whose first share is <= t
    int lo = 0, hi = count - 1;
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (tab[mid].share0 <= t) lo = mid;
      else hi = mid - 1;
    }
    const FbBatchEntry& e = tab[lo];
    const int64_t i = t - e.share0;
    const int64_t r0 = i * e.rows_per_wg;
    const int64_t r1 = r0 + e.rows_per_wg < e.N ? r0 + e.rows_per_wg : e.N;
    fused_tile<DM, WANTY, MT, LT, FB_NCH, false, true>(e.A, e.lda, e.N, e.n, e.lq, e.l, e.seed, e.omT, r0,
                                                r1, (e.n + FB_CHUNK - 1) / FB_CHUNK,
                                                e.part + i * e.lq * e.n, WANTY ? e.Y : nullptr,
                                                nullptr);
  }
}

// Omega's values (n x l, row-major: the single-matrix layout) and Omega^T in
// bfloat16 with 128 zero-padded rows (the batched kernel's Y tiles) for every
// matrix (blockIdx.y); the queue counters are cleared by block (0, 0).  Both
// come from the same generator call, so they are the values the
// single-matrix path forms.
__global__ void k_batch_omega(const FbBatchEntry* __restrict__ tab, int dm_fp8,
                              unsigned int* __restrict__ queue) {
  const FbBatchEntry& e = tab[blockIdx.y];
  if (blockIdx.x == 0 && blockIdx.y == 0 && threadIdx.x < FB_NCLASS) queue[threadIdx.x] = 0u;
  const int ng = (e.l + 3) >> 2;
  for (int w = blockIdx.x * blockDim.x + threadIdx.x; w < e.n * ng; w += gridDim.x * blockDim.x) {
    const int k = w / ng, g = w - k * ng;
    float z[4];
    gauss4(e.seed, 0u, (uint64_t)k, (uint32_t)g, z);
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int c = 4 * g + u;
      if (c < e.l) {
        e.omega[(int64_t)k * e.l + c] = z[u];
        e.omT[c * FB_NPAD + k] = to_bf16(dm_fp8 ? e4m3_value(z[u]) : z[u]);
      }
    }
  }
  // the zero padding of Omega^T: columns k >= n of rows c < l, rows l .. 127
  for (int e2 = blockIdx.x * blockDim.x + threadIdx.x; e2 < 128 * FB_NPAD; e2 += gridDim.x * blockDim.x) {
    const int c = e2 / FB_NPAD, k = e2 - c * FB_NPAD;
    if (c >= e.l || k >= e.n) e.omT[e2] = to_bf16(0.0f);
  }
}

// W of every matrix (blockIdx.y): the fixed-order FP64 sum of its partials,
// the order of k_reduce_partials_f32
__global__ void k_reduce_partials_batch(const FbBatchEntry* __restrict__ tab) {
  const FbBatchEntry& m = tab[blockIdx.y];
  const int64_t count = (int64_t)m.lq * m.n;
  const int64_t nparts = m.nshares;
  // global (not flat) accesses through the table's pointers
  const __attribute__((address_space(1))) float* __restrict__ part =
      (const __attribute__((address_space(1))) float*)m.part;
  __attribute__((address_space(1))) double* Wm = (__attribute__((address_space(1))) double*)m.W;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < count;
       e += (int64_t)gridDim.x * blockDim.x) {
    double s[8] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    int64_t g = 0;
    for (; g + 8 <= nparts; g += 8)
#pragma unroll
      for (int u = 0; u < 8; ++u) s[u] += (double)part[(g + u) * count + e];
    for (; g < nparts; ++g) s[0] += (double)part[g * count + e];
    Wm[e] = ((s[0] + s[1]) + (s[2] + s[3])) + ((s[4] + s[5]) + (s[6] + s[7]));
  }
}

bool fused_bf16_batch_supported(int64_t n, int lq, int l, int64_t lda, const void* A) {
  return n >= 1 && n <= FB_NPAD && lq <= 160 && l <= 128 && (lda % 4) == 0 &&
         ((uintptr_t)A % 16) == 0;
}

int fused_bf16_batch_class(int lq, int l, bool want_y) {
  if (!want_y) return 0;
  return lq <= 64 ? 2 : l <= 64 ? 1 : 0;
}

hipError_t launch_sketch_batch_setup(hipStream_t st, int dmode, bool want_y,
                                     const FbBatchEntry* d_tab, int count, int max_n,
                                     unsigned int* queue) {
  if (count < 1) return hipSuccess;
  if (want_y) {
    const unsigned bx = (unsigned)((max_n * 32 + 255) / 256 < 64 ? (max_n * 32 + 255) / 256 : 64);
    hipLaunchKernelGGL(k_batch_omega, dim3(bx < 1 ? 1 : bx, (unsigned)count), dim3(256), 0, st, d_tab,
                       dmode == FB_FP8 ? 1 : 0, queue);
  } else {
    hipLaunchKernelGGL(k_zero_queue, dim3(1), dim3(64), 0, st, queue);
  }
  return hipGetLastError();
}

hipError_t launch_sketch_batch_class(hipStream_t st, int dmode, bool want_y,
                                     const FbBatchEntry* d_tab, const FbBatchClass& k,
                                     unsigned int* queue, int num_cu) {
  if (k.count < 1 || k.nshares < 1) return hipSuccess;
  if (k.cls < 0 || k.cls >= FB_NCLASS || (!want_y && k.cls != 0)) return hipErrorInvalidValue;
  const int64_t g64 = k.nshares < num_cu ? k.nshares : num_cu;
  const dim3 grid((unsigned)g64), block(FB_THREADS);
  const FbBatchEntry* tab = d_tab + k.first;
  unsigned int* q = queue + k.cls;
#define SID_FB_BATCH(DM_, WY_, MT_, LT_)                                                       \
  hipLaunchKernelGGL((k_sketch_fused_bf16_batch<DM_, WY_, MT_, LT_>), grid, block, 0, st, tab, \
                     k.count, k.nshares, q)
#define SID_FB_BATCH_Y(DM_)                            \
  if (!want_y) SID_FB_BATCH(DM_, false, 10, 8);        \
  else if (k.cls == 0) SID_FB_BATCH(DM_, true, 10, 8); \
  else if (k.cls == 1) SID_FB_BATCH(DM_, true, 10, 4); \
  else SID_FB_BATCH(DM_, true, 4, 4);
  if (dmode == FB_BF16X2) {
    SID_FB_BATCH_Y(FB_BF16X2)
  } else if (dmode == FB_FP8) {
    SID_FB_BATCH_Y(FB_FP8)
  } else {
    SID_FB_BATCH_Y(FB_BF16)
  }
#undef SID_FB_BATCH_Y
#undef SID_FB_BATCH
  return hipGetLastError();
}

hipError_t launch_reduce_partials_batch(hipStream_t st, const FbBatchEntry* d_tab, int count,
                                        int64_t max_lqn) {
  if (count < 1) return hipSuccess;
  int64_t bx = (max_lqn + 255) / 256;
  if (bx > 256) bx = 256;
  hipLaunchKernelGGL(k_reduce_partials_batch, dim3((unsigned)bx, (unsigned)count), dim3(256), 0, st,
                     d_tab);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// The FP32 sketch pass ("FP32 plain": FP32 data, Gaussians and products,
// FP32 accumulation within a workgroup, FP64 across) on the FP32 matrix
// instruction v_mfma_f32_16x16x4_f32 (K = 4).  The work layout is the one
// of the bf16 pass above, with 32-row panels (eight K steps of 4) so that
// Psi in FP32 fits LDS twice:
//   A (16 x 4): lane l holds row l%16, k = l/16;  B (4 x 16): col l%16,
//   k = l/16;  C as above.
// W: the K order within a panel is permuted so that K step s = 4h + t pairs
// lane group g with panel row 16h + 4g + t: a lane's two 16-byte loads
// (rows 16h + 4g .. +3 of its column) are exactly its B operands.  Psi is
// stored in LDS in slot order 4s + g.
// Y: the chunk is written to LDS row-major in FP32; the B operand (Omega)
// comes from a copy of Omega^T whose k index is permuted per chunk so that a
// lane's 32 values for the chunk's 32 K steps are contiguous
// (omP[c][128 j + 32 g + s] = Omega(128 j + 4 s + g, c)).
// ---------------------------------------------------------------------------
constexpr int F3_PR = 32;                    // rows per panel
constexpr int F3_KSW = F3_PR / 4;            // K steps of W per panel
constexpr int F3_KSY = FB_CHUNK / 4;         // K steps of Y per chunk
constexpr int F3_PROW = F3_PR + 4;           // LDS row stride of Psi (floats)
constexpr int F3_CROW = FB_CHUNK + 4;        // LDS row stride of a chunk (floats)

// slot of panel row r (r = 16h + 4g + t -> K step s = 4h + t, slot 4s + g)
__device__ __forceinline__ int f3_slot(int r) {
  const int h = r >> 4, g = (r >> 2) & 3, t = r & 3;
  return 4 * (4 * h + t) + g;
}

__device__ __forceinline__ void gen_psi_f32(float* __restrict__ s_psi, uint64_t seed, int64_t p0,
                                            int64_t r1, int lq, int i0, int i1, int tid) {
  asm volatile("" : "+v"(tid));
#pragma unroll 1
  for (int w = i0 + tid; w < i1; w += FB_THREADS) {
    const int kk = w & (F3_PR - 1), g = w / F3_PR;
    float z[4] = {0.f, 0.f, 0.f, 0.f};
    if (p0 + kk < r1) gauss4(seed, 1u, (uint64_t)(p0 + kk), (uint32_t)g, z);
    const int pos = f3_slot(kk);
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int m = 4 * g + e;
      if (m < lq) s_psi[m * F3_PROW + pos] = z[e];
    }
  }
}

template <bool WANTY, int MT, int LT, int NCH>
__global__ __launch_bounds__(FB_THREADS) void k_sketch_fused_f32(
    const float* __restrict__ A, int64_t lda, int64_t N, int n, int lq, int l, uint64_t seed,
    const float* __restrict__ omP /* LT*16 x FB_NPAD, permuted per chunk, zero padded */,
    int64_t rows_per_wg, float* __restrict__ part /* grid x lq x n */, float* __restrict__ Y) {
  static_assert(FB_WAVES % LT == 0 || LT % FB_WAVES == 0, "Y tiles split evenly over the waves");
  static_assert(2 * LT >= FB_WAVES && NCH <= FB_NCH, "tile counts");
  constexpr int YR = 2 * LT / FB_WAVES;           // Y row tiles per wave (2 per panel)
  constexpr int MTR = MT < FB_MTR ? MT : FB_MTR;  // W row tiles in registers
  constexpr int MTX = MT - MTR;                   // W row tiles accumulated in LDS
  __shared__ __attribute__((aligned(16))) float s_psi[2][MT * 16 * F3_PROW];
  __shared__ __attribute__((aligned(16))) float s_chk[F3_PR * F3_CROW];
  __shared__ __attribute__((aligned(16))) float s_wx[MTX > 0 ? MTX * NCH * FB_THREADS * 4 : 4];

  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int lr = lane & 15, lg = lane >> 4;
  const int64_t r0 = (int64_t)blockIdx.x * rows_per_wg;
  int64_t r1 = r0 + rows_per_wg;
  if (r1 > N) r1 = N;
  const int lq4 = (lq + 3) >> 2;
  const int gen_items = F3_PR * lq4;

  for (int e = tid; e < 2 * MT * 16 * F3_PROW; e += FB_THREADS) (&s_psi[0][0])[e] = 0.0f;
  if constexpr (MTX > 0)
    for (int e = tid; e < MTX * NCH * FB_THREADS * 4; e += FB_THREADS) s_wx[e] = 0.0f;

  f32x4_t wacc[MTR][NCH];
#pragma unroll
  for (int mt = 0; mt < MTR; ++mt)
#pragma unroll
    for (int j = 0; j < NCH; ++j) wacc[mt][j] = f32x4_t{0.f, 0.f, 0.f, 0.f};
  f32x4_t yacc[YR];
#pragma unroll
  for (int r = 0; r < YR; ++r) yacc[r] = f32x4_t{0.f, 0.f, 0.f, 0.f};
  const int yc = wave % LT, rt0 = (wave / LT) * YR;

  const int64_t r1f = r0 + ((r1 - r0) / F3_PR) * F3_PR;
  const int col_w = 16 * wave + lr;
  typedef const __attribute__((address_space(1))) f32x4_t* gptr4;
  // a lane's 8 values of its column: v[4h + t] = row 16h + 4lg + t
  auto load8 = [&](const float* pc, int col, float (&v)[8]) {
    const float* base = chunk_col(pc, lda, n, col, lg);
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const f32x4_t a = __builtin_nontemporal_load((gptr4)(base + 16 * h));
#pragma unroll
      for (int t = 0; t < 4; ++t) v[4 * h + t] = a[t];
    }
  };
  auto load8_tail = [&](const float* pc, int col, int rows_left, float (&v)[8]) {
    typedef const __attribute__((address_space(1))) float* gptr;
    const gptr base = (gptr)(chunk_col(pc, lda, n, col, lg) - 4 * lg);
#pragma unroll
    for (int h = 0; h < 2; ++h)
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        const int r = 16 * h + 4 * lg + t;
        const bool ok = r < rows_left;
        const float x = base[ok ? r : rows_left - 1];
        v[4 * h + t] = ok ? x : 0.0f;
      }
  };
  float v[8];
  if (r0 < r1f) load8(A + r0, col_w, v);
  lds_barrier();
  if (r0 < r1) gen_psi_f32(s_psi[0], seed, r0, r1, lq, 0, gen_items, tid);
  const uint32_t om_lane = (uint32_t)((yc * 16 + lr) * FB_NPAD + 32 * lg);

  auto panel = [&](auto tail_tag, int64_t p0, int pb) {
    constexpr bool TAIL = decltype(tail_tag)::value;
    const int64_t pn = p0 + F3_PR;
    const int rows = TAIL ? (int)(r1 - p0) : F3_PR;
    const float* psi = s_psi[pb];
#pragma unroll
    for (int j = 0; j < NCH; ++j) {
      const bool col_ok = col_w + FB_CHUNK * j < n;
      if constexpr (TAIL) load8_tail(A + p0, col_w + FB_CHUNK * j, rows, v);
      lds_barrier();
      // (1) Omega fragments of this chunk (32 K steps)
      f32x4_t of[F3_KSY / 4];
      if constexpr (WANTY) {
        uintptr_t om_addr = (uintptr_t)omP;
        asm volatile("" : "+s"(om_addr));
        const gptr4 om = (gptr4)(om_addr + 4u * (om_lane + (uint32_t)(FB_CHUNK * j)));
#pragma unroll
        for (int u = 0; u < F3_KSY / 4; ++u) of[u] = om[u];
      }
      // (2) B operands of W and the row-major chunk copy for Y
      float b[8];
#pragma unroll
      for (int i = 0; i < 8; ++i) {
        b[i] = col_ok ? v[i] : 0.0f;
        if constexpr (WANTY) s_chk[(16 * (i >> 2) + 4 * lg + (i & 3)) * F3_CROW + col_w] = b[i];
      }
      // (3) the next chunk's loads
      __builtin_amdgcn_sched_barrier(0);
      if constexpr (!TAIL) {
        if (j + 1 < NCH) load8(A + p0, col_w + FB_CHUNK * (j + 1), v);
        else if (pn < r1f) load8(A + pn, col_w, v);
      }
      __builtin_amdgcn_sched_barrier(0);
      // (4) W(:, chunk) += Psi(:, panel) A(panel, chunk)
#pragma unroll
      for (int s = 0; s < F3_KSW; ++s)
#pragma unroll
        for (int mt = 0; mt < MTR; ++mt) {
          const float a = psi[(mt * 16 + lr) * F3_PROW + 4 * s + lg];
          wacc[mt][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(a, b[s], wacc[mt][j], 0, 0, 0);
        }
      if constexpr (MTX > 0) {
#pragma unroll
        for (int mx = 0; mx < MTX; ++mx) {
          f32x4_t* wx = reinterpret_cast<f32x4_t*>(&s_wx[(((mx * NCH + j) * FB_WAVES + wave) * 64 + lane) * 4]);
          f32x4_t acc = f32x4_t{0.f, 0.f, 0.f, 0.f};
#pragma unroll
          for (int s = 0; s < F3_KSW; ++s) {
            const float a = psi[((MTR + mx) * 16 + lr) * F3_PROW + 4 * s + lg];
            acc = __builtin_amdgcn_mfma_f32_16x16x4f32(a, b[s], acc, 0, 0, 0);
          }
          *wx += acc;
        }
      }
      // (5) slice j of Psi(:, next panel)
      if (!TAIL && pn < r1)
        gen_psi_f32(s_psi[pb ^ 1], seed, pn, r1, lq, gen_items * j / NCH, gen_items * (j + 1) / NCH,
                    tid);
      lds_barrier();  // chunk buffer complete
      // (6) Y(panel, this wave's tiles) += A(panel, chunk) Omega(chunk, :)
      if constexpr (WANTY) {
#pragma unroll
        for (int s = 0; s < F3_KSY; ++s) {
#pragma unroll
          for (int r = 0; r < YR; ++r) {
            const float a = s_chk[((rt0 + r) * 16 + lr) * F3_CROW + 4 * s + lg];
            yacc[r] = __builtin_amdgcn_mfma_f32_16x16x4f32(a, of[s >> 2][s & 3], yacc[r], 0, 0, 0);
          }
        }
      }
    }
    if constexpr (WANTY) {
      int lg4 = 4 * lg;
      asm volatile("" : "+v"(lg4));
      float* yp = Y + p0 * (int64_t)l;
      const int c = yc * 16 + lr;
#pragma unroll
      for (int r = 0; r < YR; ++r) {
#pragma unroll
        for (int t = 0; t < 4; ++t) {
          const int rr = (rt0 + r) * 16 + lg4 + t;
          if (c < l && (!TAIL || rr < rows)) yp[rr * l + c] = yacc[r][t];
        }
        yacc[r] = f32x4_t{0.f, 0.f, 0.f, 0.f};
      }
    }
  };

  int pb = 0;
  int64_t p0 = r0;
  for (; p0 < r1f; p0 += F3_PR, pb ^= 1) panel(std::false_type{}, p0, pb);
  if (p0 < r1) panel(std::true_type{}, p0, pb);

  float* dst = part + (int64_t)blockIdx.x * lq * n;
#pragma unroll
  for (int j = 0; j < NCH; ++j) {
    const int col = FB_CHUNK * j + col_w;
    if (col >= n) continue;
#pragma unroll
    for (int mt = 0; mt < MT; ++mt) {
      f32x4_t w4;
      if (mt < MTR) {
        w4 = wacc[mt < MTR ? mt : 0][j];
      } else {
        w4 = *reinterpret_cast<const f32x4_t*>(
            &s_wx[((((mt - MTR) * NCH + j) * FB_WAVES + wave) * 64 + lane) * 4]);
      }
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        const int m = mt * 16 + 4 * lg + t;
        if (m < lq) dst[m + (int64_t)lq * col] = w4[t];
      }
    }
  }
}

// Omega^T in FP32, k permuted per 128-column chunk: out[c * FB_NPAD + 128 j + 32 g + s] =
// Omega(128 j + 4 s + g, c), zero padded
__global__ void k_omega_p_f32(const float* __restrict__ omega /* n x l row-major */, int n, int l,
                              int lpad, float* __restrict__ out) {
  for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < lpad * FB_NPAD; e += gridDim.x * blockDim.x) {
    const int c = e / FB_NPAD, q = e - c * FB_NPAD;
    const int j = q / FB_CHUNK, rem = q - j * FB_CHUNK, g = rem / 32, s = rem - 32 * g;
    const int k = FB_CHUNK * j + 4 * s + g;
    out[e] = (c < l && k < n) ? omega[k * l + c] : 0.0f;
  }
}

// Omega^T in bfloat16 (FP8 mode: the e4m3 values, exact in bfloat16), zero
// padded: out[c * FB_NPAD + k] = value of G(seed, 0, k, c)
__global__ void k_omega_t_bf16(const float* __restrict__ omega /* n x l row-major */, int n, int l,
                               int lpad, int fp8, __bf16* __restrict__ out) {
  for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < lpad * FB_NPAD; e += gridDim.x * blockDim.x) {
    const int c = e / FB_NPAD, k = e - c * FB_NPAD;
    const float z = (c < l && k < n) ? omega[k * l + c] : 0.0f;
    out[e] = to_bf16(fp8 ? e4m3_value(z) : z);
  }
}

// W = sum of the workgroup partials, in FP64, in a fixed order (eight
// interleaved running sums, then their sum), so the result is reproducible
__global__ void k_reduce_partials_f32(const float* __restrict__ part, int64_t nparts, int64_t count,
                                      double* __restrict__ out) {
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < count;
       e += (int64_t)gridDim.x * blockDim.x) {
    double s[8] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    int64_t g = 0;
    for (; g + 8 <= nparts; g += 8)
#pragma unroll
      for (int u = 0; u < 8; ++u) s[u] += (double)part[(g + u) * count + e];
    for (; g < nparts; ++g) s[0] += (double)part[g * count + e];
    out[e] = ((s[0] + s[1]) + (s[2] + s[3])) + ((s[4] + s[5]) + (s[6] + s[7]));
  }
}

hipError_t launch_sketch_fused_f32(hipStream_t st, const float* A, int64_t lda, int64_t N, int n,
                                   int lq, int l, uint64_t seed, const float* omega, float* omP,
                                   int num_cu, float* part, double* W, float* Y) {
  const int lpad = ((l + 63) / 64) * 64;
  if (Y)
    hipLaunchKernelGGL(k_omega_p_f32, dim3(256), dim3(256), 0, st, omega, n, l, lpad, omP);
  int64_t rpw = 0;
  const int64_t grid = fused_bf16_grid(N, num_cu, &rpw);  // rows per workgroup: a multiple of 64
  const int mt = (lq + 15) / 16;
  const int nch = (n + FB_CHUNK - 1) / FB_CHUNK;
#define SID_F3(WY, MT_, LT_, NCH_)                                                      \
  hipLaunchKernelGGL((k_sketch_fused_f32<WY, MT_, LT_, NCH_>), dim3((unsigned)grid),   \
                     dim3(FB_THREADS), 0, st, A, lda, N, n, lq, l, seed, omP, rpw, part, Y)
#define SID_F3_NCH(WY, MT_, LT_)                   \
  if (nch <= 1) SID_F3(WY, MT_, LT_, 1);           \
  else if (nch <= 2) SID_F3(WY, MT_, LT_, 2);      \
  else SID_F3(WY, MT_, LT_, 4);
#define SID_F3_MT(WY, LT_)                                 \
  if (mt <= 4) { SID_F3_NCH(WY, 4, LT_) }                  \
  else { SID_F3_NCH(WY, 10, LT_) }
  if (!Y) { SID_F3_MT(false, 8) }
  else if (lpad <= 64) { SID_F3_MT(true, 4) }
  else { SID_F3_MT(true, 8) }
#undef SID_F3_MT
#undef SID_F3_NCH
#undef SID_F3
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const int64_t count = (int64_t)lq * n;
  int64_t b = (count + 255) / 256;
  if (b > 2048) b = 2048;
  hipLaunchKernelGGL(k_reduce_partials_f32, dim3((unsigned)b), dim3(256), 0, st, part, grid, count, W);
  return hipGetLastError();
}

bool fused_bf16_supported(int64_t n, int lq, int l, int64_t lda, const void* A, bool has_rows) {
  // a row list gathers single values: no alignment needed (W only; checked by the caller)
  return n <= FB_NPAD && lq <= 160 && l <= 128 &&
         (has_rows || ((lda % 4) == 0 && ((uintptr_t)A % 16) == 0));
}

int64_t fused_bf16_grid(int64_t N, int num_cu, int64_t* rows_per_wg) {
  int64_t g = num_cu;
  int64_t rpw = (N + g - 1) / g;
  rpw = (rpw + FB_PR - 1) / FB_PR * FB_PR;
  if (rpw < FB_PR) rpw = FB_PR;
  g = (N + rpw - 1) / rpw;
  *rows_per_wg = rpw;
  return g;
}

hipError_t launch_sketch_fused_bf16(hipStream_t st, int dmode, const float* A, int64_t lda,
                                    int64_t N, int n, int lq, int l, uint64_t seed,
                                    const float* omega, __bf16* omT, int num_cu, float* part,
                                    double* W, float* Y, int64_t* nparts_out,
                                    const int64_t* rows) {
  if (rows && (Y || dmode == FB_FP8)) return hipErrorInvalidValue;  // row lists: W only, bf16
  const int lpad = ((l + 63) / 64) * 64;  // Y tiles: a multiple of 4 tiles of 16
  if (Y) {
    hipLaunchKernelGGL(k_omega_t_bf16, dim3(256), dim3(256), 0, st, omega, n, l, lpad,
                       dmode == FB_FP8 ? 1 : 0, omT);
  }
  int64_t rpw = 0;
  const int64_t grid = fused_bf16_grid(N, num_cu, &rpw);
  *nparts_out = grid;
  const int mt = (lq + 15) / 16;
  const int nch = (n + FB_CHUNK - 1) / FB_CHUNK;
#define SID_FUSED(SP, WY, MT_, LT_, NCH_)                                                  \
  hipLaunchKernelGGL((k_sketch_fused_bf16<SP, WY, MT_, LT_, NCH_>), dim3((unsigned)grid), \
                     dim3(FB_THREADS), 0, st, A, lda, N, n, lq, l, seed, omT, rpw, part, Y,  \
                     nullptr)
#define SID_FUSED_R(SP, MT_, NCH_)                                                          \
  hipLaunchKernelGGL((k_sketch_fused_bf16<SP, false, MT_, 8, NCH_, true>),                  \
                     dim3((unsigned)grid), dim3(FB_THREADS), 0, st, A, lda, N, n, lq, l, seed, \
                     omT, rpw, part, Y, rows)
#define SID_FUSED_RN(SP, MT_)                   \
  if (nch <= 1) SID_FUSED_R(SP, MT_, 1);        \
  else if (nch <= 2) SID_FUSED_R(SP, MT_, 2);   \
  else SID_FUSED_R(SP, MT_, 4);
#define SID_FUSED_RM(SP)                        \
  if (mt <= 4) { SID_FUSED_RN(SP, 4) }          \
  else { SID_FUSED_RN(SP, 10) }
#define SID_FUSED_NCH(SP, WY, MT_, LT_)         \
  if (nch <= 1) SID_FUSED(SP, WY, MT_, LT_, 1); \
  else if (nch <= 2) SID_FUSED(SP, WY, MT_, LT_, 2); \
  else SID_FUSED(SP, WY, MT_, LT_, 4);
#define SID_FUSED_MT(SP, WY, LT_)                          \
  if (mt <= 4) { SID_FUSED_NCH(SP, WY, 4, LT_) }           \
  else { SID_FUSED_NCH(SP, WY, 10, LT_) }
#define SID_FUSED_SP(SP)                                     \
  if (!Y) { SID_FUSED_MT(SP, false, 8) }                     \
  else if (lpad <= 64) { SID_FUSED_MT(SP, true, 4) }         \
  else { SID_FUSED_MT(SP, true, 8) }
  if (rows) {
    if (dmode == FB_BF16X2) { SID_FUSED_RM(FB_BF16X2) }
    else { SID_FUSED_RM(FB_BF16) }
  } else if (dmode == FB_BF16X2) { SID_FUSED_SP(FB_BF16X2) }
  else if (dmode == FB_FP8) { SID_FUSED_SP(FB_FP8) }
  else { SID_FUSED_SP(FB_BF16) }
#undef SID_FUSED_RM
#undef SID_FUSED_RN
#undef SID_FUSED_R
#undef SID_FUSED_SP
#undef SID_FUSED_MT
#undef SID_FUSED_NCH
#undef SID_FUSED
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const int64_t count = (int64_t)lq * n;
  int64_t blocks = (count + 255) / 256;
  if (blocks > 4096) blocks = 4096;
  hipLaunchKernelGGL(k_reduce_partials_f32, dim3((unsigned)blocks), dim3(256), 0, st, part, grid,
                     count, W);
  return hipGetLastError();
}


// ---------------------------------------------------------------------------
// Skeleton estimate of the single pass, AJ = Y T (N x k), on the matrix
// cores.  Computed as AJ^T = T^T Y^T so that each MFMA output tile is
// (16 skeleton columns) x (16 rows of A) and lands as coalesced column-major
// stores.  v_mfma_{f32,f64}_16x16x4 layouts: A (16 x 4): lane l holds row
// l%16, k = l/16; B (4 x 16): lane l holds col l%16, k = l/16; C: col l%16,
// element t = row 4*(l/16) + t (f32) or row l/16 + 4*t (f64).  A lane reads 4 consecutive entries of one Y row at a
// time; entry s of that quad feeds MFMA s, whose A operand therefore holds
// T(kb + 4*(l/16) + s, m) -- the K order is permuted, the sum is the same.
// T^T (kpad x lpad, zero padded) lives in LDS; each wave owns 32 rows of A
// (two 16-row tiles) and all skeleton columns.
// ---------------------------------------------------------------------------
template <typename TE>
struct MfmaK4;
// crow(lg, t): output row held in accumulator element t by lanes 16*lg ..
// 16*lg+15 (the FP32 and FP64 forms arrange the 16 x 16 result differently).
template <>
struct MfmaK4<float> {
  typedef float acc_t __attribute__((ext_vector_type(4)));
  static __device__ __forceinline__ acc_t run(float a, float b, acc_t c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int crow(int lg, int t) { return 4 * lg + t; }
};
template <>
struct MfmaK4<double> {
  typedef double acc_t __attribute__((ext_vector_type(4)));
  static __device__ __forceinline__ acc_t run(double a, double b, acc_t c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int crow(int lg, int t) { return lg + 4 * t; }
};

constexpr int AT_WAVES = 4;
constexpr int AT_RT = 2;  // 16-row tiles per wave

template <typename TE, typename OutT, int CT>
__global__ __launch_bounds__(64 * AT_WAVES) void k_apply_t_mfma(
    const TE* __restrict__ Y, int64_t N, int l, const double* __restrict__ Tm /* l x k, ld l */,
    int k, OutT* __restrict__ AJ, int64_t ldaj) {
  using M = MfmaK4<TE>;
  extern __shared__ __attribute__((aligned(16))) unsigned char s_raw[];
  TE* s_tt = reinterpret_cast<TE*>(s_raw);  // T^T: [CT*16][lst], m-major
  const int lpad = (l + 15) & ~15;
  const int lst = lpad + 1;  // odd stride: the 16 rows read together hit 16 banks
  for (int e = threadIdx.x; e < CT * 16 * lst; e += blockDim.x) {
    const int m = e / lst, c = e - m * lst;
    s_tt[e] = (m < k && c < l) ? (TE)Tm[c + (int64_t)l * m] : TE(0);
  }
  __syncthreads();
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int lr = lane & 15, lg = lane >> 4;
  const bool vec = (l % 4) == 0;
  // persistent workgroups: T^T is staged once and the row blocks are walked
  // with a grid stride
  const int64_t nblk = (N + AT_WAVES * AT_RT * 16 - 1) / (AT_WAVES * AT_RT * 16);
  for (int64_t blk = blockIdx.x; blk < nblk; blk += gridDim.x) {
  const int64_t row0 = (blk * AT_WAVES + wave) * (AT_RT * 16);
  typename M::acc_t acc[AT_RT][CT];
#pragma unroll
  for (int r = 0; r < AT_RT; ++r)
#pragma unroll
    for (int c = 0; c < CT; ++c) acc[r][c] = typename M::acc_t{0, 0, 0, 0};
  for (int kb = 0; kb < lpad; kb += 16) {
    TE yv[AT_RT][4];
#pragma unroll
    for (int r = 0; r < AT_RT; ++r) {
      const int64_t row = row0 + r * 16 + lr;
      const int c0 = kb + 4 * lg;
      if (row < N && vec && c0 + 4 <= l) {
        typedef TE te4 __attribute__((ext_vector_type(4)));
        const te4 q4 = *reinterpret_cast<const te4*>(Y + row * l + c0);
#pragma unroll
        for (int s = 0; s < 4; ++s) yv[r][s] = q4[s];
      } else {
#pragma unroll
        for (int s = 0; s < 4; ++s) yv[r][s] = (row < N && c0 + s < l) ? Y[row * l + c0 + s] : TE(0);
      }
    }
#pragma unroll
    for (int s = 0; s < 4; ++s) {
#pragma unroll
      for (int c = 0; c < CT; ++c) {
        const TE a = s_tt[(c * 16 + lr) * lst + kb + 4 * lg + s];
#pragma unroll
        for (int r = 0; r < AT_RT; ++r) acc[r][c] = M::run(a, yv[r][s], acc[r][c]);
      }
    }
  }
#pragma unroll
  for (int r = 0; r < AT_RT; ++r) {
    const int64_t row = row0 + r * 16 + lr;
    if (row >= N) continue;
#pragma unroll
    for (int c = 0; c < CT; ++c)
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        const int m = c * 16 + M::crow(lg, t);
        if (m < k) AJ[row + ldaj * m] = (OutT)acc[r][c][t];
      }
  }
  }
}

template <typename TE, typename OutT>
static hipError_t apply_t_dispatch(hipStream_t st, const TE* Y, int64_t N, int l,
                                   const double* Tm, int k, OutT* AJ, int64_t ldaj, int num_cu) {
  const int ct = (k + 15) / 16;
  const int lpad = (l + 15) & ~15;
  const int64_t rows_per_block = AT_WAVES * AT_RT * 16;
  int64_t nblk = (N + rows_per_block - 1) / rows_per_block;
  if (nblk > (int64_t)num_cu * 4) nblk = (int64_t)num_cu * 4;  // persistent: a few per CU
  const dim3 grid((unsigned)nblk);
#define SID_AT(CT_)                                                                        \
  {                                                                                        \
    const size_t shm = sizeof(TE) * (size_t)(CT_) * 16 * (lpad + 1);                       \
    auto kern = k_apply_t_mfma<TE, OutT, CT_>;                                             \
    if (shm > 65536) (void)hipFuncSetAttribute((const void*)kern,                          \
                                               hipFuncAttributeMaxDynamicSharedMemorySize, \
                                               (int)shm);                                  \
    hipLaunchKernelGGL(kern, grid, dim3(64 * AT_WAVES), shm, st, Y, N, l, Tm, k, AJ, ldaj); \
  }
  if (ct <= 2) SID_AT(2)
  else if (ct <= 4) SID_AT(4)
  else if (ct <= 7) SID_AT(7)
  else if (ct <= 10) SID_AT(10)
  else return hipErrorInvalidValue;
#undef SID_AT
  return hipGetLastError();
}

bool apply_t_mfma_supported(int k, int l, bool y_f64) {
  const int ct = (k + 15) / 16;
  const int ctt = ct <= 2 ? 2 : ct <= 4 ? 4 : ct <= 7 ? 7 : 10;  // template tile count
  const size_t shm = (y_f64 ? 8 : 4) * (size_t)ctt * 16 * (((l + 15) & ~15) + 1);
  return ct <= 10 && shm <= 160 * 1024;
}

hipError_t launch_apply_t_mfma(hipStream_t st, const void* Y, bool y_f64, int64_t N, int l,
                               const double* Tm, int k, void* AJ, bool aj_f64, int64_t ldaj, int num_cu) {
  if (y_f64) {
    if (aj_f64) return apply_t_dispatch<double, double>(st, (const double*)Y, N, l, Tm, k, (double*)AJ, ldaj, num_cu);
    return apply_t_dispatch<double, float>(st, (const double*)Y, N, l, Tm, k, (float*)AJ, ldaj, num_cu);
  }
  if (aj_f64) return apply_t_dispatch<float, double>(st, (const float*)Y, N, l, Tm, k, (double*)AJ, ldaj, num_cu);
  return apply_t_dispatch<float, float>(st, (const float*)Y, N, l, Tm, k, (float*)AJ, ldaj, num_cu);
}


// ---------------------------------------------------------------------------
// Skeleton estimate of the single pass for the bfloat16 sketch precisions,
// AJ = Y T on the bf16 matrix cores.  Y (N x l, row-major FP32) and T (l x k,
// FP64) are each split into bf16 hi + lo parts and the product is formed from
// the three terms Y_hi T_hi + Y_hi T_lo + Y_lo T_hi (the dropped Y_lo T_lo is
// below 2^-16 of the product), accumulated in FP32.  Orientation as in
// k_apply_t_mfma: AJ^T = T^T Y^T, so a C tile is (16 skeleton columns) x
// (16 rows of A) and its stores run down the columns of AJ.
//   A operand: T^T tile (16 x 32) from LDS, lane = skeleton column l%16,
//              entries 8*(l/16) .. +7 of a 32-wide slice of l;
//   B operand: Y^T tile (32 x 16), lane = row l%16 of A, 8 consecutive Y
//              entries of that row (two 16-byte loads).
// Each wave owns 32 rows (two row tiles) of a 128-row block; workgroups loop
// over blocks so that the T split is staged in LDS once per workgroup.
// ---------------------------------------------------------------------------
constexpr int AB_THREADS = 256;
constexpr int AB_LPAD = 128;               // l <= 128: four K steps of 32
constexpr int AB_LS = AB_LPAD + 8;         // LDS row stride (bf16)
constexpr int AB_ROWS = 4 * 32;            // rows per block

// AL: l % 4 == 0 (16-byte aligned rows of Y: two 16-byte loads per lane
// and K step); otherwise eight 4-byte loads, the entries past l zero
template <int KT, typename OutT, bool AL = true>
__global__ __launch_bounds__(AB_THREADS) void k_apply_t_bf16(
    const float* __restrict__ Y, int64_t N, int l, const double* __restrict__ Tm /* l x k */,
    int k, OutT* __restrict__ AJ, int64_t ldaj) {
  __shared__ __attribute__((aligned(16))) __bf16 s_th[KT * 16 * AB_LS];
  __shared__ __attribute__((aligned(16))) __bf16 s_tl[KT * 16 * AB_LS];
  for (int e = threadIdx.x; e < KT * 16 * AB_LPAD; e += AB_THREADS) {
    const int m = e / AB_LPAD, c = e - m * AB_LPAD;
    const float x = (m < k && c < l) ? (float)Tm[c + (int64_t)l * m] : 0.0f;
    const __bf16 h = to_bf16(x);
    s_th[m * AB_LS + c] = h;
    s_tl[m * AB_LS + c] = to_bf16(x - (float)h);
  }
  __syncthreads();
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int lr = lane & 15, lg = lane >> 4;
  const int nks = (l + 31) >> 5;
  const int64_t nblk = (N + AB_ROWS - 1) / AB_ROWS;
  typedef const __attribute__((address_space(1))) f32x4_t* gptr4;
  // Y entries of one block for this lane: y[rt][ks] = Y(row0 + 16 rt + lr,
  // 32 ks + 8 lg .. +7); the next block's are loaded while this one is
  // multiplied
  f32x4_t y[2][4][2];
  auto load_block = [&](int64_t b) {
    const int64_t row0 = b * AB_ROWS + wave * 32;
#pragma unroll
    for (int rt = 0; rt < 2; ++rt) {
      const int64_t row = row0 + rt * 16 + lr;
#pragma unroll
      for (int ks = 0; ks < 4; ++ks)
#pragma unroll
        for (int h = 0; h < 2; ++h) {
          const int c = 32 * ks + 8 * lg + 4 * h;
          if constexpr (AL) {
            y[rt][ks][h] = (row < N && c + 4 <= l) ? *(gptr4)(Y + row * l + c)
                                                   : f32x4_t{0.f, 0.f, 0.f, 0.f};
          } else {
#pragma unroll
            for (int t = 0; t < 4; ++t) y[rt][ks][h][t] = (row < N && c + t < l) ? Y[row * l + c + t] : 0.f;
          }
        }
    }
  };
  int64_t b = blockIdx.x;
  if (b < nblk) load_block(b);
  for (; b < nblk; b += gridDim.x) {
    const int64_t row0 = b * AB_ROWS + wave * 32;
    bf16x8_t bh[2][4], bl[2][4];
#pragma unroll
    for (int rt = 0; rt < 2; ++rt)
#pragma unroll
      for (int ks = 0; ks < 4; ++ks)
#pragma unroll
        for (int i = 0; i < 8; ++i) {
          const float x = y[rt][ks][i >> 2][i & 3];
          const __bf16 hv = to_bf16(x);
          bh[rt][ks][i] = hv;
          bl[rt][ks][i] = to_bf16(x - (float)hv);
        }
    if (b + gridDim.x < nblk) load_block(b + gridDim.x);
    f32x4_t acc[2][KT];
#pragma unroll
    for (int rt = 0; rt < 2; ++rt)
#pragma unroll
      for (int kt = 0; kt < KT; ++kt) acc[rt][kt] = f32x4_t{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int ks = 0; ks < 4; ++ks) {
      if (ks >= nks) break;
#pragma unroll
      for (int kt = 0; kt < KT; ++kt) {
        const int ti = (kt * 16 + lr) * AB_LS + 32 * ks + 8 * lg;
        const bf16x8_t th = *reinterpret_cast<const bf16x8_t*>(&s_th[ti]);
        const bf16x8_t tl = *reinterpret_cast<const bf16x8_t*>(&s_tl[ti]);
#pragma unroll
        for (int rt = 0; rt < 2; ++rt) {
          acc[rt][kt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(th, bh[rt][ks], acc[rt][kt], 0, 0, 0);
          acc[rt][kt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(th, bl[rt][ks], acc[rt][kt], 0, 0, 0);
          acc[rt][kt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(tl, bh[rt][ks], acc[rt][kt], 0, 0, 0);
        }
      }
    }
#pragma unroll
    for (int rt = 0; rt < 2; ++rt) {
      const int64_t row = row0 + rt * 16 + lr;
      if (row >= N) continue;
#pragma unroll
      for (int kt = 0; kt < KT; ++kt)
#pragma unroll
        for (int t = 0; t < 4; ++t) {
          const int m = kt * 16 + 4 * lg + t;
          if (m < k) AJ[row + ldaj * m] = (OutT)acc[rt][kt][t];
        }
    }
  }
}

bool apply_t_bf16_supported(int k, int l) {
  return k >= 1 && k <= 128 && l >= 1 && l <= AB_LPAD;
}

hipError_t launch_apply_t_bf16(hipStream_t st, const float* Y, int64_t N, int l, const double* Tm,
                               int k, void* AJ, bool aj_f64, int64_t ldaj, int num_cu) {
  if (!apply_t_bf16_supported(k, l)) return hipErrorInvalidValue;
  const int64_t nblk = (N + AB_ROWS - 1) / AB_ROWS;
  int64_t g = (int64_t)num_cu * 4;
  if (g > nblk) g = nblk;
  const dim3 grid((unsigned)g), block(AB_THREADS);
  const bool al = (l % 4) == 0;
#define SID_AB2(KT_, AL_)                                                                          \
  if (aj_f64) hipLaunchKernelGGL((k_apply_t_bf16<KT_, double, AL_>), grid, block, 0, st, Y, N, l, \
                                 Tm, k, (double*)AJ, ldaj);                                        \
  else hipLaunchKernelGGL((k_apply_t_bf16<KT_, float, AL_>), grid, block, 0, st, Y, N, l, Tm, k,   \
                          (float*)AJ, ldaj);
#define SID_AB(KT_)              \
  if (al) { SID_AB2(KT_, true) } \
  else { SID_AB2(KT_, false) }
  if (k <= 32) { SID_AB(2) }
  else if (k <= 64) { SID_AB(4) }
  else { SID_AB(8) }
#undef SID_AB
#undef SID_AB2
  return hipGetLastError();
}

}  // namespace sid
