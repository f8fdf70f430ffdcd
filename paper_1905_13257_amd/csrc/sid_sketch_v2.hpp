// sid_sketch_v2.hpp -- the bfloat16 sketch pass (bf16 / bf16x2 / fp8 forms)
// on 32x32x16 matrix instructions, with the data staged through LDS by
// direct global-to-LDS loads.
//
// One streaming read of A forms both sketches of the single-pass ID
// (Alg. 4 sketch step; the two-sided sketch of Halko et al. Sec. 5.5 items
// (1)-(2), quoted in Sec. 2.3):
//   W = Psi A   (lq x n)     Y = A Omega   (N x l)
//
// Work layout.  Workgroups of four waves, one per CU (one wave per SIMD, so
// a wave may hold up to 512 registers).  Two workgroups on the same XCD
// (blocks b and b + 8: blocks are dealt to the eight XCDs round-robin) form
// a pair that owns one contiguous range of rows; both read every row and
// column of it (the second read of a line is served by the XCD's L2 or the
// Infinity Cache, not HBM), and they split the work that has to stay on
// chip: half h forms the W rows of its half of Psi (hsplit rows each, so
// the Gaussian work splits evenly too) and the Y columns 32 LT h .. of its
// half.  The W partial of the pair's whole row range then fits the
// accumulator registers: MT x NCT tiles of 32 x 32 per wave.
// The range is walked in panels of 64 rows; a panel is consumed in NCT
// chunks of 128 columns, and wave w owns columns 32w .. 32w+31 of a chunk.
//   * Data: each wave moves its 64 x 32 FP32 block of a chunk from HBM into
//     its own part of a two-stage LDS ring with eight global_load_lds_dwordx4
//     (32 columns x 32 bytes each).  A stage is read into registers K step
//     by K step (two ds_read_b128 per lane, bank-conflict free by the
//     placement of the 16-byte pieces) and refilled with the chunk two
//     ahead right after its last read, so up to two chunks (64 KB per CU)
//     are in flight while the current one is multiplied.  No wave reads
//     another wave's ring part: the ring needs no barrier.
//   * W(:, chunk) += Psi(:, panel) A(panel, chunk): A operand = a 32-row tile
//     of the half's Psi from LDS, B operand = the lane's 8 rows of its
//     column (bf16 hi, and lo in the split form).
//   * Y(panel, :) += A(panel, chunk) Omega(chunk, :) needs rows of A: the
//     converted values are written transposed into a row-major chunk buffer
//     (column c of the chunk at position 2 (c mod 64) + c / 64, so the 32
//     lanes of a write hit 32 banks); Omega^T is stored with its k index in
//     the same order, so the products pair up.
//   * Psi(half's rows, next panel) is generated (Philox + Box-Muller) into
//     the other half of a double-buffered LDS array, a slice per chunk; a
//     thread draws one panel row and four Psi rows, and adjacent lanes
//     (adjacent panel rows) swap two values so that each writes two Psi rows
//     as 32-bit pairs.
// The W partial of each pair is written once at the end (FP32, row-major
// lq x n per pair, each half its rows) and summed in a fixed order in FP64.
//
// v_mfma_f32_32x32x16_bf16 (wave64): A (32 x 16): lane l holds row l%32,
// k = 8 (l/32) .. +7; B (16 x 32): lane l holds column l%32, k = 8 (l/32) ..
// +7; D (32 x 32): lane l holds column l%32, rows 8 (e/4) + 4 (l/32) + e%4 in
// element e.
#pragma once
#include <type_traits>

#include "sid_kernels.hpp"

namespace sid {
namespace v2 {

typedef __bf16 bf16x8_t __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x2_t __attribute__((ext_vector_type(2)));
typedef float f32x4_t __attribute__((ext_vector_type(4)));
typedef float f32x16_t __attribute__((ext_vector_type(16)));

constexpr int V2_WAVES = 4;
constexpr int V2_THREADS = 64 * V2_WAVES;
constexpr int V2_PR = 64;                      // rows per panel (4 K steps of 16)
constexpr int V2_CHUNK = 32 * V2_WAVES;        // columns per chunk
constexpr int V2_WFL = V2_PR * 32;             // floats of one wave's block (8 KB)
constexpr int V2_STAGE = V2_WAVES * V2_WFL;    // floats of one ring stage (32 KB)
constexpr int V2_CS = V2_CHUNK + 8;            // chunk buffer row stride (bf16)
constexpr int V2_PS = V2_PR;                   // Psi row stride (bf16, XOR-placed 16 B pieces)
constexpr int V2_MAXNCT = 4;                   // chunks per launch: n <= 512

__device__ __forceinline__ f32x16_t mfma32(bf16x8_t a, bf16x8_t b, f32x16_t c) {
  return __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, c, 0, 0, 0);
}

// position of chunk column c (0..127) in a row of the chunk buffer
__device__ __forceinline__ int chk_pos(int c) { return 2 * (c & 63) + (c >> 6); }

// ring: a wave's 64 x 32 block is 8 DMA instructions q of 64 lanes x 16
// bytes; instruction q carries rows 32 (q/4) .. +31 (one whole 128-byte
// line) of the 8 columns 8 (q%4) .. +7: lane i takes column 8 (q%4) + i/8
// and rows 32 (q/4) + 4x .. +3 with x = (i%8) ^ (i/8), so that the eight
// lanes of a 16-byte read group hit eight different 16-byte bank groups.
// Slot of (row half rh, column cc, rows 4x ..):
__device__ __forceinline__ int ring_slot(int rh, int cc, int x) {
  return 64 * (4 * rh + (cc >> 3)) + 8 * (cc & 7) + (x ^ (cc & 7));
}

// Psi element (row m, panel row k) in a buffer of MT*32 rows
__device__ __forceinline__ int psi_idx(int m, int k) {
  return m * V2_PS + ((((k >> 3) ^ m) & 7) << 3) + (k & 7);
}

}  // namespace v2

using namespace v2;

// DM: FB_BF16 / FB_BF16X2 / FB_FP8 (as in the first pass).  WANTY: form Y.
// MT: 32-row tiles of W per half (hsplit and lq - hsplit <= 32 MT); NCT:
// chunks of 128 columns (n <= 128 NCT); LT: 32-column tiles of Y per half
// (2 or 4: l <= 64 LT).
template <int DM, bool WANTY, int MT, int NCT, int LT>
__global__ __launch_bounds__(V2_THREADS, 1) void k_sketch_v2(
    const float* __restrict__ A, int64_t lda, int64_t N, int n, int lq, int hsplit, int l,
    uint64_t seed, const __bf16* __restrict__ omT /* 64 LT x 128 NCT, k in chunk-buffer order */,
    int64_t rows_per_pair, float* __restrict__ part /* pairs x lq x n, row-major per pair */,
    float* __restrict__ Y /* N x l row-major */, int yadd /* 1: Y += A Omega */,
    const __bf16* __restrict__ psi_img /* optional: Psi images (MT = 4 only) */) {
  static_assert(LT == 2 || LT == 4, "Y column tiles per half");
  // Psi images are taken for MT = 4 only (MT pieces per thread: the counts
  // of the waits at (2))
  constexpr bool PSI_IMG_OK = MT == 4;
  constexpr bool SPLIT = DM == FB_BF16X2;
  constexpr bool FP8 = DM == FB_FP8;
  constexpr int NH = SPLIT ? 2 : 1;
  // Y tiles of a wave: LT = 2: one tile (row tile w/2, column tile w%2);
  // LT = 4: both row tiles of column tile w
  constexpr int YR = LT == 2 ? 1 : 2;          // Y row tiles per wave
  constexpr int NPADO = 128 * NCT;             // row length of omT

  __shared__ __attribute__((aligned(16))) float s_ring[2 * V2_STAGE];
  __shared__ __attribute__((aligned(16))) __bf16 s_psi[2][MT * 32 * V2_PS];
  __shared__ __attribute__((aligned(16))) __bf16 s_chk[NH][V2_PR * V2_CS];

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int lc = lane & 31, hl = lane >> 5;
  // pair and half: blocks b and b + 8 (same XCD) share a row range
  const int64_t b = blockIdx.x;
  const int64_t pair = (b >> 4) * 8 + (b & 7);
  const int half = (int)((b >> 3) & 1);
  const int64_t r0 = pair * rows_per_pair;
  int64_t r1 = r0 + rows_per_pair;
  if (r1 > N) r1 = N;
  if (r1 < r0) r1 = r0;  // a pair past the end has no rows and writes a zero partial
  const int64_t r1f = r0 + ((r1 - r0) / V2_PR) * V2_PR;  // end of the full panels
  const int64_t nfull = (r1f - r0) / V2_PR;
  // this half's Psi (= W) rows [mb, mb + mc) and Y columns [yb, yb + 32 LT)
  const int mb = half ? hsplit : 0;
  const int mc = half ? lq - hsplit : hsplit;
  const int yb = half * 32 * LT;
  const int gen_items = V2_PR * ((mc + 3) >> 2);          // per panel: (panel row, group of 4)
  const int gen_iters = (gen_items + V2_THREADS - 1) / V2_THREADS;

  // Psi rows >= mc stay zero in both buffers
  for (int e = tid; e < 2 * MT * 32 * V2_PS / 2; e += V2_THREADS)
    reinterpret_cast<uint32_t*>(&s_psi[0][0])[e] = 0u;

  // ---- data movement -----------------------------------------------------
  // this lane's column within its wave's block, and its global column of
  // chunk j
  const int colw = 32 * wave;
  typedef const __attribute__((address_space(1))) void* gvoid;
  typedef __attribute__((address_space(3))) void* lvoid;
  // DMA of (panel starting at p0, chunk j) into ring stage st: instruction q
  // to slot 64 q + lane of the wave's part (placement above)
  const int dma_ci = lane >> 3;
  const int dma_x = (lane & 7) ^ dma_ci;
  auto dma = [&](int64_t p0, int j, int st) __attribute__((always_inline)) {
    float* dst = s_ring + st * V2_STAGE + wave * V2_WFL;
#pragma unroll
    for (int c4 = 0; c4 < 4; ++c4) {
      int col = V2_CHUNK * j + colw + 8 * c4 + dma_ci;
      col = col < n ? col : n - 1;
      const float* src = A + (int64_t)col * lda + p0 + 4 * dma_x;
#pragma unroll
      for (int rh = 0; rh < 2; ++rh)
        __builtin_amdgcn_global_load_lds((gvoid)(src + 32 * rh), (lvoid)(dst + 256 * (4 * rh + c4)),
                                         16, 0, 0);
    }
  };
  // the lane's 8 values of K step ks (rows 16 ks + 8 hl + 0..7 of its
  // column) from ring stage st
  auto ring_read = [&](int st, int ks, float (&v)[8]) __attribute__((always_inline)) {
    const float* base = s_ring + st * V2_STAGE + wave * V2_WFL;
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int xx = 4 * (ks & 1) + 2 * hl + h;
      const f32x4_t a =
          *reinterpret_cast<const f32x4_t*>(base + 4 * ring_slot(ks >> 1, lc, xx));
#pragma unroll
      for (int t = 0; t < 4; ++t) v[4 * h + t] = a[t];
    }
  };

  // ---- accumulators ------------------------------------------------------
  f32x16_t wacc[MT][NCT];
#pragma unroll
  for (int mt = 0; mt < MT; ++mt)
#pragma unroll
    for (int j = 0; j < NCT; ++j)
#pragma unroll
      for (int e = 0; e < 16; ++e) wacc[mt][j][e] = 0.0f;
  f32x16_t yacc[YR];
#pragma unroll
  for (int r = 0; r < YR; ++r)
#pragma unroll
    for (int e = 0; e < 16; ++e) yacc[r][e] = 0.0f;
  const int yrt0 = LT == 2 ? (wave >> 1) : 0;      // first Y row tile
  const int yc = LT == 2 ? (wave & 1) : wave;      // Y column tile within the half
  const int ycol = yb + 32 * yc + lc;              // this lane's Y column

  // ---- Psi generation ------------------------------------------------------
  // iterations [it0, it1) of panel pn's items into buffer pb; item w: panel
  // row k = w % 64, group g = w / 64 (the half's Psi rows 4g .. 4g+3).  Lanes
  // 2i and 2i+1 (rows k, k+1 of one group) swap two draws, then the even
  // lane writes Psi rows 4g, 4g+1 and the odd lane rows 4g+2, 4g+3 as
  // (k, k+1) pairs.  At most GMAX iterations per chunk (straight-line code).
  constexpr int GMAX = (MT * 8 * V2_PR + V2_THREADS - 1) / V2_THREADS / NCT + 1;
  auto gen = [&](int64_t pn, int pb, int it0, int it1) __attribute__((always_inline)) {
    int t = tid;
    asm volatile("" : "+v"(t));
    const bool odd = (t & 1) != 0;
#pragma unroll
    for (int u = 0; u < GMAX; ++u) {
      const int it = it0 + u;
      if (it >= it1) break;
      const int w = it * V2_THREADS + t;
      if (w < gen_items) {  // whole groups of 64: both lanes of a pair agree
        const int k = w & (V2_PR - 1), g = w >> 6;
        float z[4] = {0.f, 0.f, 0.f, 0.f};
        const int64_t r = pn + k;
        if (r < r1) gauss4(seed, 1u, (uint64_t)r, (uint32_t)((mb >> 2) + g), z);
        if constexpr (FP8) {
#pragma unroll
          for (int e = 0; e < 4; ++e) z[e] = e4m3_value(z[e]);
        }
        // send z[2], z[3] (even) / z[0], z[1] (odd) to the neighbour
        const float s0 = odd ? z[0] : z[2], s1 = odd ? z[1] : z[3];
        const float q0 = __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(s0), 0xB1, 0xF, 0xF, false));
        const float q1 = __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(s1), 0xB1, 0xF, 0xF, false));
        bf16x2_t p0, p1;
        p0[0] = (__bf16)(odd ? q0 : z[0]);
        p0[1] = (__bf16)(odd ? z[2] : q0);
        p1[0] = (__bf16)(odd ? q1 : z[1]);
        p1[1] = (__bf16)(odd ? z[3] : q1);
        const int m0 = 4 * g + (odd ? 2 : 0);
        const int ke = k & ~1;
        if (m0 < mc) *reinterpret_cast<bf16x2_t*>(&s_psi[pb][psi_idx(m0, ke)]) = p0;
        if (m0 + 1 < mc) *reinterpret_cast<bf16x2_t*>(&s_psi[pb][psi_idx(m0 + 1, ke)]) = p1;
      }
    }
  };

  // Y(panel, this wave's tiles), then reset.  Offsets in 32 bits from the
  // uniform base (N l 4 bytes < 4 GiB is checked by the host); the row steps
  // are uniform multiples of l
  auto store_y = [&](int64_t p0, int rows) __attribute__((always_inline)) {
    if constexpr (WANTY) {
#pragma unroll
      for (int r = 0; r < YR; ++r) {
        const int rb = 32 * (yrt0 + r) + 4 * hl;
        const uint32_t ob = (uint32_t)(((p0 + rb) * l + ycol) * 4);
        f32x16_t t = yacc[r];
        asm volatile("" : "+v"(t));
        if (yadd) {
          // Y += this pass's part: all sixteen old values are loaded before
          // the first sum, and the sums are those of a separate Y + part pass
          float old[16];
#pragma unroll
          for (int e = 0; e < 16; ++e) {
            const int dr = 8 * (e >> 2) + (e & 3);
            old[e] = (ycol < l && rb + dr < rows)
                         ? *reinterpret_cast<const float*>(reinterpret_cast<const char*>(Y) +
                                                           (ob + (uint32_t)(dr * l * 4)))
                         : 0.0f;
          }
#pragma unroll
          for (int e = 0; e < 16; ++e) t[e] = old[e] + t[e];
        }
#pragma unroll
        for (int e = 0; e < 16; ++e) {
          const int dr = 8 * (e >> 2) + (e & 3);
          if (ycol < l && rb + dr < rows)
            *reinterpret_cast<float*>(reinterpret_cast<char*>(Y) + (ob + (uint32_t)(dr * l * 4))) = t[e];
          yacc[r][e] = 0.0f;
        }
        __builtin_amdgcn_sched_barrier(0);
      }
    }
  };

  // ---- one chunk -----------------------------------------------------------
  // TAIL: the ragged last panel (rows_left < 64), read with guarded loads
  // straight from A; otherwise from ring stage st.
  auto chunk = [&](auto tail_tag, int64_t p0, int j, int pb, int st, int64_t next_p0, int next_j,
                   bool next_ok, bool store_prev, bool one_more) __attribute__((always_inline)) {
    constexpr bool TAIL = decltype(tail_tag)::value;
    const int rows_left = TAIL ? (int)(r1 - p0) : V2_PR;
    const int col = V2_CHUNK * j + colw + lc;
    const bool col_ok = col < n;
    // (0) with Psi images: the first chunk of a panel loads the next panel's
    //     image of this half (MT pieces of 16 bytes per thread), written to
    //     LDS at (5); issued first, so that the waits below count them
    const bool img = PSI_IMG_OK && psi_img && !TAIL && j == 0 && p0 + V2_PR < r1;
    bf16x8_t imv[MT];
    if (img) {
      typedef const __attribute__((address_space(1))) bf16x8_t* gimg;
      const gimg src = (gimg)(psi_img + ((p0 / V2_PR + 1) * 2 + half) * (int64_t)(MT * 32 * V2_PS));
#pragma unroll
      for (int i = 0; i < MT; ++i) imv[i] = src[tid + V2_THREADS * i];
    }
    // (1) Omega^T fragments of this chunk (used at its end)
    bf16x8_t of[8];
    if constexpr (WANTY) {
#pragma unroll
      for (int ks = 0; ks < 8; ++ks)
        of[ks] = *reinterpret_cast<const bf16x8_t*>(omT + (int64_t)ycol * NPADO + V2_CHUNK * j +
                                                    16 * ks + 8 * hl);
    }
    // (2) the chunk's values: 32 per lane.  The first chunk of a panel also
    // stores the previous panel's Y (after the wait, so that the count of
    // the next wait stays exact: those stores are older than the DMA of the
    // next chunk)
    float v[4][8];
    if constexpr (TAIL) {
      if (store_prev) store_y(p0 - V2_PR, V2_PR);
      // no DMA is in flight any more: fill ring stage st with the same
      // placement, rows past the end of the range read as zero
      {
        typedef const __attribute__((address_space(1))) float* gptr;
        float* dst = s_ring + st * V2_STAGE + wave * V2_WFL + 4 * lane;
#pragma unroll 1
        for (int q = 0; q < 8; ++q) {
          int cc = V2_CHUNK * j + colw + 8 * (q & 3) + dma_ci;
          cc = cc < n ? cc : n - 1;
          const gptr src = (gptr)(A + (int64_t)cc * lda + p0);
          f32x4_t a;
#pragma unroll
          for (int t = 0; t < 4; ++t) {
            const int r = 32 * (q >> 2) + 4 * dma_x + t;
            const float x = src[r < rows_left ? r : rows_left - 1];
            a[t] = r < rows_left ? x : 0.0f;
          }
          *reinterpret_cast<f32x4_t*>(dst + 256 * q) = a;
        }
      }
#pragma unroll
      for (int ks = 0; ks < 4; ++ks) ring_read(st, ks, v[ks]);
    } else {
      // the DMA of this chunk was issued two chunks ago; the one of the next
      // chunk (8 loads, if there is a next chunk: one_more) and this chunk's
      // Omega fragments (8) may still be outstanding
      // (with an image load this chunk: its MT = 4 loads as well)
      if constexpr (WANTY) {
        if (img) {
          if (one_more) asm volatile("s_waitcnt vmcnt(20)" ::: "memory");
          else asm volatile("s_waitcnt vmcnt(12)" ::: "memory");
        } else {
          if (one_more) asm volatile("s_waitcnt vmcnt(16)" ::: "memory");
          else asm volatile("s_waitcnt vmcnt(8)" ::: "memory");
        }
      } else {
        if (img) {
          if (one_more) asm volatile("s_waitcnt vmcnt(12)" ::: "memory");
          else asm volatile("s_waitcnt vmcnt(4)" ::: "memory");
        } else {
          if (one_more) asm volatile("s_waitcnt vmcnt(8)" ::: "memory");
          else asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
        }
      }
      if (store_prev) store_y(p0 - V2_PR, V2_PR);
      if constexpr (FP8) {
        // the tile scale needs all 64 rows first
#pragma unroll
        for (int ks = 0; ks < 4; ++ks) ring_read(st, ks, v[ks]);
      }
    }
    // (3) FP8: the column's 64-row tile scale (the other 32 rows are in lane
    // l ^ 32)
    float fs = 1.0f, fsi = 1.0f;
    if constexpr (FP8 && !TAIL) {
      // the stage is in registers: refill it with the chunk two ahead
      asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory");
      __builtin_amdgcn_sched_barrier(0);
      if (next_ok) dma(next_p0, next_j, st);
      __builtin_amdgcn_sched_barrier(0);
    }
    if constexpr (FP8) {
      float amax = 0.0f;
#pragma unroll
      for (int ks = 0; ks < 4; ++ks)
#pragma unroll
        for (int i = 0; i < 8; ++i) amax = fmaxf(amax, fabsf(v[ks][i]));
      amax = fmaxf(amax, __shfl_xor(amax, 32, 64));
      fs = fp8_tile_scale(amax, fsi);
    }
    // (4) the chunk buffer is free once every wave's Y products of the
    // previous chunk are done
    lds_barrier();
    const int pos = chk_pos(colw + lc);
    const __bf16* psi = s_psi[pb];
#pragma unroll
    for (int ks = 0; ks < 4; ++ks) {
      if constexpr (!FP8 && !TAIL) {
        // K step by K step from the ring; after the last read the stage is
        // refilled with the chunk two ahead
        ring_read(st, ks, v[ks]);
        if (ks == 3) {
          asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory");
          __builtin_amdgcn_sched_barrier(0);
          if (next_ok) dma(next_p0, next_j, st);
          __builtin_amdgcn_sched_barrier(0);
        }
      }
      bf16x8_t bh, bl;
#pragma unroll
      for (int i = 0; i < 8; ++i) {
        float x = col_ok ? v[ks][i] : 0.0f;
        if constexpr (FP8) x = e4m3_value(x * fsi) * fs;
        const __bf16 h = (__bf16)x;
        bh[i] = h;
        const int ci = (16 * ks + 8 * hl + i) * V2_CS + pos;
        if constexpr (WANTY) s_chk[0][ci] = h;
        if constexpr (SPLIT) {
          const __bf16 lo = (__bf16)(x - (float)h);
          bl[i] = lo;
          if constexpr (WANTY) s_chk[NH - 1][ci] = lo;
        }
      }
      // W(:, chunk) += Psi(:, panel) A(panel, chunk), K step ks
#pragma unroll
      for (int mt = 0; mt < MT; ++mt) {
        const int m = 32 * mt + lc;  // local Psi row
        const bf16x8_t af = *reinterpret_cast<const bf16x8_t*>(&psi[psi_idx(m, 16 * ks + 8 * hl)]);
        wacc[mt][j] = mfma32(af, bh, wacc[mt][j]);
        if constexpr (SPLIT) wacc[mt][j] = mfma32(af, bl, wacc[mt][j]);
      }
      __builtin_amdgcn_sched_barrier(0);
    }
    // (5) slice j of Psi(:, next panel), or the whole of it from its image
    if (PSI_IMG_OK && psi_img) {
      if (img) {
        bf16x8_t* dstp = reinterpret_cast<bf16x8_t*>(&s_psi[pb ^ 1][0]);
#pragma unroll
        for (int i = 0; i < MT; ++i) dstp[tid + V2_THREADS * i] = imv[i];
      }
    } else if (!TAIL && p0 + V2_PR < r1) {
      gen(p0 + V2_PR, pb ^ 1, gen_iters * j / NCT, gen_iters * (j + 1) / NCT);
    }
    lds_barrier();  // chunk buffer complete (and, after the last chunk, the next Psi)
    // (6) Y(panel, this wave's tiles) += A(panel, chunk) Omega(chunk, :)
    if constexpr (WANTY) {
#pragma unroll
      for (int ks = 0; ks < 8; ++ks) {
#pragma unroll
        for (int r = 0; r < YR; ++r) {
          const int ci = (32 * (yrt0 + r) + lc) * V2_CS + 16 * ks + 8 * hl;
          const bf16x8_t ah = *reinterpret_cast<const bf16x8_t*>(&s_chk[0][ci]);
          yacc[r] = mfma32(ah, of[ks], yacc[r]);
          if constexpr (SPLIT) {
            const bf16x8_t al = *reinterpret_cast<const bf16x8_t*>(&s_chk[NH - 1][ci]);
            yacc[r] = mfma32(al, of[ks], yacc[r]);
          }
        }
      }
    }
  };

  // ---- the row range -------------------------------------------------------
  // chunk sequence of the full panels: c = NCT * panel + j
  const int64_t nchunk = nfull * NCT;
  if (nchunk > 0) dma(r0, 0, 0);
  if (nchunk > 1) dma(r0 + (NCT > 1 ? 0 : V2_PR), NCT > 1 ? 1 : 0, 1);
  lds_barrier();  // zeroed Psi visible
  if (r0 < r1) {
    // in the chunks' slices (each within the unrolled bound GMAX)
#pragma unroll
    for (int j = 0; j < NCT; ++j) gen(r0, 0, gen_iters * j / NCT, gen_iters * (j + 1) / NCT);
    lds_barrier();
  }
  int pb = 0;
  int64_t c = 0;
  for (int64_t p = 0; p < nfull; ++p, pb ^= 1) {
    const int64_t p0 = r0 + p * V2_PR;
#pragma unroll
    for (int j = 0; j < NCT; ++j, ++c) {
      const int64_t cn = c + 2;
      const int64_t np0 = r0 + (cn / NCT) * V2_PR;
      chunk(std::false_type{}, p0, j, pb, (int)(c & 1), np0, (int)(cn % NCT), cn < nchunk,
            j == 0 && p > 0, c + 1 < nchunk);
    }
  }
  if (r1f < r1) {
#pragma unroll
    for (int j = 0; j < NCT; ++j)
      chunk(std::true_type{}, r1f, j, pb, 0, 0, 0, false, j == 0 && nfull > 0, false);
    store_y(r1f, (int)(r1 - r1f));
  } else if (nfull > 0) {
    store_y(r1f - V2_PR, V2_PR);
  }

  // ---- W partial of this workgroup (FP32, row-major lq x n) ----------------
  char* dst = reinterpret_cast<char*>(part + (pair * lq + mb) * (int64_t)n);
#pragma unroll
  for (int j = 0; j < NCT; ++j) {
    const int col = V2_CHUNK * j + colw + lc;
    const uint32_t ob = (uint32_t)((4 * hl * n + col) * 4);
#pragma unroll
    for (int mt = 0; mt < MT; ++mt) {
      f32x16_t t = wacc[mt][j];
      asm volatile("" : "+v"(t));  // read out here, tile by tile
#pragma unroll
      for (int e = 0; e < 16; ++e) {
        const int dm = 32 * mt + 8 * (e >> 2) + (e & 3);
        if (dm + 4 * hl < mc && col < n)
          *reinterpret_cast<float*>(dst + (ob + (uint32_t)(dm * n * 4))) = t[e];
      }
      // one tile at a time (its registers are read out just before its stores)
      __builtin_amdgcn_sched_barrier(0);
    }
  }
}

// W rows of the first half of the pair: a multiple of 4 near lq / 2
inline int v2_hsplit(int lq) { return 4 * ((lq + 7) / 8); }
// template W row tiles per half and Y column tiles per half of a shape
inline int v2_mt(int lq) { return (v2_hsplit(lq) + 31) / 32; }
inline int v2_lt(int l) { return l <= 128 ? 2 : 4; }

// accumulator registers per lane of a launch with nct chunks: W (MT x NCT
// tiles of 16) and, with Y, its tiles and the Omega fragments of a chunk;
// kept <= 288 so that the rest of the state fits the 512 a wave may hold
// without spilling
constexpr bool v2_fits_t(int mt, int nct, int lt, bool wanty) {
  return mt >= 1 && mt <= 4 && nct >= 1 && nct <= V2_MAXNCT &&
         mt * nct * 16 + (wanty ? (lt == 2 ? 1 : 2) * 16 + 32 : 0) <= 288;
}
inline bool v2_fits(int nct, int lq, int l, bool wanty) {
  return lq >= 2 && lq <= 256 && l >= 1 && l <= 256 &&
         v2_fits_t(v2_mt(lq), nct, v2_lt(l), wanty);
}

// launch of one template instance (none for shapes that do not fit)
template <int DM, bool WY, int MT, int NCT, int LT>
hipError_t v2_launch_one(hipStream_t st, dim3 grid, const float* A, int64_t lda, int64_t N, int n,
                         int lq, int l, uint64_t seed, const __bf16* omT, int64_t rpp, float* part,
                         float* Y, int yadd, const __bf16* psi_img) {
  if constexpr (v2_fits_t(MT, NCT, LT, WY)) {
    hipLaunchKernelGGL((k_sketch_v2<DM, WY, MT, NCT, LT>), grid, dim3(V2_THREADS), 0, st, A, lda,
                       N, n, lq, v2_hsplit(lq), l, seed, omT, rpp, part, Y, yadd,
                       MT == 4 ? psi_img : nullptr);
    return hipGetLastError();
  } else {
    return hipErrorInvalidValue;
  }
}

// every template instance of one data mode: MT 1..4, NCT 1..4, LT 2 or 4
template <int DM>
hipError_t v2_launch_dm(hipStream_t st, dim3 grid, const float* A, int64_t lda, int64_t N, int n,
                        int lq, int l, uint64_t seed, const __bf16* omT, int64_t rpp, float* part,
                        float* Y, int yadd, const __bf16* psi_img) {
  const int mt = v2_mt(lq), lt = v2_lt(l), nct = (n + V2_CHUNK - 1) / V2_CHUNK;
#define SID_V2(WY, MT_, NCT_, LT_) \
  return v2_launch_one<DM, WY, MT_, NCT_, LT_>(st, grid, A, lda, N, n, lq, l, seed, omT, rpp, part, Y, \
                                               yadd, psi_img)
#define SID_V2_LT(MT_, NCT_)                     \
  if (!Y) SID_V2(false, MT_, NCT_, 2);           \
  else if (lt == 2) SID_V2(true, MT_, NCT_, 2);  \
  else SID_V2(true, MT_, NCT_, 4);
#define SID_V2_NCT(MT_)                          \
  if (nct == 1) { SID_V2_LT(MT_, 1) }            \
  else if (nct == 2) { SID_V2_LT(MT_, 2) }       \
  else if (nct == 3) { SID_V2_LT(MT_, 3) }       \
  else { SID_V2_LT(MT_, 4) }
  if (mt == 1) { SID_V2_NCT(1) }
  else if (mt == 2) { SID_V2_NCT(2) }
  else if (mt == 3) { SID_V2_NCT(3) }
  else { SID_V2_NCT(4) }
#undef SID_V2_NCT
#undef SID_V2_LT
#undef SID_V2
}

hipError_t v2_launch_bf16(hipStream_t st, dim3 grid, const float* A, int64_t lda, int64_t N, int n,
                          int lq, int l, uint64_t seed, const __bf16* omT, int64_t rpp, float* part,
                          float* Y, int yadd, const __bf16* psi_img);
hipError_t v2_launch_bf16x2(hipStream_t st, dim3 grid, const float* A, int64_t lda, int64_t N,
                            int n, int lq, int l, uint64_t seed, const __bf16* omT, int64_t rpw,
                            float* part, float* Y, int yadd, const __bf16* psi_img);
hipError_t v2_launch_fp8(hipStream_t st, dim3 grid, const float* A, int64_t lda, int64_t N, int n,
                         int lq, int l, uint64_t seed, const __bf16* omT, int64_t rpw, float* part,
                         float* Y, int yadd, const __bf16* psi_img);

}  // namespace sid
