// sid_interp.hip -- single-pass ID with interpolation (Alg. 6, Sec. 2.6):
// the coarse skeleton A(S, J), the coarse-to-fine product Mf ACJ, and the
// fused reconstruction Ahat = Mf ACJ P (eq. (single_ID)) on the matrix cores.
//
// Mf is trilinear (piecewise linear per dimension, Sec. 3), applied as a
// tensor product from three 1-D tables: a fine point (c, ix, iy, iz) reads
// the 8 coarse rows ((c*mx + X)*my + Y)*mz + Z, X in {lo_x, hi_x} etc., with
// weight wx * (wy * wz) (the lower node of a dimension weighs 1 - w).
#include <hip/hip_runtime.h>

#include "sid_device.hpp"
#include "sid_interp.hpp"

namespace sid {

namespace {

typedef __bf16 bf16x8_t __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x2_t __attribute__((ext_vector_type(2)));
typedef float f32x2_t __attribute__((ext_vector_type(2)));
typedef float f32x4_t __attribute__((ext_vector_type(4)));
typedef float f32x16_t __attribute__((ext_vector_type(16)));
typedef uint32_t u32x4_t __attribute__((ext_vector_type(4)));

// two floats rounded to bfloat16 (nearest even) in one dword, first in the
// low half
__device__ __forceinline__ uint32_t pack_bf16x2(float a, float b) {
  return __builtin_bit_cast(uint32_t, __builtin_convertvector(f32x2_t{a, b}, bf16x2_t));
}

template <typename W>
__device__ __forceinline__ W table_weight(const InterpDev& t, int j);
template <>
__device__ __forceinline__ float table_weight<float>(const InterpDev& t, int j) {
  return t.w32[j];
}
template <>
__device__ __forceinline__ double table_weight<double>(const InterpDev& t, int j) {
  return t.w64[j];
}

// The 8 coarse rows and weights of fine row i (i < N < 2^31).
template <typename W>
__device__ __forceinline__ void stencil8(const InterpDev& t, uint32_t i, uint32_t idx[8],
                                        W w[8]) {
  const uint32_t nz = (uint32_t)t.nz, nyz = (uint32_t)t.ny * nz;
  const uint32_t per = (uint32_t)t.nx * nyz;
  const uint32_t c = i / per;
  uint32_t r = i - c * per;
  const uint32_t ix = r / nyz;
  r -= ix * nyz;
  const uint32_t iy = r / nz;
  const uint32_t iz = r - iy * nz;
  const int jy = t.nx + (int)iy, jz = t.nx + t.ny + (int)iz;
  const uint32_t xl = (uint32_t)t.lo[ix], xh = (uint32_t)t.hi[ix];
  const uint32_t yl = (uint32_t)t.lo[jy], yh = (uint32_t)t.hi[jy];
  const uint32_t zl = (uint32_t)t.lo[jz], zh = (uint32_t)t.hi[jz];
  const W wx1 = table_weight<W>(t, (int)ix), wy1 = table_weight<W>(t, jy),
          wz1 = table_weight<W>(t, jz);
  const W wx0 = W(1) - wx1, wy0 = W(1) - wy1, wz0 = W(1) - wz1;
  const uint32_t mx = (uint32_t)t.mx, my = (uint32_t)t.my, mz = (uint32_t)t.mz;
#pragma unroll
  for (int q = 0; q < 8; ++q) {
    const uint32_t X = (q & 4) ? xh : xl, Y = (q & 2) ? yh : yl, Z = (q & 1) ? zh : zl;
    w[q] = ((q & 4) ? wx1 : wx0) * (((q & 2) ? wy1 : wy0) * ((q & 1) ? wz1 : wz0));
    idx[q] = ((c * mx + X) * my + Y) * mz + Z;
  }
}

template <typename T>
__global__ void k_gather_coarse_skeleton(const T* __restrict__ A, int64_t lda,
                                         const int64_t* __restrict__ rows, int64_t Ns,
                                         const int64_t* __restrict__ piv,
                                         const int64_t* __restrict__ keff_p, T* __restrict__ dst,
                                         int64_t ldd) {
  const int keff = (int)*keff_p;
  const int t = blockIdx.y;
  const T* col = (t < keff) ? A + lda * piv[t] : nullptr;
  T* d = dst + ldd * t;
  for (int64_t s = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; s < Ns;
       s += (int64_t)gridDim.x * blockDim.x)
    d[s] = col ? col[rows[s]] : T(0);
}

// B(i, c) = sum_q w_q ACJ(idx_q, c): one thread per fine row, 16 columns per
// block row of the grid.
template <typename T>
__global__ __launch_bounds__(256) void k_interp_apply(InterpDev t, const T* __restrict__ ACJ,
                                                      int64_t ldacj, int k, T* __restrict__ B,
                                                      int64_t ldb) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= t.N) return;
  uint32_t idx[8];
  T w[8];
  stencil8<T>(t, (uint32_t)i, idx, w);
  const int c0 = blockIdx.y * 16;
  const int c1 = c0 + 16 < k ? c0 + 16 : k;
  for (int c = c0; c < c1; ++c) {
    const T* col = ACJ + ldacj * c;
    T acc = T(0);
#pragma unroll
    for (int q = 0; q < 8; ++q) acc = fma(w[q], col[idx[q]], acc);
    B[i + ldb * c] = acc;
  }
}

// acjt(s, c) = ACJ(s, c) for c < k, 0 for k <= c < kp (row-major, kp <= 128)
__global__ __launch_bounds__(256) void k_pack_acjt(const float* __restrict__ ACJ, int64_t ldacj,
                                                   int64_t Nc, int k, int kp,
                                                   float* __restrict__ acjt) {
  __shared__ float tile[64][129];
  const int64_t s0 = (int64_t)blockIdx.x * 64;
  for (int e = threadIdx.x; e < 64 * kp; e += 256) {
    const int s = e & 63, c = e >> 6;
    tile[s][c] = (s0 + s < Nc && c < k) ? ACJ[s0 + s + ldacj * c] : 0.0f;
  }
  __syncthreads();
  for (int e = threadIdx.x; e < 64 * kp; e += 256) {
    const int s = e / kp, c = e - s * kp;
    if (s0 + s < Nc) acjt[(s0 + s) * kp + c] = tile[s][c];
  }
}

// P as matrix-core B operands for 32x32x16 products: entry
// e = ((cb * ks_n + ks) * 2 + h) * 64 + lane holds
// P(16 ks + 8 (lane/32) + 0..7, 32 cb + lane%32), h = 0 the bfloat16
// rounding hi, h = 1 the rounding of the remainder lo (zero outside k x n).
__global__ __launch_bounds__(256) void k_pack_p(const float* __restrict__ P, int64_t ldp, int k,
                                                int64_t n, int ks_n, int64_t total,
                                                bf16x8_t* __restrict__ pb) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= total) return;
  const int lane = (int)(e & 63), h = (int)((e >> 6) & 1);
  const int64_t rest = e >> 7;
  const int ks = (int)(rest % ks_n);
  const int64_t cb = rest / ks_n;
  const int64_t col = cb * 32 + (lane & 31);
  const int kb = ks * 16 + 8 * (lane >> 5);
  bf16x8_t v;
#pragma unroll
  for (int i = 0; i < 8; ++i) {
    const int kk = kb + i;
    const float x = (kk < k && col < n) ? P[kk + ldp * col] : 0.0f;
    const __bf16 hb = (__bf16)x;
    v[i] = h ? (__bf16)(x - (float)hb) : hb;
  }
  pb[e] = v;
}

// Ahat = Mf ACJ P for 256 fine rows per block (4 waves of 64 rows, each two
// 32-row tiles of 32x32x16 bf16 MFMAs; k padded to KS = kp/16 steps).  Two
// blocks share a CU (LDS <= 80 KiB each), so one block's operand formation
// overlaps the other's products.
//  * Row tiles: blocks are dealt to the 8 XCDs round-robin, so block b
//    takes row tile XCD-major: each XCD works on one contiguous eighth of
//    the rows and its L2 holds the coarse rows that eighth's stencils read.
//  * Operands: each lane forms its slice of the interpolated skeleton rows
//    B = Mf ACJ (row lane%32 of each tile, columns 16 ks + 8 (lane/32) + 0..7)
//    from the row-major copy acjt, in FP32, and keeps it in registers split
//    into bfloat16 hi + lo for the whole block.
//  * P: the block walks the 32-column blocks of P (packed operands) through a
//    ring of 3 LDS buffers: the block's threads load column block cb + 3
//    while the waves multiply block cb and write it to LDS one block later,
//    so a load has two blocks' work to arrive; one barrier per block.
//  * Products: three MFMAs per tile and k-step (hi*hi + hi*lo + lo*hi),
//    consecutive MFMAs on different tiles' accumulators.
//  * Output: each wave turns its 64 x 32 result around in its own LDS tile
//    so that a store (or, ERR, a load of A to compare with) covers 4
//    columns x 64 consecutive rows, 256 contiguous bytes per column.
constexpr int IM_WAVES = 4;
constexpr int IM_ROWS = 64 * IM_WAVES;

// IDENT: the plain ID, Ahat = AJ P (eq. (ID)): row i of B is row i of AJ,
// read straight from the column-major N x kk skeleton `acjt` (ld ldaj); the
// operator tables are not used (t.N only).
template <int KS, bool ERR, bool VEC, bool IDENT = false>
__global__ __launch_bounds__(64 * IM_WAVES, 2) void k_interp_mfma(
    InterpDev t, const float* __restrict__ acjt, const bf16x8_t* __restrict__ pb, int64_t n,
    float* __restrict__ out, int64_t ldo, const float* __restrict__ A, int64_t lda,
    double* __restrict__ part, int64_t ldaj = 0, int kk = 0) {
  constexpr int KP = 16 * KS;
  constexpr int NT = 64 * IM_WAVES;
  constexpr int PCH = KS * 128;             // packed operands per 32-column block
  constexpr int PPT = (PCH + NT - 1) / NT;  // of them per thread in the block's copy
  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int hl = lane >> 5, lc = lane & 31;
  const int g = lane >> 4, li = lane & 15;
  const int64_t nbk = gridDim.x, b = blockIdx.x;
  const int64_t Q = nbk / 8, R = nbk % 8, xcd = b % 8;
  const int64_t tile = xcd * Q + (xcd < R ? xcd : R) + b / 8;
  const int64_t r0 = tile * IM_ROWS + wave * 64;
  const int64_t N = t.N;

  u32x4_t ah[2][KS], al[2][KS];  // 8 bfloat16 each, packed two per dword
#pragma unroll
  for (int rt = 0; rt < 2; ++rt) {
    // rows past N (ragged last block) take row N-1's stencil with zero
    // weights: no branch, so the load groups below stay in order
    const int64_t i = r0 + 32 * rt + lc;
    uint32_t idx[8];
    float w[8];
    if constexpr (!IDENT) stencil8<float>(t, (uint32_t)(i < N ? i : N - 1), idx, w);
    const float live = i < N ? 1.0f : 0.0f;
#pragma unroll
    for (int q = 0; q < 8; ++q) w[q] = IDENT ? live : w[q] * live;
#pragma unroll
    for (int ks = 0; ks < KS; ++ks) {
      float acc[8];
#pragma unroll
      for (int e = 0; e < 8; ++e) acc[e] = 0.0f;
      if constexpr (IDENT) {
        // eight skeleton columns of one row: lanes 0-31 and 32-63 each read
        // 32 consecutive rows (128 bytes) of one column per load
        const int64_t ic = i < N ? i : N - 1;
#pragma unroll
        for (int e = 0; e < 8; ++e) {
          const int c = 16 * ks + 8 * hl + e;
          acc[e] = c < kk ? w[0] * acjt[(int64_t)c * ldaj + ic] : 0.0f;
        }
      } else {
#pragma unroll
        for (int q = 0; q < 8; ++q) {
          const f32x4_t* src =
              reinterpret_cast<const f32x4_t*>(acjt + (size_t)idx[q] * KP + 16 * ks + 8 * hl);
          const f32x4_t v0 = src[0], v1 = src[1];
#pragma unroll
          for (int e = 0; e < 4; ++e) {
            acc[e] = fmaf(w[q], v0[e], acc[e]);
            acc[4 + e] = fmaf(w[q], v1[e], acc[4 + e]);
          }
        }
      }
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const uint32_t h = pack_bf16x2(acc[2 * e], acc[2 * e + 1]);
        ah[rt][ks][e] = h;
        al[rt][ks][e] = pack_bf16x2(acc[2 * e] - __uint_as_float(h << 16),
                                    acc[2 * e + 1] - __uint_as_float(h & 0xffff0000u));
      }
      // one (tile, k-step) group of 16 loads in flight at a time: hoisting
      // all of them would need more registers than the operands themselves.
      // The empty asm takes this group's operands and clobbers memory, so
      // they are formed before the next group's loads are issued.
      asm volatile("" ::"v"(ah[rt][ks]), "v"(al[rt][ks]) : "memory");
    }
  }

  __shared__ bf16x8_t s_p[3][PCH];
  // per wave: 32 columns x 64 rows, rows contiguous, padded against bank
  // conflicts (except at KS = 8, where the padding would not leave two
  // blocks room in a CU's LDS); only this wave touches it, and a wave's LDS
  // accesses execute in order, so the exchange needs no barrier (the empty
  // asms below keep the compiler from reordering across it)
  constexpr int TS = KS < 8 ? 68 : 64;
  __shared__ __attribute__((aligned(16))) float s_t[IM_WAVES][32 * TS];
  float* tw = s_t[wave];
  const int64_t ncb = (n + 31) / 32;
  // pb holds 3 column blocks of operands beyond the last one, so the loads
  // ahead need no bound
  auto gload = [&](int64_t cbl, bf16x8_t* Rg) {
#pragma unroll
    for (int k2 = 0; k2 < PPT; ++k2) {
      const int e = tid + NT * k2;
      if (e < PCH) Rg[k2] = pb[cbl * PCH + e];
    }
  };
  auto stash = [&](int buf, const bf16x8_t* Rg) {
#pragma unroll
    for (int k2 = 0; k2 < PPT; ++k2) {
      const int e = tid + NT * k2;
      if (e < PCH) s_p[buf][e] = Rg[k2];
    }
  };
  bf16x8_t RA[PPT], RB[PPT];
  gload(0, RA);
  stash(0, RA);
  gload(1, RA);
  stash(1, RA);
  gload(2, RA);

  // ERR: the 8 x 4 values of A this lane compares in a column block (store
  // layout), loaded before the block's MFMAs so their latency overlaps them
  const int64_t row = r0 + 4 * li;
  // error sums; the largest |A - Ahat| / |A| is kept as the pair (num, den)
  // and compared by cross-multiplication (exact: both differences and |A|
  // are FP32 values or exact differences of two, their products fit FP64),
  // so the loop divides nothing
  double se = 0.0, sa = 0.0, mabs = 0.0, rnum = 0.0, rden = 1.0;

  // The column-block loop, instantiated for the block's rows all below N or
  // not (TAIL) and, within it, for the last column block or not (LAST): the
  // steady state has no branch around a memory access, so the compiler
  // waits for each P load by its exact place in the wave's (in-order) count
  // of memory operations instead of for all of them, and the stores of a
  // block stay in flight while the next block is multiplied.
  auto run = [&](auto tail_tag) {
    constexpr bool TAIL = decltype(tail_tag)::value;
    constexpr bool FULL = VEC && !TAIL;  // 16-byte accesses for every lane
    // A for columns 16 half + 0..15 of block cbl, in the store layout
    auto load_a = [&](int64_t cbl, int half, f32x4_t* dst4, auto last_tag) {
      constexpr bool LAST = decltype(last_tag)::value;
#pragma unroll
      for (int s4 = 0; s4 < 4; ++s4) {
        const int64_t j = cbl * 32 + 16 * half + 4 * s4 + g;
        const float* src = A + j * lda + row;
        if constexpr (FULL) {
          if (!LAST || j < n) dst4[s4] = *reinterpret_cast<const f32x4_t*>(src);
          else dst4[s4] = f32x4_t{0.0f, 0.0f, 0.0f, 0.0f};
        } else {
#pragma unroll
          for (int e = 0; e < 4; ++e)
            dst4[s4][e] = ((!LAST || j < n) && (!TAIL || row + e < N)) ? src[e] : 0.0f;
        }
      }
    };
    // one column block: Rl receives block cb + 3, Rs (block cb + 2, loaded
    // one step earlier) goes to LDS
    auto step = [&](int64_t cb, bf16x8_t* Rl, const bf16x8_t* Rs, auto last_tag) {
      constexpr bool LAST = decltype(last_tag)::value;
      gload(cb + 3, Rl);
      // ERR: the first half of the block's A before the MFMAs, the second
      // right after them (all eight at once would not fit the registers)
      f32x4_t Ac0[4], Ac1[4];
      if constexpr (ERR) load_a(cb, 0, Ac0, last_tag);
      const bf16x8_t* pw = s_p[cb % 3];
      f32x16_t acc[2];
#pragma unroll
      for (int rt = 0; rt < 2; ++rt)
#pragma unroll
        for (int e = 0; e < 16; ++e) acc[rt][e] = 0.0f;
      // consecutive MFMAs go to different tiles' accumulators
#pragma unroll
      for (int ks = 0; ks < KS; ++ks) {
        const bf16x8_t bh = pw[(ks * 2 + 0) * 64 + lane];
        const bf16x8_t bl = pw[(ks * 2 + 1) * 64 + lane];
#pragma unroll
        for (int rt = 0; rt < 2; ++rt)
          acc[rt] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(
              __builtin_bit_cast(bf16x8_t, ah[rt][ks]), bh, acc[rt], 0, 0, 0);
#pragma unroll
        for (int rt = 0; rt < 2; ++rt)
          acc[rt] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(
              __builtin_bit_cast(bf16x8_t, ah[rt][ks]), bl, acc[rt], 0, 0, 0);
#pragma unroll
        for (int rt = 0; rt < 2; ++rt)
          acc[rt] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(
              __builtin_bit_cast(bf16x8_t, al[rt][ks]), bh, acc[rt], 0, 0, 0);
      }
      if constexpr (ERR) load_a(cb, 1, Ac1, last_tag);
      // MFMA layout: lane (lc, hl) holds column lc, rows
      // 32 rt + 8 (e/4) + 4 hl + e%4 in accumulator e
#pragma unroll
      for (int rt = 0; rt < 2; ++rt)
#pragma unroll
        for (int jq = 0; jq < 4; ++jq)
          *reinterpret_cast<f32x4_t*>(tw + lc * TS + 32 * rt + 8 * jq + 4 * hl) =
              f32x4_t{acc[rt][4 * jq], acc[rt][4 * jq + 1], acc[rt][4 * jq + 2],
                      acc[rt][4 * jq + 3]};
      asm volatile("" ::: "memory");
      // store layout: lane (li, g) takes column 4 s + g, rows 4 li + 0..3
#pragma unroll
      for (int s8 = 0; s8 < 8; ++s8) {
        const int col = 4 * s8 + g;
        const f32x4_t v = *reinterpret_cast<const f32x4_t*>(tw + col * TS + 4 * li);
        const int64_t j = cb * 32 + col;
        const bool jok = !LAST || j < n;
        if constexpr (!ERR) {
          float* dst = out + j * ldo + row;
          if constexpr (FULL) {
            if (jok) __builtin_nontemporal_store(v, reinterpret_cast<f32x4_t*>(dst));
          } else {
#pragma unroll
            for (int e = 0; e < 4; ++e)
              if (jok && (!TAIL || row + e < N)) dst[e] = v[e];
          }
        } else {
#pragma unroll
          for (int e = 0; e < 4; ++e) {
            if (jok && (!TAIL || row + e < N)) {
              const double a = (double)(s8 < 4 ? Ac0[s8 & 3][e] : Ac1[s8 & 3][e]);
              const double d = a - (double)v[e];
              se = fma(d, d, se);
              sa = fma(a, a, sa);
              const double ad = fabs(d), aa = fabs(a);
              mabs = fmax(mabs, ad);
              const bool better = a != 0.0 && ad * rden > rnum * aa;
              rnum = better ? ad : rnum;
              rden = better ? aa : rden;
            }
          }
          // one column's entries at a time: without this the scheduler
          // interleaves all entries' FP64 work and runs out of registers
          asm volatile("" : "+v"(se), "+v"(sa), "+v"(mabs), "+v"(rnum), "+v"(rden));
        }
      }
      asm volatile("" ::: "memory");
      stash((int)((cb + 2) % 3), Rs);
      __syncthreads();
    };
    using F = std::false_type;
    using T = std::true_type;
    // steady pairs (unrolled so that RA and RB swap roles without copies)
    // while at least one block follows them, then the last one or two
    int64_t cb = 0;
    for (; cb + 2 < ncb; cb += 2) {
      step(cb, RB, RA, F{});
      step(cb + 1, RA, RB, F{});
    }
    if (cb + 1 < ncb) {
      step(cb, RB, RA, F{});
      step(cb + 1, RA, RB, T{});
    } else {
      step(cb, RB, RA, T{});
    }
  };
  __syncthreads();
  const bool tail_block = tile * IM_ROWS + IM_ROWS > N;
  if (tail_block) run(std::true_type{});
  else run(std::false_type{});

  if constexpr (ERR) {
    // the reduction reuses the transposition tiles (the loop ended with a
    // barrier, so no wave still reads them)
    double(*s_r)[4] = reinterpret_cast<double(*)[4]>(&s_t[0][0]);
    double mrel = rnum / rden;
    se = wave_sum(se);
    sa = wave_sum(sa);
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
      mrel = fmax(mrel, __shfl_xor(mrel, o, 64));
      mabs = fmax(mabs, __shfl_xor(mabs, o, 64));
    }
    if (lane == 0) {
      s_r[wave][0] = se;
      s_r[wave][1] = sa;
      s_r[wave][2] = mrel;
      s_r[wave][3] = mabs;
    }
    __syncthreads();
    if (tid == 0) {
      double a = 0, bsum = 0, c = 0, d = 0;
      for (int v = 0; v < IM_WAVES; ++v) {
        a += s_r[v][0];
        bsum += s_r[v][1];
        c = fmax(c, s_r[v][2]);
        d = fmax(d, s_r[v][3]);
      }
      double* o = part + 4 * b;
      o[0] = a;
      o[1] = bsum;
      o[2] = c;
      o[3] = d;
    }
  }
}

// out4 = (sqrt(sum of part[4b]), sqrt(sum of part[4b+1]), max part[4b+2],
// max part[4b+3]) over the nb blocks' partials
__global__ __launch_bounds__(256) void k_interp_norms_reduce(const double* __restrict__ part,
                                                             int64_t nb,
                                                             double* __restrict__ out4) {
  __shared__ double s[4][256];
  double a = 0.0, b = 0.0, c = 0.0, d = 0.0;
  for (int64_t e = threadIdx.x; e < nb; e += 256) {
    a += part[4 * e];
    b += part[4 * e + 1];
    c = fmax(c, part[4 * e + 2]);
    d = fmax(d, part[4 * e + 3]);
  }
  s[0][threadIdx.x] = a;
  s[1][threadIdx.x] = b;
  s[2][threadIdx.x] = c;
  s[3][threadIdx.x] = d;
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if ((int)threadIdx.x < h) {
      s[0][threadIdx.x] += s[0][threadIdx.x + h];
      s[1][threadIdx.x] += s[1][threadIdx.x + h];
      s[2][threadIdx.x] = fmax(s[2][threadIdx.x], s[2][threadIdx.x + h]);
      s[3][threadIdx.x] = fmax(s[3][threadIdx.x], s[3][threadIdx.x + h]);
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    out4[0] = sqrt(s[0][0]);
    out4[1] = sqrt(s[1][0]);
    out4[2] = s[2][0];
    out4[3] = s[3][0];
  }
}

template <int KS, bool ERR, bool IDENT = false>
hipError_t launch_mfma_vec(hipStream_t st, bool vec, const InterpDev& t, const float* acjt,
                           const bf16x8_t* pb, int64_t n, float* out, int64_t ldo, const float* A,
                           int64_t lda, double* part, int64_t ldaj = 0, int kk = 0) {
  const dim3 grid((unsigned)interp_mfma_blocks(t.N));
  if (vec)
    hipLaunchKernelGGL((k_interp_mfma<KS, ERR, true, IDENT>), grid, dim3(64 * IM_WAVES), 0, st, t,
                       acjt, pb, n, out, ldo, A, lda, part, ldaj, kk);
  else
    hipLaunchKernelGGL((k_interp_mfma<KS, ERR, false, IDENT>), grid, dim3(64 * IM_WAVES), 0, st, t,
                       acjt, pb, n, out, ldo, A, lda, part, ldaj, kk);
  return hipGetLastError();
}

template <bool ERR, bool IDENT = false>
hipError_t launch_mfma_ks(hipStream_t st, int ks, bool vec, const InterpDev& t, const float* acjt,
                          const bf16x8_t* pb, int64_t n, float* out, int64_t ldo, const float* A,
                          int64_t lda, double* part, int64_t ldaj = 0, int kk = 0) {
#define SID_MKS(K_) \
  return launch_mfma_vec<K_, ERR, IDENT>(st, vec, t, acjt, pb, n, out, ldo, A, lda, part, ldaj, kk)
  switch (ks) {
    case 1: SID_MKS(1);
    case 2: SID_MKS(2);
    case 3: SID_MKS(3);
    case 4: SID_MKS(4);
    case 5: SID_MKS(5);
    case 6: SID_MKS(6);
    case 7: SID_MKS(7);
    case 8: SID_MKS(8);
    default: return hipErrorInvalidValue;
  }
#undef SID_MKS
}

}  // namespace

hipError_t launch_gather_coarse_skeleton(hipStream_t st, const void* A, bool f64, int64_t lda,
                                         const int64_t* rows, int64_t Ns, const int64_t* piv,
                                         const int64_t* keff, int kcap, void* dst, int64_t ldd) {
  int64_t bx = (Ns + 255) / 256;
  if (bx > 2048) bx = 2048;
  const dim3 grid((unsigned)bx, (unsigned)kcap);
  if (f64)
    hipLaunchKernelGGL(k_gather_coarse_skeleton<double>, grid, dim3(256), 0, st,
                       (const double*)A, lda, rows, Ns, piv, keff, (double*)dst, ldd);
  else
    hipLaunchKernelGGL(k_gather_coarse_skeleton<float>, grid, dim3(256), 0, st, (const float*)A,
                       lda, rows, Ns, piv, keff, (float*)dst, ldd);
  return hipGetLastError();
}

hipError_t launch_interp_apply(hipStream_t st, const InterpDev& t, bool f64, const void* ACJ,
                               int64_t ldacj, int k, void* B, int64_t ldb) {
  const dim3 grid((unsigned)((t.N + 255) / 256), (unsigned)((k + 15) / 16));
  if (f64)
    hipLaunchKernelGGL(k_interp_apply<double>, grid, dim3(256), 0, st, t, (const double*)ACJ,
                       ldacj, k, (double*)B, ldb);
  else
    hipLaunchKernelGGL(k_interp_apply<float>, grid, dim3(256), 0, st, t, (const float*)ACJ,
                       ldacj, k, (float*)B, ldb);
  return hipGetLastError();
}

size_t interp_pb_bytes(int64_t n, int kp) {
  // three blocks beyond the last one: the fused kernel loads ahead unguarded
  const int64_t ncb = (n + 31) / 32;
  return (size_t)(ncb + 3) * (size_t)(kp / 16) * 2 * 64 * sizeof(bf16x8_t);
}

hipError_t launch_interp_pack(hipStream_t st, const float* ACJ, int64_t ldacj, int64_t Nc, int k,
                              int kp, float* acjt, const float* P, int64_t ldp, int64_t n,
                              void* pb) {
  if (kp % 16 != 0 || kp < 16 || kp > 128 || k > kp) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_pack_acjt, dim3((unsigned)((Nc + 63) / 64)), dim3(256), 0, st, ACJ, ldacj,
                     Nc, k, kp, acjt);
  const int ks_n = kp / 16;
  const int64_t total = ((n + 31) / 32) * ks_n * 128;
  hipLaunchKernelGGL(k_pack_p, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, st, P, ldp, k,
                     n, ks_n, total, (bf16x8_t*)pb);
  return hipGetLastError();
}

int64_t interp_mfma_blocks(int64_t N) { return (N + IM_ROWS - 1) / IM_ROWS; }

hipError_t launch_interp_mfma(hipStream_t st, const InterpDev& t, int kp, const float* acjt,
                              const void* pb, int64_t n, float* out, int64_t ldo, const float* A,
                              int64_t lda, double* part, int64_t part_cap, double* out4) {
  if (kp % 16 != 0 || kp < 16 || kp > 128) return hipErrorInvalidValue;
  const int ks = kp / 16;
  const bf16x8_t* p = (const bf16x8_t*)pb;
  if (A) {
    if (interp_mfma_blocks(t.N) > part_cap) return hipErrorInvalidValue;
    const bool vec = lda % 4 == 0 && ((uintptr_t)A & 15) == 0;
    hipError_t e = launch_mfma_ks<true>(st, ks, vec, t, acjt, p, n, nullptr, 0, A, lda, part);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_interp_norms_reduce, dim3(1), dim3(256), 0, st, part,
                       interp_mfma_blocks(t.N), out4);
    return hipGetLastError();
  }
  const bool vec = ldo % 4 == 0 && ((uintptr_t)out & 15) == 0;
  return launch_mfma_ks<false>(st, ks, vec, t, acjt, p, n, out, ldo, nullptr, 0, nullptr);
}

hipError_t launch_pack_p(hipStream_t st, const float* P, int64_t ldp, int k, int kp, int64_t n,
                         void* pb) {
  if (kp % 16 != 0 || kp < 16 || kp > 128 || k > kp) return hipErrorInvalidValue;
  const int ks_n = kp / 16;
  const int64_t total = ((n + 31) / 32) * ks_n * 128;
  hipLaunchKernelGGL(k_pack_p, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, st, P, ldp, k,
                     n, ks_n, total, (bf16x8_t*)pb);
  return hipGetLastError();
}

hipError_t launch_id_mfma(hipStream_t st, const float* AJ, int64_t ldaj, int64_t N, int k, int kp,
                          const void* pb, int64_t n, float* out, int64_t ldo, const float* A,
                          int64_t lda, double* part, int64_t part_cap, double* out4) {
  if (kp % 16 != 0 || kp < 16 || kp > 128 || k > kp || N < 1) return hipErrorInvalidValue;
  InterpDev t{};
  t.N = N;
  const int ks = kp / 16;
  const bf16x8_t* p = (const bf16x8_t*)pb;
  if (A) {
    if (interp_mfma_blocks(N) > part_cap) return hipErrorInvalidValue;
    const bool vec = lda % 4 == 0 && ((uintptr_t)A & 15) == 0;
    hipError_t e = launch_mfma_ks<true, true>(st, ks, vec, t, AJ, p, n, nullptr, 0, A, lda, part,
                                              ldaj, k);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_interp_norms_reduce, dim3(1), dim3(256), 0, st, part,
                       interp_mfma_blocks(N), out4);
    return hipGetLastError();
  }
  const bool vec = ldo % 4 == 0 && ((uintptr_t)out & 15) == 0;
  return launch_mfma_ks<false, true>(st, ks, vec, t, AJ, p, n, out, ldo, nullptr, 0, nullptr, ldaj,
                                     k);
}

}  // namespace sid
