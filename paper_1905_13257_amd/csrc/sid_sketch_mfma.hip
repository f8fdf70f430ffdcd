// sid_sketch_mfma.hip -- the sketch pass as one streaming read of A on the
// gfx950 matrix cores (bfloat16 MFMA, FP32 accumulation).
//
// One pass over A forms both sketches of the single-pass ID:
//   W = Psi A   ((lq x n), the Gaussian sketch whose first l rows select the
//               skeleton, Alg. 4 "Y <- A Omega" in the paper's row orientation)
//   Y = A Omega (N x l, the range sketch of the two-sided single-pass sketch,
//               Halko et al. Sec. 5.5 items (1)-(2), quoted in Sec. 2.3).
//
// Layout of the work.  One persistent 512-thread workgroup per CU owns a
// contiguous range of rows of A and walks it in panels of 32 rows:
//   * each wave loads its 64-column slice of the panel from HBM straight into
//     registers in the MFMA B-operand layout (8 consecutive rows of one
//     column per lane), splits FP32 -> bf16 hi (+ lo) and
//       - accumulates W(:, slice) += Psi(:, panel) A(panel, slice) in
//         registers (the W partial stays on chip for the whole row range);
//       - writes the bf16 values transposed into LDS (row-major panel);
//   * Psi(:, panel) is generated in place (Philox + Box-Muller, bf16) into
//     LDS in the A-operand layout;
//   * each wave then computes a 16 x 32 block of Y(panel, :) = A(panel, :)
//     Omega from the row-major panel in LDS and Omega^T (bf16) read through
//     L2, and stores it.
// The W partial of each workgroup is written once at the end (FP32) and the
// partials are summed in a fixed order in FP64 by k_reduce_partials_f32.
//
// MFMA operand layouts used (v_mfma_f32_16x16x32_bf16, wave64):
//   A (16 x 32): lane l holds row l%16, k = 8*(l/16) .. +7
//   B (32 x 16): lane l holds col l%16, k = 8*(l/16) .. +7
//   C (16 x 16): lane l holds col l%16, rows 4*(l/16) .. +3
#include "sid_kernels.hpp"

namespace sid {

typedef __bf16 bf16x8_t __attribute__((ext_vector_type(8)));
typedef float f32x4_t __attribute__((ext_vector_type(4)));

constexpr int FB_WAVES = 4;                  // one wave per SIMD
constexpr int FB_THREADS = 64 * FB_WAVES;
constexpr int FB_PB = 32;                    // rows per panel (one K step of 32)
constexpr int FB_CTW = 8;                    // 16-column tiles per wave -> 128 columns per wave
constexpr int FB_NPAD = FB_WAVES * 16 * FB_CTW;  // 512: max columns
constexpr int FB_AROW = FB_NPAD + 8;      // LDS row stride of the panel (bf16), padded
constexpr int FB_PROW = FB_PB + 8;        // LDS row stride of Psi (bf16), padded

__device__ __forceinline__ __bf16 to_bf16(float f) { return (__bf16)f; }

// MT: 16-row tiles of W (lq <= 16*MT); LT: 16-column tiles of Y (l <= 16*LT)
template <bool SPLIT, int MT, int LT>
__global__ __launch_bounds__(FB_THREADS) void k_sketch_fused_bf16(
    const float* __restrict__ A, int64_t lda, int64_t N, int n, int lq, int l, uint64_t seed,
    const __bf16* __restrict__ omT /* LT*16 x FB_NPAD, k contiguous, zero padded */,
    int64_t rows_per_wg, float* __restrict__ part /* grid x lq x n */, float* __restrict__ Y) {
  static_assert((2 * LT) % FB_WAVES == 0, "Y tiles are split evenly over the waves");
  __shared__ __attribute__((aligned(16))) __bf16 s_ahi[FB_PB * FB_AROW];
  __shared__ __attribute__((aligned(16))) __bf16 s_alo[SPLIT ? FB_PB * FB_AROW : 8];
  __shared__ __attribute__((aligned(16))) __bf16 s_psi[MT * 16 * FB_PROW];

  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int lr = lane & 15, lg = lane >> 4;  // MFMA lane coordinates
  const int64_t r0 = (int64_t)blockIdx.x * rows_per_wg;
  int64_t r1 = r0 + rows_per_wg;
  if (r1 > N) r1 = N;

  // Psi rows >= lq stay zero for the whole kernel
  for (int e = tid; e < MT * 16 * FB_PROW; e += FB_THREADS) s_psi[e] = to_bf16(0.0f);

  f32x4_t wacc[MT][FB_CTW];
#pragma unroll
  for (int mt = 0; mt < MT; ++mt)
#pragma unroll
    for (int ct = 0; ct < FB_CTW; ++ct) wacc[mt][ct] = f32x4_t{0.f, 0.f, 0.f, 0.f};

  // Y tiles of this wave: row tile yr (0/1), column tiles yc0 .. yc0 + YT - 1
  constexpr int YT = 2 * LT / FB_WAVES;
  const int yr = wave & 1;
  const int yc0 = (wave >> 1) * YT;
  const int lq4 = (lq + 3) >> 2;

  for (int64_t p0 = r0; p0 < r1; p0 += FB_PB) {
    const int nrow = (int)((r1 - p0 < FB_PB) ? (r1 - p0) : FB_PB);
    __syncthreads();  // previous panel's LDS reads are done

    // (1) issue the loads of this wave's A slice (B-operand layout: lane =
    //     8 consecutive panel rows of one column), FP32 in registers
    float v[FB_CTW][8];
    const int rl = 8 * lg;  // first panel row of this lane
#pragma unroll
    for (int ct = 0; ct < FB_CTW; ++ct) {
      const int col = wave * (16 * FB_CTW) + ct * 16 + lr;
      if (col < n && rl + 8 <= nrow) {
        const f32x4_t* src = reinterpret_cast<const f32x4_t*>(A + (int64_t)col * lda + p0 + rl);
        const f32x4_t a0 = __builtin_nontemporal_load(src);
        const f32x4_t a1 = __builtin_nontemporal_load(src + 1);
#pragma unroll
        for (int t = 0; t < 4; ++t) {
          v[ct][t] = a0[t];
          v[ct][4 + t] = a1[t];
        }
      } else {
#pragma unroll
        for (int t = 0; t < 8; ++t)
          v[ct][t] = (col < n && rl + t < nrow) ? A[(int64_t)col * lda + p0 + rl + t] : 0.0f;
      }
    }

    // (2) Psi(0:lq, panel) in place, A-operand layout s_psi[m][k]
#pragma unroll 1
    for (int w = tid; w < FB_PB * lq4; w += FB_THREADS) {
      const int kk = w / lq4, g = w - kk * lq4;
      float z[4] = {0.f, 0.f, 0.f, 0.f};
      if (kk < nrow) gauss4(seed, 1u, (uint64_t)(p0 + kk), (uint32_t)g, z);
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int m = 4 * g + e;
        if (m < lq) s_psi[m * FB_PROW + kk] = to_bf16(z[e]);
      }
    }
    __syncthreads();

    // (3) split to bf16 hi (+ lo), with a transposed copy into the row-major
    //     panel for Y, then W(:, slice) += Psi(:, panel) A(panel, slice)
    bf16x8_t bhi[FB_CTW], blo[FB_CTW];
#pragma unroll
    for (int ct = 0; ct < FB_CTW; ++ct) {
      const int col = wave * (16 * FB_CTW) + ct * 16 + lr;
#pragma unroll
      for (int t = 0; t < 8; ++t) {
        const __bf16 h = to_bf16(v[ct][t]);
        bhi[ct][t] = h;
        s_ahi[(rl + t) * FB_AROW + col] = h;
        if constexpr (SPLIT) {
          const __bf16 lo = to_bf16(v[ct][t] - (float)h);
          blo[ct][t] = lo;
          s_alo[(rl + t) * FB_AROW + col] = lo;
        }
      }
    }
#pragma unroll
    for (int mt = 0; mt < MT; ++mt) {
      const bf16x8_t af = *reinterpret_cast<const bf16x8_t*>(&s_psi[(mt * 16 + lr) * FB_PROW + 8 * lg]);
#pragma unroll
      for (int ct = 0; ct < FB_CTW; ++ct) {
        wacc[mt][ct] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af, bhi[ct], wacc[mt][ct], 0, 0, 0);
        if constexpr (SPLIT)
          wacc[mt][ct] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af, blo[ct], wacc[mt][ct], 0, 0, 0);
      }
    }
    __syncthreads();  // row-major panel complete

    // (4) Y(panel rows yr*16.., cols yc..) = A(panel, :) Omega
    if (Y) {
      f32x4_t yacc[YT];
#pragma unroll
      for (int j = 0; j < YT; ++j) yacc[j] = f32x4_t{0.f, 0.f, 0.f, 0.f};
      const int ncol_pad = (n + 31) & ~31;
#pragma unroll 1
      for (int k0 = 0; k0 < ncol_pad; k0 += 32) {
        const bf16x8_t ah = *reinterpret_cast<const bf16x8_t*>(&s_ahi[(yr * 16 + lr) * FB_AROW + k0 + 8 * lg]);
        bf16x8_t al;
        if constexpr (SPLIT) al = *reinterpret_cast<const bf16x8_t*>(&s_alo[(yr * 16 + lr) * FB_AROW + k0 + 8 * lg]);
#pragma unroll
        for (int j = 0; j < YT; ++j) {
          const bf16x8_t of = *reinterpret_cast<const bf16x8_t*>(&omT[(int64_t)((yc0 + j) * 16 + lr) * FB_NPAD + k0 + 8 * lg]);
          yacc[j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, of, yacc[j], 0, 0, 0);
          if constexpr (SPLIT) yacc[j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al, of, yacc[j], 0, 0, 0);
        }
      }
#pragma unroll
      for (int j = 0; j < YT; ++j) {
        const int c = (yc0 + j) * 16 + lr;
        if (c < l) {
#pragma unroll
          for (int t = 0; t < 4; ++t) {
            const int rr = yr * 16 + 4 * lg + t;
            if (rr < nrow) Y[(p0 + rr) * (int64_t)l + c] = yacc[j][t];
          }
        }
      }
    }
  }

  // W partial of this workgroup (FP32, column-major lq x n)
  float* dst = part + (int64_t)blockIdx.x * lq * n;
#pragma unroll
  for (int ct = 0; ct < FB_CTW; ++ct) {
    const int col = wave * (16 * FB_CTW) + ct * 16 + lr;
    if (col >= n) continue;
#pragma unroll
    for (int mt = 0; mt < MT; ++mt)
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        const int m = mt * 16 + 4 * lg + t;
        if (m < lq) dst[m + (int64_t)lq * col] = wacc[mt][ct][t];
      }
  }
}

// Omega^T in bfloat16, zero padded: out[c * FB_NPAD + k] = bf16(G(seed, 0, k, c))
__global__ void k_omega_t_bf16(const float* __restrict__ omega /* n x l row-major */, int n, int l,
                               int lpad, __bf16* __restrict__ out) {
  for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < lpad * FB_NPAD; e += gridDim.x * blockDim.x) {
    const int c = e / FB_NPAD, k = e - c * FB_NPAD;
    out[e] = to_bf16((c < l && k < n) ? omega[k * l + c] : 0.0f);
  }
}

__global__ void k_reduce_partials_f32(const float* __restrict__ part, int64_t nparts, int64_t count,
                                      double* __restrict__ out) {
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < count;
       e += (int64_t)gridDim.x * blockDim.x) {
    double s = 0.0;
    for (int64_t g = 0; g < nparts; ++g) s += (double)part[g * count + e];
    out[e] = s;
  }
}

bool fused_bf16_supported(int64_t n, int lq, int l, int64_t lda, const void* A, bool has_rows) {
  return !has_rows && n <= FB_NPAD && lq <= 160 && l <= 128 && (lda % 4) == 0 &&
         ((uintptr_t)A % 16) == 0;
}

int64_t fused_bf16_grid(int64_t N, int num_cu, int64_t* rows_per_wg) {
  int64_t g = num_cu;
  int64_t rpw = (N + g - 1) / g;
  rpw = (rpw + FB_PB - 1) / FB_PB * FB_PB;
  if (rpw < FB_PB) rpw = FB_PB;
  g = (N + rpw - 1) / rpw;
  *rows_per_wg = rpw;
  return g;
}

hipError_t launch_sketch_fused_bf16(hipStream_t st, bool split, const float* A, int64_t lda,
                                    int64_t N, int n, int lq, int l, uint64_t seed,
                                    const float* omega, __bf16* omT, int num_cu, float* part,
                                    double* W, float* Y, int64_t* nparts_out) {
  const int lpad = ((l + 63) / 64) * 64;  // Y tiles: multiple of 4 tiles of 16
  if (Y) {
    hipLaunchKernelGGL(k_omega_t_bf16, dim3(256), dim3(256), 0, st, omega, n, l, lpad, omT);
  }
  int64_t rpw = 0;
  const int64_t grid = fused_bf16_grid(N, num_cu, &rpw);
  *nparts_out = grid;
  const int mt = (lq + 15) / 16;
#define SID_FUSED(SP, MT_, LT_)                                                                   \
  hipLaunchKernelGGL((k_sketch_fused_bf16<SP, MT_, LT_>), dim3((unsigned)grid), dim3(FB_THREADS), \
                     0, st, A, lda, N, n, lq, l, seed, omT, rpw, part, Y)
#define SID_FUSED_LT(SP, MT_) \
  if (lpad <= 64) SID_FUSED(SP, MT_, 4); else SID_FUSED(SP, MT_, 8);
#define SID_FUSED_MT(SP)                                 \
  if (mt <= 4) { SID_FUSED_LT(SP, 4) }                   \
  else if (mt <= 6) { SID_FUSED_LT(SP, 6) }              \
  else if (mt <= 8) { SID_FUSED_LT(SP, 8) }              \
  else { SID_FUSED_LT(SP, 10) }
  if (split) { SID_FUSED_MT(true) } else { SID_FUSED_MT(false) }
#undef SID_FUSED_MT
#undef SID_FUSED_LT
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
  TE* s_tt = reinterpret_cast<TE*>(s_raw);  // T^T: [CT*16][lpad], m-major
  const int lpad = (l + 15) & ~15;
  for (int e = threadIdx.x; e < CT * 16 * lpad; e += blockDim.x) {
    const int m = e / lpad, c = e - m * lpad;
    s_tt[e] = (m < k && c < l) ? (TE)Tm[c + (int64_t)l * m] : TE(0);
  }
  __syncthreads();
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int lr = lane & 15, lg = lane >> 4;
  const int64_t row0 = ((int64_t)blockIdx.x * AT_WAVES + wave) * (AT_RT * 16);
  typename M::acc_t acc[AT_RT][CT];
#pragma unroll
  for (int r = 0; r < AT_RT; ++r)
#pragma unroll
    for (int c = 0; c < CT; ++c) acc[r][c] = typename M::acc_t{0, 0, 0, 0};
  const bool vec = (l % 4) == 0;
  for (int kb = 0; kb < lpad; kb += 16) {
    TE yv[AT_RT][4];
#pragma unroll
    for (int r = 0; r < AT_RT; ++r) {
      const int64_t row = row0 + r * 16 + lr;
      const int c0 = kb + 4 * lg;
      if (row < N && vec && c0 + 4 <= l) {
        const TE* src = Y + row * l + c0;
#pragma unroll
        for (int s = 0; s < 4; ++s) yv[r][s] = src[s];
      } else {
#pragma unroll
        for (int s = 0; s < 4; ++s) yv[r][s] = (row < N && c0 + s < l) ? Y[row * l + c0 + s] : TE(0);
      }
    }
#pragma unroll
    for (int s = 0; s < 4; ++s) {
#pragma unroll
      for (int c = 0; c < CT; ++c) {
        const TE a = s_tt[(c * 16 + lr) * lpad + kb + 4 * lg + s];
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

template <typename TE, typename OutT>
static hipError_t apply_t_dispatch(hipStream_t st, const TE* Y, int64_t N, int l,
                                   const double* Tm, int k, OutT* AJ, int64_t ldaj) {
  const int ct = (k + 15) / 16;
  const int lpad = (l + 15) & ~15;
  const int64_t rows_per_block = AT_WAVES * AT_RT * 16;
  const dim3 grid((unsigned)((N + rows_per_block - 1) / rows_per_block));
#define SID_AT(CT_)                                                                        \
  {                                                                                        \
    const size_t shm = sizeof(TE) * (size_t)(CT_) * 16 * lpad;                             \
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
  const size_t shm = (y_f64 ? 8 : 4) * (size_t)ctt * 16 * ((l + 15) & ~15);
  return ct <= 10 && shm <= 160 * 1024;
}

hipError_t launch_apply_t_mfma(hipStream_t st, const void* Y, bool y_f64, int64_t N, int l,
                               const double* Tm, int k, void* AJ, bool aj_f64, int64_t ldaj) {
  if (y_f64) {
    if (aj_f64) return apply_t_dispatch<double, double>(st, (const double*)Y, N, l, Tm, k, (double*)AJ, ldaj);
    return apply_t_dispatch<double, float>(st, (const double*)Y, N, l, Tm, k, (float*)AJ, ldaj);
  }
  if (aj_f64) return apply_t_dispatch<float, double>(st, (const float*)Y, N, l, Tm, k, (double*)AJ, ldaj);
  return apply_t_dispatch<float, float>(st, (const float*)Y, N, l, Tm, k, (float*)AJ, ldaj);
}

}  // namespace sid
