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

// P as matrix-core B operands: entry e = ((cb * ks_n + ks) * 2 + h) * 64 + lane
// holds P(ks*32 + 8*(lane/16) + 0..7, cb*16 + lane%16), h = 0 the bfloat16
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
  const int64_t col = cb * 16 + (lane & 15);
  const int kb = ks * 32 + 8 * (lane >> 4);
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

// Ahat = Mf ACJ P for 256 fine rows per block (64 per wave, four 16-row
// MFMA tiles).  Each lane first forms its operand slice of the interpolated
// skeleton rows B = Mf ACJ (row lane%16 of each tile, columns
// 32 ks + 8 (lane/16) + 0..7) from the row-major copy acjt, in FP32, and
// keeps it in registers split into bfloat16 hi + lo.  The block then walks
// the 16-column blocks of P (packed operands, prefetched one block ahead)
// with three 16x16x32 bf16 MFMAs per tile and k-step (hi*hi + hi*lo +
// lo*hi), and stores its 64 x 16 result (or, ERR, compares it with A).
template <int KS, bool ERR, bool VEC>
__global__ __launch_bounds__(256, 2) void k_interp_mfma(InterpDev t,
                                                        const float* __restrict__ acjt,
                                                        const bf16x8_t* __restrict__ pb,
                                                        int64_t n, float* __restrict__ out,
                                                        int64_t ldo, const float* __restrict__ A,
                                                        int64_t lda, double* __restrict__ part) {
  constexpr int KP = 32 * KS;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int g = lane >> 4, li = lane & 15;
  const int64_t r0 = (int64_t)blockIdx.x * 256 + wave * 64;
  const int64_t N = t.N;

  u32x4_t ah[4][KS], al[4][KS];  // 8 bfloat16 each, packed two per dword
#pragma unroll
  for (int rb = 0; rb < 4; ++rb) {
    // rows past N (ragged last block) take row N-1's stencil with zero
    // weights: no branch, so the load groups below stay in order
    const int64_t i = r0 + 16 * rb + li;
    uint32_t idx[8];
    float w[8];
    stencil8<float>(t, (uint32_t)(i < N ? i : N - 1), idx, w);
    const float live = i < N ? 1.0f : 0.0f;
#pragma unroll
    for (int q = 0; q < 8; ++q) w[q] *= live;
#pragma unroll
    for (int ks = 0; ks < KS; ++ks) {
      float acc[8];
#pragma unroll
      for (int e = 0; e < 8; ++e) acc[e] = 0.0f;
#pragma unroll
      for (int q = 0; q < 8; ++q) {
        const f32x4_t* src =
            reinterpret_cast<const f32x4_t*>(acjt + (size_t)idx[q] * KP + 32 * ks + 8 * g);
        const f32x4_t v0 = src[0], v1 = src[1];
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          acc[e] = fmaf(w[q], v0[e], acc[e]);
          acc[4 + e] = fmaf(w[q], v1[e], acc[4 + e]);
        }
      }
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const uint32_t h = pack_bf16x2(acc[2 * e], acc[2 * e + 1]);
        ah[rb][ks][e] = h;
        al[rb][ks][e] = pack_bf16x2(acc[2 * e] - __uint_as_float(h << 16),
                                    acc[2 * e + 1] - __uint_as_float(h & 0xffff0000u));
      }
      // one (tile, k-step) group of 16 loads in flight at a time: hoisting
      // all of them would need more registers than the operands themselves.
      // The empty asm takes this group's operands and clobbers memory, so
      // they are formed before the next group's loads are issued.
      asm volatile("" ::"v"(ah[rb][ks]), "v"(al[rb][ks]) : "memory");
    }
  }

  double se = 0.0, sa = 0.0, mrel = 0.0, mabs = 0.0;
  const int64_t ncb = (n + 15) / 16;
  // pb holds one block of operands beyond the last column block, so the
  // prefetch below needs no bound
  bf16x8_t bh[KS], bl[KS];
#pragma unroll
  for (int ks = 0; ks < KS; ++ks) {
    bh[ks] = pb[(ks * 2 + 0) * 64 + lane];
    bl[ks] = pb[(ks * 2 + 1) * 64 + lane];
  }
  for (int64_t cb = 0; cb < ncb; ++cb) {
    bf16x8_t nh[KS], nl[KS];
    const bf16x8_t* nxt = pb + (cb + 1) * KS * 128;
#pragma unroll
    for (int ks = 0; ks < KS; ++ks) {
      nh[ks] = nxt[(ks * 2 + 0) * 64 + lane];
      nl[ks] = nxt[(ks * 2 + 1) * 64 + lane];
    }
    f32x4_t acc[4];
#pragma unroll
    for (int rb = 0; rb < 4; ++rb) acc[rb] = f32x4_t{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
    for (int ks = 0; ks < KS; ++ks) {
#pragma unroll
      for (int rb = 0; rb < 4; ++rb) {
        const bf16x8_t a_h = __builtin_bit_cast(bf16x8_t, ah[rb][ks]);
        const bf16x8_t a_l = __builtin_bit_cast(bf16x8_t, al[rb][ks]);
        acc[rb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a_h, bh[ks], acc[rb], 0, 0, 0);
        acc[rb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a_h, bl[ks], acc[rb], 0, 0, 0);
        acc[rb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a_l, bh[ks], acc[rb], 0, 0, 0);
      }
    }
    const int64_t j = cb * 16 + li;
    if (j < n) {
#pragma unroll
      for (int rb = 0; rb < 4; ++rb) {
        const int64_t row = r0 + 16 * rb + 4 * g;
        if constexpr (!ERR) {
          float* dst = out + j * ldo + row;
          if (VEC && row + 3 < N) {
            __builtin_nontemporal_store(acc[rb], reinterpret_cast<f32x4_t*>(dst));
          } else {
#pragma unroll
            for (int e = 0; e < 4; ++e)
              if (row + e < N) dst[e] = acc[rb][e];
          }
        } else {
          const float* src = A + j * lda + row;
          f32x4_t a4 = f32x4_t{0.0f, 0.0f, 0.0f, 0.0f};
          if (VEC && row + 3 < N) {
            a4 = __builtin_nontemporal_load(reinterpret_cast<const f32x4_t*>(src));
          } else {
#pragma unroll
            for (int e = 0; e < 4; ++e)
              if (row + e < N) a4[e] = src[e];
          }
#pragma unroll
          for (int e = 0; e < 4; ++e) {
            if (row + e < N) {
              const double a = (double)a4[e];
              const double d = a - (double)acc[rb][e];
              se = fma(d, d, se);
              sa = fma(a, a, sa);
              const double ad = fabs(d);
              mabs = fmax(mabs, ad);
              if (a != 0.0) mrel = fmax(mrel, ad / fabs(a));
            }
          }
        }
      }
    }
#pragma unroll
    for (int ks = 0; ks < KS; ++ks) {
      bh[ks] = nh[ks];
      bl[ks] = nl[ks];
    }
  }
  if constexpr (ERR) {
    __shared__ double s_r[4][4];
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
    if (threadIdx.x == 0) {
      double a = 0, b = 0, c = 0, d = 0;
      for (int v = 0; v < 4; ++v) {
        a += s_r[v][0];
        b += s_r[v][1];
        c = fmax(c, s_r[v][2]);
        d = fmax(d, s_r[v][3]);
      }
      double* o = part + 4 * (int64_t)blockIdx.x;
      o[0] = a;
      o[1] = b;
      o[2] = c;
      o[3] = d;
    }
  }
}

template <int KS, bool ERR>
hipError_t launch_mfma_vec(hipStream_t st, bool vec, const InterpDev& t, const float* acjt,
                           const bf16x8_t* pb, int64_t n, float* out, int64_t ldo, const float* A,
                           int64_t lda, double* part) {
  const dim3 grid((unsigned)interp_mfma_blocks(t.N));
  if (vec)
    hipLaunchKernelGGL((k_interp_mfma<KS, ERR, true>), grid, dim3(256), 0, st, t, acjt, pb, n,
                       out, ldo, A, lda, part);
  else
    hipLaunchKernelGGL((k_interp_mfma<KS, ERR, false>), grid, dim3(256), 0, st, t, acjt, pb, n,
                       out, ldo, A, lda, part);
  return hipGetLastError();
}

template <bool ERR>
hipError_t launch_mfma_ks(hipStream_t st, int ks, bool vec, const InterpDev& t, const float* acjt,
                          const bf16x8_t* pb, int64_t n, float* out, int64_t ldo, const float* A,
                          int64_t lda, double* part) {
  switch (ks) {
    case 1: return launch_mfma_vec<1, ERR>(st, vec, t, acjt, pb, n, out, ldo, A, lda, part);
    case 2: return launch_mfma_vec<2, ERR>(st, vec, t, acjt, pb, n, out, ldo, A, lda, part);
    case 3: return launch_mfma_vec<3, ERR>(st, vec, t, acjt, pb, n, out, ldo, A, lda, part);
    case 4: return launch_mfma_vec<4, ERR>(st, vec, t, acjt, pb, n, out, ldo, A, lda, part);
    default: return hipErrorInvalidValue;
  }
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
  const int64_t ncb = (n + 15) / 16;
  return (size_t)(ncb + 1) * (size_t)(kp / 32) * 2 * 64 * sizeof(bf16x8_t);
}

hipError_t launch_interp_pack(hipStream_t st, const float* ACJ, int64_t ldacj, int64_t Nc, int k,
                              int kp, float* acjt, const float* P, int64_t ldp, int64_t n,
                              void* pb) {
  if (kp % 32 != 0 || kp < 32 || kp > 128 || k > kp) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_pack_acjt, dim3((unsigned)((Nc + 63) / 64)), dim3(256), 0, st, ACJ, ldacj,
                     Nc, k, kp, acjt);
  const int ks_n = kp / 32;
  const int64_t total = ((n + 15) / 16) * ks_n * 128;
  hipLaunchKernelGGL(k_pack_p, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, st, P, ldp, k,
                     n, ks_n, total, (bf16x8_t*)pb);
  return hipGetLastError();
}

int64_t interp_mfma_blocks(int64_t N) { return (N + 255) / 256; }

hipError_t launch_reduce_norms(hipStream_t st, const double* part, int64_t nb, double* out4);

hipError_t launch_interp_mfma(hipStream_t st, const InterpDev& t, int kp, const float* acjt,
                              const void* pb, int64_t n, float* out, int64_t ldo, const float* A,
                              int64_t lda, double* part, int64_t part_cap, double* out4) {
  if (kp % 32 != 0 || kp < 32 || kp > 128) return hipErrorInvalidValue;
  const int ks = kp / 32;
  const bf16x8_t* p = (const bf16x8_t*)pb;
  if (A) {
    if (interp_mfma_blocks(t.N) > part_cap) return hipErrorInvalidValue;
    const bool vec = lda % 4 == 0 && ((uintptr_t)A & 15) == 0;
    hipError_t e = launch_mfma_ks<true>(st, ks, vec, t, acjt, p, n, nullptr, 0, A, lda, part);
    if (e != hipSuccess) return e;
    return launch_reduce_norms(st, part, interp_mfma_blocks(t.N), out4);
  }
  const bool vec = ldo % 4 == 0 && ((uintptr_t)out & 15) == 0;
  return launch_mfma_ks<false>(st, ks, vec, t, acjt, p, n, out, ldo, nullptr, 0, nullptr);
}

}  // namespace sid
