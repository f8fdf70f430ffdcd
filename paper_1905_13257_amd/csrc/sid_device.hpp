// sid_device.hpp -- device-side building blocks of the gfx950 ID compressor.
//
// * Counter-based Gaussian test matrices: Philox4x32-10 (Salmon, Moraes,
//   Dror & Shaw, SC'11) feeding a single-precision Box-Muller transform.  The
//   paper draws Omega and Psi with i.i.d. Gaussian entries (Sec. 2.2, eq.
//   (sampmatrix); Alg. 4 "Generate Omega ... with i.i.d. Gaussian entries").
//   Entries are keyed by (seed, stream, major, minor) so any tile can be
//   regenerated anywhere without storing the matrix.
// * Sketch-precision value maps (bfloat16 rounding, two-term bf16 split).
// * Wave-level reductions for 64-wide wavefronts.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace sid {

// A pointer as a global-memory pointer.  Kernel arguments are known to be
// global; a pointer read from a device job table (or a value merged from
// both) is not, and accesses through it become flat instructions, which
// count in the LDS counter as well as the vector-memory counter, so that
// every wait for an LDS access would also wait for them.  Kernels that take
// job tables access memory through these.
template <class T>
__device__ __forceinline__ __attribute__((address_space(1))) T* to_global(T* p) {
  return (__attribute__((address_space(1))) T*)p;
}

// ---------------------------------------------------------------------------
// Philox4x32-10
// ---------------------------------------------------------------------------
struct U4 { uint32_t x, y, z, w; };

__device__ __forceinline__ U4 philox10(U4 c, uint32_t k0, uint32_t k1) {
  constexpr uint32_t MA = 0xD2511F53u, MB = 0xCD9E8D57u;
  constexpr uint32_t WA = 0x9E3779B9u, WB = 0xBB67AE85u;
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    const uint64_t pa = (uint64_t)MA * c.x;
    const uint64_t pb = (uint64_t)MB * c.z;
    U4 n;
    n.x = (uint32_t)(pb >> 32) ^ c.y ^ k0;
    n.y = (uint32_t)pb;
    n.z = (uint32_t)(pa >> 32) ^ c.w ^ k1;
    n.w = (uint32_t)pa;
    c = n;
    k0 += WA;
    k1 += WB;
  }
  return c;
}

// ---------------------------------------------------------------------------
// Gaussian transform.  Every step is one IEEE single-precision operation in a
// fixed order (explicit fmaf, correctly rounded division and square root), so
// the result is a function of the two 32-bit words only.  Division and square
// root are the plain operators, correctly rounded under
// -fhip-fp32-correctly-rounded-divide-sqrt; HIP's __fsqrt_rn is not used
// because without OCML_BASIC_ROUNDED_OPERATIONS it maps to the approximate
// native square root.
//   u = ((a >> 8) + 1) 2^-24,  r = sqrt(-2 ln u)
//   ln u: u = m 2^e, m in [1, 2) (halved with e+1 when m >= sqrt 2),
//         s = (m-1)/(m+1), ln m = s (2 + s^2 (2/3 + s^2 (2/5 + s^2 (2/7 +
//         s^2 (2/9 + s^2 2/11))))), ln u = fma(e, ln 2, ln m)
//   angle: quadrant b >> 30, t = (2 ((b >> 7) mod 2^23) + 1) 2^-24,
//         phi = t pi/2, Taylor sin (to phi^13) / cos (to phi^14) in phi^2
//   z_cos = r cos(theta), z_sin = r sin(theta), theta = quadrant pi/2 + phi
// Constants are the single-precision roundings of the exact values.
// ---------------------------------------------------------------------------
__device__ __forceinline__ float bits_f(uint32_t b) { return __uint_as_float(b); }

__device__ __forceinline__ float gauss_ln(float u) {
  const uint32_t ub = __float_as_uint(u);
  int e = (int)((ub >> 23) & 0xFFu) - 127;
  float m = bits_f((ub & 0x007FFFFFu) | 0x3F800000u);
  if (m >= bits_f(0x3FB504F3u)) {  // sqrt(2)
    m = m * 0.5f;
    e += 1;
  }
  const float s = __fsub_rn(m, 1.0f) / __fadd_rn(m, 1.0f);  // correctly rounded (see build flags)
  const float s2 = __fmul_rn(s, s);
  float p = __fmaf_rn(s2, bits_f(0x3E3A2E8Cu), bits_f(0x3E638E39u));  // 2/11, 2/9
  p = __fmaf_rn(s2, p, bits_f(0x3E924925u));                          // 2/7
  p = __fmaf_rn(s2, p, bits_f(0x3ECCCCCDu));                          // 2/5
  p = __fmaf_rn(s2, p, bits_f(0x3F2AAAABu));                          // 2/3
  p = __fmaf_rn(s2, p, 2.0f);
  const float lnm = __fmul_rn(s, p);
  return __fmaf_rn((float)e, bits_f(0x3F317218u), lnm);               // ln 2
}

__device__ __forceinline__ void gauss_pair(uint32_t a, uint32_t b, float& zc, float& zs) {
  const float two_m24 = bits_f(0x33800000u);
  const float u = __fmul_rn((float)((a >> 8) + 1u), two_m24);
  const float L = gauss_ln(u);
  const float r = __builtin_sqrtf(__fmul_rn(-2.0f, L));     // correctly rounded (see build flags)
  const uint32_t quad = b >> 30;
  const uint32_t frac = (b >> 7) & 0x007FFFFFu;
  const float t = __fmul_rn((float)(2u * frac + 1u), two_m24);
  const float phi = __fmul_rn(t, bits_f(0x3FC90FDBu));  // pi/2
  const float p2 = __fmul_rn(phi, phi);
  float sp = __fmaf_rn(p2, bits_f(0x2F309231u), bits_f(0xB2D7322Bu));
  sp = __fmaf_rn(p2, sp, bits_f(0x3638EF1Du));
  sp = __fmaf_rn(p2, sp, bits_f(0xB9500D01u));
  sp = __fmaf_rn(p2, sp, bits_f(0x3C088889u));
  sp = __fmaf_rn(p2, sp, bits_f(0xBE2AAAABu));
  sp = __fmaf_rn(p2, sp, 1.0f);
  float cp = __fmaf_rn(p2, bits_f(0xAD49CBA5u), bits_f(0x310F76C7u));
  cp = __fmaf_rn(p2, cp, bits_f(0xB493F27Eu));
  cp = __fmaf_rn(p2, cp, bits_f(0x37D00D01u));
  cp = __fmaf_rn(p2, cp, bits_f(0xBAB60B61u));
  cp = __fmaf_rn(p2, cp, bits_f(0x3D2AAAABu));
  cp = __fmaf_rn(p2, cp, bits_f(0xBF000000u));
  cp = __fmaf_rn(p2, cp, 1.0f);
  const float sn = __fmul_rn(phi, sp);
  const float cs = cp;
  float c, s;
  switch (quad) {
    case 0: c = cs; s = sn; break;
    case 1: c = -sn; s = cs; break;
    case 2: c = -cs; s = -sn; break;
    default: c = sn; s = -cs; break;
  }
  zc = __fmul_rn(r, c);
  zs = __fmul_rn(r, s);
}

// Entries minor = 4*group .. 4*group+3 of (seed, stream, major).
__device__ __forceinline__ void gauss4(uint64_t seed, uint32_t stream, uint64_t major,
                                       uint32_t group, float z[4]) {
  U4 c{(uint32_t)major, group, stream, (uint32_t)(major >> 32)};
  const U4 x = philox10(c, (uint32_t)seed, (uint32_t)(seed >> 32));
  gauss_pair(x.x, x.y, z[0], z[1]);
  gauss_pair(x.z, x.w, z[2], z[3]);
}

// ---------------------------------------------------------------------------
// Sketch precisions
// ---------------------------------------------------------------------------
enum Prec : int { P_F64 = 0, P_F32 = 1, P_BF16 = 2, P_BF16X2 = 3, P_FP8 = 4 };

// bfloat16 round to nearest even, returned as the (exact) float value
__device__ __forceinline__ float bf16_value(float f) {
  uint32_t b = __float_as_uint(f);
  if ((b & 0x7F800000u) == 0x7F800000u) return f;
  b = (b + 0x7FFFu + ((b >> 16) & 1u)) & 0xFFFF0000u;
  return __uint_as_float(b);
}

// OCP FP8 e4m3fn round to nearest even (3 fraction bits, bias 7, largest
// value 448, subnormal step 2^-9), saturating; returned as the exact float.
// Normal range: round the FP32 significand to 3 fraction bits on the bit
// pattern; below 2^-6: a multiple of 2^-9 (rint is ties-to-even).
__device__ __forceinline__ float e4m3_value(float x) {
  const float ax = fabsf(x);
  const float rs = rintf(ax * 512.0f) * 0.001953125f;  // branch-free: both forms, then select
  uint32_t b = __float_as_uint(ax);
  b = (b + 0x7FFFFu + ((b >> 20) & 1u)) & 0xFFF00000u;
  const float rn = fminf(__uint_as_float(b), 448.0f);
  return copysignf(ax < 0.015625f ? rs : rn, x);
}

// value a Gaussian draw takes in each precision
template <int PREC>
__device__ __forceinline__ float gauss_value(float z) {
  if constexpr (PREC == P_BF16 || PREC == P_BF16X2) return bf16_value(z);
  else if constexpr (PREC == P_FP8) return e4m3_value(z);
  else return z;
}

// Power-of-two scale of an FP8 data tile with largest magnitude amax:
// 2^(E - 7), E = floor(log2 amax) clamped to [-100, 120]; 1 for amax = 0.
// Returns the scale and sets inv to its reciprocal (both exact).
__device__ __forceinline__ float fp8_tile_scale(float amax, float& inv) {
  int E = (int)((__float_as_uint(amax) >> 23) & 0xFFu) - 127;
  E = E < -100 ? -100 : (E > 120 ? 120 : E);
  const bool zero = !(amax > 0.0f);
  const float s = zero ? 1.0f : __uint_as_float((uint32_t)(E - 7 + 127) << 23);
  inv = zero ? 1.0f : __uint_as_float((uint32_t)(7 - E + 127) << 23);
  return s;
}

// value a data entry takes in each precision (compute type T)
template <int PREC, typename T, typename In>
__device__ __forceinline__ T data_value(In a) {
  if constexpr (PREC == P_F64) {
    return (T)(double)a;
  } else {
    const float f = (float)a;
    if constexpr (PREC == P_F32) return (T)f;
    else if constexpr (PREC == P_FP8) return (T)f;  // the general kernels get pre-quantized data
    else if constexpr (PREC == P_BF16) return (T)bf16_value(f);
    else {
      const float hi = bf16_value(f);
      const float lo = bf16_value(__fsub_rn(f, hi));
      return (T)__fadd_rn(hi, lo);
    }
  }
}

// ---------------------------------------------------------------------------
// Workgroup barrier for LDS communication only: waits for this wave's LDS
// operations, not for its global loads or stores (a plain __syncthreads also
// waits for every outstanding global access of the wave).  The compiler
// fences keep memory operations from being moved across it.
// ---------------------------------------------------------------------------
__device__ __forceinline__ void lds_barrier() {
  __builtin_amdgcn_sched_barrier(0);
  asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory");
  __builtin_amdgcn_sched_barrier(0);
}

// ---------------------------------------------------------------------------
// Reductions (wave64)
// ---------------------------------------------------------------------------
template <typename T>
__device__ __forceinline__ T wave_sum(T v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

}  // namespace sid
