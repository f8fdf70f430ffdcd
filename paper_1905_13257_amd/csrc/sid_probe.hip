// sid_probe.hip -- measurement kernels for the ceilings the design rests on
// (streaming read and store rates of HBM, the issue rate of the two bfloat16
// matrix instructions).  They compute nothing of the method; bench.py
// --probes times them.
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace sid {

typedef float f32x4_t __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8_t __attribute__((ext_vector_type(8)));
typedef float f32x16_t __attribute__((ext_vector_type(16)));

// every float4 of buf read once (grid-stride, 16-byte loads); one value per
// block written so the loads cannot be dropped
__global__ __launch_bounds__(256) void k_probe_read(const f32x4_t* __restrict__ buf, int64_t n4,
                                                    float* __restrict__ sink) {
  // four 16-byte loads in flight per lane and step
  f32x4_t acc = {0.f, 0.f, 0.f, 0.f};
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  for (; e + 3 * stride < n4; e += 4 * stride) {
    const f32x4_t x0 = buf[e], x1 = buf[e + stride], x2 = buf[e + 2 * stride],
                  x3 = buf[e + 3 * stride];
    acc += (x0 + x1) + (x2 + x3);
  }
  for (; e < n4; e += stride) acc += buf[e];
  const float v = acc[0] + acc[1] + acc[2] + acc[3];
  if (v == 1234.5f) sink[blockIdx.x] = v;  // practically never taken; keeps the sum live
}

// a column-major N x n FP32 matrix written with the reconstruction kernels'
// pattern: each wave stores 4 columns x 256 contiguous bytes per instruction
// (lane l: column 4 (l / 16) .. , rows 4 (l % 16) .. +3), or (sequential =
// 1) as one contiguous fill
__global__ __launch_bounds__(256) void k_probe_store(float* __restrict__ out, int64_t N, int n,
                                                     int sequential) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (sequential) {
    f32x4_t* o = reinterpret_cast<f32x4_t*>(out);
    const int64_t n4 = N * n / 4;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    for (; e + 3 * stride < n4; e += 4 * stride) {
      o[e] = f32x4_t{1.f, 2.f, 3.f, 4.f};
      o[e + stride] = f32x4_t{1.f, 2.f, 3.f, 4.f};
      o[e + 2 * stride] = f32x4_t{1.f, 2.f, 3.f, 4.f};
      o[e + 3 * stride] = f32x4_t{1.f, 2.f, 3.f, 4.f};
    }
    for (; e < n4; e += stride) o[e] = f32x4_t{1.f, 2.f, 3.f, 4.f};
    return;
  }
  // row tiles of 64 rows, dealt over the blocks; each wave walks column
  // groups of 4
  const int64_t tiles = N / 64;
  for (int64_t t = blockIdx.x; t < tiles; t += gridDim.x) {
    const int64_t r = t * 64 + 4 * (lane & 15);
    for (int c = 4 * wave + (lane >> 4); c < n; c += 16)
      *reinterpret_cast<f32x4_t*>(out + r + N * (int64_t)c) = f32x4_t{1.f, 2.f, 3.f, 4.f};
  }
}

// register-only matrix-instruction loop: 8 independent accumulator chains,
// `iters` rounds; shape 0: v_mfma_f32_16x16x32_bf16, 1:
// v_mfma_f32_32x32x16_bf16
template <int SHAPE>
__global__ __launch_bounds__(256) void k_probe_mfma(int iters, float* __restrict__ sink) {
  bf16x8_t a, b;
#pragma unroll
  for (int i = 0; i < 8; ++i) {
    a[i] = (__bf16)(0.001f * (threadIdx.x + i));
    b[i] = (__bf16)(0.002f * (threadIdx.x - i));
  }
  if constexpr (SHAPE == 0) {
    f32x4_t acc[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) acc[u] = f32x4_t{0.f, 0.f, 0.f, 0.f};
    for (int it = 0; it < iters; ++it)
#pragma unroll
      for (int u = 0; u < 8; ++u) acc[u] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, acc[u], 0, 0, 0);
    float s = 0.f;
#pragma unroll
    for (int u = 0; u < 8; ++u) s += acc[u][0] + acc[u][3];
    if (s == 1234.5f) sink[blockIdx.x] = s;
  } else {
    f32x16_t acc[8];
#pragma unroll
    for (int u = 0; u < 8; ++u)
#pragma unroll
      for (int e = 0; e < 16; ++e) acc[u][e] = 0.f;
    for (int it = 0; it < iters; ++it)
#pragma unroll
      for (int u = 0; u < 8; ++u) acc[u] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, acc[u], 0, 0, 0);
    float s = 0.f;
#pragma unroll
    for (int u = 0; u < 8; ++u) s += acc[u][0] + acc[u][15];
    if (s == 1234.5f) sink[blockIdx.x] = s;
  }
}

hipError_t launch_probe(hipStream_t st, int kind, void* buf, int64_t N, int64_t n, int num_cu,
                        float* sink) {
  const dim3 block(256);
  switch (kind) {
    case 0:  // read N * n floats (N * n % 4 == 0)
      hipLaunchKernelGGL(k_probe_read, dim3((unsigned)(num_cu * 8)), block, 0, st,
                         (const f32x4_t*)buf, N * n / 4, sink);
      break;
    case 1:  // column stores (N % 64 == 0)
      hipLaunchKernelGGL(k_probe_store, dim3((unsigned)(num_cu * 8)), block, 0, st, (float*)buf, N,
                         (int)n, 0);
      break;
    case 2:  // sequential fill of N * n floats (N * n % 4 == 0)
      hipLaunchKernelGGL(k_probe_store, dim3((unsigned)(num_cu * 8)), block, 0, st, (float*)buf, N,
                         (int)n, 1);
      break;
    case 3:  // 16x16x32 loop, N iterations
      hipLaunchKernelGGL((k_probe_mfma<0>), dim3((unsigned)(num_cu * 8)), block, 0, st, (int)N, sink);
      break;
    case 4:  // 32x32x16 loop, N iterations
      hipLaunchKernelGGL((k_probe_mfma<1>), dim3((unsigned)(num_cu * 8)), block, 0, st, (int)N, sink);
      break;
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace sid
