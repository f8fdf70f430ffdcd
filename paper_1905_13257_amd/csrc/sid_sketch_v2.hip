// sid_sketch_v2.hip -- host side of the 32x32x16 bfloat16 sketch pass
// (k_sketch_v2 in sid_sketch_v2.hpp; one translation unit per data mode
// instantiates its kernels): Omega^T in the chunk-buffer order, the fixed-
// order FP64 sum of the workgroup partials, shape rules and the launch.
#include "sid_sketch_v2.hpp"

namespace sid {

// Omega^T in bfloat16 (FP8 mode: the e4m3 values, exact in bfloat16) with
// the k index of each 128-column chunk in chunk-buffer order:
// out[c * npad + 128 j + chk_pos(q)] = value of Omega(128 j + q, c), zero
// padded
__global__ void k_omega_t_v2(const float* __restrict__ omega /* n x l row-major */, int n, int l,
                             int lpad, int npad, int fp8, __bf16* __restrict__ out) {
  for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < lpad * npad; e += gridDim.x * blockDim.x) {
    const int c = e / npad, pos = e - c * npad;
    const int j = pos / V2_CHUNK, pp = pos - j * V2_CHUNK;
    const int q = (pp & 1) * 64 + (pp >> 1);  // inverse of chk_pos
    const int k = V2_CHUNK * j + q;
    const float z = (c < l && k < n) ? omega[k * l + c] : 0.0f;
    out[e] = (__bf16)(fp8 ? e4m3_value(z) : z);
  }
}

// W = sum of the workgroup partials (row-major lq x n each), in FP64 and a
// fixed order (eight interleaved running sums, then their sum); W is
// column-major lq x n (ldw = lq)
__global__ void k_reduce_partials_rm(const float* __restrict__ part, int64_t nparts, int lq, int n,
                                     double* __restrict__ W) {
  const int64_t count = (int64_t)lq * n;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < count;
       e += (int64_t)gridDim.x * blockDim.x) {
    double s[8] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    int64_t g = 0;
    for (; g + 8 <= nparts; g += 8)
#pragma unroll
      for (int u = 0; u < 8; ++u) s[u] += (double)part[(g + u) * count + e];
    for (; g < nparts; ++g) s[0] += (double)part[g * count + e];
    const int m = (int)(e / n), col = (int)(e - (int64_t)m * n);
    W[m + (int64_t)lq * col] = ((s[0] + s[1]) + (s[2] + s[3])) + ((s[4] + s[5]) + (s[6] + s[7]));
  }
}

int sketch_v2_slab(int lq, int l, bool wanty) {
  for (int nct = V2_MAXNCT; nct >= 1; --nct)
    if (v2_fits(nct, lq, l, wanty)) return V2_CHUNK * nct;
  return 0;
}

bool sketch_v2_supported(int64_t n, int lq, int l, bool wanty, int64_t lda, const void* A) {
  const int slab = sketch_v2_slab(lq, l, wanty);
  return n >= 1 && slab > 0 && n <= slab && (lda % 4) == 0 && ((uintptr_t)A % 16) == 0;
}

size_t sketch_v2_omt_elems(int l, int n) {
  const int nct = (n + V2_CHUNK - 1) / V2_CHUNK;
  return (size_t)(2 * v2_lt(l) * 32) * (size_t)(V2_CHUNK * nct);
}

// pairs of workgroups (one per CU each) and rows per pair: a multiple of 64,
// the pair count a multiple of 8 (one pair per two CUs of each XCD)
int64_t sketch_v2_pairs(int64_t N, int num_cu, int64_t* rows_per_pair) {
  int64_t pairs = num_cu / 2;
  const int64_t need = (N + V2_PR - 1) / V2_PR;  // no more pairs than panels
  if (pairs > need) pairs = need;
  if (pairs < 8) pairs = 8;
  pairs = (pairs + 7) / 8 * 8;
  int64_t rpp = (N + pairs - 1) / pairs;
  rpp = (rpp + V2_PR - 1) / V2_PR * V2_PR;
  if (rpp < V2_PR) rpp = V2_PR;
  *rows_per_pair = rpp;
  return pairs;
}

// Psi images: for every panel P of 64 rows and pair half h, the LDS image of
// the half's Psi rows (MT = 4 tiles of 32 rows x 64 panel rows, bf16, the
// kernel's XOR placement) that the pass would generate for that panel: the
// same generator call per (row, group of four Psi rows), FP8-rounded in the
// FP8 form, rows past N and Psi rows past the half zero.  One thread per
// (panel row, group).
__global__ void k_psi_image(uint64_t seed, int64_t N, int lq, int hsplit, int fp8,
                            __bf16* __restrict__ img, int64_t npanels) {
  constexpr int MT = 4, PIMG = MT * 32 * V2_PS;
  const int64_t items = npanels * 2 * (MT * 8) * V2_PR;
  for (int64_t w = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; w < items;
       w += (int64_t)gridDim.x * blockDim.x) {
    const int k = (int)(w % V2_PR);
    const int g = (int)((w / V2_PR) % (MT * 8));
    const int h = (int)((w / (V2_PR * MT * 8)) % 2);
    const int64_t P = w / (V2_PR * MT * 8 * 2);
    const int mb = h ? hsplit : 0, mc = h ? lq - hsplit : hsplit;
    const int64_t r = P * V2_PR + k;
    float z[4] = {0.f, 0.f, 0.f, 0.f};
    if (r < N && 4 * g < mc) gauss4(seed, 1u, (uint64_t)r, (uint32_t)((mb >> 2) + g), z);
    __bf16* out = img + (P * 2 + h) * (int64_t)PIMG;
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int m = 4 * g + e;
      const float v = m < mc ? (fp8 ? e4m3_value(z[e]) : z[e]) : 0.0f;
      out[psi_idx(m, k)] = (__bf16)v;
    }
  }
}

size_t sketch_v2_psi_image_bytes(int64_t N, int lq) {
  if (v2_mt(lq) != 4) return 0;
  const int64_t npanels = (N + V2_PR - 1) / V2_PR;
  return sizeof(uint16_t) * (size_t)npanels * 2 * (size_t)(4 * 32 * V2_PS);
}

hipError_t launch_sketch_v2_psi_image(hipStream_t st, int dmode, uint64_t seed, int64_t N, int lq,
                                      __bf16* img) {
  if (v2_mt(lq) != 4 || N < 1) return hipErrorInvalidValue;
  const int64_t npanels = (N + V2_PR - 1) / V2_PR;
  hipLaunchKernelGGL(k_psi_image, dim3(4096), dim3(256), 0, st, seed, N, lq, v2_hsplit(lq),
                     dmode == FB_FP8 ? 1 : 0, img, npanels);
  return hipGetLastError();
}

hipError_t launch_sketch_v2(hipStream_t st, int dmode, const float* A, int64_t lda, int64_t N,
                            int n, int lq, int l, uint64_t seed, const float* omega, __bf16* omT,
                            int num_cu, float* part, double* W, float* Y, int64_t* nparts_out,
                            bool y_add, const __bf16* psi_img) {
  const int nct = (n + V2_CHUNK - 1) / V2_CHUNK;
  if (n < 1 || !v2_fits(nct, lq, l, Y != nullptr)) return hipErrorInvalidValue;
  if (Y && (uint64_t)N * (uint64_t)l * 4u >= (1ull << 32)) return hipErrorInvalidValue;
  if (Y) {
    const int lpad = 2 * 32 * v2_lt(l), npad = V2_CHUNK * nct;
    hipLaunchKernelGGL(k_omega_t_v2, dim3(256), dim3(256), 0, st, omega, n, l, lpad, npad,
                       dmode == FB_FP8 ? 1 : 0, omT);
  }
  int64_t rpp = 0;
  const int64_t pairs = sketch_v2_pairs(N, num_cu, &rpp);
  *nparts_out = pairs;
  const dim3 g((unsigned)(2 * pairs));
  const int ya = (Y && y_add) ? 1 : 0;
  const __bf16* img = v2_mt(lq) == 4 ? psi_img : nullptr;
  hipError_t e = dmode == FB_BF16X2 ? v2_launch_bf16x2(st, g, A, lda, N, n, lq, l, seed, omT, rpp, part, Y, ya, img)
                 : dmode == FB_FP8  ? v2_launch_fp8(st, g, A, lda, N, n, lq, l, seed, omT, rpp, part, Y, ya, img)
                                    : v2_launch_bf16(st, g, A, lda, N, n, lq, l, seed, omT, rpp, part, Y, ya, img);
  if (e != hipSuccess) return e;
  const int64_t count = (int64_t)lq * n;
  int64_t blocks = (count + 255) / 256;
  if (blocks > 4096) blocks = 4096;
  hipLaunchKernelGGL(k_reduce_partials_rm, dim3((unsigned)blocks), dim3(256), 0, st, part, pairs,
                     lq, n, W);
  return hipGetLastError();
}

}  // namespace sid
