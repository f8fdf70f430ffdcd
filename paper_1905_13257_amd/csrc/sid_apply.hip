// sid_apply.hip -- skeleton estimate of the single pass for the bfloat16
// sketch precisions, AJ = Y T (Sec. 2.3, Halko et al. Sec. 5.5 item 4), with
// the output written in long runs down the columns of AJ.
//
// Arithmetic.  Y (N x l, row-major FP32) and T (l x k, FP64) are each split
// into bf16 hi + lo parts and the product is formed from the three terms
// Y_hi T_hi + Y_hi T_lo + Y_lo T_hi (the dropped Y_lo T_lo is below 2^-16 of
// the product), accumulated in FP32 on v_mfma_f32_16x16x32_bf16 in the order:
// K step, skeleton-column tile, row tile, then the three terms.
//   A operand: T^T tile (16 x 32) from LDS, lane = skeleton column l%16,
//              entries 8*(l/16) .. +7 of a 32-wide slice of l;
//   B operand: Y^T tile (32 x 16), lane = row l%16 of A, 8 consecutive Y
//              entries of that row (two 16-byte loads);
//   C tile:    16 skeleton columns x 16 rows of A.
// Work.  A workgroup of four waves owns blocks of 64 rows (wave w: rows
// 16 w .. 16 w + 15, one row tile: 156 registers, so that two workgroups,
// 65 KB of LDS each, run on a CU), looping over blocks so that T's split is
// staged in LDS once per workgroup;
// the next block's Y entries are loaded while the current one is multiplied.
// The results of one 16-column tile group are turned around in LDS and the
// workgroup stores them as 256-byte runs (64 rows) of each column, four
// columns per wave and instruction.  (Two row tiles per wave: 218 registers,
// one wave per SIMD, 375 us at C2; one tile: 303 us; eight waves sharing T
// with registers capped at 128: spills, 340 us.)  Columns past k in the last group store column k - 1 again
// (same value, same address), so the stores of a full block need no column
// test; the ragged last block of rows takes a guarded path.
#include "sid_apply.hpp"

namespace sid {

namespace {

typedef __bf16 bf16x8_t __attribute__((ext_vector_type(8)));
typedef float f32x4_t __attribute__((ext_vector_type(4)));

constexpr int AS_WAVES = 4;
constexpr int AS_THREADS = 64 * AS_WAVES;
// LP: l padded to a multiple of 32 (128: four K steps, 192: six); the LDS
// row stride of T's split is LP + 8 bf16
constexpr int AS_RT = 1;                  // row tiles of 16 per wave
constexpr int AS_ROWS = AS_WAVES * 16 * AS_RT;  // rows per block (64)
constexpr int AS_OS = AS_ROWS + 4;        // LDS row stride of the output staging (floats)
constexpr int AS_SL = AS_ROWS / 4;        // threads per column in the store phase

__device__ __forceinline__ __bf16 to_bf16(float f) { return (__bf16)f; }

// AL: l % 4 == 0, so Y's rows are 16-byte aligned and each lane's 8 entries
// are two 16-byte loads; otherwise (l <= 128 only) eight 4-byte loads, the
// entries past l zero.  VEC: AJ's columns are 16-byte aligned.
//
// The body serves one problem (the arguments) or, with a job table, job
// blockIdx.y (the work of a one-problem launch, dealt over the job's first
// nwg workgroups; AL and VEC per job).  KT only bounds the column tiles: a job
// with fewer skeleton columns computes zero tiles that are never stored, so
// every entry has the bits of the one-problem launch.
template <int KT, bool VEC, int LP, bool AL, bool BATCH>
__device__ __forceinline__ void apply_runs_body(const float* __restrict__ Y, int64_t N, int l,
                                                const double* __restrict__ Tm, int k,
                                                float* __restrict__ AJ, int64_t ldaj,
                                                const ApplyJob* __restrict__ jobs) {
  constexpr int AS_LS = LP + 8;
  constexpr int NKS = LP / 32;
  __shared__ __attribute__((aligned(16))) __bf16 s_th[KT * 16 * AS_LS];
  __shared__ __attribute__((aligned(16))) __bf16 s_tl[KT * 16 * AS_LS];
  __shared__ __attribute__((aligned(16))) float s_o[16 * AS_OS];
  // every access through a job's pointers is a global (not flat) access:
  // flat accesses count in the LDS counter too, so waiting for an LDS read
  // would wait for the prefetched rows
  typedef const __attribute__((address_space(1))) double* gcd;
  typedef const __attribute__((address_space(1))) float* gcf;
  typedef __attribute__((address_space(1))) float* gf;
  bool al = AL, vec = VEC;
  int64_t nwg = gridDim.x;  // workgroups dealing the blocks
  if constexpr (BATCH) {
    const ApplyJob& jb = jobs[blockIdx.y];
    nwg = jb.nwg;
    if ((int64_t)blockIdx.x >= nwg) return;
    Y = jb.Y;
    N = jb.N;
    l = jb.l;
    Tm = jb.T;
    k = jb.k;
    AJ = jb.AJ;
    ldaj = jb.ldaj;
    al = jb.al != 0;
    vec = jb.vec != 0;
  }
  for (int e = threadIdx.x; e < KT * 16 * LP; e += AS_THREADS) {
    const int m = e / LP, c = e - m * LP;
    const float x = (m < k && c < l) ? (float)((gcd)Tm)[c + (int64_t)l * m] : 0.0f;
    const __bf16 h = to_bf16(x);
    s_th[m * AS_LS + c] = h;
    s_tl[m * AS_LS + c] = to_bf16(x - (float)h);
  }
  __syncthreads();
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int lr = lane & 15, lg = lane >> 4;
  const int nks = (l + 31) >> 5;
  const int64_t nblk = (N + AS_ROWS - 1) / AS_ROWS;
  typedef const __attribute__((address_space(1))) f32x4_t* gptr4;
  // store phase: thread t writes rows 4 (t % AS_SL) .. +3 of column
  // t / AS_SL (+ AS_THREADS / AS_SL per pass) of the group
  const int sr = 4 * (threadIdx.x % AS_SL), sc = threadIdx.x / AS_SL;
  constexpr int SPASS = 16 / (AS_THREADS / AS_SL);
  f32x4_t y[AS_RT][NKS][2];
  auto load_block = [&](int64_t b) {
    const int64_t row0 = b * AS_ROWS + wave * 16 * AS_RT;
#pragma unroll
    for (int rt = 0; rt < AS_RT; ++rt) {
      const int64_t row = row0 + rt * 16 + lr;
#pragma unroll
      for (int ks = 0; ks < NKS; ++ks)
#pragma unroll
        for (int h = 0; h < 2; ++h) {
          const int c = 32 * ks + 8 * lg + 4 * h;
          if (al) {
            y[rt][ks][h] = (row < N && c + 4 <= l) ? *(gptr4)(Y + row * l + c)
                                                   : f32x4_t{0.f, 0.f, 0.f, 0.f};
          } else {
#pragma unroll
            for (int t = 0; t < 4; ++t)
              y[rt][ks][h][t] = (row < N && c + t < l) ? ((gcf)Y)[row * l + c + t] : 0.f;
          }
        }
    }
  };
  int64_t b = blockIdx.x;
  if (b < nblk) load_block(b);
  for (; b < nblk; b += nwg) {
    const int64_t blk0 = b * AS_ROWS;
    bf16x8_t bh[AS_RT][NKS], bl[AS_RT][NKS];
#pragma unroll
    for (int rt = 0; rt < AS_RT; ++rt)
#pragma unroll
      for (int ks = 0; ks < NKS; ++ks)
#pragma unroll
        for (int i = 0; i < 8; ++i) {
          const float x = y[rt][ks][i >> 2][i & 3];
          const __bf16 hv = to_bf16(x);
          bh[rt][ks][i] = hv;
          bl[rt][ks][i] = to_bf16(x - (float)hv);
        }
    if (b + nwg < nblk) load_block(b + nwg);
    f32x4_t acc[AS_RT][KT];
#pragma unroll
    for (int rt = 0; rt < AS_RT; ++rt)
#pragma unroll
      for (int kt = 0; kt < KT; ++kt) acc[rt][kt] = f32x4_t{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int ks = 0; ks < NKS; ++ks) {
      if (ks >= nks) break;
#pragma unroll
      for (int kt = 0; kt < KT; ++kt) {
        const int ti = (kt * 16 + lr) * AS_LS + 32 * ks + 8 * lg;
        const bf16x8_t th = *reinterpret_cast<const bf16x8_t*>(&s_th[ti]);
        const bf16x8_t tl = *reinterpret_cast<const bf16x8_t*>(&s_tl[ti]);
#pragma unroll
        for (int rt = 0; rt < AS_RT; ++rt) {
          acc[rt][kt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(th, bh[rt][ks], acc[rt][kt], 0, 0, 0);
          acc[rt][kt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(th, bl[rt][ks], acc[rt][kt], 0, 0, 0);
          acc[rt][kt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(tl, bh[rt][ks], acc[rt][kt], 0, 0, 0);
        }
      }
    }
    const bool full = blk0 + AS_ROWS <= N;
#pragma unroll
    for (int kt = 0; kt < KT; ++kt) {
      if (BATCH && kt * 16 >= k) break;  // uniform: the job's last column tile is done
      // C entry (rt, t) of this lane: column 4 lg + t of the group, row
      // 16 (AS_RT wave + rt) + lr of the block
#pragma unroll
      for (int rt = 0; rt < AS_RT; ++rt)
#pragma unroll
        for (int t = 0; t < 4; ++t)
          s_o[(4 * lg + t) * AS_OS + (wave * AS_RT + rt) * 16 + lr] = acc[rt][kt][t];
      __syncthreads();
#pragma unroll
      for (int half = 0; half < SPASS; ++half) {
        const int cg = sc + (AS_THREADS / AS_SL) * half;  // column within the group
        const int m0 = kt * 16 + cg;
        const int m = m0 < k ? m0 : k - 1;            // past k: column k - 1 again
        const int cl = m - kt * 16;
        const f32x4_t v = *reinterpret_cast<const f32x4_t*>(&s_o[cl * AS_OS + sr]);
        const gf dst = (gf)(AJ + blk0 + sr + ldaj * (int64_t)m);
        if (full) {
          if (vec) {
            typedef __attribute__((address_space(1))) f32x4_t* optr4;
            __builtin_nontemporal_store(v, (optr4)dst);
          } else {
#pragma unroll
            for (int t = 0; t < 4; ++t) dst[t] = v[t];
          }
        } else {
#pragma unroll
          for (int t = 0; t < 4; ++t)
            if (blk0 + sr + t < N) dst[t] = v[t];
        }
      }
      __syncthreads();
    }
  }
}

template <int KT, bool VEC, int LP, bool AL = true>
__global__ __launch_bounds__(AS_THREADS) void k_apply_t_bf16_runs(
    const float* __restrict__ Y, int64_t N, int l, const double* __restrict__ Tm /* l x k */,
    int k, float* __restrict__ AJ, int64_t ldaj) {
  apply_runs_body<KT, VEC, LP, AL, false>(Y, N, l, Tm, k, AJ, ldaj, nullptr);
}

// every job's AJ = Y T in one launch: job blockIdx.y (l <= 128, k <= 16 KT)
template <int KT>
__global__ __launch_bounds__(AS_THREADS) void k_apply_t_bf16_runs_batch(
    const ApplyJob* __restrict__ jobs) {
  apply_runs_body<KT, true, 128, true, true>(nullptr, 0, 0, nullptr, 0, nullptr, 0, jobs);
}

}  // namespace

bool apply_t_bf16_runs_supported(int k, int l) {
  if (k < 1 || l < 1) return false;
  return (l <= 128 && k <= 128) || (l <= 192 && k <= 160 && (l % 4) == 0);
}

hipError_t launch_apply_t_bf16_runs(hipStream_t st, const float* Y, int64_t N, int l,
                                    const double* Tm, int k, float* AJ, int64_t ldaj, int num_cu) {
  if (!apply_t_bf16_runs_supported(k, l) || N < 1 || ldaj < N) return hipErrorInvalidValue;
  const int64_t nblk = (N + AS_ROWS - 1) / AS_ROWS;
  int64_t g = (int64_t)num_cu * 4;
  if (g > nblk) g = nblk;
  const dim3 grid((unsigned)g), block(AS_THREADS);
  const bool vec = (ldaj % 4) == 0 && ((uintptr_t)AJ % 16) == 0;
  const int kt = (k + 15) / 16;
  const bool al = (l % 4) == 0;
#define SID_AS_LAUNCH(KT_, V_, LP_, AL_)                                                        \
  hipLaunchKernelGGL((k_apply_t_bf16_runs<KT_, V_, LP_, AL_>), grid, block, 0, st, Y, N, l, Tm, \
                     k, AJ, ldaj)
#define SID_AS(KT_, LP_, AL_)                     \
  case KT_:                                       \
    if (vec) SID_AS_LAUNCH(KT_, true, LP_, AL_);  \
    else SID_AS_LAUNCH(KT_, false, LP_, AL_);     \
    break;
  if (l <= 128 && al) {
    switch (kt) {
      SID_AS(1, 128, true) SID_AS(2, 128, true) SID_AS(3, 128, true) SID_AS(4, 128, true)
      SID_AS(5, 128, true) SID_AS(6, 128, true) SID_AS(7, 128, true) SID_AS(8, 128, true)
      default: return hipErrorInvalidValue;
    }
  } else if (l <= 128) {
    switch (kt) {
      SID_AS(1, 128, false) SID_AS(2, 128, false) SID_AS(3, 128, false) SID_AS(4, 128, false)
      SID_AS(5, 128, false) SID_AS(6, 128, false) SID_AS(7, 128, false) SID_AS(8, 128, false)
      default: return hipErrorInvalidValue;
    }
  } else {
    // l up to 192: six K steps; T's split takes up to 128 KB of LDS (one
    // workgroup per CU)
    switch (kt) {
      SID_AS(1, 192, true) SID_AS(2, 192, true) SID_AS(3, 192, true) SID_AS(4, 192, true)
      SID_AS(5, 192, true) SID_AS(6, 192, true) SID_AS(7, 192, true) SID_AS(8, 192, true)
      SID_AS(9, 192, true) SID_AS(10, 192, true)
      default: return hipErrorInvalidValue;
    }
  }
#undef SID_AS
#undef SID_AS_LAUNCH
  return hipGetLastError();
}

int apply_batch_workgroups(int64_t N, int num_cu) {
  // at least APPLY_MIN_BLOCKS blocks per workgroup, so that staging T is
  // spread over them; at most the one-problem launch's grid
  const int64_t nblk = (N + AS_ROWS - 1) / AS_ROWS;
  int64_t g = (nblk + APPLY_MIN_BLOCKS - 1) / APPLY_MIN_BLOCKS;
  if (g > (int64_t)num_cu * 4) g = (int64_t)num_cu * 4;
  return (int)(g < 1 ? 1 : g);
}

hipError_t launch_apply_t_bf16_runs_batch(hipStream_t st, const ApplyJob* jobs, int njobs,
                                          int max_nwg, int kmax) {
  if (njobs < 1 || max_nwg < 1) return hipSuccess;
  if (kmax < 1 || kmax > 128) return hipErrorInvalidValue;
  const dim3 grid((unsigned)max_nwg, (unsigned)njobs), block(AS_THREADS);
#define SID_ASB(KT_)                                                                  \
  case KT_:                                                                           \
    hipLaunchKernelGGL((k_apply_t_bf16_runs_batch<KT_>), grid, block, 0, st, jobs);   \
    break;
  switch ((kmax + 15) / 16) {
    SID_ASB(1) SID_ASB(2) SID_ASB(3) SID_ASB(4) SID_ASB(5) SID_ASB(6) SID_ASB(7) SID_ASB(8)
    default: return hipErrorInvalidValue;
  }
#undef SID_ASB
  return hipGetLastError();
}

}  // namespace sid
