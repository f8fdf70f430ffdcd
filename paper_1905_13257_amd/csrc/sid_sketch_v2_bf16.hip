// sid_sketch_v2_bf16.hip -- the bf16 instances of the 32x32x16 sketch pass
// (kernel in sid_sketch_v2.hpp); a translation unit of its own so that the
// data modes compile in parallel.
#include "sid_sketch_v2.hpp"

namespace sid {

hipError_t v2_launch_bf16(hipStream_t st, dim3 grid, const float* A, int64_t lda, int64_t N, int n,
                         int lq, int l, uint64_t seed, const __bf16* omT, int64_t rpp, float* part,
                         float* Y, int yadd, const __bf16* psi_img) {
  return v2_launch_dm<FB_BF16>(st, grid, A, lda, N, n, lq, l, seed, omT, rpp, part, Y, yadd, psi_img);
}

}  // namespace sid
