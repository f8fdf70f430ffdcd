// sid_adaptive.hpp -- tolerance-driven rank choice from the held-out probe
// rows (Remark 2.2, with the probe estimator as the stopping test).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace sid {

// After mgsqr of W's selection rows (pivots piv, R row-major k x n with
// leading dimension n, keff steps), shrink keff to the smallest rank k' whose
// probe fit ||W_pr - W_pr(:, J') P'||_F <= tol ||W_pr||_F, where W_pr are
// rows [r0, r0 + q) of W (column-major, leading dimension lq) and P' the ID
// coefficients of the first k' pivots; keff is left as it is when no prefix
// meets the tolerance; pivots past the chosen rank become -1.  Workspace:
// R11 (kcap x kcap), Z (q x kcap), part (probe_adapt_blocks(q, n) x
// (kcap + 1)), e2 (kcap + 1, the squared prefix errors).  kcap <= 256.
int64_t probe_adapt_blocks(int q, int n);
hipError_t launch_probe_adapt(hipStream_t st, const double* W, int lq, int r0, int q, int n,
                              int64_t* piv, int64_t* keff, const double* R, int kcap,
                              double* R11, double* Z, double* part, double* e2, double tol);

}  // namespace sid
