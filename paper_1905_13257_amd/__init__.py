"""MI355X (gfx950) pass-efficient interpolative-decomposition compressor.

Python binding of ``libsid.so`` (C ABI in ``include/sid.h``).  The binding only
marshals arguments: every step of the compression runs in the library's HIP
kernels.  torch supplies device memory and the current stream.

Method: Dunton, Jofre, Iaccarino & Doostan, "Pass-efficient methods for
compression of high-dimensional turbulent flow data" (arXiv:1905.13257):
randomized ID (Alg. 4), sub-sampled ID (Alg. 5), a single-pass ID that
estimates the skeleton from a second sketch (two-sided single-pass sketch,
Sec. 2.3), and the paper's single-pass ID that keeps the coarse skeleton and
interpolates it back to the fine grid (Alg. 6), here in column orientation:
A (N x n, one snapshot per column) ~ A(:, J) P, or ~ Mf A(S, J) P.
"""
from __future__ import annotations

from ._native import (  # noqa: F401
    SID_F32, SID_F64, PRECISIONS, MODES, Context, Compressed, Interp, RowSet, SidError, Stream,
    Batch, batch_streams, probe, compress, compress_batched, reconstruct, reserve, error_norms, fill_gaussian, sketch, sketch_noalloc, sync,
    interp_reconstruct, interp_error_norms, SVD, sbr_svd, SvdStream,
    library_path,
    load,
)
