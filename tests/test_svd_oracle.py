"""Pins of the SBR-SVD oracle (Alg. 2) against the mathematics: with the same
Omega it returns the two-pass R-SVD (Alg. 1) (Q spans A_p Omega and B =
Q^T A_p, so the SVDs agree), it recovers a matrix of rank <= k exactly, and
its error is within the expected-error bound (1 + k/(p-1))^{1/2} times the
optimal rank-k error (Sec. 2.3) on matrices with a known spectrum."""
import numpy as np
import pytest

import synth
from oracle import svd as osvd


def _mat(N=900, n=70, decay=0.8, seed=3, noise=0.0):
    sig = decay ** np.arange(n)
    return synth.lowrank_exact_spectrum(N, n, sig, seed=seed, noise=noise).numpy(), sig


@pytest.mark.parametrize("block", [5, 10, 30])
def test_sbr_svd_equals_two_pass_rsvd(block):
    A, _ = _mat()
    a = osvd.sbr_svd(A, 20, 10, block, seed=4)
    b = osvd.rsvd(A, 20, 10, seed=4)
    np.testing.assert_allclose(a.S, b.S, rtol=1e-9, atol=1e-13 * b.S[0])
    # the leading singular vectors agree up to sign (well separated values)
    for j in range(10):
        assert abs(abs(a.U[:, j] @ b.U[:, j]) - 1.0) < 1e-8
        assert abs(abs(a.V[:, j] @ b.V[:, j]) - 1.0) < 1e-8


def test_sbr_svd_exact_low_rank():
    """Rank 12 with l = 12 (A_p Omega of full column rank): the blocks span
    the whole range and the factorization is exact; with l = 20 > 12 the
    blocks past the rank are stopped and the result is exact as well."""
    sig = 0.5 ** np.arange(12)
    A = synth.lowrank_exact_spectrum(600, 50, sig, seed=8).numpy()
    for (k, p, b) in ((12, 0, 4), (15, 5, 4)):
        r = osvd.sbr_svd(A, k, p, b, seed=1)
        np.testing.assert_allclose(osvd.reconstruct(r), A, atol=1e-10 * np.abs(A).max())
        np.testing.assert_allclose(r.S[:12], sig, rtol=1e-8)
        assert np.all(r.S[12:] < 1e-10)


def test_sbr_svd_expected_error_bound():
    """Mean over seeds of ||A - U S V^T||_F <= (1 + k/(p-1))^{1/2} times the
    optimal rank-k error (the bound holds for the expectation)."""
    sig = np.arange(1, 81, dtype=np.float64) ** -1.0
    A = synth.lowrank_exact_spectrum(1200, 80, sig, seed=2).numpy()
    k, p = 15, 5
    opt = np.sqrt(np.sum(sig[k:] ** 2))
    errs = [np.linalg.norm(A - osvd.reconstruct(osvd.sbr_svd(A, k, p, 5, seed=s)))
            for s in range(6)]
    assert np.mean(errs) <= np.sqrt(1 + k / (p - 1)) * opt
    assert min(errs) >= opt * (1 - 1e-9)       # never better than Eckart-Young
