"""GPU parity of SBR-SVD (Alg. 2) against the oracle.  Marked gpu."""
import ctypes
import sys

import numpy as np
import pytest
import torch

import synth

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def sid():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1905_13257_amd as m
    m.load()
    return m


@pytest.fixture(scope="module")
def osvd():
    import oracle
    oracle.build()
    from oracle import svd
    return svd


def host(t):
    return t.detach().cpu().numpy()


def to_gpu(A64, dtype):
    return synth.as_colmajor(torch.from_numpy(np.asfortranarray(A64)).to(dtype)).cuda()


def recon(U, S, V):
    return (V * S[None, :]) @ U.T


# rho: sigma_j = rho^j.  The block loop's error at sigma_j is about
# eps sigma_1^2 / sigma_j (both sides), so rho keeps sigma_k^2 >= 1e-8 where
# the singular values are compared at rtol 1e-8; l = 140 (> 128) takes the
# Jacobi solver's global-memory form, l = 15 its odd-size dummy index, and
# n b = 16000 the block QR's in-place form.
@pytest.mark.parametrize("N,n,k,p,b,rho", [(3000, 120, 20, 10, 10, 0.85), (2049, 77, 12, 4, 8, 0.85),
                                           (5000, 300, 40, 20, 20, 0.85),
                                           (40013, 100, 30, 10, 10, 0.85),
                                           (3001, 90, 13, 2, 5, 0.85),
                                           (6000, 200, 120, 20, 20, 0.95),
                                           (4000, 800, 40, 20, 20, 0.85)])
def test_f64_parity(sid, osvd, N, n, k, p, b, rho):
    """FP64 data and sketch: singular values and the leading singular
    vectors (up to sign) equal the oracle's; so does the reconstruction."""
    say("sbr-svd f64", N, n, k, p, b, rho)
    sig = rho ** np.arange(n)
    A64 = synth.lowrank_exact_spectrum(N, n, sig, seed=N + n).numpy()
    g = sid.sbr_svd(to_gpu(A64, torch.float64), k, p, b, seed=3, prec="f64")
    o = osvd.sbr_svd(A64, k, p, b, seed=3, prec="f64")
    assert g.rank == k + p
    S = host(g.S)
    np.testing.assert_allclose(S, o.S, rtol=1e-8, atol=1e-12 * o.S[0])
    U, V = host(g.U), host(g.V)
    for j in range(min(k, 10)):
        assert abs(abs(U[:, j] @ o.U[:, j]) - 1.0) < 1e-7
        assert abs(abs(V[:, j] @ o.V[:, j]) - 1.0) < 1e-7
    np.testing.assert_allclose(recon(U, S, V), osvd.reconstruct(o),
                               atol=1e-9 * np.abs(A64).max())


def test_fp32_bf16x2(sid, osvd):
    """FP32 data, bf16x2 single pass (H in FP64 from the data): singular
    values within 1e-4 and the reconstruction error within 1 % of the
    oracle's on the same rounding of the sketch."""
    say("sbr-svd fp32 bf16x2")
    sig = np.arange(1, 161, dtype=np.float64) ** -1.5
    A64 = synth.lowrank_exact_spectrum(8000, 160, sig, seed=2).numpy()
    A32 = A64.astype(np.float32).astype(np.float64)
    g = sid.sbr_svd(to_gpu(A32, torch.float32), 30, 10, 10, seed=5, prec="bf16x2")
    o = osvd.sbr_svd(A32, 30, 10, 10, seed=5, prec="bf16x2")
    np.testing.assert_allclose(host(g.S), o.S, rtol=1e-4, atol=1e-6 * o.S[0])
    eg = np.linalg.norm(A32 - recon(host(g.U).astype(np.float64), host(g.S),
                                    host(g.V).astype(np.float64)))
    eo = np.linalg.norm(A32 - osvd.reconstruct(o))
    assert eg == pytest.approx(eo, rel=1e-2)
    # the expected-error bound of Sec. 2.3 against the optimal rank-30 error
    assert eg <= np.sqrt(1 + 30 / 9) * np.sqrt(np.sum(sig[30:] ** 2))


@pytest.mark.parametrize("k,p,b", [(12, 0, 4), (15, 5, 4)])
def test_exact_rank(sid, osvd, k, p, b):
    """Rank 12: l = 12 spans the range exactly; l = 20 stops after three
    blocks (rank 12 reached) and is exact as well."""
    say("sbr-svd exact rank", k, p, b)
    sig = 0.5 ** np.arange(12)
    A64 = synth.lowrank_exact_spectrum(1500, 60, sig, seed=8).numpy()
    g = sid.sbr_svd(to_gpu(A64, torch.float64), k, p, b, seed=1, prec="f64")
    assert g.rank == 12
    S = host(g.S)
    np.testing.assert_allclose(S[:12], sig, rtol=1e-8)
    assert np.all(S[12:] == 0.0)
    np.testing.assert_allclose(recon(host(g.U), S, host(g.V)), A64, atol=1e-10 * np.abs(A64).max())


def test_equals_two_pass_rsvd(sid, osvd):
    """Same Omega: SBR-SVD's singular values equal the two-pass R-SVD's
    (Alg. 1, oracle) in FP64."""
    say("sbr-svd vs r-svd")
    sig = 0.9 ** np.arange(100)
    A64 = synth.lowrank_exact_spectrum(4000, 100, sig, seed=4, noise=1e-6).numpy()
    g = sid.sbr_svd(to_gpu(A64, torch.float64), 25, 15, 8, seed=9, prec="f64")
    r = osvd.rsvd(A64, 25, 15, seed=9, prec="f64")
    np.testing.assert_allclose(host(g.S), r.S, rtol=1e-8)


def test_full_size_properties(sid):
    """The 1,572,864 x 500 FP32 channel-like matrix at k = 100, p = 20, block
    20, FP64 sketch (the benchmarked launch): U and V orthonormal, A U = V S
    (B = Q^T A_p in exact arithmetic, so V S = A Q U~ = A U), singular values
    descending, and the rank-100 error no larger than the single-pass ID's
    at the same rank."""
    say("sbr-svd full size")
    A = synth.spectral_snapshots(synth.SpectralConfig(), device="cuda")
    out = sid.sbr_svd(A, 100, 20, 20, seed=0, prec="f64")
    assert out.rank == 120
    S = out.S
    assert bool(torch.all(S[:-1] >= S[1:])) and float(S[-1]) > 0.0
    U, V = out.U.double(), out.V.double()
    eye = torch.eye(100, dtype=torch.float64, device="cuda")
    assert float((U.T @ U - eye).abs().max()) < 1e-5
    assert float((V.T @ V - eye).abs().max()) < 1e-5
    AU = A.double() @ U
    resid = torch.linalg.norm(AU - V * S[None, :]) / torch.linalg.norm(S)
    assert float(resid) < 1e-5
    err = sid.error_norms(A, out.V * S.float()[None, :], out.U.T.contiguous())["rel_fro"]
    ide = sid.compress(A, 100, 20, seed=0, mode="single_pass", prec="f64", probe_rows=10)
    err_id = sid.error_norms(A, ide.AJ, ide.P)["rel_fro"]
    # the optimal rank-100 error from the spectrum of A^T A (FP64)
    lam = np.linalg.eigvalsh(host(A.double().T @ A.double()))[::-1]
    opt = float(np.sqrt(lam[100:].clip(min=0).sum() / lam.clip(min=0).sum()))
    say("sbr-svd rel_fro", err, "single-pass ID", err_id, "optimal", opt)
    assert err <= err_id
    # the expected-error bound of Sec. 2.3: factor (1 + k / (p - 1))^(1/2) over the
    # optimum (which the error, formed from FP32 factors, may undercut by rounding only)
    assert opt * (1 - 1e-4) <= err <= np.sqrt(1 + 100 / 19) * opt


@pytest.mark.parametrize("dt,prec,blocks", [
    (torch.float32, "bf16x2", [37, 200, 1, 300, 162]),      # stage flushes at 512, then 188
    (torch.float64, "f64", [600, 100]),                      # 512 sketched in place, stage 188
    (torch.float32, "f32", [50, 150]),                        # one flush at finish
])
def test_stream_equals_whole(sid, dt, prec, blocks):
    """Alg. 2's single pass over column blocks (sid_svd_stream_*): each
    sketched block adds its part of H in column order, so S, U, V equal the
    whole-matrix sid_sbr_svd bit for bit."""
    say("sbr-svd stream", dt, prec, blocks)
    n = sum(blocks)
    sig = 0.9 ** np.arange(n)
    A64 = synth.lowrank_exact_spectrum(20000, n, sig, seed=n, noise=1e-7).numpy()
    A = to_gpu(A64, dt)
    whole = sid.sbr_svd(A, 24, 16, 8, seed=7, prec=prec)
    st = sid.SvdStream(20000, n, 24, 16, 8, seed=7, prec=prec, dtype=dt)
    c0 = 0
    for nb in blocks:
        st.push(A[:, c0:c0 + nb])
        c0 += nb
    assert st.cols() == n
    out = st.finish()
    assert out.rank == whole.rank == 40
    assert torch.equal(out.S, whole.S)
    assert torch.equal(out.U, whole.U)
    assert torch.equal(out.V, whole.V)


def test_stream_rules(sid):
    """An SBR-SVD stream cannot be ended as an ID stream or saved, and needs
    k + oversample <= the columns pushed."""
    say("sbr-svd stream rules")
    A = to_gpu(np.random.default_rng(0).standard_normal((3000, 60)), torch.float32)
    st = sid.SvdStream(3000, 60, 10, 10, 10)
    st.push(A[:, :15])
    L, h = st.ctx._lib, st._h
    assert L.sid_stream_save(h, None, ctypes.byref(ctypes.c_size_t(0))) == -1
    with pytest.raises(sid.SidError):
        st.finish()                                 # 15 columns < l = 20
    st2 = sid.SvdStream(3000, 60, 10, 10, 10)
    st2.push(A)
    z = torch.zeros(1, dtype=torch.int64, device="cuda")
    assert L.sid_stream_finish(st2._h, ctypes.c_void_p(z.data_ptr()), None, 1, None, 1, None,
                               None) == -1
    out = st2.finish()
    assert out.rank == 20
