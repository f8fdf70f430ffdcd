"""Pins of the CPU oracle against facts fixed outside the oracle itself:
library routines (rocRAND's Philox, LAPACK pivoted QR, least squares, SVD),
closed forms, the paper's printed values, error bounds, invariants and brute
force on tiny inputs.  CPU only."""
import itertools
import math
import os
import shutil
import subprocess

import numpy as np
import pytest
import scipy.linalg
import scipy.stats

import synth

HERE = os.path.dirname(os.path.abspath(__file__))


# ---------------------------------------------------------------------------
# Generator
# ---------------------------------------------------------------------------

@pytest.fixture(scope="module")
def rocrand_philox(tmp_path_factory):
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc):
        pytest.skip("hipcc not available")
    exe = str(tmp_path_factory.mktemp("philox") / "philox_ref")
    src = os.path.join(HERE, "helpers", "philox_rocrand_ref.cpp")
    subprocess.check_call([hipcc, "-O1", "-o", exe, src], cwd="/tmp")
    return exe


def test_philox_matches_rocrand(oracle_mod, rocrand_philox):
    """Philox4x32-10 equals rocRAND's library implementation (counter words
    placed through its (subsequence, offset) seeding)."""
    rng = np.random.default_rng(5)
    cases = [(0, 0, 0, 0, 0, 0), (0xFFFFFFFF, 0x3FFFFFFF, 0xFFFFFFFF, 0xFFFFFFFF, 0xFFFFFFFF, 0xFFFFFFFF)]
    for _ in range(200):
        c = rng.integers(0, 2**32, size=6, dtype=np.uint64)
        c[1] &= 0x3FFFFFFF
        cases.append(tuple(int(v) for v in c))
    inp = "\n".join(" ".join(f"{v:x}" for v in c) for c in cases) + "\n"
    out = subprocess.run([rocrand_philox], input=inp, capture_output=True, text=True, check=True).stdout
    ref = [tuple(int(w, 16) for w in line.split()) for line in out.strip().splitlines()]
    assert len(ref) == len(cases)
    for c, r in zip(cases, ref):
        got = tuple(int(v) for v in oracle_mod.philox(c[:4], c[4:]))
        assert got == r


def _draw_pairs(oracle_mod, n_major=20000, seed=3):
    z = oracle_mod.gaussian(seed, 1, np.arange(n_major, dtype=np.int64), 0, 64)
    return z


def test_gaussian_moments_and_ks(oracle_mod):
    """Draws are standard normal: mean, variance, kurtosis within sampling
    error, and a Kolmogorov-Smirnov test against the normal CDF."""
    z = oracle_mod.gaussian(11, 0, np.arange(40000, dtype=np.int64), 0, 64).astype(np.float64).ravel()
    n = z.size  # 2.56e6
    assert abs(z.mean()) < 5 / math.sqrt(n)
    assert abs(z.var() - 1.0) < 5 * math.sqrt(2.0 / n)
    kurt = np.mean(z ** 4) / np.mean(z ** 2) ** 2
    assert abs(kurt - 3.0) < 5 * math.sqrt(24.0 / n)
    ks = scipy.stats.kstest(z[:500000], "norm")
    assert ks.pvalue > 1e-3


def test_box_muller_structure(oracle_mod):
    """Each Box-Muller pair satisfies z0^2 + z1^2 = -2 ln u and
    atan2(z1, z0) = (quadrant + t) pi/2 with u, quadrant, t read from the
    Philox words (checked with numpy's own log/atan2 to single precision)."""
    seed, stream = 123456789, 1
    for major in [0, 1, 7, 2**33 + 5]:
        for group in range(6):
            ctr = [major & 0xFFFFFFFF, group, stream, major >> 32]
            key = [seed & 0xFFFFFFFF, seed >> 32]
            x = [int(v) for v in oracle_mod.philox(ctr, key)]
            z = [float(oracle_mod.lib().oracle_gauss(seed, stream, major, 4 * group + e)) for e in range(4)]
            for (a, b), (z0, z1) in [((x[0], x[1]), (z[0], z[1])), ((x[2], x[3]), (z[2], z[3]))]:
                u = ((a >> 8) + 1) * 2.0 ** -24
                r2 = -2.0 * math.log(u)
                assert abs(z0 * z0 + z1 * z1 - r2) <= 2e-6 * max(r2, 1e-3)
                quad = b >> 30
                t = (2 * ((b >> 7) & 0x7FFFFF) + 1) * 2.0 ** -24
                ang = (quad + t) * math.pi / 2
                got = math.atan2(z1, z0) % (2 * math.pi)
                d = abs(got - ang)
                d = min(d, 2 * math.pi - d)
                assert d < 1e-5


def test_gaussian_keying(oracle_mod):
    """Entries depend only on (seed, stream, major, minor): blocks agree with
    single-entry evaluation; streams and seeds decorrelate."""
    blk = oracle_mod.gaussian(9, 1, np.array([3, 100, 5000], dtype=np.int64), 2, 9)
    for s, major in enumerate([3, 100, 5000]):
        for t in range(9):
            assert blk[s, t] == np.float32(oracle_mod.lib().oracle_gauss(9, 1, major, 2 + t))
    a = oracle_mod.gaussian(9, 0, np.arange(2000), 0, 16).ravel()
    b = oracle_mod.gaussian(9, 1, np.arange(2000), 0, 16).ravel()
    c = oracle_mod.gaussian(10, 0, np.arange(2000), 0, 16).ravel()
    assert abs(np.corrcoef(a, b)[0, 1]) < 0.03
    assert abs(np.corrcoef(a, c)[0, 1]) < 0.03


def test_rounding_maps(oracle_mod):
    """bfloat16 and e4m3 rounding: representable values are fixed points,
    halfway cases go to even, e4m3 saturates at 448 (OCP FP8 definition)."""
    r = oracle_mod.round_values
    assert r(np.array([1.0, -2.5, 3.140625]), "bf16").tolist() == [1.0, -2.5, 3.140625]
    # 1 + 2^-8 is halfway between 1 and 1 + 2^-7 -> even (1.0)
    assert r(np.array([1.0 + 2 ** -8]), "bf16")[0] == 1.0
    assert r(np.array([1.0 + 3 * 2 ** -8]), "bf16")[0] == 1.0 + 2 ** -6
    assert r(np.array([1.0625]), "e4m3")[0] == 1.0          # halfway -> even
    assert r(np.array([1.1875]), "e4m3")[0] == 1.25
    assert r(np.array([1000.0, -500.0]), "e4m3").tolist() == [448.0, -448.0]
    assert r(np.array([2 ** -9, 3 * 2 ** -10]), "e4m3").tolist() == [2 ** -9, 2 ** -8]


def test_e4m3_matches_torch_cast(oracle_mod):
    """The oracle's e4m3 rounding equals torch's float8_e4m3fn conversion (an
    independent implementation) on every FP32 value of a wide sweep below the
    saturation point, including the subnormal range and halfway cases."""
    import torch
    rng = np.random.default_rng(3)
    x = np.concatenate([
        rng.standard_normal(20000) * 10.0 ** rng.uniform(-4, 2.3, 20000),
        np.arange(-2048, 2049) * 2.0 ** -12,                # subnormals and halfway points
        # normal-range halfway points (1 + (2m + 1)/16) 2^e
        ((1.0 + (2 * np.arange(8) + 1) / 16.0)[None, :] * 2.0 ** np.arange(-6, 8)[:, None]).ravel(),
    ]).astype(np.float32)
    x = x[np.abs(x) < 448.0]
    ours = oracle_mod.round_values(x.astype(np.float64), "e4m3")
    ref = torch.from_numpy(x).to(torch.float8_e4m3fn).float().numpy().astype(np.float64)
    assert np.array_equal(ours, ref)


def test_fp8_tile_scaled_values(oracle_mod):
    """FP8 data values: every 64-row tile of a column is scaled by a power of
    two that puts its largest magnitude in [128, 256); the result equals
    torch's e4m3 cast of the scaled tile, scaled back; relative error <= 2^-4
    for entries not in the subnormal range; scaling a tile by 2^m scales its
    values by 2^m exactly; all-zero tiles stay zero."""
    import torch
    rng = np.random.default_rng(4)
    N, n = 300, 6
    A = (rng.standard_normal((N, n)) * np.array([1.0, 1e-3, 1e4, 0.0, 7.0, 2.0 ** -20])).astype(np.float32)
    A[70:100, 4] = 0.0
    A64 = A.astype(np.float64)
    V = oracle_mod.data_values(A64, "fp8")
    for t0 in range(0, N, 64):
        blk = A64[t0:t0 + 64]
        for j in range(n):
            col = blk[:, j]
            amax = np.abs(col).max()
            if amax == 0:
                assert np.all(V[t0:t0 + 64, j] == 0)
                continue
            s = 2.0 ** (math.floor(math.log2(amax)) - 7)
            assert 128 <= amax / s < 256
            ref = torch.from_numpy((col / s).astype(np.float32)).to(torch.float8_e4m3fn)
            assert np.array_equal(V[t0:t0 + 64, j], ref.double().numpy() * s)
            big = np.abs(col) >= s * 2.0 ** -6
            assert np.all(np.abs(V[t0:t0 + 64, j][big] - col[big]) <= 2.0 ** -4 * np.abs(col[big]))
    B = A64.copy()
    B[64:128] *= 2.0 ** 5
    VB = oracle_mod.data_values(B, "fp8")
    assert np.array_equal(VB[64:128], V[64:128] * 2.0 ** 5)
    assert np.array_equal(VB[:64], V[:64]) and np.array_equal(VB[128:], V[128:])


# ---------------------------------------------------------------------------
# Sketches
# ---------------------------------------------------------------------------

def _small(N=600, n=40, seed=1):
    rng = np.random.default_rng(seed)
    return rng.standard_normal((N, n)).astype(np.float32).astype(np.float64)


def test_sketch_matches_matmul(oracle_mod):
    """W and Y equal a library matmul of the explicitly formed test matrices."""
    A = _small()
    N, n = A.shape
    lq, l = 23, 17
    W = oracle_mod.sketch_w(A, None, lq, seed=4, prec="f64")
    Psi = oracle_mod.psi(4, np.arange(N), lq, "f64")
    np.testing.assert_allclose(W, Psi @ A, rtol=1e-12, atol=1e-12)
    Om = oracle_mod.omega(4, n, l, "f64")
    Y = oracle_mod.sketch_y(A, Om, "f64")
    np.testing.assert_allclose(Y, A @ Om, rtol=1e-12, atol=1e-12)


def test_fp8_sketch_matches_matmul(oracle_mod):
    """FP8 sketches: W and Y equal a library matmul of the Gaussian draws cast
    to e4m3 by torch and the tile-scaled e4m3 data; the FP8 ID of a
    well-separated low-rank matrix stays within the e4m3 precision of it."""
    import torch
    A = _small(640, 24, 5)
    N, n = A.shape
    lq, l = 19, 12
    z = oracle_mod.gaussian(9, 1, np.arange(N), 0, lq)
    Psi = torch.from_numpy(z).to(torch.float8_e4m3fn).double().numpy().T
    Ad = oracle_mod.data_values(A, "fp8")
    W = oracle_mod.sketch_w(A, None, lq, 9, "fp8")
    np.testing.assert_allclose(W, Psi @ Ad, rtol=1e-12, atol=1e-12)
    zo = oracle_mod.gaussian(9, 0, np.arange(n), 0, l)
    Om = torch.from_numpy(zo).to(torch.float8_e4m3fn).double().numpy()
    assert np.array_equal(Om, oracle_mod.omega(9, n, l, "fp8"))
    np.testing.assert_allclose(oracle_mod.sketch_y(A, Om, "fp8"), Ad @ Om, rtol=1e-12, atol=1e-12)
    rng = np.random.default_rng(6)
    L = rng.standard_normal((2000, 5)) @ rng.standard_normal((5, 40))
    for mode in ("two_pass", "single_pass"):
        res = oracle_mod.compress(L, k=5, oversample=5, seed=2, mode=mode, prec="fp8",
                                  sp_rcond=1e-3)
        e = oracle_mod.error_norms(L, res.AJ, res.P)
        assert e["rel_fro"] < 0.1, (mode, e)


def test_sketch_identity_and_scaling(oracle_mod):
    """Psi Y = W Omega (both are Psi A Omega); scaling A by 2^s scales W
    exactly; a coarse sketch equals the full sketch of A(S, :)."""
    A = _small(500, 30, 2)
    N, n = A.shape
    lq, l = 20, 14
    W = oracle_mod.sketch_w(A, None, lq, 7, "f64")
    Om = oracle_mod.omega(7, n, l, "f64")
    Y = oracle_mod.sketch_y(A, Om, "f64")
    lhs = oracle_mod.psi_times(np.arange(N), lq, 7, "f64", Y)
    np.testing.assert_allclose(lhs, W @ Om, rtol=1e-10, atol=1e-9)
    W8 = oracle_mod.sketch_w(8.0 * A, None, lq, 7, "f64")
    assert np.array_equal(W8, 8.0 * W)
    S = np.arange(3, N, 4)
    Wc = oracle_mod.sketch_w(A, S, lq, 7, "f64")
    Psi_S = oracle_mod.psi(7, S, lq, "f64")
    np.testing.assert_allclose(Wc, Psi_S @ A[S], rtol=1e-12, atol=1e-12)


def test_precision_value_maps(oracle_mod):
    """bf16x2 split reproduces the single-precision value to 2^-16 relative
    and hi/lo are bf16-representable; bf16 values round-trip."""
    rng = np.random.default_rng(3)
    a = rng.standard_normal(10000).astype(np.float32).astype(np.float64)
    v = oracle_mod.data_values(a, "bf16x2")
    assert np.max(np.abs(v - a) / np.abs(a)) <= 2.0 ** -16
    b = oracle_mod.data_values(a, "bf16")
    assert np.max(np.abs(b - a) / np.abs(a)) <= 2.0 ** -8
    assert np.array_equal(oracle_mod.data_values(b, "bf16"), b)


# ---------------------------------------------------------------------------
# mgsqr and coefficients
# ---------------------------------------------------------------------------

def _generic_wide(l=20, n=60, seed=0):
    rng = np.random.default_rng(seed)
    # decaying column scales make pivot choices well separated
    return rng.standard_normal((l, n)) * np.exp(-np.linspace(0, 3, n))[None, rng.permutation(n)]


def test_cpqr_matches_lapack_pivots(oracle_mod):
    """J equals LAPACK dgeqp3 pivots (scipy) on generic inputs whose pivot
    margins are well above roundoff; Q orthonormal; W(:, J) = Q R11."""
    for seed in range(6):
        W = _generic_wide(seed=seed)
        k = 12
        cp = oracle_mod.cpqr(W, k)
        assert cp.margins.min() > 1e-8
        _, Rl, piv = scipy.linalg.qr(W, pivoting=True, mode="economic")
        assert list(cp.J) == list(piv[:k])
        assert cp.J[0] == int(np.argmax(np.linalg.norm(W, axis=0)))
        np.testing.assert_allclose(cp.Q.T @ cp.Q, np.eye(k), atol=1e-13)
        np.testing.assert_allclose(W[:, cp.J], cp.Q @ cp.R[:, cp.J], rtol=1e-12, atol=1e-12)
        # |R11| diagonal equals |R| diagonal of LAPACK
        np.testing.assert_allclose(np.abs(np.diag(cp.R[:, cp.J])), np.abs(np.diag(Rl)[:k]),
                                   rtol=1e-10)


def test_coefficients_identity_lstsq_and_bound(oracle_mod):
    """P(:, J) = I bitwise; P = W(:, J)^+ W (least squares); ||P||_2 <=
    sqrt(1 + k (n - k)) (the coefficient bound quoted after Thm 2.1)."""
    for seed in range(4):
        W = _generic_wide(l=25, n=70, seed=seed)
        k = 15
        cp = oracle_mod.cpqr(W, k)
        P = oracle_mod.id_coefficients(cp.R, cp.J, W.shape[1])
        assert np.array_equal(P[:, cp.J], np.eye(k))
        X, *_ = np.linalg.lstsq(W[:, cp.J], W, rcond=None)
        np.testing.assert_allclose(P, X, rtol=1e-9, atol=1e-10)
        assert np.linalg.norm(P, 2) <= math.sqrt(1 + k * (W.shape[1] - k))


def test_rank_tolerance_stop(oracle_mod):
    """Exact rank r: mgsqr stops at k_eff = r under a relative tolerance and
    the discarded residual is at roundoff (Remark 2.2 stopping rule)."""
    rng = np.random.default_rng(2)
    r = 6
    W = rng.standard_normal((30, r)) @ rng.standard_normal((r, 50))
    cp = oracle_mod.cpqr(W, 20, rank_tol=1e-10)
    assert cp.k_eff == r
    cp0 = oracle_mod.cpqr(np.zeros((5, 8)), 3)
    assert cp0.k_eff == 0


def test_brute_force_subsets(oracle_mod):
    """Tiny inputs: for every subset of k columns the least-squares error is
    at least the best subset's; the deterministic ID's P is the least-squares
    optimum for its J, so its error equals that subset's minimum."""
    rng = np.random.default_rng(8)
    A = rng.standard_normal((15, 10)) @ np.diag(np.exp(-np.arange(10) / 2.0))
    for k in (1, 2, 3):
        cp = oracle_mod.cpqr(A, k)
        P = oracle_mod.id_coefficients(cp.R, cp.J, A.shape[1])
        e_id = np.linalg.norm(A - A[:, cp.J] @ P)
        best = min(np.linalg.norm(A - A[:, list(S)] @ np.linalg.lstsq(A[:, list(S)], A, rcond=None)[0])
                   for S in itertools.combinations(range(A.shape[1]), k))
        sub = A[:, cp.J]
        e_ls = np.linalg.norm(A - sub @ np.linalg.lstsq(sub, A, rcond=None)[0])
        assert abs(e_id - e_ls) <= 1e-12 * np.linalg.norm(A)
        assert e_id >= best - 1e-12
        s = np.linalg.svd(A, compute_uv=False)
        assert best >= np.sqrt(np.sum(s[k:] ** 2)) - 1e-12


def test_deterministic_id_spectral_bound(oracle_mod):
    """Deterministic ID (mgsqr on A itself) obeys
    ||A - A(:, J) P||_2 <= sqrt(1 + k (n - k)) sigma_{k+1}  (eq. (id_bound_orig))."""
    for seed in range(3):
        A = np.asarray(synth.lowrank_exact_spectrum(300, 40, np.exp(-np.arange(1, 41) / 4.0), seed=seed))
        for k in (5, 10, 20):
            cp = oracle_mod.cpqr(A, k)
            P = oracle_mod.id_coefficients(cp.R, cp.J, A.shape[1])
            e2 = np.linalg.norm(A - A[:, cp.J] @ P, 2)
            s = np.linalg.svd(A, compute_uv=False)
            assert e2 <= math.sqrt(1 + k * (A.shape[1] - k)) * s[k] * (1 + 1e-10)
            assert e2 >= s[k] * (1 - 1e-10)           # Eckart-Young, 2-norm


# ---------------------------------------------------------------------------
# Whole compressor
# ---------------------------------------------------------------------------

def _c1_like(N=1024, n=96, noise=1e-8, seed=1000):
    sig = np.exp(-np.arange(1, n + 1) / 10.0)
    return np.asarray(synth.lowrank_exact_spectrum(N, n, sig, seed=seed, noise=noise)), sig


def test_exact_recovery_both_modes(oracle_mod):
    """rank(A) = r <= k: both modes reproduce A to roundoff."""
    rng = np.random.default_rng(4)
    r = 7
    A = rng.standard_normal((800, r)) @ rng.standard_normal((r, 60))
    for mode in ("two_pass", "single_pass"):
        res = oracle_mod.compress(A, k=10, oversample=6, seed=1, mode=mode)
        e = oracle_mod.error_norms(A, res.AJ, res.P)
        assert e["rel_fro"] < 1e-12, (mode, e)


def test_closed_form_optimum_and_eckart_young(oracle_mod):
    """sigma_j = exp(-j/10): the optimal rank-k error is exp(-k/10)
    (geometric tail); the ID error is never below it and stays within a
    small factor of it (randomized ID error, Sec. 2.4)."""
    A, sig = _c1_like()
    k = 20
    opt = math.sqrt(np.sum(sig[k:] ** 2) / np.sum(sig ** 2))
    assert abs(opt - math.exp(-k / 10.0)) < 1e-3
    for mode in ("two_pass", "single_pass"):
        res = oracle_mod.compress(A, k=k, oversample=10, seed=0, mode=mode)
        e = oracle_mod.error_norms(A, res.AJ, res.P)["rel_fro"]
        assert e >= opt * (1 - 1e-6)
        assert e <= 6 * opt


def test_single_pass_shares_selection_with_two_pass(oracle_mod):
    """Single-pass and two-pass ID select bit-identical J and P from the same
    sketch (Alg. 5 and Alg. 6 share their selection steps), and the
    single-pass skeleton satisfies the interpolation identity
    Psi_sel A_J_hat = W_sel(:, J)."""
    A, _ = _c1_like(N=700, n=64)
    r2 = oracle_mod.compress(A, 12, 8, seed=3, mode="two_pass")
    r1 = oracle_mod.compress(A, 12, 8, seed=3, mode="single_pass")
    assert np.array_equal(r1.J, r2.J) and np.array_equal(r1.P, r2.P)
    lz = 20 + 8   # selection rows + extra co-range rows
    lhs = oracle_mod.psi_times(np.arange(A.shape[0]), lz + 10, 3, "f64", r1.AJ)[:lz]
    # least-squares fit on a tall system: the identity holds up to the
    # residual of the fit, which is the part of W(:, J) outside Psi range(Y)
    proj = r1.W[:lz][:, r1.J]
    assert np.linalg.norm(lhs - proj) <= 0.5 * np.linalg.norm(proj)
    # exact when A has rank <= l
    rng = np.random.default_rng(1)
    B = rng.standard_normal((400, 6)) @ rng.standard_normal((6, 40))
    rb = oracle_mod.compress(B, 5, 4, seed=3, mode="single_pass")
    lhs = oracle_mod.psi_times(np.arange(400), 19, 3, "f64", rb.AJ)[:9 + 4]
    np.testing.assert_allclose(lhs, rb.W[:13][:, rb.J], rtol=1e-9, atol=1e-9 * np.abs(rb.W).max())


def test_probe_estimator_tracks_true_error(oracle_mod):
    """err_probe is within [0.5, 2] of the true relative error in at least
    95% of seeded trials (held-out Psi rows are independent of J, P)."""
    A, _ = _c1_like(N=600, n=80)
    ok = 0
    trials = 40
    for s in range(trials):
        res = oracle_mod.compress(A, 10, 5, seed=s, mode="two_pass", probe_rows=10)
        e = oracle_mod.error_norms(A, res.AJ, res.P)["rel_fro"]
        ok += 0.5 <= res.err_probe / e <= 2.0
    assert ok >= 0.95 * trials


def test_permutation_metamorphic(oracle_mod):
    """Permuting A's columns permutes the sketch's columns, hence J (pivot
    margins large), and leaves the error unchanged."""
    A, _ = _c1_like(N=500, n=50)
    perm = np.random.default_rng(1).permutation(50)
    r = oracle_mod.compress(A, 8, 6, seed=2)
    rp = oracle_mod.compress(A[:, perm], 8, 6, seed=2)
    assert r.cp.margins.min() > 1e-6
    assert list(perm[rp.J]) == list(r.J)


def test_subsampled_bound_thm21(oracle_mod):
    """Sub-sampled ID (mgsqr on the coarse rows A_c = A(S, :), literal
    Alg. 5) obeys Thm 2.1: ||A - A_hat||_2 <= min over tau of rho_k(tau)."""
    x = np.linspace(0, 1, 257)
    t = np.linspace(0, 1, 40)
    A = np.array([[np.sin(2 * np.pi * (xi - 0.3 * tj)) * np.exp(-tj) + 0.3 * np.cos(6 * np.pi * xi * (1 + tj))
                   for tj in t] for xi in x])
    S = np.arange(0, 257, 4)
    Ac = A[S]
    n = A.shape[1]
    for k in (3, 5, 8):
        cp = oracle_mod.cpqr(Ac, k)
        P = oracle_mod.id_coefficients(cp.R, cp.J, n)
        err = np.linalg.norm(A - A[:, cp.J] @ P, 2)
        sc = np.linalg.svd(Ac, compute_uv=False)
        ec = np.linalg.norm(Ac - Ac[:, cp.J] @ P, 2)
        pn = np.linalg.norm(P, 2)
        G = A.T @ A
        Gc = Ac.T @ Ac
        best = np.inf
        for tau in np.linspace(0.0, 3 * len(x) / len(S), 400):
            eps = max(np.linalg.eigvalsh(G - tau * Gc).max(), 0.0)
            rho = (1 + pn) * math.sqrt(tau * sc[k] ** 2 + eps) + ec * math.sqrt(tau + eps / sc[k - 1] ** 2)
            best = min(best, rho)
        assert err <= best * (1 + 1e-9)


def test_compression_factor_printed_values(oracle_mod):
    """The Table 1 storage count k(m + n) reproduces the compression factors
    printed in Fig. 7's caption (golden fixture) and the temporal factor
    n/k = 100 of Sec. 3.3 (10000 steps at k = 100)."""
    rows = np.loadtxt(os.path.join(HERE, "golden", "compression_factor_fig7.txt"))
    for k, printed, m, nsp in rows:
        cf = oracle_mod.compression_factor(int(nsp), int(m), int(k))
        assert round(cf / 10) * 10 == printed or abs(cf - printed) / printed < 0.002
    assert oracle_mod.temporal_compression_factor(10000, 100) == 100.0


def test_refinement_least_squares(oracle_mod):
    """Refinement of P (the least-squares coefficients of the refinement
    sketch with J fixed), pinned without its library solve: (1) with the
    refinement sketch equal to the first one it returns the first P, which
    mgsqr and back substitution formed (R11^-1 R12); (2) the residual of the
    refinement sketch is orthogonal to its pivot columns (normal equations)
    and P(:, J) = I exactly; (3) on a matrix of rank k the refined ID is
    exact, whatever the precision of the first sketch; (4) from an FP8
    first sketch the refined ID is at least as accurate as the unrefined
    one."""
    rng = np.random.default_rng(31)
    N, n, k, p = 3000, 60, 8, 6
    A = (rng.standard_normal((N, 12)) @ rng.standard_normal((12, n))
         * np.exp(-np.arange(n) / 15.0)).astype(np.float32).astype(np.float64)
    l = k + p
    res = oracle_mod.compress(A, k, p, seed=5, mode="two_pass", prec="bf16x2", probe_rows=0)
    P1 = oracle_mod.refine(A, res, seed=5, refine_prec="bf16x2", l=l)
    assert np.max(np.abs(P1 - res.P)) <= 1e-9 * np.max(np.abs(res.P))
    res8 = oracle_mod.compress(A, k, p, seed=5, mode="two_pass", prec="fp8", probe_rows=0)
    J = res8.cp.J
    P8 = oracle_mod.refine(A, res8, seed=5, refine_prec="f64", l=l)
    assert np.array_equal(P8[:, J], np.eye(k))
    Wp = oracle_mod.sketch_w(A, None, l, 5, "f64")
    ne = Wp[:, J].T @ (Wp - Wp[:, J] @ P8)
    assert np.max(np.abs(ne)) <= 1e-11 * np.linalg.norm(Wp[:, J]) * np.linalg.norm(Wp)
    e0 = oracle_mod.error_norms(A, A[:, J], res8.P)["rel_fro"]
    e1 = oracle_mod.error_norms(A, A[:, J], P8)["rel_fro"]
    assert e1 <= e0
    Lk = rng.standard_normal((N, k)) @ rng.standard_normal((k, n))
    r8 = oracle_mod.compress(Lk, k, p, seed=7, mode="two_pass", prec="fp8", probe_rows=0)
    Pk = oracle_mod.refine(Lk, r8, seed=7, refine_prec="f64", l=l)
    assert oracle_mod.error_norms(Lk, Lk[:, r8.cp.J], Pk)["rel_fro"] < 1e-12


def test_literal_subsampled_id_matches_lapack(oracle_mod):
    """Alg. 5 literal: mgsqr directly on A(S, :).  With well-separated
    pivots its J equals LAPACK's pivoted QR (dgeqp3) of A(S, :); with S all
    rows and rank(A) <= k the ID is exact."""
    rng = np.random.default_rng(41)
    N, n, k = 400, 30, 6
    A = rng.standard_normal((N, n)) * np.exp(-np.linspace(0, 4, n))[None, rng.permutation(n)]
    S = np.arange(1, N, 3)
    res = oracle_mod.compress_literal(A, k, S)
    _, _, piv = scipy.linalg.qr(A[S], pivoting=True, mode="economic")
    assert res.J.tolist() == piv[:k].tolist()
    assert np.isnan(res.err_probe)
    L = rng.standard_normal((N, 4)) @ rng.standard_normal((4, n))
    r2 = oracle_mod.compress_literal(L, 6, np.arange(N), rank_tol=1e-10)
    assert r2.k_eff == 4
    assert oracle_mod.error_norms(L, r2.AJ[:, :4], r2.P[:4])["rel_fro"] < 1e-12


# ---------------------------------------------------------------------------
# Tolerance-driven rank from the probe rows (Remark 2.2)
# ---------------------------------------------------------------------------

def test_adaptive_rank_exact_rank_matrix(oracle_mod):
    """A matrix of exact rank r: every pivot prefix shorter than r leaves a
    probe error of the order of the next singular value, the prefix of length
    r leaves rounding only, so any tolerance between them selects k_eff = r."""
    r = 12
    sig = 0.7 ** np.arange(r)
    A = synth.lowrank_exact_spectrum(700, 90, sig, seed=31).numpy()
    for tol in (1e-9, 1e-7):
        res = oracle_mod.compress(A, 30, 10, seed=2, mode="two_pass", prec="f64", probe_rows=10,
                              probe_tol=tol)
        assert res.k_eff == r, (tol, res.k_eff)
        assert res.err_probe <= tol
        assert np.all(res.J[r:] == -1) and np.all(res.P[r:] == 0.0)
    # a loose tolerance stops at the first prefix that meets it
    res = oracle_mod.compress(A, 30, 10, seed=2, mode="two_pass", prec="f64", probe_rows=10,
                          probe_tol=10.0)
    assert res.k_eff == 1


def test_adaptive_rank_prefix_errors_two_formulations(oracle_mod):
    """The prefix errors from the definition (coefficients of every prefix)
    equal the one-solve form ||W_pr - Z(:, :k') R(:k', :)|| with
    Z = W_pr(:, J) R11^-1 (a triangular inverse restricted to a leading block
    is that block's inverse); and the chosen rank is the first prefix under
    the tolerance."""
    sig = np.arange(1, 61, dtype=np.float64) ** -2.0
    A = synth.lowrank_exact_spectrum(500, 60, sig, seed=5, noise=1e-6).numpy()
    W = oracle_mod.sketch_w(A, np.arange(500), 30 + 10, 4, "f64")
    cp = oracle_mod.cpqr(W[:30], 25)
    Wpr = W[30:]
    e = oracle_mod.probe_prefix_errors(cp, Wpr, 60)
    R11 = cp.R[:, cp.J]
    Z = np.linalg.solve(R11.T, Wpr[:, cp.J].T).T
    nrm = np.linalg.norm(Wpr)
    for kp in range(1, cp.k_eff + 1):
        alt = np.linalg.norm(Wpr - Z[:, :kp] @ cp.R[:kp]) / nrm
        assert alt == pytest.approx(e[kp], rel=1e-9, abs=1e-13)
    tol = 0.5 * (e[8] + e[9]) if e[9] < e[8] else e[9]
    cp2 = oracle_mod.adaptive_rank(cp, Wpr, 60, tol)
    assert e[cp2.k_eff] <= tol and all(e[i] > tol for i in range(1, cp2.k_eff))


def test_err_sketch_hand_case_and_mgs_residual(oracle_mod):
    """err_sketch (the sketch-fit estimate, Remark 2.2) pinned two ways.

    Hand case: W = [[3, 0, 1], [4, 0, 0]], k = 1.  mgsqr picks column 0
    (norm 5), q = (0.6, 0.8); column 2 gets the coefficient (q . w_2) / 5 =
    0.12 and keeps the residual (0.64, -0.48) of norm 0.8, so ||W - W(:, J) P||_F / ||W||_F = 0.8 / sqrt(26).
    Generic case: the same ratio equals ||R22||_F / ||W||_F, the norm of
    mgsqr's own final residual (the columns it did not pick, after k
    projections), computed without P."""
    W = np.array([[3.0, 0.0, 1.0], [4.0, 0.0, 0.0]])
    cp = oracle_mod.cpqr(W, 1)
    assert cp.J.tolist() == [0]
    np.testing.assert_allclose(cp.final_residual[:, 2], [0.64, -0.48], rtol=0, atol=1e-15)
    P = oracle_mod.id_coefficients(cp.R, cp.J, 3)
    np.testing.assert_allclose(P, [[1.0, 0.0, 0.12]], rtol=0, atol=1e-15)  # (q . w_2) / 5
    # compress() reports the ratio on the selection rows of its own sketch;
    # feed the hand matrix through the same fit
    fit = np.linalg.norm(W - W[:, cp.J] @ P) / np.linalg.norm(W)
    assert abs(fit - 0.8 / math.sqrt(26.0)) <= 1e-15
    rng = np.random.default_rng(41)
    A = rng.standard_normal((400, 9)) @ rng.standard_normal((9, 60)) + 1e-3 * rng.standard_normal((400, 60))
    for mode in ("two_pass", "single_pass"):
        k, p = 7, 5
        res = oracle_mod.compress(A, k, p, seed=4, mode=mode, prec="f64", probe_rows=6)
        Wsel = res.W[:k + p]
        r22 = np.linalg.norm(res.cp.final_residual) / np.linalg.norm(Wsel)
        assert abs(res.err_sketch - r22) <= 1e-12 * r22, (mode, res.err_sketch, r22)


def test_error_norms_relative_max_hand_case(oracle_mod):
    """Relative entry-wise error (Sec. 3.1): max |A_ij - Ahat_ij| / |A_ij| over
    the nonzero entries of A, with the absolute maximum beside it.  Hand case
    with Ahat = AJ P = [[1.1, 0.5], [2, 3]] against A = [[1, 0], [2, 4]]:
    relative errors 0.1 and 0.25 (the zero entry, absolute error 0.5, is
    excluded), absolute maximum 1; ||A - Ahat||_F^2 = 0.01 + 0.25 + 1."""
    A = np.array([[1.0, 0.0], [2.0, 4.0]])
    AJ = np.array([[1.1, 0.5], [2.0, 3.0]])
    P = np.eye(2)
    e = oracle_mod.error_norms(A, AJ, P)
    assert abs(e["rel_max"] - 0.25) <= 1e-15
    assert abs(e["max_abs"] - 1.0) <= 1e-15
    assert abs(e["fro_err"] - math.sqrt(1.26)) <= 1e-15
    assert abs(e["fro_a"] - math.sqrt(21.0)) <= 1e-15
    # all-zero column and a rank-1 product: the zero entries never enter
    A = np.array([[0.0, 2.0], [0.0, -4.0]])
    AJ = np.array([[1.0], [1.0]])
    P = np.array([[1.0, 2.5]])
    e = oracle_mod.error_norms(A, AJ, P)
    assert abs(e["rel_max"] - 1.625) <= 1e-15      # |-4 - 2.5| / 4
    assert abs(e["max_abs"] - 6.5) <= 1e-15
