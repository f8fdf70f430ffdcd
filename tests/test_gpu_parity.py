"""GPU parity: the HIP path (through the C ABI) against the CPU oracle on the
same seeded inputs.  Marked gpu."""
import ctypes
import math
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


def to_gpu(A64: np.ndarray, dtype=torch.float32, ld: int | None = None) -> torch.Tensor:
    """Column-major device copy; ld > N pads every column (leading dimension)."""
    t = torch.from_numpy(np.asfortranarray(A64)).to(dtype)
    if ld is None:
        return synth.as_colmajor(t).cuda()
    N, n = A64.shape
    store = torch.zeros((n, ld), dtype=dtype, device="cuda")
    out = store.T[:N]
    out.copy_(t.cuda())
    return out


def ld4(N: int) -> int:
    return (N + 3) // 4 * 4


def host(t: torch.Tensor) -> np.ndarray:
    return t.detach().cpu().numpy()


# sketch tolerance: relative to sum |Psi||A| per entry (accumulation error bound)
# |err| <= 10 sqrt(L) u * sum|Psi||A| with L <= 8192 terms per partial sum
RTOL = {"f64": 1e-13, "f32": 5e-5, "bf16": 5e-5, "bf16x2": 5e-5, "fp8": 5e-5}


def _absbound(A64, rows, lq, seed, prec, oracle_mod):
    Psi = oracle_mod.psi(seed, rows, lq, prec)
    return np.abs(Psi) @ np.abs(oracle_mod.data_values(A64[rows], prec))


def test_gaussian_bit_identical(sid, oracle_mod):
    """Device generator == oracle generator, bit for bit, both streams."""
    for seed in (0, 7, 2**40 + 3):
        for stream, major0, nmajor, minor0, nminor in [(0, 0, 513, 0, 120), (1, 10**6, 257, 3, 131),
                                                       (1, 2**32 - 5, 20, 0, 9)]:
            say("gauss", seed, stream, major0, nmajor, minor0, nminor)
            g = host(sid.fill_gaussian(seed, stream, major0, nmajor, minor0, nminor))
            o = oracle_mod.gaussian(seed, stream, np.arange(major0, major0 + nmajor, dtype=np.int64),
                                    minor0, nminor)
            assert np.array_equal(g.view(np.uint32), o.view(np.uint32))


@pytest.mark.parametrize("prec", ["f64", "f32", "bf16", "bf16x2"])
@pytest.mark.parametrize("shape", [(1000, 77, 6, 4, 3), (4096, 256, 20, 10, 10), (333, 5, 3, 2, 0)])
def test_sketch_parity(sid, oracle_mod, prec, shape):
    N, n, k, p, q = shape
    say("sketch", prec, shape)
    rng = np.random.default_rng(N + n)
    A64 = rng.standard_normal((N, n)).astype(np.float32).astype(np.float64)
    A = to_gpu(A64, torch.float64 if prec == "f64" else torch.float32)
    seed = 5
    W, Y = sid.sketch(A, k, p, seed=seed, prec=prec, probe_rows=q, want_y=True)
    l = k + p
    lq = l + p + q
    Wo = oracle_mod.sketch_w(A64, None, lq, seed, prec)
    bound = _absbound(A64, np.arange(N), lq, seed, prec, oracle_mod)
    err = np.abs(host(W) - Wo)
    assert np.all(err <= RTOL[prec] * bound + 1e-300), (err / bound).max()
    Yo = oracle_mod.sketch_y(A64, oracle_mod.omega(seed, n, l, prec), prec)
    ybound = np.abs(oracle_mod.data_values(A64, prec)) @ np.abs(oracle_mod.omega(seed, n, l, prec))
    yerr = np.abs(host(Y).astype(np.float64) - Yo)
    assert np.all(yerr <= RTOL[prec] * ybound + 1e-300), (yerr / ybound).max()


@pytest.mark.parametrize("prec", ["bf16", "bf16x2", "fp8", "f32"])
@pytest.mark.parametrize("shape", [(2597, 500, 100, 20, 10), (49394, 500, 100, 20, 10),
                                   (700, 129, 7, 3, 2), (5000, 300, 60, 10, 5),
                                   (3001, 1100, 30, 10, 5)])
def test_sketch_parity_streaming_sizes(sid, oracle_mod, prec, shape):
    """Shapes that exercise the streaming matrix-core pass (FP32 data with a
    leading dimension padded to a multiple of 4): n up to 512 (four
    128-column chunks), lq up to 160 (W rows beyond 128 kept in LDS), l up to
    128, workgroups with full panels plus a ragged tail, and a workgroup that
    owns only a tail; n = 1100 runs as three column slabs.  The data span
    several decades per column so that the FP8 tile scales differ from tile
    to tile."""
    N, n, k, p, q = shape
    say("sketch streaming", prec, shape)
    rng = np.random.default_rng(N + 7 * n)
    A64 = rng.standard_normal((N, n)) * np.exp(rng.uniform(-3, 3, (N // 64 + 1, n))).repeat(64, 0)[:N]
    A64 = A64.astype(np.float32).astype(np.float64)
    A = to_gpu(A64, torch.float32, ld=ld4(N))
    seed = 11
    W, Y = sid.sketch(A, k, p, seed=seed, prec=prec, probe_rows=q, want_y=True)
    l = k + p
    lq = l + p + q
    Wo = oracle_mod.sketch_w(A64, None, lq, seed, prec)
    bound = _absbound(A64, np.arange(N), lq, seed, prec, oracle_mod)
    err = np.abs(host(W) - Wo)
    assert np.all(err <= RTOL[prec] * bound), (err / bound).max()
    Om = oracle_mod.omega(seed, n, l, prec)
    Yo = oracle_mod.sketch_y(A64, Om, prec)
    ybound = np.abs(oracle_mod.data_values(A64, prec)) @ np.abs(Om)
    yerr = np.abs(host(Y).astype(np.float64) - Yo)
    assert np.all(yerr <= RTOL[prec] * ybound), (yerr / ybound).max()


def test_sketch_coarse_rows(sid, oracle_mod):
    N, n, k, p, q = 2000, 40, 5, 5, 4
    say("coarse sketch")
    rng = np.random.default_rng(3)
    A64 = rng.standard_normal((N, n)).astype(np.float32).astype(np.float64)
    A = to_gpu(A64, torch.float64)
    S = np.sort(rng.choice(N, size=300, replace=False)).astype(np.int64)
    rs = sid.RowSet(S, N)
    W, _ = sid.sketch(A, k, p, seed=9, coarse=rs, prec="f64", probe_rows=q, want_y=False)
    Wo = oracle_mod.sketch_w(A64, S, k + p + q, 9, "f64")
    np.testing.assert_allclose(host(W), Wo, rtol=1e-12, atol=1e-12 * np.abs(Wo).max())


def c1_matrix(N=4096, n=256, seed=1000):
    sig = np.exp(-np.arange(1, n + 1) / 10.0)
    return np.asarray(synth.lowrank_exact_spectrum(N, n, sig, seed=seed, noise=1e-8)), sig


@pytest.mark.parametrize("mode", ["two_pass", "single_pass"])
def test_c1_fp64_bit_exact_pivots(sid, oracle_mod, mode):
    """FP64 mode on the 4096 x 256 exact-spectrum matrix (k=20, p=10):
    J identical to the oracle, P and errors to FP64 roundoff."""
    say("c1 fp64", mode)
    A64, sig = c1_matrix()
    A = to_gpu(A64, torch.float64)
    k, p, q = 20, 10, 10
    out = sid.compress(A, k, p, seed=0, mode=mode, prec="f64", probe_rows=q)
    torch.cuda.synchronize()
    ref = oracle_mod.compress(A64, k, p, seed=0, mode=mode, prec="f64", probe_rows=q)
    assert ref.cp.margins.min() > 1e-10
    assert host(out.J).tolist() == ref.J.tolist()
    assert int(host(out.k_eff)[0]) == k
    P = host(out.P)
    np.testing.assert_allclose(P, ref.P, rtol=0, atol=1e-10 * np.abs(ref.P).max())
    assert np.array_equal(P[:, ref.J], np.eye(k))
    e = host(out.err)
    say("c1 fp64", mode, "rel diff err_sketch", abs(e[1] - ref.err_sketch) / ref.err_sketch,
        "err_probe", abs(e[0] - ref.err_probe) / ref.err_probe)
    assert abs(e[1] - ref.err_sketch) <= 1e-10 * ref.err_sketch
    # single pass: the probe estimate passes through the skeleton solve (the
    # GPU's least squares on mgsqr of M = W Omega against the oracle's
    # Householder Q of Y and SVD pseudo-inverse), which agree to ~1e-10
    assert abs(e[0] - ref.err_probe) <= (1e-10 if mode == "two_pass" else 1e-8) * ref.err_probe
    AJ = host(out.AJ)
    if mode == "two_pass":
        assert np.array_equal(AJ, A64[:, ref.J])
    else:
        np.testing.assert_allclose(AJ, ref.AJ, rtol=0, atol=1e-9 * np.abs(ref.AJ).max())
    eg = sid.error_norms(A, out.AJ, out.P)
    eo = oracle_mod.error_norms(A64, ref.AJ, ref.P)
    say("c1 fp64", mode, "rel diff rel_fro", abs(eg["rel_fro"] - eo["rel_fro"]) / eo["rel_fro"])
    # two pass: the error of the exact columns A(:, J) and P; single pass also
    # carries the skeleton estimate (AJ within 1e-9 of the oracle's above)
    tol = 1e-10 if mode == "two_pass" else 1e-9
    assert abs(eg["rel_fro"] - eo["rel_fro"]) <= tol * eo["rel_fro"] + 1e-14
    opt = math.sqrt(np.sum(sig[k:] ** 2) / np.sum(sig ** 2))
    assert eg["rel_fro"] >= opt * (1 - 1e-6)


@pytest.mark.parametrize("prec", ["f32", "bf16x2", "bf16", "fp8"])
def test_low_precision_modes(sid, oracle_mod, prec):
    """FP32 data, low-precision sketches: pivots agree with the oracle (run
    in the same sketch precision) until its first near-tie, and the error is
    within a stated factor of the oracle's."""
    say("lowprec", prec)
    A64, _ = c1_matrix(N=4096, n=256, seed=1001)
    A64 = A64.astype(np.float32).astype(np.float64)
    A = to_gpu(A64, torch.float32)
    k, p, q = 20, 10, 10
    for mode in ("two_pass", "single_pass"):
        out = sid.compress(A, k, p, seed=1, mode=mode, prec=prec, probe_rows=q)
        torch.cuda.synchronize()
        ref = oracle_mod.compress(A64, k, p, seed=1, mode=mode, prec=prec, probe_rows=q)
        J = host(out.J)
        tie = {"f32": 1e-5, "bf16x2": 1e-4, "bf16": 1e-2, "fp8": 3e-2}[prec]
        ist = next((i for i, m in enumerate(ref.cp.margins) if m <= tie), k)
        assert J[:ist].tolist() == ref.J[:ist].tolist(), (prec, mode, ist)
        eg = sid.error_norms(A, out.AJ, out.P)["rel_fro"]
        eo = oracle_mod.error_norms(A64, ref.AJ, ref.P)["rel_fro"]
        fac = {"f32": 1.01, "bf16x2": 1.05, "bf16": 1.5, "fp8": 1.5}[prec]
        say("lowprec", prec, mode, "gpu", eg, "oracle", eo)
        assert eg <= fac * eo + 1e-6, (prec, mode, eg, eo)
        assert eg >= eo / fac - 1e-6, (prec, mode, eg, eo)


def test_exact_rank_recovery(sid):
    """rank(A) = 7 <= k: both modes reproduce A (FP64 and FP32)."""
    rng = np.random.default_rng(4)
    A64 = rng.standard_normal((3000, 7)) @ rng.standard_normal((7, 90))
    for dt, prec, tol in [(torch.float64, "f64", 1e-11), (torch.float32, "f32", 5e-6)]:
        A = to_gpu(A64, dt)
        for mode in ("two_pass", "single_pass"):
            say("exact rank", prec, mode)
            out = sid.compress(A, 10, 6, seed=2, mode=mode, prec=prec)
            e = sid.error_norms(A, out.AJ, out.P)
            assert e["rel_fro"] < tol, (prec, mode, e)


def test_rank_tolerance_and_degenerate(sid):
    say("rank tol")
    rng = np.random.default_rng(5)
    A64 = rng.standard_normal((500, 5)) @ rng.standard_normal((5, 40))
    A = to_gpu(A64, torch.float64)
    out = sid.compress(A, 12, 4, seed=0, prec="f64", rank_tol=1e-9)
    keff = int(host(out.k_eff)[0])
    assert keff == 5
    J = host(out.J)
    assert (J[keff:] == -1).all()
    assert np.all(host(out.P)[keff:] == 0)
    Z = torch.zeros((300, 20), dtype=torch.float64, device="cuda").T.contiguous().T
    out = sid.compress(Z, 4, 2, prec="f64")
    assert int(host(out.k_eff)[0]) == 0


def test_edge_shapes(sid, oracle_mod):
    """k = n, k = 1, no oversampling, no probe rows, n not a multiple of the
    tile, tiny N."""
    rng = np.random.default_rng(6)
    for (N, n, k, p, q) in [(70, 12, 12, 0, 0), (129, 3, 1, 0, 2), (65, 65, 30, 5, 1), (1, 1, 1, 0, 0)]:
        say("edge", N, n, k, p, q)
        A64 = rng.standard_normal((N, n))
        A = to_gpu(A64, torch.float64)
        for mode in ("two_pass", "single_pass"):
            out = sid.compress(A, k, p, seed=3, mode=mode, prec="f64", probe_rows=q)
            torch.cuda.synchronize()
            ref = oracle_mod.compress(A64, k, p, seed=3, mode=mode, prec="f64", probe_rows=q)
            kk = ref.k_eff
            assert host(out.J)[:kk].tolist() == ref.J[:kk].tolist()
            np.testing.assert_allclose(host(out.P), ref.P, atol=1e-9 * max(1, np.abs(ref.P).max()))


def test_reconstruct_matches_oracle(sid, oracle_mod):
    say("reconstruct")
    rng = np.random.default_rng(7)
    AJ64 = rng.standard_normal((1000, 13))
    P64 = rng.standard_normal((13, 70))
    for dt, tol in [(torch.float64, 1e-13), (torch.float32, 1e-5)]:
        out = sid.reconstruct(to_gpu(AJ64, dt), to_gpu(P64, dt))
        ref = oracle_mod.reconstruct(AJ64, P64)
        np.testing.assert_allclose(host(out), ref, rtol=0, atol=tol * np.abs(ref).max())
    # FP32 on the matrix cores (k <= 128): per entry within 2^-15 of
    # |AJ| |P| of the product of the FP32 values; ragged shapes around the
    # 64-row, 32-column and 16-k tiles, k = 128, a leading dimension > N
    for (N, k, n, ld) in [(1000, 13, 70, 1000), (4099, 128, 33, 4100), (64, 1, 1, 64),
                          (257, 17, 95, 300), (70001, 100, 500, 70004)]:
        AJ32 = rng.standard_normal((N, k)).astype(np.float32)
        P32 = rng.standard_normal((k, n)).astype(np.float32)
        AJd = to_gpu(AJ32.astype(np.float64), torch.float32, ld=ld)
        out = sid.reconstruct(AJd, to_gpu(P32.astype(np.float64), torch.float32))
        A64, P64b = AJ32.astype(np.float64), P32.astype(np.float64)
        ref = A64 @ P64b
        bound = 2.0 ** -15 * (np.abs(A64) @ np.abs(P64b)) + 1e-30
        err = np.abs(host(out).astype(np.float64) - ref)
        say("reconstruct mfma", N, k, n, "max err / bound", (err / bound).max())
        assert np.all(err <= bound), (N, k, n)



@pytest.mark.timeout(400)
def test_c2_full_size_sampled(sid, oracle_mod):
    """The benchmarked workload at full size (1,572,864 x 500 FP32 channel-like
    snapshots; single pass, bf16x2, k = 100, p = 20, e = 20, q = 10), in the
    launch configuration the benchmark times.  The oracle forms W over every
    row (its own Psi, row block by row block, with the |Psi||A| bound beside
    it) and Y on sampled rows; J is compared up to the oracle's first
    near-tie; P(:, J) = I exactly; the error of the returned decomposition is
    compared with the oracle's error routine on sampled rows."""
    k, p, q = 100, 20, 10
    l, lz = k + p, k + 2 * p
    lq = lz + q
    seed, prec = 0, "bf16x2"
    say("c2 full size: synthesizing")
    A = synth.spectral_snapshots(synth.SpectralConfig(), device="cuda")
    N, n = A.shape
    assert (N, n) == (1572864, 500)
    W, Y = sid.sketch(A, k, p, seed=seed, prec=prec, probe_rows=q, want_y=True)
    out = sid.compress(A, k, p, seed=seed, mode="single_pass", prec=prec, probe_rows=q)
    torch.cuda.synchronize()
    Wg, Yg = host(W), host(Y)
    Acpu = A.cpu()
    say("c2 full size: oracle W over all rows")
    Wo = np.zeros((lq, n))
    Wb = np.zeros((lq, n))
    blk = 1 << 16
    for r0 in range(0, N, blk):
        rows = np.arange(r0, min(N, r0 + blk))
        M = oracle_mod.data_values(Acpu[r0:r0 + rows.size].double().numpy(), prec)
        Ps = oracle_mod.psi(seed, rows, lq, prec)
        Wo += Ps @ M
        Wb += np.abs(Ps) @ np.abs(M)
        if (r0 // blk) % 6 == 5:
            say("c2 full size: oracle rows done", r0 + rows.size)
    assert Wg.shape == (lq, n)
    err = np.abs(Wg - Wo)
    say("c2 full size: W max err / bound", (err / Wb).max())
    assert np.all(err <= RTOL[prec] * Wb), (err / Wb).max()
    say("c2 full size: Y on sampled rows")
    rng = np.random.default_rng(12)
    rows = np.sort(rng.choice(N, size=4096, replace=False))
    A_rows = Acpu[rows].double().numpy()
    Om = oracle_mod.omega(seed, n, l, prec)
    Yo = oracle_mod.sketch_y(A_rows, Om, prec)
    ybound = np.abs(oracle_mod.data_values(A_rows, prec)) @ np.abs(Om)
    yerr = np.abs(Yg[rows].astype(np.float64) - Yo)
    assert np.all(yerr <= RTOL[prec] * ybound), (yerr / ybound).max()
    say("c2 full size: pivots against the oracle's mgsqr of its own W")
    cp = oracle_mod.cpqr(Wo[:l], k)
    assert cp.k_eff == k and int(host(out.k_eff)[0]) == k
    J = host(out.J)
    tie = np.nonzero(cp.margins <= 1e-4)[0]
    ist = int(tie[0]) if tie.size else k
    say("c2 full size: pivots compared up to", ist)
    assert ist >= 10
    assert J[:ist].tolist() == cp.J[:ist].tolist()
    assert len(set(J.tolist())) == k and J.min() >= 0 and J.max() < n
    P = host(out.P).astype(np.float64)
    assert np.array_equal(P[:, J], np.eye(k))
    say("c2 full size: error of the decomposition on sampled rows")
    AJ = out.AJ[torch.from_numpy(rows).cuda()]
    eg = sid.error_norms(A[torch.from_numpy(rows).cuda()], AJ, out.P)
    eo = oracle_mod.error_norms(A_rows, host(AJ).astype(np.float64), P)
    assert abs(eg["fro_err"] - eo["fro_err"]) <= 1e-9 * eo["fro_err"], (eg, eo)
    assert abs(eg["fro_a"] - eo["fro_a"]) <= 1e-12 * eo["fro_a"], (eg, eo)
    full = sid.error_norms(A, out.AJ, out.P)
    say("c2 full size: rel_fro sampled", eo["rel_fro"], "whole", full["rel_fro"])
    assert full["rel_fro"] < 1e-2 and eo["rel_fro"] < 1e-2


def test_fp8_general_path(sid, oracle_mod):
    """FP8 where the streaming pass does not apply (an unpadded leading
    dimension that is not a multiple of 4, FP64 data, a coarse row set, and
    l = 180 > 128 as in the streaming FP8 workload): the e4m3 data values
    are formed by a quantizing pass and the general kernels sketch them;
    W and Y within the per-entry bound of the oracle, and compress runs."""
    rng = np.random.default_rng(8)
    cases = []
    A64 = (rng.standard_normal((333, 20)) * np.exp(rng.uniform(-3, 3, 20))).astype(np.float32).astype(np.float64)
    cases.append(("lda333", A64, to_gpu(A64, torch.float32), None, 5, 5, 3))
    cases.append(("f64", A64, to_gpu(A64, torch.float64, ld=336), None, 5, 5, 3))
    S = np.arange(0, 333, 3).astype(np.int64)
    cases.append(("coarse", A64, to_gpu(A64, torch.float32, ld=336), S, 5, 5, 3))
    B64 = rng.standard_normal((4096, 300)).astype(np.float32).astype(np.float64)
    cases.append(("l180", B64, to_gpu(B64, torch.float32), None, 150, 30, 10))
    for name, X64, X, rows, k, p, q in cases:
        say("fp8 general", name)
        rs = sid.RowSet(rows, X64.shape[0]) if rows is not None else None
        W, Y = sid.sketch(X, k, p, seed=6, prec="fp8", probe_rows=q, coarse=rs, want_y=True)
        l = k + p
        lq = l + p + q
        Wo = oracle_mod.sketch_w(X64, rows, lq, 6, "fp8")
        rr = np.arange(X64.shape[0]) if rows is None else rows
        Psi = oracle_mod.psi(6, rr, lq, "fp8")
        bound = np.abs(Psi) @ np.abs(oracle_mod.data_values(X64, "fp8")[rr])
        assert np.all(np.abs(host(W) - Wo) <= RTOL["fp8"] * bound + 1e-30), name
        Om = oracle_mod.omega(6, X64.shape[1], l, "fp8")
        Yo = oracle_mod.sketch_y(X64, Om, "fp8")
        yb = np.abs(oracle_mod.data_values(X64, "fp8")) @ np.abs(Om)
        assert np.all(np.abs(host(Y).astype(np.float64) - Yo) <= RTOL["fp8"] * yb + 1e-30), name
        mode = "two_pass" if rows is not None else "single_pass"
        out = sid.compress(X, k, p, seed=6, prec="fp8", probe_rows=q, coarse=rs, mode=mode)
        torch.cuda.synchronize()
        ref = oracle_mod.compress(X64, k, p, seed=6, prec="fp8", probe_rows=q, coarse_rows=rows, mode=mode)
        ist = next((i for i, m in enumerate(ref.cp.margins) if m <= 1e-3), k)
        assert host(out.J)[:ist].tolist() == ref.J[:ist].tolist(), name

def _blocks(n, widths):
    c0, out, i = 0, [], 0
    while c0 < n:
        w = min(widths[i % len(widths)], n - c0)
        out.append((c0, w))
        c0 += w
        i += 1
    return out


@pytest.mark.parametrize("prec,dt", [("f64", torch.float64), ("f32", torch.float32),
                                     ("bf16x2", torch.float32), ("fp8", torch.float32)])
def test_stream_equals_whole_matrix(sid, oracle_mod, prec, dt):
    """Single-pass stream of ragged column blocks (one wider than the
    512-column stage, sketched in place) == sid_compress of the whole matrix:
    identical pivots, P and AJ to rounding of the Y sums, and the oracle's
    pivots until its first near-tie."""
    N, n, k, p, q = 4096, 700, 24, 8, 6
    say("stream", prec)
    A64, _ = c1_matrix(N=N, n=n, seed=1002)
    A64 = A64.astype(np.float32).astype(np.float64)
    A = to_gpu(A64, dt)
    st = sid.Stream(N, n, k, p, seed=4, dtype=dt, mode="single_pass", prec=prec, probe_rows=q)
    for c0, w in _blocks(n, [530, 7, 1, 100, 33]):
        st.push(A[:, c0:c0 + w])
    assert st.info()["cols"] == n
    got = st.finish()
    ref = sid.compress(A, k, p, seed=4, mode="single_pass", prec=prec, probe_rows=q)
    torch.cuda.synchronize()
    assert host(got.J).tolist() == host(ref.J).tolist()
    rt = 1e-9 if prec == "f64" else 2e-4
    np.testing.assert_allclose(host(got.P), host(ref.P), rtol=0, atol=rt * np.abs(host(ref.P)).max())
    np.testing.assert_allclose(host(got.AJ), host(ref.AJ), rtol=0,
                               atol=rt * np.abs(host(ref.AJ)).max())
    orc = oracle_mod.compress(A64, k, p, seed=4, mode="single_pass", prec=prec, probe_rows=q)
    tie = {"f64": 1e-10, "f32": 1e-5, "bf16x2": 1e-4, "fp8": 3e-2}[prec]
    ist = next((i for i, m in enumerate(orc.cp.margins) if m <= tie), k)
    assert host(got.J)[:ist].tolist() == orc.J[:ist].tolist()


def test_stream_general_kernels_chunk_cap(sid):
    """FP64 stream of a 300,000 x 700 matrix in ragged blocks: the general
    kernels cap their row chunks by the column count, and a stream's passes
    use the chunk count of the whole stream, so its W, J and P equal the
    resident call's bit for bit (two-pass, FP64 sketch)."""
    N, n, k, p, q = 300000, 700, 16, 8, 4
    say("stream chunk cap")
    g = torch.Generator(device="cuda").manual_seed(77)
    A = torch.randn((n, N), dtype=torch.float64, device="cuda", generator=g).T
    A = A * torch.exp(-torch.arange(n, device="cuda", dtype=torch.float64) / 60.0)
    A = synth.as_colmajor(A)
    st = sid.Stream(N, n, k, p, seed=6, dtype=torch.float64, mode="two_pass", prec="f64",
                    probe_rows=q)
    for c0, w in _blocks(n, [100, 37]):
        st.push(A[:, c0:c0 + w])
    got = st.finish(want_skeleton=False)
    ref = sid.compress(A, k, p, seed=6, mode="two_pass", prec="f64", probe_rows=q)
    torch.cuda.synchronize()
    assert host(got.J).tolist() == host(ref.J).tolist()
    assert np.array_equal(host(got.P), host(ref.P))
    assert np.array_equal(host(got.err), host(ref.err))


def test_stream_save_restore_and_two_pass(sid):
    """A stream checkpointed after part of the columns and restored into a
    new stream finishes like the uninterrupted one; a two-pass stream gives
    the two-pass J and P and refuses to return a skeleton; columns past n_max
    are rejected."""
    N, n, k, p = 3000, 260, 16, 8
    rng = np.random.default_rng(12)
    A64 = (rng.standard_normal((N, 30)) @ rng.standard_normal((30, n))) * np.exp(-np.arange(n) / 80)
    A = to_gpu(A64, torch.float32)
    kw = dict(seed=2, dtype=torch.float32, mode="single_pass", prec="bf16x2", probe_rows=5)
    s1 = sid.Stream(N, n, k, p, **kw)
    for c0, w in _blocks(n, [50, 13]):
        s1.push(A[:, c0:c0 + w])
    full = s1.finish()
    s2 = sid.Stream(N, n, k, p, **kw)
    for c0, w in _blocks(120, [50, 13]):
        s2.push(A[:, c0:c0 + w])
    state = s2.save()
    s2.close()
    s3 = sid.Stream.restore(state)
    assert s3.info()["cols"] == 120
    for c0, w in _blocks(n - 120, [50, 13]):
        s3.push(A[:, 120 + c0:120 + c0 + w])
    with pytest.raises(sid.SidError):
        s3.push(A[:, :1])
    res = s3.finish()
    torch.cuda.synchronize()
    assert host(res.J).tolist() == host(full.J).tolist()
    np.testing.assert_allclose(host(res.P), host(full.P), atol=1e-4 * np.abs(host(full.P)).max())
    np.testing.assert_allclose(host(res.AJ), host(full.AJ), atol=1e-4 * np.abs(host(full.AJ)).max())
    tp = sid.Stream(N, n, k, p, seed=2, dtype=torch.float32, mode="two_pass", prec="f32")
    for c0, w in _blocks(n, [64]):
        tp.push(A[:, c0:c0 + w])
    r2 = tp.finish(want_skeleton=False)
    ref = sid.compress(A, k, p, seed=2, mode="two_pass", prec="f32")
    assert host(r2.J).tolist() == host(ref.J).tolist()
    np.testing.assert_allclose(host(r2.P), host(ref.P), atol=1e-5 * np.abs(host(ref.P)).max())
    tp2 = sid.Stream(N, n, k, p, seed=2, dtype=torch.float32, mode="two_pass", prec="f32")
    tp2.push(A)
    AJ = torch.empty((k, N), dtype=torch.float32, device="cuda").T
    L = sid.load()
    st = L.sid_stream_finish(tp2._h, None, None, 1, ctypes.c_void_p(AJ.data_ptr()), N, None, None)
    tp2._h = None
    assert st == -1


@pytest.mark.parametrize("mode,prec", [("single_pass", "bf16x2"), ("two_pass", "f32"),
                                       ("single_pass", "fp8")])
def test_batched_equals_individual(sid, oracle_mod, mode, prec):
    """A batch of matrices of mixed shapes and ranks (spectrum j^-1.5, as in
    the batched workload) == one sid_compress per matrix, bit for bit in J
    and P (same kernels, own workspace per internal stream), and the
    oracle's pivots until its first near-tie.  The shapes cover both
    one-workgroup mgsqr kernels (run as batched launches) and, at l = 100,
    n = 400, the multi-workgroup one (run in the problem's own sequence)."""
    rng = np.random.default_rng(21)
    shapes = [(16384, 64, 8), (5120, 300, 40), (40000, 128, 20), (2048, 512, 64), (9000, 90, 12),
              (30000, 200, 33), (4096, 77, 9), (12000, 400, 90)]
    mats, A64s = [], []
    for (N, n, k) in shapes:
        sig = np.arange(1, n + 1) ** -1.5
        A64 = np.asarray(synth.lowrank_exact_spectrum(N, n, sig, seed=int(rng.integers(1 << 30)),
                                                      noise=0.0)).astype(np.float32).astype(np.float64)
        A64s.append(A64)
        mats.append(to_gpu(A64, torch.float32))
    ks = [s[2] for s in shapes]
    seeds = list(range(3, 3 + len(shapes)))
    say("batched", mode, prec)
    outs = sid.compress_batched(mats, ks, oversample=10, seed=seeds, mode=mode, prec=prec,
                                probe_rows=6)
    torch.cuda.synchronize()
    for b, A in enumerate(mats):
        ref = sid.compress(A, ks[b], 10, seed=seeds[b], mode=mode, prec=prec, probe_rows=6)
        torch.cuda.synchronize()
        assert np.array_equal(host(outs[b].J), host(ref.J)), b
        assert np.array_equal(host(outs[b].P), host(ref.P)), b
        assert np.array_equal(host(outs[b].AJ), host(ref.AJ)), b
        assert np.array_equal(host(outs[b].err), host(ref.err)), b
    b = 2
    orc = oracle_mod.compress(A64s[b], ks[b], 10, seed=seeds[b], mode=mode, prec=prec, probe_rows=6)
    tie = {"f32": 1e-5, "bf16x2": 1e-4, "fp8": 3e-2}[prec]
    ist = next((i for i, m in enumerate(orc.cp.margins) if m <= tie), ks[b])
    assert host(outs[b].J)[:ist].tolist() == orc.J[:ist].tolist()


def test_refinement_pass(sid, oracle_mod):
    """Refinement of P on a second sketch (both modes): the same precision is
    a no-op; an FP8 first sketch refined on a bf16x2 sketch matches the
    oracle's refinement (least squares on that sketch with J fixed) and, two
    pass, does not increase the error of the ID."""
    A64, _ = c1_matrix(N=4096, n=256, seed=1003)
    A64 = A64.astype(np.float32).astype(np.float64)
    A = to_gpu(A64, torch.float32)
    k, p, q = 20, 10, 10
    for mode in ("two_pass", "single_pass"):
        say("refine", mode)
        base = sid.compress(A, k, p, seed=6, mode=mode, prec="bf16x2", probe_rows=q)
        same = sid.compress(A, k, p, seed=6, mode=mode, prec="bf16x2", probe_rows=q, refine=True,
                            refine_prec="bf16x2")
        torch.cuda.synchronize()
        assert np.array_equal(host(same.J), host(base.J))
        np.testing.assert_allclose(host(same.P), host(base.P), atol=1e-6 * np.abs(host(base.P)).max())
        r0 = sid.compress(A, k, p, seed=6, mode=mode, prec="fp8", probe_rows=q)
        r1 = sid.compress(A, k, p, seed=6, mode=mode, prec="fp8", probe_rows=q, refine=True,
                          refine_prec="bf16x2")
        torch.cuda.synchronize()
        orc = oracle_mod.compress(A64, k, p, seed=6, mode=mode, prec="fp8", probe_rows=q)
        assert orc.cp.margins.min() > 1e-4   # same e4m3 values on both sides; sums differ ~1e-6
        assert host(r1.J).tolist() == orc.J.tolist()
        P1o = oracle_mod.refine(A64, orc, seed=6, refine_prec="bf16x2", l=k + p)
        P1 = host(r1.P).astype(np.float64)
        np.testing.assert_allclose(P1, P1o, atol=2e-4 * np.abs(P1o).max())
        assert np.array_equal(P1[:, orc.J], np.eye(k))
        e0 = sid.error_norms(A, r0.AJ, r0.P)["rel_fro"]
        e1 = sid.error_norms(A, r1.AJ, r1.P)["rel_fro"]
        say("refine", mode, "fp8 error", e0, "refined", e1)
        # single pass keeps the skeleton estimated from the FP8 Y, which a
        # refit of P does not repair: reported only
        if mode == "two_pass":
            assert e1 <= e0 * 1.001


@pytest.mark.parametrize("Ns_step,dt,prec", [(3, torch.float64, "f64"), (25, torch.float64, "f64"),
                                             (3, torch.float32, "f32")])
def test_literal_subsampled_id(sid, oracle_mod, Ns_step, dt, prec):
    """Alg. 5 as written (mgsqr on the coarse rows A(S, :)): pivots equal the
    oracle's, P to FP64 roundoff, AJ the exact columns, err[0] NaN."""
    N, n, k = 5000, 60, 12
    rng = np.random.default_rng(51)
    A64 = (rng.standard_normal((N, n)) * np.exp(-np.linspace(0, 5, n))[None, rng.permutation(n)])
    A64 = A64.astype(np.float32).astype(np.float64)
    A = to_gpu(A64, dt)
    S = np.arange(0, N, Ns_step).astype(np.int64)
    say("literal", Ns_step, prec, S.size)
    rs = sid.RowSet(S, N)
    out = sid.compress(A, k, 0, coarse=rs, mode="two_pass", prec=prec, select="literal")
    torch.cuda.synchronize()
    ref = oracle_mod.compress_literal(A64, k, S, prec=prec)
    assert ref.cp.margins.min() > 1e-8
    assert host(out.J).tolist() == ref.J.tolist()
    np.testing.assert_allclose(host(out.P), ref.P, atol=1e-9 * np.abs(ref.P).max())
    assert np.array_equal(host(out.AJ).astype(np.float64), A64[:, ref.J])
    e = host(out.err)
    assert np.isnan(e[0])
    assert abs(e[1] - ref.err_sketch) <= 1e-8 * max(ref.err_sketch, 1e-300)


@pytest.mark.parametrize("prec", ["bf16", "bf16x2", "fp8", "f32"])
def test_streaming_pass_edge_shapes(sid, oracle_mod, prec):
    """The matrix-core pass on degenerate shapes: fewer rows than one panel,
    one column, k = n, no probe rows, all-zero columns (FP8 tiles with scale
    1), exact-rank data; W and Y within the per-entry bound and compress
    equal to the oracle up to its first near-tie."""
    rng = np.random.default_rng(61)
    for (N, n, k, p, q) in [(8, 5, 2, 1, 1), (64, 1, 1, 0, 0), (200, 12, 12, 0, 3), (1000, 40, 5, 5, 0),
                            (65, 129, 9, 4, 2)]:
        say("edge streaming", prec, N, n, k, p, q)
        A64 = rng.standard_normal((N, n)).astype(np.float32).astype(np.float64)
        if n > 3:
            A64[:, 2] = 0.0
        A = to_gpu(A64, torch.float32, ld=ld4(N))
        l = k + p
        lq = l + p + q
        W, Y = sid.sketch(A, k, p, seed=3, prec=prec, probe_rows=q, want_y=True)
        Wo = oracle_mod.sketch_w(A64, None, lq, 3, prec)
        bound = _absbound(A64, np.arange(N), lq, 3, prec, oracle_mod)
        assert np.all(np.abs(host(W) - Wo) <= RTOL[prec] * bound + 1e-30)
        Om = oracle_mod.omega(3, n, l, prec)
        Yo = oracle_mod.sketch_y(A64, Om, prec)
        ybound = np.abs(oracle_mod.data_values(A64, prec)) @ np.abs(Om)
        assert np.all(np.abs(host(Y).astype(np.float64) - Yo) <= RTOL[prec] * ybound + 1e-30)
        for mode in ("two_pass", "single_pass"):
            out = sid.compress(A, k, p, seed=3, mode=mode, prec=prec, probe_rows=q)
            torch.cuda.synchronize()
            ref = oracle_mod.compress(A64, k, p, seed=3, mode=mode, prec=prec, probe_rows=q)
            ke = int(host(out.k_eff)[0])
            assert ke == ref.k_eff
            tie = next((i for i, m in enumerate(ref.cp.margins) if m <= 1e-3), ref.k_eff)
            assert host(out.J)[:tie].tolist() == ref.J[:tie].tolist()
            J = host(out.J)[:ke]
            assert np.array_equal(host(out.P)[:ke][:, J], np.eye(ke))


@pytest.mark.parametrize("prec", ["bf16x2", "fp8"])
def test_pair_pass_y_over_column_slabs(sid, oracle_mod, prec):
    """The workgroup-pair pass (l = 180 > 128) over a matrix wider than its
    column slab: every slab after the first adds its part of Y in the kernel.
    W and Y against the oracle (per-entry bound); a single-pass stream of
    ragged blocks (each flush after the first adds in the kernel as well)
    against the resident call: the same W bit for bit (J, P identical) and
    AJ to rounding of the Y sums."""
    N, n, k, p, q = 3000, 900, 150, 30, 6
    l, lq = k + p, k + 2 * p + q
    A64, _ = c1_matrix(N=N, n=n, seed=1006)
    A64 = A64.astype(np.float32).astype(np.float64)
    A = to_gpu(A64, torch.float32)
    say("pair-pass Y slabs", prec)
    W, Y = sid.sketch(A, k, p, seed=5, prec=prec, probe_rows=q, want_y=True)
    Wo = oracle_mod.sketch_w(A64, None, lq, 5, prec)
    bound = _absbound(A64, np.arange(N), lq, 5, prec, oracle_mod)
    assert np.all(np.abs(host(W) - Wo) <= RTOL[prec] * bound + 1e-30)
    Om = oracle_mod.omega(5, n, l, prec)
    Yo = oracle_mod.sketch_y(A64, Om, prec)
    ybound = np.abs(oracle_mod.data_values(A64, prec)) @ np.abs(Om)
    assert np.all(np.abs(host(Y).astype(np.float64) - Yo) <= RTOL[prec] * ybound + 1e-30)
    st = sid.Stream(N, n, k, p, seed=5, dtype=torch.float32, mode="single_pass", prec=prec,
                    probe_rows=q)
    for c0, w in _blocks(n, [300, 7, 450, 64]):
        st.push(A[:, c0:c0 + w])
    got = st.finish()
    ref = sid.compress(A, k, p, seed=5, mode="single_pass", prec=prec, probe_rows=q)
    torch.cuda.synchronize()
    assert host(got.J).tolist() == host(ref.J).tolist()
    assert np.array_equal(host(got.P), host(ref.P))
    np.testing.assert_allclose(host(got.AJ), host(ref.AJ), rtol=0,
                               atol=2e-4 * np.abs(host(ref.AJ)).max())
    # AJ = Y T at l = 180, k = 150 on the bf16 matrix cores (hi + lo splits of
    # Y and T, three products): T = M^+ W(0:lz, J) with M = W(0:lz, :) Omega
    # formed from the GPU's W (no truncation on either side), each entry of AJ
    # within 2^-15 of sum_t |Y(i, t)| |T(t, j)|
    tight = sid.compress(A, k, p, seed=5, mode="single_pass", prec=prec, probe_rows=q,
                         sp_rcond=1e-12)
    torch.cuda.synchronize()
    J = host(tight.J)
    Wg = host(W).astype(np.float64)
    Yg = host(Y).astype(np.float64)
    lz = l + p
    M = Wg[:lz] @ Om
    T = np.linalg.pinv(M, rcond=1e-12) @ Wg[:lz][:, J]
    AJo = Yg @ T
    bound = 2.0 ** -15 * (np.abs(Yg) @ np.abs(T)) + 1e-30
    dAJ = np.abs(host(tight.AJ).astype(np.float64) - AJo)
    say("pair-pass AJ max |dAJ| / bound", (dAJ / bound).max())
    assert np.all(dAJ <= bound)


@pytest.mark.parametrize("k,p", [(37, 10), (61, 6)])
def test_apply_rows_not_16_byte_aligned(sid, oracle_mod, k, p):
    """AJ = Y T on the bf16 matrix cores when l % 4 != 0 (Y's rows are not
    16-byte aligned, so each lane reads its entries one by one): each entry
    of AJ within 2^-15 of sum_t |Y(i, t)| |T(t, j)|, with T = M^+ W(0:lz, J)
    formed from the GPU's W and Omega (ragged last row block)."""
    N, n, q = 5000, 300, 6
    l, lz = k + p, k + 2 * p
    assert l % 4 != 0
    A64, _ = c1_matrix(N=N, n=n, seed=1007)
    A = to_gpu(A64.astype(np.float32).astype(np.float64), torch.float32)
    say("unaligned apply", k, p)
    W, Y = sid.sketch(A, k, p, seed=9, prec="bf16x2", probe_rows=q, want_y=True)
    out = sid.compress(A, k, p, seed=9, mode="single_pass", prec="bf16x2", probe_rows=q,
                       sp_rcond=1e-12)
    torch.cuda.synchronize()
    J = host(out.J)
    Wg = host(W).astype(np.float64)
    Yg = host(Y).astype(np.float64)
    Om = oracle_mod.omega(9, n, l, "bf16x2")
    M = Wg[:lz] @ Om
    T = np.linalg.pinv(M, rcond=1e-12) @ Wg[:lz][:, J]
    AJo = Yg @ T
    bound = 2.0 ** -15 * (np.abs(Yg) @ np.abs(T)) + 1e-30
    dAJ = np.abs(host(out.AJ).astype(np.float64) - AJo)
    say("unaligned AJ max |dAJ| / bound", (dAJ / bound).max())
    assert np.all(dAJ <= bound)


def test_cooperative_launch_matches_plain(sid, oracle_mod):
    """The multi-workgroup pivoted QR (W_sel of 120 x 500 takes it) as the
    default plain launch and as the opt-in cooperative one (SID_COOPERATIVE=1
    when the context is created): the same pivots, P, AJ and estimates bit
    for bit, and both contexts report no failed device-side wait."""
    import os
    A64, _ = c1_matrix(N=6000, n=500, seed=1008)
    A = to_gpu(A64.astype(np.float32).astype(np.float64), torch.float32)
    say("cooperative vs plain QR launch")
    kw = dict(seed=4, mode="single_pass", prec="bf16x2", probe_rows=10)
    plain = sid.compress(A, 100, 20, **kw)
    old = os.environ.get("SID_COOPERATIVE")
    os.environ["SID_COOPERATIVE"] = "1"
    try:
        ctx = sid.Context()
    finally:
        if old is None:
            del os.environ["SID_COOPERATIVE"]
        else:
            os.environ["SID_COOPERATIVE"] = old
    coop = sid.compress(A, 100, 20, ctx=ctx, **kw)
    ctx.sync()
    sid.sync()
    torch.cuda.synchronize()
    for a, b in ((plain.J, coop.J), (plain.P, coop.P), (plain.AJ, coop.AJ), (plain.err, coop.err),
                 (plain.k_eff, coop.k_eff)):
        assert torch.equal(a, b)
    assert int(plain.k_eff[0]) == 100
    ctx.close()


@pytest.mark.parametrize("prec", ["f64", "bf16x2"])
def test_ties_across_qr_workgroups(sid, oracle_mod, prec):
    """Exact ties decided across the workgroups of the multi-workgroup QR
    (W_sel of 100 x 500: 128 columns per workgroup): duplicated columns in
    different workgroups give equal candidates, and both sides take the
    smallest index (Sec. 2.4 mgsqr).  Ties at steps 0, 4 and 6 (140 / 420,
    10 / 300, 3 / 260); every other step's margin is above 4e-5, so the
    GPU's pivots on its own W must equal the oracle's mgsqr of that W."""
    rng = np.random.default_rng(45)
    N, n, k, p = 3000, 500, 80, 20
    A64 = rng.standard_normal((N, n)) * (0.985 ** np.arange(n))
    pairs = [(10, 300), (140, 420), (3, 260), (200, 499)]
    for a, b in pairs:
        A64[:, b] = A64[:, a]
    A64[:, 140] *= 20.0
    A64[:, 420] = A64[:, 140]
    dt = torch.float64 if prec == "f64" else torch.float32
    if dt == torch.float32:
        A64 = A64.astype(np.float32).astype(np.float64)
    A = to_gpu(A64, dt)
    say("ties across QR workgroups", prec)
    for mode in ("two_pass", "single_pass"):
        out = sid.compress(A, k, p, seed=5, mode=mode, prec=prec, probe_rows=4)
        Wg, _ = sid.sketch(A, k, p, seed=5, prec=prec, probe_rows=4, want_y=(mode == "single_pass"))
        torch.cuda.synchronize()
        Wg = host(Wg)
        for a, b in pairs:
            assert np.array_equal(Wg[:, a], Wg[:, b]), (prec, a, b)
        cp = oracle_mod.cpqr(Wg[:k + p], k)
        J = host(out.J)
        assert J[0] == 140, (prec, mode, J[:3])
        assert J.tolist() == cp.J.tolist(), (prec, mode)
        m = np.asarray(cp.margins)
        assert np.count_nonzero(m == 0) >= 3 and m[m > 0].min() > 1e-5


@pytest.mark.parametrize("prec", ["bf16x2", "fp8"])
def test_pair_pass_psi_images_bitwise(sid, oracle_mod, prec):
    """Over more than one column slab the workgroup-pair pass reads Psi from
    images formed once (instead of generating it in every slab's launch):
    W of the first slab's columns equals, bit for bit, the sketch of those
    columns alone (one launch, Psi generated in the kernel); a ragged last
    row panel is covered (N = 3000).  (W and Y of the wide call against the
    oracle: test_pair_pass_y_over_column_slabs.)"""
    N, n, k, p, q = 3000, 900, 150, 30, 6
    A64, _ = c1_matrix(N=N, n=n, seed=1009)
    A = to_gpu(A64.astype(np.float32).astype(np.float64), torch.float32)
    say("pair pass Psi images", prec)
    W_all, _ = sid.sketch(A, k, p, seed=7, prec=prec, probe_rows=q, want_y=True)
    W_one, _ = sid.sketch(A[:, :384].contiguous(), k, p, seed=7, prec=prec, probe_rows=q,
                          want_y=True)
    torch.cuda.synchronize()
    assert torch.equal(W_all[:, :384], W_one)


def test_graph_capture_replay(sid, oracle_mod):
    """sid_reserve covers every allocation of a compress call; the call is
    then captured into a HIP graph and replayed several times, with eager
    work and host synchronization between replays, and reproduces the eager
    results bit for bit."""
    A64, _ = c1_matrix(N=4096, n=256, seed=1004)
    A = to_gpu(A64.astype(np.float32).astype(np.float64), torch.float32)
    q = 10
    stream = torch.cuda.Stream()
    cases = [
        ("single_pass", "bf16x2", 20, 10, {}),
        ("two_pass", "f32", 20, 10, {}),
        # l = 180: the FP8 streaming workload's shape
        ("single_pass", "fp8", 150, 30, {}),
        # refinement in another precision than the first sketch
        ("two_pass", "fp8", 20, 10, dict(refine=True, refine_prec="bf16x2")),
        ("single_pass", "bf16", 20, 10, dict(refine=True, refine_prec="f32")),
        ("two_pass", "f64", 20, 10, dict(refine=True, refine_prec="bf16x2")),
    ]
    for mode, prec, k, p, kw in cases:
        say("graph", mode, prec, k, p, kw)
        with torch.cuda.stream(stream):
            ctx = sid.Context(stream=stream)
            sid.reserve(A.shape[0], A.shape[1], k, p, mode=mode, prec=prec, probe_rows=q, ctx=ctx,
                        **kw)
            held = ctx.workspace_bytes()
            out = sid.compress(A, k, p, seed=2, mode=mode, prec=prec, probe_rows=q, ctx=ctx, **kw)
            assert ctx.workspace_bytes() == held       # the reservation covered the call
            eager = sid.compress(A, k, p, seed=2, mode=mode, prec=prec, probe_rows=q, ctx=ctx,
                                 **kw)
        ctx.sync()
        torch.cuda.synchronize()
        ref = [host(t).copy() for t in (eager.J, eager.P, eager.AJ, eager.err)]
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g, stream=stream):
            sid.compress(A, k, p, seed=2, mode=mode, prec=prec, probe_rows=q, ctx=ctx, out=out,
                         **kw)
        assert ctx.workspace_bytes() == held
        for rep in range(3):
            for t in (out.J, out.P, out.AJ, out.err):
                t.zero_()
            torch.cuda.synchronize()
            g.replay()
            torch.cuda.synchronize()
            ctx.sync()
            got = [host(t) for t in (out.J, out.P, out.AJ, out.err)]
            for a, b in zip(got, ref):
                assert np.array_equal(a, b, equal_nan=True), (mode, prec, rep)
            _ = (A * 2.0).sum().item()  # unrelated eager work between replays
        ctx.close()


@pytest.mark.parametrize("prec", ["bf16", "bf16x2"])
@pytest.mark.parametrize("shape", [(50000, 300, 20, 10, 5, 2), (9001, 700, 30, 10, 4, 3), (4000, 64, 8, 4, 2, 0)])
def test_coarse_rows_streaming_pass(sid, oracle_mod, prec, shape):
    """The sub-sampled sketch W = Psi(:, S) A(S, :) on the matrix-core pass
    (row list staged per panel, Psi keyed by the global row): every-other
    rows, every-third rows, and random rows (step 0), including n = 700 in
    column slabs and workgroups with ragged tails; then the two-pass
    compression on it against the oracle."""
    N, n, k, p, q, step = shape
    say("coarse streaming", prec, shape)
    rng = np.random.default_rng(N + n)
    A64 = (rng.standard_normal((N, 40)) @ rng.standard_normal((40, n))
           + 0.01 * rng.standard_normal((N, n))).astype(np.float32).astype(np.float64)
    A = to_gpu(A64, torch.float32)
    S = (np.arange(1, N, step) if step else np.sort(rng.choice(N, size=N // 5, replace=False))).astype(np.int64)
    rs = sid.RowSet(S, N)
    lq = k + p + q
    W, _ = sid.sketch(A, k, p, seed=13, coarse=rs, prec=prec, probe_rows=q, want_y=False)
    Wo = oracle_mod.sketch_w(A64, S, lq, 13, prec)
    bound = np.abs(oracle_mod.psi(13, S, lq, prec)) @ np.abs(oracle_mod.data_values(A64[S], prec))
    err = np.abs(host(W) - Wo)
    assert np.all(err <= RTOL[prec] * bound + 1e-30), (err / bound).max()
    out = sid.compress(A, k, p, seed=13, coarse=rs, mode="two_pass", prec=prec, probe_rows=q)
    torch.cuda.synchronize()
    ref = oracle_mod.compress(A64, k, p, seed=13, coarse_rows=S, mode="two_pass", prec=prec, probe_rows=q)
    ist = next((i for i, m in enumerate(ref.cp.margins) if m <= 1e-3), k)
    assert host(out.J)[:ist].tolist() == ref.J[:ist].tolist()
    assert np.array_equal(host(out.AJ).astype(np.float64)[:, :ist], A64[:, ref.J[:ist]])


@pytest.mark.parametrize("N,k", [(3001, 16), (4097, 40), (2113, 70), (3001, 90), (4093, 100),
                                 (2113, 128)])
def test_single_pass_skeleton_store_paths(sid, N, k):
    """AJ = Y T of the bf16 sketch precisions: FP32 data takes the kernel that
    stores 256-byte column runs, FP64 data holding the same values takes the
    one that stores straight from the matrix tiles; their FP32 sums are
    formed in the same order, so the two AJ agree bit for bit (k from 16 to
    128 covers every column-tile count; N leaves a ragged last row block).
    N is odd so that both inputs reach the sketch through the same FP32
    staging copy and the two Y are identical."""
    say("skeleton store paths", N, k)
    rng = np.random.default_rng(N + k)
    n = 160
    A64 = (rng.standard_normal((N, n)) @ np.diag(0.97 ** np.arange(n))).astype(np.float32)
    A64 = A64.astype(np.float64)
    o32 = sid.compress(to_gpu(A64, torch.float32), k, 0, seed=5, mode="single_pass",
                       prec="bf16x2", probe_rows=0)
    o64 = sid.compress(to_gpu(A64, torch.float64), k, 0, seed=5, mode="single_pass",
                       prec="bf16x2", probe_rows=0)
    torch.cuda.synchronize()
    assert torch.equal(o32.J, o64.J)
    assert torch.equal(o32.AJ.double(), o64.AJ)


@pytest.mark.parametrize("N,n,k,p,q,dt", [(5000, 77, 20, 10, 10, torch.float32),
                                          (20011, 300, 100, 20, 10, torch.float32),
                                          (3001, 200, 40, 20, 0, torch.float64),
                                          (70000, 130, 100, 20, 10, torch.float64),
                                          (4099, 90, 30, 10, 5, torch.float32),
                                          (9001, 260, 150, 20, 10, torch.float32)])
def test_f64_sketch_tiled_equals_general(sid, oracle_mod, N, n, k, p, q, dt):
    """The F64 sketches over all rows run on the register-tiled kernels; a
    row set holding every row sends the same sketch through the general
    kernels.  Both sum each entry in the same order with the same FMAs (W:
    row chunks, then the chunks in order), so W and Y agree bit for bit
    (row tiles of 64, 128 and 160 rows and two-tile cases, several column
    tiles, l above 64 and above 128, ragged edges);
    the tiled W is also within the F64 bound of the oracle's."""
    say("f64 tiled sketch", N, n, k, p, q, dt)
    rng = np.random.default_rng(N)
    A64 = rng.standard_normal((N, n))
    if dt == torch.float32:
        A64 = A64.astype(np.float32).astype(np.float64)
    A = to_gpu(A64, dt)
    every = sid.RowSet(np.arange(N, dtype=np.int64), N)
    for want_y in (False, True):
        Wt, Yt = sid.sketch(A, k, p, seed=4, prec="f64", probe_rows=q, want_y=want_y)
        Wg, Yg = sid.sketch(A, k, p, seed=4, prec="f64", probe_rows=q, want_y=want_y,
                            coarse=every)
        torch.cuda.synchronize()
        assert torch.equal(Wt, Wg)
        if want_y:
            assert torch.equal(Yt, Yg)
    Wt, _ = sid.sketch(A, k, p, seed=4, prec="f64", probe_rows=q, want_y=False)
    lq = Wt.shape[0]
    Wo = oracle_mod.sketch_w(A64, None, lq, 4, "f64")
    bound = _absbound(A64, np.arange(N), lq, 4, "f64", oracle_mod)
    assert np.all(np.abs(host(Wt) - Wo) <= RTOL["f64"] * bound + 1e-30)


@pytest.mark.parametrize("prec", ["f64", "bf16x2", "f32"])
def test_exact_pivot_ties_smallest_index(sid, oracle_mod, prec):
    """Duplicated snapshot columns give exactly equal sketch columns, hence
    exactly tied residual norms in mgsqr; both sides take the smallest column
    index (Sec. 2.4 mgsqr with ties broken towards the first column).  The
    tied pairs are placed so that the larger of each pair comes first in
    norm order, and the pivots must equal the oracle's, which picks the
    first maximum."""
    say("ties", prec)
    rng = np.random.default_rng(44)
    N, n, k, p = 3000, 48, 12, 8
    base = rng.standard_normal((N, 16)) * np.exp(-np.arange(16) / 4.0)
    A64 = base @ rng.standard_normal((16, n))
    # exact duplicates: columns 5 <- 30, 9 <- 40, 17 <- 17 + 20, 2 <- 46
    for dst, src in [(30, 5), (40, 9), (37, 17), (46, 2)]:
        A64[:, dst] = A64[:, src]
    # make a duplicated column the largest, so the very first pivot is a tie
    A64[:, 9] *= 40.0
    A64[:, 40] = A64[:, 9]
    dt = torch.float64 if prec == "f64" else torch.float32
    A64 = A64.astype(np.float32).astype(np.float64) if dt == torch.float32 else A64
    A = to_gpu(A64, dt)
    for mode in ("two_pass", "single_pass"):
        out = sid.compress(A, k, p, seed=5, mode=mode, prec=prec, probe_rows=4)
        torch.cuda.synchronize()
        Wg, _ = sid.sketch(A, k, p, seed=5, prec=prec, probe_rows=4, want_y=(mode == "single_pass"))
        Wg = host(Wg)
        for a, b in [(5, 30), (9, 40), (17, 37), (2, 46)]:
            assert np.array_equal(Wg[:, a], Wg[:, b]), (prec, a, b)
        cp = oracle_mod.cpqr(Wg[:k + p], k)
        J = host(out.J)
        assert J[0] == 9, (prec, mode, J[:3])
        assert J.tolist() == cp.J.tolist(), (prec, mode, J, cp.J)
        if prec == "f64":
            ref = oracle_mod.compress(A64, k, p, seed=5, mode=mode, prec=prec, probe_rows=4)
            assert J.tolist() == ref.J.tolist()
