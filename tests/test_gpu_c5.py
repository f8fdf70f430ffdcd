"""The streaming FP8 workload: 1,572,864 x 2000 FP32 channel-like snapshots
arriving in blocks of 32 columns (62 blocks of 32 and one of 16), single pass,
FP8 e4m3 sketch, k = 150, p = 30 (l = 180, e = 30, q = 10: 220 sketch rows),
the shape the workgroup-pair matrix-core pass takes (l > 128).

* the stream gives the pivots and coefficients of the resident call;
* W on sampled columns over every row and Y on sampled rows against the
  oracle entry by entry (per-entry bound |Psi| |A| in FP8 values);
* mgsqr and the coefficients of the oracle on the GPU's W: the same pivots;
* errors of FP8, FP8 + one refinement pass (FP32 sketch), bf16x2 and FP32,
  single and two pass, side by side; two pass, FP8 + refinement is within
  5 % of FP32.

Marked gpu."""
import sys

import numpy as np
import pytest
import torch

import synth

pytestmark = pytest.mark.gpu

K, P_OV, Q_PR = 150, 30, 10
L, LZ = K + P_OV, K + 2 * P_OV
LQ = LZ + Q_PR
RTOL = 5e-5     # FP32 accumulation of the sketch: per entry, relative to sum |Psi| |A|


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


def host(t):
    return t.detach().cpu().numpy()


@pytest.mark.timeout(900)
def test_c5_fp8_stream(sid, oracle_mod):
    seed, prec = 0, "fp8"
    say("c5: synthesizing")
    A = synth.spectral_snapshots(synth.streaming_config(), device="cuda")
    torch.cuda.synchronize()
    N, n = A.shape
    assert (N, n) == (1572864, 2000)
    kw = dict(seed=seed, mode="single_pass", prec=prec, probe_rows=Q_PR)
    st = sid.Stream(N, n, K, P_OV, dtype=torch.float32, **kw)
    for c0 in range(0, n, 32):
        st.push(A[:, c0:c0 + 32])
    got = st.finish()
    ref = sid.compress(A, K, P_OV, **kw)
    torch.cuda.synchronize()
    assert got.rank() == K and ref.rank() == K
    J = host(got.J)
    assert J.tolist() == host(ref.J).tolist()
    assert np.array_equal(host(got.P), host(ref.P))

    say("c5: W on sampled columns against the oracle")
    W, Y = sid.sketch(A, K, P_OV, seed=seed, prec=prec, probe_rows=Q_PR, want_y=True)
    torch.cuda.synchronize()
    Wg = host(W)
    assert Wg.shape == (LQ, n)
    rng = np.random.default_rng(55)
    cols = np.unique(np.concatenate([rng.choice(n, size=20, replace=False),
                                     [0, 31, 32, 1983, 1984, 1999]]))
    Acols = A[:, torch.from_numpy(cols).cuda()].double().cpu().numpy()
    Wo = oracle_mod.sketch_w(Acols, None, LQ, seed, prec)
    Wb = np.zeros_like(Wo)
    blk = 1 << 17
    for r0 in range(0, N, blk):
        rows = np.arange(r0, min(N, r0 + blk))
        Wb += np.abs(oracle_mod.psi(seed, rows, LQ, prec)) @ np.abs(
            oracle_mod.data_values(Acols[r0:r0 + rows.size], prec))
    werr = np.abs(Wg[:, cols] - Wo)
    say("c5: W max err / bound", (werr / Wb).max())
    assert np.all(werr <= RTOL * Wb)

    say("c5: Y on sampled rows against the oracle")
    rows = np.sort(rng.choice(N, size=2048, replace=False))
    # the FP8 values of a row depend on its 64-row tile: take each sampled
    # row's tile from the device copy
    tiles = np.unique(rows // 64)
    trows = (tiles[:, None] * 64 + np.arange(64)[None, :]).ravel()
    At = A[torch.from_numpy(trows).cuda()].double().cpu().numpy()
    Vt = oracle_mod.data_values(At, prec)
    pos = {t: i for i, t in enumerate(tiles.tolist())}
    V = np.stack([Vt[pos[r // 64] * 64 + r % 64] for r in rows])
    Om = oracle_mod.omega(seed, n, L, prec)
    Yo = V @ Om
    ybound = np.abs(V) @ np.abs(Om)
    yerr = np.abs(host(Y)[rows].astype(np.float64) - Yo)
    live = ybound > 0            # rows at the walls are zero in two components
    say("c5: Y max err / bound", (yerr[live] / ybound[live]).max())
    assert np.all(yerr <= RTOL * ybound)
    del At, Vt, V

    say("c5: the oracle's mgsqr on the GPU's W")
    cp = oracle_mod.cpqr(Wg[:L], K)
    tie = np.nonzero(cp.margins <= 1e-10)[0]
    ist = int(tie[0]) if tie.size else K
    say("c5: smallest pivot margin", cp.margins.min(), "compared up to", ist)
    assert J[:ist].tolist() == cp.J[:ist].tolist()
    Po = oracle_mod.id_coefficients(cp.R, cp.J, n)
    Pg = host(got.P).astype(np.float64)
    if ist == K:
        bound = 2.0 ** -24 * np.abs(Po) * (1 + 1e-6) + 1e-11 * np.abs(Po).max()
        assert np.all(np.abs(Pg - Po) <= bound)

    say("c5: errors")
    errs = precision_errors(sid, A, K, P_OV, Q_PR, seed, "c5")
    for mode in ("single_pass", "two_pass"):
        assert errs[mode, "f32"] <= errs[mode, "fp8"]
    # two pass: the skeleton is A(:, J) itself and the refinement recomputes
    # P on an FP32 sketch, so FP8 + refinement reaches the FP32 error (the
    # pivots differ; measured 0.78 x FP32 here).  Single pass: the skeleton
    # comes from the FP8 Y, which the refinement of P cannot repair
    # (reported only)
    assert errs["two_pass", "fp8+refine"] <= errs["two_pass", "fp8"]
    assert errs["two_pass", "fp8+refine"] <= 1.05 * errs["two_pass", "f32"]


def precision_errors(sid, A, k, p, q, seed, tag):
    """Relative Frobenius errors of FP8, FP8 + one FP32 refinement pass, bf16x2
    and FP32 sketches, single and two pass, on the same matrix."""
    errs = {}
    for mode in ("single_pass", "two_pass"):
        for name, kwx in [("fp8", dict(prec="fp8")),
                          ("fp8+refine", dict(prec="fp8", refine=True, refine_prec="f32")),
                          ("bf16x2", dict(prec="bf16x2")), ("f32", dict(prec="f32"))]:
            o = sid.compress(A, k, p, seed=seed, mode=mode, probe_rows=q, **kwx)
            torch.cuda.synchronize()
            errs[mode, name] = sid.error_norms(A, o.AJ, o.P)["rel_fro"]
            say(tag + ":", mode, name, "rel_fro", errs[mode, name], "probe estimate",
                float(o.err[0]), "ratio to f32", errs[mode, name] / errs.get((mode, "f32"), np.nan))
        for name in ("fp8", "fp8+refine", "bf16x2"):
            say(tag + ":", mode, name, "/ f32 =", errs[mode, name] / errs[mode, "f32"])
    return errs
