"""Pins of the single-pass ID oracle (Alg. 6) against what the mathematics
fixes: the interpolation property and partition of unity of piecewise linear
nodal bases, exact reproduction of (tri)linear functions, the textbook
interpolation error bound H^2/8 max|f''| with its H^2 rate (Sec. 2.6, the
discussion after Theorem 2.2), the full-rank limit where the single-pass ID
error equals the interpolation error, and the inequalities of Theorem 2.2."""
import math

import numpy as np
import pytest
import torch

import synth
from oracle import spid


def _grid(rng, n, lo=0.0, hi=1.0):
    x = np.sort(rng.uniform(lo, hi, size=n))
    x[0], x[-1] = lo, hi
    return x


def _subset(rng, n, m):
    return np.sort(rng.choice(n, size=m, replace=False)).astype(np.int64)


@pytest.mark.parametrize("period", [0.0, 1.5])
def test_hat_nodal_and_partition_of_unity(period):
    rng = np.random.default_rng(3)
    for trial in range(20):
        n = int(rng.integers(2, 40))
        m = int(rng.integers(1, n + 1))
        x = _grid(rng, n, 0.0, 1.0 if period == 0.0 else 1.4)
        c = _subset(rng, n, m)
        H = spid.hat_matrix(x, c, period)
        assert H.shape == (n, m)
        np.testing.assert_allclose(H[c], np.eye(m), atol=1e-14)
        np.testing.assert_allclose(H.sum(1), 1.0, atol=1e-13)
        # at most two coarse nodes per fine point (t = 2 per dimension)
        assert np.all((np.abs(H) > 0).sum(1) <= 2)


def test_hat_reproduces_linear_functions_bounded():
    rng = np.random.default_rng(4)
    for trial in range(20):
        n = int(rng.integers(3, 50))
        m = int(rng.integers(2, n + 1))
        x = _grid(rng, n, -1.0, 2.0)
        c = _subset(rng, n, m)
        H = spid.hat_matrix(x, c)
        a, b = rng.normal(size=2)
        f = a + b * x
        # interior points and the continued end elements alike
        np.testing.assert_allclose(H @ f[c], f, atol=1e-12)


def test_hat_periodic_wraps_last_element():
    # nodes at 0, 1, 2 of a period-4 circle: fine point 3 sits half way
    # between node 2 and node 0 + 4, fine point -1 (= 3) likewise
    x = np.array([0.0, 1.0, 2.0, 3.0])
    H = spid.hat_matrix(x, np.array([0, 1, 2]), period=4.0)
    np.testing.assert_allclose(H[3], [0.5, 0.0, 0.5])
    x2 = np.array([0.0, 0.5, 1.0, 2.0, 3.5])
    H2 = spid.hat_matrix(x2, np.array([0, 2, 3]), period=4.0)
    # 3.5 lies in the wrapping element [2, 4]: weight 0.75 on node 0 (at 4)
    np.testing.assert_allclose(H2[4], [0.75, 0.0, 0.25])
    # bounded: beyond the last node the last element's line continues
    H3 = spid.hat_matrix(np.array([0.0, 1.0, 2.0, 3.0]), np.array([0, 2]))
    np.testing.assert_allclose(H3[3], [-0.5, 1.5])


@pytest.mark.parametrize("periodic", [False, True])
def test_interpolation_error_bound_and_h2_rate(periodic):
    """max |f - I_H f| <= H^2/8 max|f''| for piecewise linear interpolation,
    and the error falls by ~4 when H halves (the H^2 rate named after
    Theorem 2.2)."""
    errs = []
    for nf in (65, 129, 257):
        if periodic:
            L = 2.0 * math.pi
            x = np.arange(nf - 1) * (L / (nf - 1))
            f = np.sin(x) + 0.5 * np.cos(2 * x)
            fpp = 1.0 + 2.0
        else:
            L = 0.0
            x = np.linspace(0.0, math.pi, nf)
            f = np.sin(x)
            fpp = 1.0
        c = np.arange(0, len(x), 2)
        Hs = 2.0 * (x[1] - x[0])
        E = np.max(np.abs(spid.hat_matrix(x, c, L) @ f[c] - f))
        assert E <= Hs * Hs / 8.0 * fpp * (1 + 1e-9)
        errs.append(E)
    for a, b in zip(errs, errs[1:]):
        assert 3.6 < a / b < 4.4


def _mesh(ncomp, n, strides, period=(0.0, 0.0, 0.0), seed=5):
    rng = np.random.default_rng(seed)
    coords = tuple(_grid(rng, n_d, 0.0, 1.0) for n_d in n)
    coarse = tuple(np.arange(0, n_d, s, dtype=np.int64) for n_d, s in zip(n, strides))
    return synth.StructuredMesh(ncomp, tuple(n), coords, coarse, tuple(period))


def test_trilinear_reproduction_and_ordering():
    """Mf reproduces every product of affine functions of x, y, z exactly,
    per component; with unequal dimensions this fixes the Kronecker order and
    the row numbering (z fastest, then y, x, component)."""
    mesh = _mesh(2, (6, 5, 7), (2, 3, 2))
    Mf = spid.interp_operator(mesh)
    nx, ny, nz = mesh.n
    assert Mf.shape == (mesh.rows, len(mesh.coarse_rows))
    x, y, z = mesh.coords
    c = np.arange(2)
    F = ((1.0 + c)[:, None, None, None] * (1 + 2 * x)[None, :, None, None]
         * (3 - y)[None, None, :, None] * (0.5 + z)[None, None, None, :]).reshape(-1)
    np.testing.assert_allclose(Mf @ F[mesh.coarse_rows], F, rtol=1e-12, atol=1e-12)
    # eight coarse points per fine point at most (t = 8), rows sum to one
    nnz = np.diff(Mf.indptr)
    assert nnz.max() <= 8
    np.testing.assert_allclose(np.asarray(Mf.sum(1)).ravel(), 1.0, atol=1e-13)


def test_trilinear_h2_rate_3d():
    errs = []
    for n in (17, 33, 65):
        t = np.linspace(0.0, 1.0, n)
        mesh = synth.StructuredMesh(1, (n, n, n), (t, t, t),
                                    tuple(np.arange(0, n, 2) for _ in range(3)), (0.0, 0.0, 0.0))
        F = (np.sin(2 * t)[:, None, None] * np.cos(t)[None, :, None]
             * np.exp(t)[None, None, :]).reshape(-1)
        Mf = spid.interp_operator(mesh)
        errs.append(np.max(np.abs(Mf @ F[mesh.coarse_rows] - F)))
    for a, b in zip(errs, errs[1:]):
        assert 3.3 < a / b < 4.6


def _field(nx=16, ny=8, nz=8, n=40, drift=0.02):
    cfg = synth.SpectralConfig(nx=nx, ny=ny, nz=nz, n_snapshots=n, n_modes=40, drift=drift,
                               seed=77)
    A = synth.spectral_snapshots(cfg, dtype=torch.float64).numpy()
    return cfg, A


def test_full_rank_limit_equals_interpolation_error():
    """With k = n the coarse ID is exact (A(S, J) P = A(S, :)), so the
    single-pass ID reduces to Mf A(S, :) and its error to ||E_I||: the
    saturation the paper observes as the rank grows."""
    cfg, A = _field(n=12)
    mesh = synth.channel_mesh(cfg, (2, 2, 2))
    Mf = spid.interp_operator(mesh)
    res = spid.spid_compress(A, mesh, k=12, oversample=4, seed=3)
    assert res.k_eff == 12
    Ahat = spid.spid_reconstruct(Mf, res.ACJ, res.P)
    ref = Mf @ A[mesh.coarse_rows]
    np.testing.assert_allclose(Ahat, ref, rtol=0, atol=1e-10 * np.abs(ref).max())
    # and the coarse skeleton is the coarse rows of the skeleton columns
    np.testing.assert_array_equal(res.ACJ, A[np.ix_(mesh.coarse_rows, res.J)])


@pytest.mark.parametrize("literal", [False, True])
def test_theorem_2_2(literal):
    """||A - A_hat||_2 <= ||E_I||_2 + ||Mf||_2 ||A_c - A_c(:, J) P||_2 (the
    proof's middle inequality, always true) and the theorem's bound with the
    ID bound sqrt(1 + k(n - k)) sigma_{k+1}(A_c)."""
    cfg, A = _field()
    mesh = synth.channel_mesh(cfg, (2, 2, 2))
    Mf = spid.interp_operator(mesh)
    k = 8
    res = spid.spid_compress(A, mesh, k=k, oversample=6, seed=11, literal=literal)
    t = spid.thm22_terms(A, mesh, Mf, res)
    n = A.shape[1]
    assert t["err"] <= t["EI"] + t["M"] * t["coarse_err"] * (1 + 1e-12)
    assert t["err"] <= t["EI"] + t["M"] * math.sqrt(1 + k * (n - k)) * t["sigma_k1"]
    # J and P are those of the sub-sampled ID on the same coarse rows
    base = res.base
    np.testing.assert_array_equal(res.J, base.J)
    np.testing.assert_array_equal(res.P, base.P)


def test_rows_sampler_matches_full_reconstruction():
    cfg, A = _field(n=20)
    mesh = synth.channel_mesh(cfg, (2, 2, 2), periodic=True)
    Mf = spid.interp_operator(mesh)
    res = spid.spid_compress(A, mesh, k=6, oversample=4, seed=2)
    Ahat = spid.spid_reconstruct(Mf, res.ACJ, res.P)
    rows = np.array([0, 5, 17, mesh.rows - 1])
    np.testing.assert_allclose(spid.spid_rows(Mf, res.ACJ, res.P, rows), Ahat[rows],
                               rtol=1e-13, atol=1e-13)


def test_interp_rows_match_operator():
    mesh = _mesh(2, (6, 5, 7), (2, 3, 2), period=(1.5, 0.0, 0.0))
    Mf = spid.interp_operator(mesh)
    rows = np.array([0, 1, 37, 104, 105, mesh.rows - 1])
    np.testing.assert_array_equal(spid.interp_rows(mesh, rows).toarray(), Mf[rows].toarray())


def _sweep(k, strides=(2, 4, 8)):
    cfg = synth.SpectralConfig(nx=65, ny=9, nz=65, n_snapshots=60, n_modes=40, drift=0.3,
                               seed=77, kmax=1.5)
    A = synth.spectral_snapshots(cfg, dtype=torch.float64).numpy()
    nA = np.linalg.norm(A)
    out = []
    for st in strides:
        mesh = synth.channel_mesh(cfg, (st, 1, st), keep_last=True)
        Mf = spid.interp_operator(mesh)
        res = spid.spid_compress(A, mesh, k, 10, seed=1)
        ke = res.k_eff
        e_spid = np.linalg.norm(A - spid.spid_reconstruct(Mf, res.ACJ, res.P)) / nA
        e_sub = np.linalg.norm(A - A[:, res.J[:ke]] @ res.P[:ke]) / nA
        e_int = np.linalg.norm(A - Mf @ A[mesh.coarse_rows]) / nA
        out.append((e_spid, e_sub, e_int))
    return out


def test_subsampling_sweep_interpolation_dominated():
    """Sub-sampling in x and z by 2, 4, 8 on a field resolved on those grids,
    at a rank above the field's numerical rank: the single-pass ID error
    saturates at the interpolation error and grows like H^2 (x4 per halving
    of the resolution), while the sub-sampled ID with the fine skeleton stays
    at its (rounding-level) ID error: the contrast the paper draws in Sec. 2.6
    and Fig. 4 (right)."""
    rows = _sweep(20)
    for (sp, sb, ei) in rows:
        assert sp == pytest.approx(ei, rel=0.05)
        assert sb < 1e-6 * sp
    for a, b in zip(rows, rows[1:]):
        assert 3.0 < b[0] / a[0] < 5.0


def test_subsampling_sweep_truncation_dominated():
    """At a rank well below the field's: both errors are the rank-k
    truncation, nearly equal and nearly independent of the sub-sampling
    (Theorem 2.2's sigma_{k+1} term dominates the interpolation term).  At a
    sub-sampling of 8 per dimension the interpolation error of this field
    reaches half the truncation error, so the sweep stops at 4."""
    rows = _sweep(10, strides=(2, 4))
    for (sp, sb, ei) in rows:
        assert sp == pytest.approx(sb, rel=0.3)
        assert ei < 0.5 * sp
    assert max(r[1] for r in rows) < 1.5 * min(r[1] for r in rows)
