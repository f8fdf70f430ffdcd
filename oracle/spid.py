"""CPU FP64 oracle of the single-pass ID with interpolation (Alg. 6).

TEST INFRASTRUCTURE ONLY, like ``oracle.oracle``: only ``tests/``,
``__graft_entry__.smoke()`` and the benchmark's ``cpu_baseline`` leg may use
it.  It shares no code with the HIP product path.

Reference: Dunton, Jofre, Iaccarino & Doostan, arXiv:1905.13257, Sec. 2.6
(single-pass ID), Alg. 6, eq. (single_ID), Theorem 2.2; Sec. 3 states that
the interpolation used is piecewise linear.

Orientation (as in ``oracle.oracle``): A is N x n with one snapshot per
column, rows are grid points.  The paper's A_p ~ P_c A_p,c(I_c, :) M with a
coarse-to-fine operator M (n_c x n in the paper's row-snapshot layout)
becomes here

    A ~ Mf A(S, J) P,      Mf = M^T (N x N_c),

where S are the coarse rows (the sub-sampled grid, eq. (A_c)), J and P are
the column ID of A(S, :) (the same J and P as the sub-sampled ID, Alg. 5),
and A(S, J) = A_c(:, J) is the coarse skeleton that Alg. 6 stores instead of
the fine one.

The operator.  On a tensor-product grid (components x nx x ny x nz, z
fastest) piecewise linear interpolation in each dimension is the tensor
product of three 1-D operators, Mf = I_ncomp (x) Mx (x) My (x) Mz (trilinear,
t = 8 coarse points per fine point).  Each 1-D operator has entries
Md[i, a] = phi_a(x_i): the piecewise linear nodal ("hat") basis function of
coarse node a, evaluated at fine coordinate x_i.  Readings where the paper
is silent (how the ends are treated):
  * bounded dimension: the first and the last element's linear functions
    are continued beyond the outermost coarse nodes (linear extrapolation);
  * periodic dimension of period L: the nodes lie on a circle, the last
    element joins node m-1 to node 0 + L;
  * a dimension with a single coarse node is constant.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np
import scipy.sparse as sp

from . import oracle as _o


def hat_matrix(x: np.ndarray, coarse: np.ndarray, period: float = 0.0) -> np.ndarray:
    """Dense 1-D piecewise linear interpolation matrix, n_fine x n_coarse:
    entry (i, a) is the nodal basis function of coarse node a at x[i].

    x: fine coordinates (strictly increasing); coarse: kept indices into x
    (strictly increasing).  Written element by element: every fine point is
    located in one element [X_a, X_b] of the coarse nodes (the end elements
    continued for a bounded dimension, the wrapping element for a periodic
    one) and receives the two linear shape functions of that element."""
    x = np.asarray(x, np.float64)
    coarse = np.asarray(coarse, np.int64)
    X = x[coarse]
    nf, m = len(x), len(X)
    H = np.zeros((nf, m))
    if m == 1:
        H[:, 0] = 1.0
        return H
    # the elements: (left node, right node, left coordinate, right coordinate)
    elems = [(a, a + 1, X[a], X[a + 1]) for a in range(m - 1)]
    if period > 0.0:
        elems.append((m - 1, 0, X[m - 1], X[0] + period))
    for i in range(nf):
        xi = x[i]
        if period > 0.0:
            # map into [X_0, X_0 + L): the nodes cover one period from X_0
            xi = X[0] + np.mod(xi - X[0], period)
            e = next(e for e in elems if e[2] <= xi <= e[3])
        else:
            if xi < X[0]:
                e = elems[0]
            elif xi > X[-1]:
                e = elems[-1]
            else:
                e = next(e for e in elems if e[2] <= xi <= e[3])
        a, b, xa, xb = e
        s = (xi - xa) / (xb - xa)          # local coordinate, 0 at node a, 1 at node b
        H[i, a] += 1.0 - s
        H[i, b] += s
    return H


def interp_operator(mesh) -> sp.csr_matrix:
    """Mf = I_ncomp (x) Mx (x) My (x) Mz as a sparse N x N_c matrix (rows and
    columns ordered component, x, y, z with z fastest)."""
    Hs = [sp.csr_matrix(hat_matrix(mesh.coords[d], mesh.coarse[d], mesh.period[d]))
          for d in range(3)]
    Mf = sp.kron(Hs[0], sp.kron(Hs[1], Hs[2], format="csr"), format="csr")
    return sp.kron(sp.identity(mesh.ncomp, format="csr"), Mf, format="csr")


def interp_rows(mesh, rows) -> sp.csr_matrix:
    """Selected rows of Mf (len(rows) x N_c) without forming Mf: row
    ((c * nx + i) * ny + j) * nz + k is e_c (x) Mx[i] (x) My[j] (x) Mz[k]."""
    Hs = [hat_matrix(mesh.coords[d], mesh.coarse[d], mesh.period[d]) for d in range(3)]
    nx, ny, nz = mesh.n
    blk = Hs[0].shape[1] * Hs[1].shape[1] * Hs[2].shape[1]
    out = []
    for r in np.asarray(rows, np.int64):
        c, rem = divmod(int(r), nx * ny * nz)
        i, rem = divmod(rem, ny * nz)
        j, k = divmod(rem, nz)
        row = sp.kron(sp.csr_matrix(Hs[0][i:i + 1]),
                      sp.kron(sp.csr_matrix(Hs[1][j:j + 1]), sp.csr_matrix(Hs[2][k:k + 1])))
        e = sp.csr_matrix(([1.0], ([0], [c])), shape=(1, mesh.ncomp))
        out.append(sp.kron(e, row, format="csr"))
    M = sp.vstack(out, format="csr")
    assert M.shape[1] == mesh.ncomp * blk
    return M


@dataclass
class SPIDResult:
    J: np.ndarray            # k skeleton snapshot indices (pivot order; -1 past k_eff)
    P: np.ndarray            # k x n coefficients (rows past k_eff zero)
    ACJ: np.ndarray          # N_c x k coarse skeleton A(S, J) (columns past k_eff zero)
    k_eff: int
    base: _o.Result          # the ID of the coarse data it came from


def spid_compress(A, mesh, k: int, oversample: int, seed: int = 0, prec: str = "f64",
                  probe_rows: int = 10, literal: bool = False) -> SPIDResult:
    """Alg. 6: subsample A to the coarse rows, compute the ID of A(S, :)
    (the Gaussian-sketched sub-sampled ID, or with ``literal`` mgsqr on
    A(S, :) itself), and keep the coarse skeleton A(S, J) in place of the
    fine one.  J and P are those of the sub-sampled ID."""
    A = np.asarray(A)
    rows = mesh.coarse_rows
    if literal:
        res = _o.compress_literal(A, k, rows, prec=prec)
    else:
        res = _o.compress(A, k, oversample, seed=seed, coarse_rows=rows, mode="two_pass",
                          prec=prec, probe_rows=probe_rows)
    ACJ = np.zeros((len(rows), k))
    ke = res.k_eff
    ACJ[:, :ke] = np.asarray(A, np.float64)[np.ix_(rows, res.J[:ke])]
    return SPIDResult(J=res.J, P=res.P, ACJ=ACJ, k_eff=ke, base=res)


def spid_reconstruct(Mf, ACJ: np.ndarray, P: np.ndarray) -> np.ndarray:
    """A_hat = Mf A(S, J) P (eq. (single_ID), transposed)."""
    return np.asarray(Mf @ np.asarray(ACJ, np.float64)) @ np.asarray(P, np.float64)


def spid_rows(Mf, ACJ: np.ndarray, P: np.ndarray, rows) -> np.ndarray:
    """Selected rows of A_hat (for samples of a matrix too large to
    reconstruct): A_hat(i, :) = Mf(i, :) A(S, J) P.  ``Mf`` is the operator
    or the rows of it (``interp_rows``) already selected (rows=None)."""
    Mr = Mf if rows is None else Mf[np.asarray(rows, np.int64)]
    return np.asarray(Mr @ np.asarray(ACJ, np.float64)) @ np.asarray(P, np.float64)


def error_norms(A, Ahat) -> dict:
    """Relative Frobenius and entry-wise errors of a formed approximation
    (Sec. 3 error measures, as ``oracle.error_norms``)."""
    A = np.asarray(A, np.float64)
    D = A - np.asarray(Ahat, np.float64)
    fro_a = float(np.linalg.norm(A))
    nz = A != 0
    return dict(rel_fro=float(np.linalg.norm(D)) / fro_a if fro_a > 0 else 0.0,
                fro_err=float(np.linalg.norm(D)), fro_a=fro_a,
                rel_max=float(np.max(np.abs(D[nz]) / np.abs(A[nz]))) if nz.any() else 0.0,
                max_abs=float(np.max(np.abs(D))))


def thm22_terms(A, mesh, Mf, res: SPIDResult) -> dict:
    """The quantities of Theorem 2.2 in spectral norms: the interpolation
    error E_I = A - Mf A(S, :), the coarse ID error A(S, :) - A(S, J) P,
    ||Mf||_2, sigma_{k+1} of A(S, :), and the single-pass ID error."""
    A = np.asarray(A, np.float64)
    Ac = A[mesh.coarse_rows]
    Mfd = Mf.toarray()
    ke = res.k_eff
    EI = A - Mfd @ Ac
    Ecoarse = Ac - res.ACJ[:, :ke] @ res.P[:ke]
    Ahat = Mfd @ res.ACJ[:, :ke] @ res.P[:ke]
    s_c = np.linalg.svd(Ac, compute_uv=False)
    return dict(err=float(np.linalg.norm(A - Ahat, 2)), EI=float(np.linalg.norm(EI, 2)),
                coarse_err=float(np.linalg.norm(Ecoarse, 2)), M=float(np.linalg.norm(Mfd, 2)),
                sigma_k1=float(s_c[ke]) if ke < len(s_c) else 0.0)
