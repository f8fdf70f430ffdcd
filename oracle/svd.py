"""CPU FP64 oracle of the randomized SVDs (Sec. 2.3): the basic two-pass
R-SVD (Alg. 1) and the single-pass blocked randomized SVD, SBR-SVD (Alg. 2).

TEST INFRASTRUCTURE ONLY, like ``oracle.oracle``: only ``tests/``,
``__graft_entry__.smoke()`` and the benchmark's ``cpu_baseline`` leg may use
it.  It shares no code with the HIP product path.

Orientation.  The paper's A_p (m x n_p: m snapshots in rows, n_p grid points)
is A^T here (A: N x n, one snapshot per column).  Its Gaussian test matrix
Omega (n_p x l) is Psi^T, the same Psi as the ID's (Psi(r, i) keyed by the
global row index i, stream 1), so G = A_p Omega = (Psi A)^T = W^T and
H = A_p^T G = A W^T.  The result A_p ~ U_k S_k V_k^T reads
A ~ V_k S_k U_k^T: V_k (N x k) spatial, U_k (n x k) temporal.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

from . import oracle as _o


@dataclass
class SVDResult:
    U: np.ndarray   # n x k (temporal, the paper's U_k)
    S: np.ndarray   # k
    V: np.ndarray   # N x k (spatial, the paper's V_k)


def _omega(A: np.ndarray, l: int, seed: int, prec: str) -> np.ndarray:
    """Omega = Psi^T (N x l) with the sketch's rounding of the Gaussians."""
    return _o.psi(seed, np.arange(A.shape[0]), l, prec).T


def rsvd(A, k: int, oversample: int, seed: int = 0, prec: str = "f64") -> SVDResult:
    """Alg. 1 in the paper's notation on A_p = A^T: Q R = qr(A_p Omega),
    B = Q^T A_p, B = U~ S V^T, U = Q U~ (two passes over A)."""
    Ap = np.asarray(A, np.float64).T
    l = k + oversample
    Om = _omega(A, l, seed, prec)
    Q, _ = np.linalg.qr(Ap @ Om)
    B = Q.T @ Ap
    Ut, S, Vt = np.linalg.svd(B, full_matrices=False)
    U = Q @ Ut
    return SVDResult(U=U[:, :k], S=S[:k], V=Vt[:k].T)


def sbr_svd(A, k: int, oversample: int, block: int, seed: int = 0,
            prec: str = "f64", stop_tol: float = 1e-12) -> SVDResult:
    """Alg. 2 (SBR-SVD), steps in the paper's order on A_p = A^T.

    One pass: for every row a of A_p (a snapshot), g = a Omega is appended
    to G and H += a^T g.  Then for each of the s = l / b blocks of Omega's
    columns: Y_i = G_i - Q (B Omega_i); (Q_i, R_i) = qr(Y_i); (Q_i, R~_i) =
    qr(Q_i - Q (Q^T Q_i)); R_i = R~_i R_i;
    B_i = R_i^-T (H_i^T - Y_i^T Q B - Omega_i^T B^T B); Q = [Q, Q_i];
    B = [B; B_i].  Finally B = U~ S V^T and U = Q U~.

    Alg. 2 needs A_p Omega of full column rank l; this reading stops before a
    block whose R_i has a diagonal entry <= stop_tol ||G||_F (the earlier
    blocks then span A_p Omega) and returns the rank reached (S padded with
    zeros, U and V with zero columns, up to k)."""
    Ap = np.asarray(A, np.float64).T
    m, npg = Ap.shape
    l = k + oversample
    if l % block != 0:
        raise ValueError("l = k + oversample must be a multiple of the block size")
    s = l // block
    Om = _omega(A, l, seed, prec)
    # the single pass over the rows of A_p (snapshots)
    G = np.zeros((m, l))
    H = np.zeros((npg, l))
    Ad = _o.data_values(np.asarray(A), prec).T    # the values the sketch reads
    for r in range(m):
        g = Ad[r] @ Om
        G[r] = g
        H += np.outer(Ap[r], g)
    Q = np.zeros((m, 0))
    B = np.zeros((0, npg))
    gnorm = np.linalg.norm(G)
    for i in range(s):
        cols = slice(i * block, (i + 1) * block)
        Om_i = Om[:, cols]
        Y = G[:, cols] - Q @ (B @ Om_i)
        Qi, Ri = np.linalg.qr(Y)
        Qi, Rt = np.linalg.qr(Qi - Q @ (Q.T @ Qi))
        Ri = Rt @ Ri
        # A_p Omega of rank below l: the block's R_i is singular and
        # R_i^-T undefined; the blocks so far already span A_p Omega
        if np.min(np.abs(np.diag(Ri))) <= stop_tol * gnorm:
            break
        rhs = H[:, cols].T - Y.T @ Q @ B - Om_i.T @ B.T @ B
        Bi = np.linalg.solve(Ri.T, rhs)
        Q = np.hstack([Q, Qi])
        B = np.vstack([B, Bi])
    Ut, S, Vt = np.linalg.svd(B, full_matrices=False)
    U = Q @ Ut
    kk = min(k, len(S))
    Uk, Sk, Vk = np.zeros((m, k)), np.zeros(k), np.zeros((npg, k))
    Uk[:, :kk], Sk[:kk], Vk[:, :kk] = U[:, :kk], S[:kk], Vt[:kk].T
    return SVDResult(U=Uk, S=Sk, V=Vk)


def reconstruct(res: SVDResult) -> np.ndarray:
    """A ~ V_k S_k U_k^T (N x n)."""
    return (res.V * res.S[None, :]) @ res.U.T
