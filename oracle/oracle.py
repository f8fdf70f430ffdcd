"""CPU FP64 oracle of the pass-efficient interpolative decomposition.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
benchmark's ``cpu_baseline`` leg may import this module.  It shares no code with
the HIP product path (``paper_1905_13257_amd``); the only common dependency is
the seeded input generator module ``synth``.

Reference: Dunton, Jofre, Iaccarino & Doostan, "Pass-efficient methods for
compression of high-dimensional turbulent flow data", arXiv:1905.13257.

Orientation.  The paper stores time in rows (A_p is m x n, m snapshots) and
computes a row ID A_p ~ P A_p(I,:) (Sec. 2.4, eq. (ID)).  Here A = A_p^T is
N x n with one snapshot per column and the same decomposition appears as the
column ID A ~ A(:, J) P, J a list of k snapshot indices, P a k x n matrix with
P(:, J) = I (Remark 2.1: the column ID is the analogous form).

Steps, each written as the plain definition in the paper's order:

* ``sketch`` -- W = Psi(:, S) A(S, :) and Y = A Omega with i.i.d. Gaussian
  Psi, Omega (Sec. 2.2 eq. (sampmatrix); Alg. 4 "Y <- A Omega"; the two-sided
  single-pass sketch of Halko et al. Sec. 5.5 quoted in Sec. 2.3, items (1)-(2)).
  S is an optional coarse row subset (Sec. 2.5, eq. (A_c), "direct injection").
* ``cpqr`` -- the paper's mgsqr: column-pivoted modified Gram-Schmidt, k steps
  (Sec. 2.4, Alg. 3-5 step "Q, R, I <- mgsqr(., k)").
* ``id_coefficients`` -- C = R11^+ R12 by back substitution, P = [I | C]
  placed by the pivot permutation (Alg. 3-5, the two steps after mgsqr).
* ``estimates`` -- relative residual of the sketch fit and of held-out probe
  rows of Psi (the paper states only a CPQR-residual stopping rule,
  Remark 2.2; the probe estimator is this implementation's reading).
* ``skeleton_single_pass`` -- the skeleton columns A(:, J) estimated from the
  sketches without a second pass: Q = orth(Y), Z = Psi(:,S) Q(S,:),
  X = Z^+ W(:, J), A_J ~ Q X (the minimum-residual solve of Halko et al.
  Sec. 5.5 item (4), quoted in Sec. 2.3).
* ``error_norms`` -- relative Frobenius and relative max errors (Sec. 3,
  Tables 4-7 captions; Sec. 3.1 "relative entry-wise error").
* ``compression_factor`` -- Sec. 3.1 definitions and Table 1 storage counts.

Sketch precisions.  The Gaussian values of Psi and Omega are single-precision
draws (``gaussian``); a low-precision mode stores them rounded to bfloat16 or
FP8 e4m3, and the data rounded the way that mode reads them.  ``prec`` selects
the rounding; all arithmetic after the rounding is FP64.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass, field

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB = None

STREAM_OMEGA = 0
STREAM_PSI = 1
PRECISIONS = ("f64", "f32", "bf16", "bf16x2", "fp8")


def build(force: bool = False) -> str:
    """Compile the oracle's C core (plain gcc, OpenMP, no fast-math)."""
    src = os.path.join(_HERE, "oracle_core.c")
    out = os.path.join(_HERE, "liboracle.so")
    if force or not os.path.exists(out) or os.path.getmtime(out) < os.path.getmtime(src):
        import subprocess
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-ffp-contract=off", "-fPIC",
                               "-shared", "-o", out, src])
    return out


def lib():
    global _LIB
    if _LIB is None:
        path = os.path.join(_HERE, "liboracle.so")
        if not os.path.exists(path):
            build()
        L = ctypes.CDLL(path)
        i64, u64, u32 = ctypes.c_int64, ctypes.c_uint64, ctypes.c_uint32
        vp = ctypes.c_void_p
        L.oracle_philox4x32_10.argtypes = [vp, vp, vp]
        L.oracle_gauss.argtypes = [u64, u32, u64, u64]
        L.oracle_gauss.restype = ctypes.c_float
        L.oracle_fill_gaussian.argtypes = [u64, u32, vp, i64, i64, i64, i64, vp]
        L.oracle_sketch_w.argtypes = [u64, ctypes.c_int, vp, i64, i64, vp, i64, i64, vp]
        L.oracle_sketch_y.argtypes = [vp, i64, i64, i64, vp, i64, vp]
        L.oracle_error_norms.argtypes = [vp, i64, vp, i64, vp, i64, i64, i64, i64, vp]
        L.oracle_round_bf16.argtypes = [ctypes.c_double]
        L.oracle_round_bf16.restype = ctypes.c_double
        L.oracle_round_e4m3.argtypes = [ctypes.c_double]
        L.oracle_round_e4m3.restype = ctypes.c_double
        L.oracle_round_e4m3_array.argtypes = [vp, i64]
        _LIB = L
    return _LIB


def _ptr(a: np.ndarray):
    return ctypes.c_void_p(a.ctypes.data)


# --------------------------------------------------------------------------
# Random test matrices
# --------------------------------------------------------------------------

def philox(counter, key) -> np.ndarray:
    c = np.ascontiguousarray(counter, dtype=np.uint32)
    k = np.ascontiguousarray(key, dtype=np.uint32)
    out = np.zeros(4, dtype=np.uint32)
    lib().oracle_philox4x32_10(_ptr(c), _ptr(k), _ptr(out))
    return out


def gaussian(seed: int, stream: int, majors, minor0: int, nminor: int) -> np.ndarray:
    """G(seed, stream, major, minor) for each major in ``majors`` (array of
    int64) and minor in [minor0, minor0+nminor); shape (len(majors), nminor),
    float32 values."""
    majors = np.ascontiguousarray(majors, dtype=np.int64)
    out = np.empty((majors.size, nminor), dtype=np.float32)
    lib().oracle_fill_gaussian(ctypes.c_uint64(seed), stream, _ptr(majors), 0, majors.size,
                               minor0, nminor, _ptr(out))
    return out


def round_values(x: np.ndarray, kind: str) -> np.ndarray:
    """Round FP32-exact values to bfloat16 or e4m3 (nearest, ties to even)."""
    x = np.asarray(x, dtype=np.float64)
    if kind == "bf16":
        f = x.astype(np.float32).view(np.uint32).astype(np.uint64)
        lsb = (f >> np.uint64(16)) & np.uint64(1)
        r = ((f + np.uint64(0x7FFF) + lsb) & np.uint64(0xFFFF0000)).astype(np.uint32)
        return r.view(np.float32).astype(np.float64)
    if kind == "e4m3":
        flat = np.array(x, dtype=np.float64, copy=True).reshape(-1)
        lib().oracle_round_e4m3_array(_ptr(flat), flat.size)
        return flat.reshape(x.shape)
    raise ValueError(kind)


def test_matrix_values(z: np.ndarray, prec: str) -> np.ndarray:
    """Values a sketch precision stores for the Gaussian draws z (float32)."""
    if prec in ("f64", "f32"):
        return z.astype(np.float64)
    if prec in ("bf16", "bf16x2"):
        return round_values(z, "bf16")
    if prec == "fp8":
        return round_values(z, "e4m3")
    raise ValueError(prec)


def data_values(A: np.ndarray, prec: str) -> np.ndarray:
    """Values of the data as a sketch precision reads them.

    f64: as given.  f32: rounded to single.  bf16: rounded to bfloat16.
    bf16x2: hi + lo with hi = bf16(a), lo = bf16(a - hi) (a two-term split of
    the single-precision value).  fp8 reads per-tile scaled e4m3 values
    (see ``fp8_data_values``; A must then hold whole 64-row tiles from row
    0 of the matrix)."""
    A = np.asarray(A, dtype=np.float64)
    if prec == "f64":
        return A
    if prec == "f32":
        return A.astype(np.float32).astype(np.float64)
    if prec == "bf16":
        return round_values(A.astype(np.float32), "bf16")
    if prec == "bf16x2":
        a32 = A.astype(np.float32)
        hi = round_values(a32, "bf16")
        lo = round_values((a32.astype(np.float64) - hi).astype(np.float32), "bf16")
        return hi + lo
    if prec == "fp8":
        return fp8_data_values(A)
    raise ValueError(prec)


FP8_TILE_ROWS = 64


def fp8_data_values(A: np.ndarray) -> np.ndarray:
    """Values of FP32 data as the FP8 (e4m3) sketch reads them.

    The rows of A are cut into tiles of 64 consecutive rows (the last one
    ragged); each (tile, column) pair gets a power-of-two scale
    s = 2^(E - 7), E = floor(log2 max|a|) over the tile's entries, clamped to
    [-100, 120] (s = 1 for an all-zero tile), so that |a| / s < 256 <= 448,
    the largest e4m3 value.  Each entry becomes s * e4m3(a / s), nearest with
    ties to even.  The paper fixes no low-precision format; this per-tile
    scaling is the usual way of putting data of any magnitude into e4m3's
    narrow exponent range."""
    A = np.asarray(A, dtype=np.float64).astype(np.float32).astype(np.float64)
    N, n = A.shape
    out = np.empty_like(A)
    for t0 in range(0, N, FP8_TILE_ROWS):
        blk = A[t0:t0 + FP8_TILE_ROWS]
        amax = np.abs(blk).max(axis=0)
        _, ex = np.frexp(amax)                 # amax = f 2^ex, f in [0.5, 1)
        E = np.clip(ex - 1, -100, 120)
        s = np.where(amax > 0, np.ldexp(1.0, E - 7), 1.0)
        out[t0:t0 + FP8_TILE_ROWS] = round_values(blk / s, "e4m3") * s
    return out


def omega(seed: int, n: int, l: int, prec: str = "f64", col0: int = 0) -> np.ndarray:
    """Omega (n x l): Omega(j, c) = G(seed, 0, col0 + j, c)."""
    z = gaussian(seed, STREAM_OMEGA, np.arange(col0, col0 + n, dtype=np.int64), 0, l)
    return test_matrix_values(z, prec)


def psi(seed: int, rows, lq: int, prec: str = "f64") -> np.ndarray:
    """Psi(:, rows) ((l+q) x len(rows)): Psi(r, i) = G(seed, 1, i, r), keyed by
    the global row index i of A."""
    z = gaussian(seed, STREAM_PSI, np.asarray(rows, dtype=np.int64), 0, lq)
    return test_matrix_values(z, prec).T


# --------------------------------------------------------------------------
# Sketches
# --------------------------------------------------------------------------

def sketch_w(A: np.ndarray, rows, lq: int, seed: int, prec: str = "f64") -> np.ndarray:
    """W = Psi(:, rows) A(rows, :) in FP64, ((l+q) x n)."""
    A = np.asfortranarray(data_values(A, prec))
    N, n = A.shape
    rows = np.ascontiguousarray(np.arange(N) if rows is None else rows, dtype=np.int64)
    W = np.zeros((n, lq), dtype=np.float64)          # column-major lq x n == row-major n x lq
    rmode = 0 if prec in ("f64", "f32") else (2 if prec == "fp8" else 1)
    lib().oracle_sketch_w(ctypes.c_uint64(seed), rmode, _ptr(A), A.strides[1] // 8, n,
                          _ptr(rows), rows.size, lq, _ptr(W))
    return W.T.copy()


def sketch_y(A: np.ndarray, Om: np.ndarray, prec: str = "f64") -> np.ndarray:
    """Y = A Omega in FP64, (N x l)."""
    A = np.asfortranarray(data_values(A, prec))
    N, n = A.shape
    Om = np.ascontiguousarray(Om, dtype=np.float64)
    l = Om.shape[1]
    Y = np.empty((N, l), dtype=np.float64)
    lib().oracle_sketch_y(_ptr(A), A.strides[1] // 8, N, n, _ptr(Om), l, _ptr(Y))
    return Y


# --------------------------------------------------------------------------
# mgsqr and the ID coefficients
# --------------------------------------------------------------------------

@dataclass
class CPQR:
    J: np.ndarray              # pivot columns, in pivot order
    R: np.ndarray              # k_eff x n, R[i, J[i]] = residual norm at step i
    Q: np.ndarray              # l x k_eff orthonormal directions
    k_eff: int
    margins: np.ndarray        # relative gap between best and second-best norm
    pivot_norms: np.ndarray    # residual norm of the chosen column at each step
    final_residual: np.ndarray = field(default=None)  # l x n residual after k_eff steps


def cpqr(W: np.ndarray, k: int, rank_tol: float = 0.0) -> CPQR:
    """Column-pivoted modified Gram-Schmidt (the paper's mgsqr), k steps.

    Step i: every not-yet-chosen column's residual norm is recomputed; the
    largest is the pivot (ties: smallest column index); its residual is
    normalized to q_i; R[i, p] = norm; every remaining column j gets
    R[i, j] = q_i^T r_j and r_j -= R[i, j] q_i.  The loop stops early when the
    pivot norm is zero or, with rank_tol > 0, at most rank_tol times the first
    pivot norm (Remark 2.2: ID stops on the decay seen by the rank-revealing
    QR)."""
    Wr = np.array(W, dtype=np.float64, copy=True)
    l, n = Wr.shape
    kmax = min(k, l, n)
    R = np.zeros((kmax, n))
    Q = np.zeros((l, kmax))
    alive = np.ones(n, dtype=bool)
    J, margins, pnorms = [], [], []
    first = None
    for i in range(kmax):
        norms = np.sqrt(np.sum(Wr * Wr, axis=0))
        cand = np.where(alive, norms, -1.0)
        p = int(np.argmax(cand))
        top = cand[p]
        rest = cand.copy()
        rest[p] = -1.0
        second = rest.max() if n > 1 else -1.0
        if top <= 0.0 or (first is not None and rank_tol > 0.0 and top <= rank_tol * first):
            break
        if first is None:
            first = top
        margins.append((top - max(second, 0.0)) / top)
        pnorms.append(top)
        q = Wr[:, p] / top
        Q[:, i] = q
        R[i, p] = top
        alive[p] = False
        Wr[:, p] = 0.0
        idx = np.nonzero(alive)[0]
        coef = q @ Wr[:, idx]
        R[i, idx] = coef
        Wr[:, idx] -= np.outer(q, coef)
        J.append(p)
    k_eff = len(J)
    return CPQR(J=np.array(J, dtype=np.int64), R=R[:k_eff], Q=Q[:, :k_eff], k_eff=k_eff,
                margins=np.array(margins), pivot_norms=np.array(pnorms), final_residual=Wr)


def id_coefficients(R: np.ndarray, J: np.ndarray, n: int) -> np.ndarray:
    """P (k x n) with P(:, J) = I and P(:, j) = R11^{-1} R(:, j) otherwise,
    R11 = R(:, J) upper triangular in pivot order (C = R11^+ R12, P = Z[I|C]^T
    of Alg. 3-5), by back substitution."""
    k = len(J)
    P = np.zeros((k, n))
    if k == 0:
        return P
    R11 = R[:, J]
    others = np.setdiff1d(np.arange(n), J)
    rhs = R[:, others]
    X = np.zeros_like(rhs)
    for b in range(k - 1, -1, -1):
        acc = rhs[b] - R11[b, b + 1:] @ X[b + 1:]
        X[b] = acc / R11[b, b]
    P[:, others] = X
    for i, j in enumerate(J):
        P[:, j] = 0.0
        P[i, j] = 1.0
    return P


# --------------------------------------------------------------------------
# Single-pass skeleton and the whole compressor
# --------------------------------------------------------------------------

def psi_times(rows, lq: int, seed: int, prec: str, M: np.ndarray, block: int = 1 << 16) -> np.ndarray:
    """Psi(:, rows) @ M for M with len(rows) rows, generating Psi blockwise."""
    rows = np.asarray(rows, dtype=np.int64)
    out = np.zeros((lq, M.shape[1]))
    for s0 in range(0, rows.size, block):
        P = psi(seed, rows[s0:s0 + block], lq, prec)
        out += P @ M[s0:s0 + block]
    return out


def skeleton_single_pass(Y: np.ndarray, W: np.ndarray, J: np.ndarray, lz: int, rows,
                         seed: int, prec: str, rcond: float = 1e-12):
    """Estimate A(:, J) from the sketches alone.

    Q = orth(Y) by Householder QR; Z = Psi(:, S) Q(S, :) over all rows of
    Psi; X = pinv(Z[:lz]) W[:lz](:, J) with singular values below rcond*s_max
    dropped; A_J ~ Q X.  lz = l + extra co-range rows: with lz = l the solve
    is the square minimum-residual problem of Halko et al. Sec. 5.5 item (4),
    whose matrix the paper notes is typically ill-conditioned (Sec. 2.3);
    extra rows make Z a tall Gaussian-like matrix.  Returns (AJ_hat, Z, X)."""
    Q, _ = np.linalg.qr(Y)
    lq = W.shape[0]
    rows = np.arange(Y.shape[0]) if rows is None else np.asarray(rows)
    Zfull = psi_times(rows, lq, seed, prec, Q[rows])
    X = np.linalg.pinv(Zfull[:lz], rcond=rcond) @ W[:lz][:, J]
    return Q @ X, Zfull, X


def probe_prefix_errors(cp: CPQR, Wpr: np.ndarray, n: int) -> np.ndarray:
    """Relative probe fit of every prefix of the pivots: entry k' (1 <= k' <=
    k_eff) is ||W_pr - W_pr(:, J') P'|| / ||W_pr|| with J' the first k'
    pivots and P' their ID coefficients (from the first k' rows of R), each
    formed from its definition."""
    out = np.full(cp.k_eff + 1, np.nan)
    out[0] = 1.0
    for kp in range(1, cp.k_eff + 1):
        Jp = cp.J[:kp]
        Pp = id_coefficients(cp.R[:kp], Jp, n)
        out[kp] = _rel_fit(Wpr, Wpr[:, Jp] @ Pp)
    return out


def adaptive_rank(cp: CPQR, Wpr: np.ndarray, n: int, tol: float) -> CPQR:
    """Tolerance-driven rank (Remark 2.2: ID stops on a criterion instead of
    a fixed k), with the held-out probe rows as the stopping test: the
    smallest k' whose relative probe fit is <= tol (k_eff unchanged when no
    prefix meets it); the first k' pivot steps of mgsqr are those of a run
    stopped at k'."""
    e = probe_prefix_errors(cp, Wpr, n)
    hit = [kp for kp in range(1, cp.k_eff + 1) if e[kp] <= tol]
    if not hit:
        return cp
    kp = hit[0]
    return CPQR(J=cp.J[:kp], R=cp.R[:kp], Q=cp.Q[:, :kp], k_eff=kp, margins=cp.margins[:kp],
                pivot_norms=cp.pivot_norms[:kp], final_residual=None)


def _rel_fit(Wpart: np.ndarray, approx: np.ndarray) -> float:
    den = np.linalg.norm(Wpart)
    return float(np.linalg.norm(Wpart - approx) / den) if den > 0 else 0.0


@dataclass
class Result:
    J: np.ndarray
    P: np.ndarray
    AJ: np.ndarray
    k_eff: int
    err_probe: float
    err_sketch: float
    W: np.ndarray
    Y: np.ndarray | None
    cp: CPQR


def compress_literal(A, k: int, coarse_rows, prec: str = "f64", rank_tol: float = 0.0) -> Result:
    """The sub-sampled ID exactly as Alg. 5 writes it: mgsqr directly on the
    coarse rows A(S, :) (no Gaussian sketch), P from its R, and the skeleton
    columns A(:, J) copied from the full matrix (two-pass).  err_sketch is
    the residual of the mgsqr fit on A(S, :); there are no probe rows
    (err_probe = NaN)."""
    A = np.asarray(A)
    N, n = A.shape
    rows = np.asarray(coarse_rows, np.int64)
    if rows.size <= k or np.any(np.diff(rows) <= 0) or rows[0] < 0 or rows[-1] >= N:
        raise ValueError("coarse rows must be sorted, unique, in range and more than k")
    if prec not in ("f64", "f32"):
        raise ValueError("the literal form reads the data in F64 or F32")
    W = data_values(A[rows], prec)
    cp = cpqr(W, k, rank_tol)
    Pk = id_coefficients(cp.R, cp.J, n)
    P = np.zeros((k, n))
    P[:cp.k_eff] = Pk
    J = np.full(k, -1, dtype=np.int64)
    J[:cp.k_eff] = cp.J
    AJk = np.zeros((N, k))
    AJk[:, :cp.k_eff] = np.asarray(A, dtype=np.float64)[:, cp.J]
    return Result(J=J, P=P, AJ=AJk, k_eff=cp.k_eff, err_probe=float("nan"),
                  err_sketch=_rel_fit(W, W[:, cp.J] @ Pk), W=W, Y=None, cp=cp)


def compress(A, k: int, oversample: int, seed: int = 0, coarse_rows=None,
             mode: str = "two_pass", prec: str = "f64", probe_rows: int = 10,
             rank_tol: float = 0.0, sp_rcond: float = 1e-12,
             corange_extra: int | None = None, probe_tol: float = 0.0,
             timings: dict | None = None) -> Result:
    """Randomized / sub-sampled ID (Alg. 4-5) or its single-pass form.

    A: N x n array (any float type; FP32 data are promoted exactly).
    Psi rows: [0, l) select J and P (l = k + oversample, Alg. 4); in single
    pass [l, l + e) are extra co-range rows used only by the skeleton solve
    (e = corange_extra, default = oversample); the last probe_rows rows are
    held out for the error estimate.
    Returns J (pivot order), P (k x n; rows beyond k_eff zero), the skeleton
    (two_pass: A(:, J) copied; single_pass: estimated from the sketches),
    and the two error estimates (err_probe: held-out probe rows; err_sketch:
    residual of the sketch fit itself).  If `timings` is a dict, the wall
    time of each phase (sketch, mgsqr, coefficients, skeleton) is added to
    it in seconds."""
    import time as _time
    tick = [_time.perf_counter()]

    def phase(name):
        if timings is not None:
            t = _time.perf_counter()
            timings[name] = timings.get(name, 0.0) + t - tick[0]
            tick[0] = t
    A = np.asarray(A)
    N, n = A.shape
    l = k + oversample
    if not (1 <= k <= min(n, l)):
        raise ValueError("need 1 <= k <= min(n, k + oversample)")
    rows = np.arange(N, dtype=np.int64) if coarse_rows is None else np.asarray(coarse_rows, np.int64)
    if coarse_rows is not None:
        if rows.size <= k or np.any(np.diff(rows) <= 0) or rows[0] < 0 or rows[-1] >= N:
            raise ValueError("coarse rows must be sorted, unique, in range and more than k")
    if corange_extra is None:
        corange_extra = oversample
    e = corange_extra if mode == "single_pass" else 0
    lz = l + e
    lq = lz + probe_rows
    W = sketch_w(A, rows, lq, seed, prec)
    Y = None
    if mode == "single_pass":
        Y = sketch_y(A, omega(seed, n, l, prec), prec)
    phase("sketch")
    cp = cpqr(W[:l], k, rank_tol)
    if probe_tol > 0.0:
        cp = adaptive_rank(cp, W[lz:], n, probe_tol)
    phase("mgsqr")
    Pk = id_coefficients(cp.R, cp.J, n)
    phase("coefficients")
    P = np.zeros((k, n))
    P[:cp.k_eff] = Pk
    J = np.full(k, -1, dtype=np.int64)
    J[:cp.k_eff] = cp.J
    err_sketch = _rel_fit(W[:l], W[:l][:, cp.J] @ Pk)
    if mode == "two_pass":
        AJ = np.asarray(A, dtype=np.float64)[:, cp.J]
        err_probe = _rel_fit(W[lz:], W[lz:][:, cp.J] @ Pk) if probe_rows else float("nan")
    elif mode == "single_pass":
        AJ, Zfull, X = skeleton_single_pass(Y, W, cp.J, lz, rows, seed, prec, sp_rcond)
        err_probe = _rel_fit(W[lz:], (Zfull[lz:] @ X) @ Pk) if probe_rows else float("nan")
    else:
        raise ValueError(mode)
    AJk = np.zeros((N, k))
    AJk[:, :cp.k_eff] = AJ
    phase("skeleton")
    return Result(J=J, P=P, AJ=AJk, k_eff=cp.k_eff, err_probe=err_probe,
                  err_sketch=err_sketch, W=W, Y=Y, cp=cp)


def refine(A, res: Result, seed: int, refine_prec: str, l: int, coarse_rows=None) -> np.ndarray:
    """Refinement of the coefficients P on a second, more precise sketch of
    A.  The paper stops at the ID; this is this implementation's reading of
    a refinement pass: the pivots J of the first sketch are kept and P is
    recomputed as the least-squares solution that defines it (the ID
    coefficients of Sec. 2.4 are R11^-1 R12, the least-squares fit of the
    sketch's columns by its pivot columns), now on the sketch
    W' = Psi_sel(:, S) A(S, :) taken in ``refine_prec``:

      P1 = argmin_X ||W'(:, J) X - W'||_F = W'(:, J)^+ W',  P1(:, J) = I.

    (A one-step correction that reuses the first sketch's R11 is cheaper but
    diverges when the first sketch's rounding, e.g. FP8, swamps the small
    singular values of R11.)  Returns P1 (k x n, rows past k_eff zero)."""
    A = np.asarray(A)
    N, n = A.shape
    rows = np.arange(N, dtype=np.int64) if coarse_rows is None else np.asarray(coarse_rows, np.int64)
    ke = res.k_eff
    J = res.cp.J
    Wp = sketch_w(A, rows, l, seed, refine_prec)
    X = np.linalg.lstsq(Wp[:, J], Wp, rcond=None)[0]
    X[:, J] = np.eye(ke)
    P1 = np.zeros_like(res.P)
    P1[:ke] = X
    return P1


def reconstruct(AJ: np.ndarray, P: np.ndarray) -> np.ndarray:
    """A_hat = A_J P (the ID of eq. (ID), transposed)."""
    return np.asarray(AJ, np.float64) @ np.asarray(P, np.float64)


def error_norms(A, AJ, P) -> dict:
    """Relative Frobenius error and relative max error of A ~ A_J P, entry by
    entry in FP64 without forming A_hat."""
    A = np.asfortranarray(np.asarray(A, dtype=np.float64))
    AJ = np.asfortranarray(np.asarray(AJ, dtype=np.float64))
    P = np.asfortranarray(np.asarray(P, dtype=np.float64))
    N, n = A.shape
    k = AJ.shape[1]
    out = np.zeros(4)
    lib().oracle_error_norms(_ptr(A), A.strides[1] // 8, _ptr(AJ), max(AJ.strides[1] // 8, 1),
                             _ptr(P), max(P.strides[1] // 8, 1), N, k, n, _ptr(out))
    fro_err, fro_a = np.sqrt(out[0]), np.sqrt(out[1])
    return dict(rel_fro=float(fro_err / fro_a) if fro_a > 0 else 0.0,
                fro_err=float(fro_err), fro_a=float(fro_a),
                rel_max=float(out[2]), max_abs=float(out[3]))


def compression_factor(N: int, n: int, k: int, n_coarse: int | None = None,
                       stencil: int = 0) -> float:
    """Entries of A over entries stored (Sec. 3.1).  ID stores k(N + n)
    (Table 1); storing the coarse skeleton (Alg. 6) stores k(N_c + n) + t N."""
    if n_coarse is None:
        return N * n / (k * (N + n))
    return N * n / (k * (n_coarse + n) + stencil * N)


def temporal_compression_factor(n: int, k: int) -> float:
    """Snapshots over target rank (Sec. 3.1)."""
    return n / k
