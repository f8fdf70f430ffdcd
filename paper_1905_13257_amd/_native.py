"""ctypes binding of libsid.so.  Argument marshalling only."""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIBPATH = os.path.join(_HERE, "libsid.so")
_LIB = None

SID_F64, SID_F32 = 0, 1
PRECISIONS = {"f64": 0, "f32": 1, "bf16": 2, "bf16x2": 3, "fp8": 4}
MODES = {"two_pass": 0, "single_pass": 1, "coarse_skeleton": 2}
SELECT = {"gauss": 0, "literal": 1}
_STATUS = {0: "SID_OK", -1: "SID_EINVAL", -2: "SID_ENOMEM", -3: "SID_EDEVICE",
           -4: "SID_ESTATE", -5: "SID_ENONFINITE", -6: "SID_ERANK"}

EXPORTS = [
    "sid_params_init", "sid_create", "sid_destroy", "sid_last_error", "sid_workspace_bytes",
    "sid_set_workspace_limit", "sid_rowset_create", "sid_rowset_destroy", "sid_reserve",
    "sid_compress", "sid_reconstruct", "sid_error_norms", "sid_fill_gaussian", "sid_sketch",
    "sid_stream_begin", "sid_stream_push", "sid_stream_finish", "sid_stream_info", "sid_stream_abort",
    "sid_stream_save", "sid_stream_restore", "sid_compress_batched", "sid_reserve_batched",
    "sid_batch_streams",
    "sid_interp_create", "sid_interp_destroy", "sid_interp_rowset", "sid_interp_info",
    "sid_interp_reconstruct", "sid_interp_error_norms", "sid_svd_params_init", "sid_sbr_svd",
    "sid_svd_stream_begin", "sid_svd_stream_finish", "sid_sync", "sid_sketch_noalloc", "sid_probe",
]


class SidError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{_STATUS.get(status, status)}: {msg}")
        self.status = status


class _Params(ctypes.Structure):
    _fields_ = [
        ("k", ctypes.c_int64),
        ("oversample", ctypes.c_int64),
        ("seed", ctypes.c_uint64),
        ("coarse", ctypes.c_void_p),
        ("mode", ctypes.c_int),
        ("prec", ctypes.c_int),
        ("probe_rows", ctypes.c_int32),
        ("corange_rows", ctypes.c_int32),
        ("rank_tol", ctypes.c_double),
        ("sp_rcond", ctypes.c_double),
        ("refine", ctypes.c_int32),
        ("refine_prec", ctypes.c_int),
        ("select", ctypes.c_int),
        ("probe_tol", ctypes.c_double),
    ]


class _SvdParams(ctypes.Structure):
    _fields_ = [
        ("k", ctypes.c_int64),
        ("oversample", ctypes.c_int64),
        ("block", ctypes.c_int64),
        ("seed", ctypes.c_uint64),
        ("prec", ctypes.c_int),
    ]


class _Mesh(ctypes.Structure):
    _fields_ = [
        ("ncomp", ctypes.c_int32),
        ("reserved", ctypes.c_int32),
        ("n", ctypes.c_int64 * 3),
        ("coord", ctypes.c_void_p * 3),
        ("coarse", ctypes.c_void_p * 3),
        ("ncoarse", ctypes.c_int64 * 3),
        ("period", ctypes.c_double * 3),
    ]


def library_path() -> str:
    return _LIBPATH


def load():
    """Load libsid.so; raises if it has not been built (no fallback path)."""
    global _LIB
    if _LIB is not None:
        return _LIB
    if not os.path.exists(_LIBPATH):
        raise ImportError(f"{_LIBPATH} is missing: build it with "
                          "`python -m paper_1905_13257_amd.build`")
    L = ctypes.CDLL(_LIBPATH)
    i64, u64, vp, dbl = ctypes.c_int64, ctypes.c_uint64, ctypes.c_void_p, ctypes.c_double
    pp = ctypes.POINTER(_Params)
    L.sid_params_init.argtypes = [pp, i64]
    L.sid_params_init.restype = None
    L.sid_create.argtypes = [ctypes.POINTER(vp), ctypes.c_int, vp]
    L.sid_destroy.argtypes = [vp]
    L.sid_last_error.argtypes = [vp]
    L.sid_last_error.restype = ctypes.c_char_p
    L.sid_workspace_bytes.argtypes = [vp]
    L.sid_workspace_bytes.restype = ctypes.c_size_t
    L.sid_set_workspace_limit.argtypes = [vp, ctypes.c_size_t]
    L.sid_sync.argtypes = [vp]
    L.sid_rowset_create.argtypes = [vp, vp, i64, i64, ctypes.POINTER(vp)]
    L.sid_rowset_destroy.argtypes = [vp]
    L.sid_reserve.argtypes = [vp, i64, i64, pp]
    L.sid_compress.argtypes = [vp, vp, ctypes.c_int, i64, i64, i64, pp, vp, vp, i64, vp, i64,
                               vp, vp]
    L.sid_reconstruct.argtypes = [vp, vp, i64, vp, i64, ctypes.c_int, i64, i64, i64, vp, i64]
    L.sid_error_norms.argtypes = [vp, vp, i64, vp, i64, vp, i64, ctypes.c_int, i64, i64, i64, vp]
    L.sid_fill_gaussian.argtypes = [vp, u64, ctypes.c_int, i64, i64, i64, i64, vp]
    L.sid_sketch.argtypes = [vp, vp, ctypes.c_int, i64, i64, i64, pp, vp, vp]
    L.sid_sketch_noalloc.argtypes = [vp, vp, ctypes.c_int, i64, i64, i64, pp, vp, vp]
    L.sid_stream_begin.argtypes = [vp, ctypes.c_int, i64, i64, pp, ctypes.POINTER(vp)]
    L.sid_stream_push.argtypes = [vp, vp, i64, i64]
    L.sid_stream_finish.argtypes = [vp, vp, vp, i64, vp, i64, vp, vp]
    L.sid_stream_abort.argtypes = [vp]
    L.sid_compress_batched.argtypes = [vp, vp, i64, ctypes.c_int]
    L.sid_reserve_batched.argtypes = [vp, vp, i64, ctypes.c_int, ctypes.c_int]
    L.sid_batch_streams.argtypes = [vp]
    L.sid_batch_streams.restype = ctypes.c_int
    L.sid_probe.argtypes = [vp, ctypes.c_int, vp, i64, i64]
    L.sid_stream_info.argtypes = [vp, ctypes.POINTER(i64), ctypes.POINTER(i64), ctypes.POINTER(i64),
                                  ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_int)]
    L.sid_stream_save.argtypes = [vp, vp, ctypes.POINTER(ctypes.c_size_t)]
    L.sid_stream_restore.argtypes = [vp, vp, ctypes.c_size_t, ctypes.POINTER(vp)]
    L.sid_svd_params_init.argtypes = [ctypes.POINTER(_SvdParams), i64]
    L.sid_svd_params_init.restype = None
    L.sid_sbr_svd.argtypes = [vp, vp, ctypes.c_int, i64, i64, i64, ctypes.POINTER(_SvdParams), vp,
                              vp, i64, vp, i64, ctypes.POINTER(i64)]
    L.sid_svd_stream_begin.argtypes = [vp, ctypes.c_int, i64, i64, ctypes.POINTER(_SvdParams),
                                       ctypes.POINTER(vp)]
    L.sid_svd_stream_finish.argtypes = [vp, vp, vp, i64, vp, i64, ctypes.POINTER(i64)]
    L.sid_interp_create.argtypes = [vp, ctypes.POINTER(_Mesh), ctypes.POINTER(vp)]
    L.sid_interp_destroy.argtypes = [vp]
    L.sid_interp_rowset.argtypes = [vp]
    L.sid_interp_rowset.restype = vp
    L.sid_interp_info.argtypes = [vp, ctypes.POINTER(i64), ctypes.POINTER(i64)]
    L.sid_interp_reconstruct.argtypes = [vp, vp, vp, i64, vp, i64, ctypes.c_int, i64, i64, vp,
                                         i64]
    L.sid_interp_error_norms.argtypes = [vp, vp, vp, i64, vp, i64, vp, i64, ctypes.c_int, i64,
                                         i64, vp]
    for name in ("sid_create", "sid_destroy", "sid_set_workspace_limit", "sid_rowset_create",
                 "sid_rowset_destroy", "sid_reserve", "sid_compress", "sid_reconstruct",
                 "sid_error_norms", "sid_fill_gaussian", "sid_sketch", "sid_stream_begin",
                 "sid_stream_push", "sid_stream_finish", "sid_stream_info", "sid_stream_abort",
                 "sid_stream_save", "sid_compress_batched",
                 "sid_stream_restore", "sid_interp_create", "sid_interp_destroy",
                 "sid_interp_info", "sid_interp_reconstruct", "sid_interp_error_norms",
                 "sid_sbr_svd", "sid_svd_stream_begin", "sid_svd_stream_finish"):
        getattr(L, name).restype = ctypes.c_int
    _LIB = L
    return L


def _ptr(t: torch.Tensor | None):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else ctypes.c_void_p(0)


def _colmajor(A: torch.Tensor) -> tuple[torch.Tensor, int]:
    """(tensor with stride (1, ld), ld) for a 2-D matrix."""
    if A.dim() != 2:
        raise ValueError("expected a 2-D matrix")
    if A.stride(0) == 1 and A.stride(1) >= max(A.shape[0], 1):
        return A, A.stride(1)
    B = torch.empty((A.shape[1], A.shape[0]), dtype=A.dtype, device=A.device).T
    B.copy_(A)
    return B, max(A.shape[0], 1)


def _dtype_code(t: torch.Tensor) -> int:
    if t.dtype == torch.float64:
        return SID_F64
    if t.dtype == torch.float32:
        return SID_F32
    raise TypeError("data must be float32 or float64")


class Context:
    """A libsid context bound to one device and one stream (default: the
    current torch stream of that device when the context is made)."""

    def __init__(self, device: int | None = None, stream: torch.cuda.Stream | None = None):
        L = load()
        if device is None:
            device = torch.cuda.current_device()
        if stream is None:
            stream = torch.cuda.current_stream(device)
        self.device = device
        self.stream = stream
        h = ctypes.c_void_p()
        st = L.sid_create(ctypes.byref(h), int(device), ctypes.c_void_p(stream.cuda_stream))
        if st != 0:
            raise SidError(st, "sid_create failed")
        self._h = h
        self._lib = L

    def check(self, st: int):
        if st != 0:
            raise SidError(st, self._lib.sid_last_error(self._h).decode())

    @property
    def handle(self):
        return self._h

    def workspace_bytes(self) -> int:
        return int(self._lib.sid_workspace_bytes(self._h))

    def set_workspace_limit(self, nbytes: int):
        self.check(self._lib.sid_set_workspace_limit(self._h, nbytes))

    def sync(self):
        """Wait for the context's work; raises if a device-side wait failed
        since the last sync (sid_sync)."""
        self.check(self._lib.sid_sync(self._h))

    def close(self):
        if getattr(self, "_h", None):
            self._lib.sid_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


_CTX: dict = {}


def default_context(device: torch.device | int | None = None) -> Context:
    dev = torch.device("cuda", torch.cuda.current_device()) if device is None else torch.device(device)
    idx = dev.index if dev.index is not None else torch.cuda.current_device()
    stream = torch.cuda.current_stream(idx)
    key = (idx, stream.cuda_stream)
    if key not in _CTX:
        _CTX[key] = Context(idx, stream)
    return _CTX[key]


def sync(device: torch.device | int | None = None):
    """sid_sync on the default context of `device` (current stream)."""
    default_context(device).sync()


class RowSet:
    """Coarse row set S (sorted, unique row indices of A), uploaded once."""

    def __init__(self, rows, N: int, ctx: Context | None = None):
        import numpy as np
        self.ctx = ctx or default_context()
        arr = np.ascontiguousarray(np.asarray(rows, dtype=np.int64))
        h = ctypes.c_void_p()
        self.ctx.check(self.ctx._lib.sid_rowset_create(
            self.ctx.handle, ctypes.c_void_p(arr.ctypes.data), arr.size, N, ctypes.byref(h)))
        self._h = h
        self.count = arr.size
        self.N = N

    def close(self):
        if getattr(self, "_h", None):
            self.ctx._lib.sid_rowset_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _params(k, oversample, seed, coarse, mode, prec, probe_rows, rank_tol, sp_rcond,
            corange_rows=-1, refine=False, refine_prec="bf16x2", select="gauss",
            probe_tol=0.0) -> _Params:
    p = _Params()
    load().sid_params_init(ctypes.byref(p), int(k))
    p.oversample = int(oversample)
    p.seed = int(seed)
    p.coarse = coarse._h if coarse is not None else None
    p.mode = MODES[mode]
    p.prec = PRECISIONS[prec]
    p.probe_rows = int(probe_rows)
    p.corange_rows = int(corange_rows)
    p.rank_tol = float(rank_tol)
    p.sp_rcond = float(sp_rcond)
    p.refine = 1 if refine else 0
    p.refine_prec = PRECISIONS[refine_prec]
    p.select = SELECT[select]
    p.probe_tol = float(probe_tol)
    return p


@dataclass
class Compressed:
    J: torch.Tensor          # int64 [k], pivot order, -1 past k_eff
    P: torch.Tensor          # k x n
    AJ: torch.Tensor | None  # N x k skeleton (copy or single-pass estimate)
    err: torch.Tensor        # float64 [2]: probe estimate, sketch residual
    k_eff: torch.Tensor      # int64 [1]; -1: a device-wide wait failed (invalid)

    def rank(self) -> int:
        """k_eff as an int (synchronizes); raises on a failed result."""
        r = int(self.k_eff.item())
        if r < 0:
            raise SidError(-3, "k_eff = -1: a device-wide wait of the pivoted QR timed out")
        return r


class _Problem(ctypes.Structure):
    _fields_ = [("A", ctypes.c_void_p), ("N", ctypes.c_int64), ("n", ctypes.c_int64),
                ("lda", ctypes.c_int64), ("params", _Params), ("J", ctypes.c_void_p),
                ("P", ctypes.c_void_p), ("ldp", ctypes.c_int64), ("AJ", ctypes.c_void_p),
                ("ldaj", ctypes.c_int64), ("err", ctypes.c_void_p), ("k_eff", ctypes.c_void_p)]


def _new_outputs(N: int, n: int, k: int, dtype, dev, want_skeleton: bool) -> Compressed:
    J = torch.empty(k, dtype=torch.int64, device=dev)
    P = torch.empty((n, k), dtype=dtype, device=dev).T
    AJ = torch.empty((k, N), dtype=dtype, device=dev).T if want_skeleton else None
    err = torch.empty(2, dtype=torch.float64, device=dev)
    keff = torch.empty(1, dtype=torch.int64, device=dev)
    return Compressed(J, P, AJ, err, keff)


class Batch:
    """A fixed set of problems for sid_compress_batched.  The problem table,
    the inputs and the outputs live as long as the object, so the call can be
    repeated, reserved ahead (reserve: sid_reserve_batched, optionally with
    the autotuner) and captured in a HIP graph (run under capture after
    reserve).  k, oversample, seed and probe_rows may be scalars or one value
    per matrix; all matrices share dtype, mode and precision."""

    def __init__(self, mats: list, k, oversample=10, seed=0, mode: str = "two_pass",
                 prec: str = "f32", probe_rows=10, rank_tol: float = 0.0, sp_rcond: float = 0.0,
                 want_skeleton: bool = True, ctx: Context | None = None,
                 probe_tol: float = 0.0):
        if not mats:
            raise ValueError("no matrices")
        self.ctx = ctx or default_context(mats[0].device)
        m = len(mats)
        per = lambda v: list(v) if isinstance(v, (list, tuple)) else [v] * m
        ks, ovs, seeds, qs = per(k), per(oversample), per(seed), per(probe_rows)
        dtype = mats[0].dtype
        self.dtype_code = _dtype_code(mats[0])
        self.probs = (_Problem * m)()
        self.keep, self.outs = [], []
        for b, A in enumerate(mats):
            if A.dtype != dtype:
                raise ValueError("all matrices must share one dtype")
            A, lda = _colmajor(A)
            N, n = A.shape
            o = _new_outputs(N, n, ks[b], dtype, A.device, want_skeleton)
            p = _params(ks[b], ovs[b], seeds[b], None, mode, prec, qs[b], rank_tol, sp_rcond,
                        probe_tol=probe_tol)
            self.probs[b] = _Problem(ctypes.c_void_p(A.data_ptr()), N, n, lda, p, _ptr(o.J),
                                     _ptr(o.P), o.P.stride(1), _ptr(o.AJ),
                                     o.AJ.stride(1) if o.AJ is not None else 1, _ptr(o.err),
                                     _ptr(o.k_eff))
            self.keep.append(A)
            self.outs.append(o)
        self.count = m

    def reserve(self, tune: bool = False) -> "Batch":
        """sid_reserve_batched: the plan, child streams and workspaces; with
        tune=True the autotuner times the stream counts on this batch."""
        self.ctx.check(self.ctx._lib.sid_reserve_batched(self.ctx.handle, self.probs, self.count,
                                                         self.dtype_code, 1 if tune else 0))
        return self

    def run(self) -> list:
        self.ctx.check(self.ctx._lib.sid_compress_batched(self.ctx.handle, self.probs, self.count,
                                                          self.dtype_code))
        return self.outs


def compress_batched(mats: list, k, oversample=10, seed=0, mode: str = "two_pass",
                     prec: str = "f32", probe_rows=10, rank_tol: float = 0.0,
                     sp_rcond: float = 0.0, want_skeleton: bool = True,
                     ctx: Context | None = None, probe_tol: float = 0.0) -> list:
    """Rank-k column IDs of several matrices in one call (sid_compress_batched).
    k, oversample, seed and probe_rows may be scalars or one value per matrix;
    all matrices share dtype, mode and precision."""
    if not mats:
        return []
    return Batch(mats, k, oversample, seed, mode, prec, probe_rows, rank_tol, sp_rcond,
                 want_skeleton, ctx, probe_tol).run()


PROBES = {"read": 0, "store_columns": 1, "store_sequential": 2, "mfma_16x16x32": 3,
          "mfma_32x32x16": 4}


def probe(kind: str, buf: torch.Tensor | None = None, rounds: int = 0,
          ctx: Context | None = None) -> None:
    """sid_probe: one launch of a measurement kernel (no part of the method).
    buf: an N x n FP32 column-major device matrix for the memory probes;
    rounds for the matrix-instruction probes."""
    ctx = ctx or default_context(torch.device("cuda"))
    code = PROBES[kind]
    if code <= 2:
        if buf is None or buf.dtype != torch.float32:
            raise ValueError("the memory probes take an FP32 device matrix")
        b, ld = _colmajor(buf)
        if ld != b.shape[0]:
            raise ValueError("probe buffer: contiguous columns")
        ctx.check(ctx._lib.sid_probe(ctx.handle, code, _ptr(b), b.shape[0], b.shape[1]))
    else:
        ctx.check(ctx._lib.sid_probe(ctx.handle, code, None, rounds, 1))


def batch_streams(ctx: Context | None = None) -> int:
    """Child streams the batched calls of ctx use (set by the autotuner)."""
    ctx = ctx or default_context(torch.device("cuda"))
    return int(ctx._lib.sid_batch_streams(ctx.handle))


def compress(A: torch.Tensor, k: int, oversample: int = 10, seed: int = 0,
             coarse: RowSet | None = None, mode: str = "two_pass", prec: str = "f32",
             probe_rows: int = 10, rank_tol: float = 0.0, sp_rcond: float = 0.0,
             corange_rows: int = -1, want_skeleton: bool = True, ctx: Context | None = None,
             out: Compressed | None = None, refine: bool = False,
             refine_prec: str = "bf16x2", select: str = "gauss",
             probe_tol: float = 0.0) -> Compressed:
    """Rank-k column ID of A (N x n, float32/float64 on the GPU); refine=True
    adds one refinement pass of P on a refine_prec sketch; select="literal"
    runs mgsqr on the coarse rows A(S, :) themselves (Alg. 5 as written);
    probe_tol > 0 picks the smallest rank <= k whose probe estimate meets it
    (out.k_eff)."""
    ctx = ctx or default_context(A.device)
    A, lda = _colmajor(A)
    N, n = A.shape
    dev = A.device
    if out is None:
        J = torch.empty(k, dtype=torch.int64, device=dev)
        P = torch.empty((n, k), dtype=A.dtype, device=dev).T
        # the coarse skeleton (Alg. 6) has the coarse rows only
        rows = coarse.count if (mode == "coarse_skeleton" and coarse is not None) else N
        AJ = torch.empty((k, rows), dtype=A.dtype, device=dev).T if want_skeleton else None
        err = torch.empty(2, dtype=torch.float64, device=dev)
        keff = torch.empty(1, dtype=torch.int64, device=dev)
        out = Compressed(J, P, AJ, err, keff)
    p = _params(k, oversample, seed, coarse, mode, prec, probe_rows, rank_tol, sp_rcond,
                corange_rows, refine, refine_prec, select, probe_tol)
    ldaj = out.AJ.stride(1) if out.AJ is not None else 1
    ctx.check(ctx._lib.sid_compress(
        ctx.handle, _ptr(A), _dtype_code(A), N, n, lda, ctypes.byref(p), _ptr(out.J),
        _ptr(out.P), out.P.stride(1), _ptr(out.AJ), ldaj, _ptr(out.err), _ptr(out.k_eff)))
    return out


def reserve(N: int, n: int, k: int, oversample: int = 10, mode: str = "two_pass",
            prec: str = "f32", probe_rows: int = 10, coarse: RowSet | None = None,
            corange_rows: int = -1, refine: bool = False, refine_prec: str = "bf16x2",
            select: str = "gauss", probe_tol: float = 0.0,
            ctx: Context | None = None) -> None:
    """Allocate ahead of time everything a compress of this shape needs
    (sid_reserve); later compress calls allocate nothing (graph capture)."""
    ctx = ctx or default_context()
    p = _params(k, oversample, 0, coarse, mode, prec, probe_rows, 0.0, 0.0, corange_rows,
                refine, refine_prec, select, probe_tol)
    ctx.check(ctx._lib.sid_reserve(ctx.handle, N, n, ctypes.byref(p)))


def sketch(A: torch.Tensor, k: int, oversample: int = 10, seed: int = 0,
           coarse: RowSet | None = None, prec: str = "f32", probe_rows: int = 10,
           want_y: bool = True, corange_rows: int = -1, ctx: Context | None = None):
    """W = Psi(:, S) A(S, :) (lw x n, float64; lw = l + e + q with the
    single-pass co-range rows e when want_y) and Y = A Omega (N x l)."""
    ctx = ctx or default_context(A.device)
    A, lda = _colmajor(A)
    N, n = A.shape
    l = k + oversample
    e = (oversample if corange_rows < 0 else corange_rows) if want_y else 0
    lq = l + e + probe_rows
    W = torch.empty((n, lq), dtype=torch.float64, device=A.device).T
    Y = None
    if want_y:
        ydt = torch.float64 if prec == "f64" else torch.float32
        Y = torch.empty((N, l), dtype=ydt, device=A.device)
    p = _params(k, oversample, seed, coarse, "single_pass" if want_y else "two_pass", prec,
                probe_rows, 0.0, 0.0, corange_rows)
    ctx.check(ctx._lib.sid_sketch(ctx.handle, _ptr(A), _dtype_code(A), N, n, lda,
                                  ctypes.byref(p), _ptr(W), _ptr(Y)))
    return W, Y


def sketch_noalloc(A: torch.Tensor, k: int, W: torch.Tensor, Y: torch.Tensor | None = None,
                   oversample: int = 10, seed: int = 0, prec: str = "bf16x2",
                   probe_rows: int = 10, corange_rows: int = -1, ctx: Context | None = None):
    """sid_sketch_noalloc: sid_sketch without any allocation (scratch in the
    library's static device array).  The caller passes the outputs: W (lw x n
    float64, column-major, lw = l + e + q with e only when Y is given) and
    optionally Y (N x l float32, row-major)."""
    ctx = ctx or default_context(A.device)
    if A.stride(0) != 1:
        raise ValueError("A must be column-major")
    N, n = A.shape
    p = _params(k, oversample, seed, None, "single_pass" if Y is not None else "two_pass", prec,
                probe_rows, 0.0, 0.0, corange_rows)
    ctx.check(ctx._lib.sid_sketch_noalloc(ctx.handle, _ptr(A), _dtype_code(A), N, n, A.stride(1),
                                          ctypes.byref(p), _ptr(W), _ptr(Y)))
    return W, Y


def reconstruct(AJ: torch.Tensor, P: torch.Tensor, out: torch.Tensor | None = None,
                ctx: Context | None = None) -> torch.Tensor:
    """Ahat = AJ P (N x n)."""
    ctx = ctx or default_context(AJ.device)
    AJ, ldaj = _colmajor(AJ)
    P, ldp = _colmajor(P.to(AJ.dtype))
    N, k = AJ.shape
    n = P.shape[1]
    if out is None:
        out = torch.empty((n, N), dtype=AJ.dtype, device=AJ.device).T
    ctx.check(ctx._lib.sid_reconstruct(ctx.handle, _ptr(AJ), ldaj, _ptr(P), ldp,
                                       _dtype_code(AJ), N, k, n, _ptr(out), out.stride(1)))
    return out


def error_norms(A: torch.Tensor, AJ: torch.Tensor, P: torch.Tensor,
                ctx: Context | None = None) -> dict:
    """||A - AJ P||_F, ||A||_F, relative max error, max abs error (FP64)."""
    ctx = ctx or default_context(A.device)
    A, lda = _colmajor(A)
    AJ, ldaj = _colmajor(AJ.to(A.dtype))
    P, ldp = _colmajor(P.to(A.dtype))
    N, n = A.shape
    k = AJ.shape[1]
    out = (ctypes.c_double * 4)()
    ctx.check(ctx._lib.sid_error_norms(ctx.handle, _ptr(A), lda, _ptr(AJ), ldaj, _ptr(P), ldp,
                                       _dtype_code(A), N, k, n, out))
    fe, fa = out[0], out[1]
    return dict(fro_err=fe, fro_a=fa, rel_fro=fe / fa if fa > 0 else 0.0, rel_max=out[2],
                max_abs=out[3])


def fill_gaussian(seed: int, stream: int, major0: int, nmajor: int, minor0: int, nminor: int,
                  device=None, ctx: Context | None = None) -> torch.Tensor:
    """The generator's entries G(seed, stream, major, minor) as a
    (nmajor, nminor) float32 tensor on the GPU."""
    ctx = ctx or default_context(device)
    out = torch.empty((nmajor, nminor), dtype=torch.float32, device=torch.device("cuda", ctx.device))
    ctx.check(ctx._lib.sid_fill_gaussian(ctx.handle, int(seed), int(stream), major0, nmajor,
                                         minor0, nminor, _ptr(out)))
    return out


class Stream:
    """Streaming compression: push column blocks, then finish (sid_stream_*).
    J indexes columns in arrival order."""

    def __init__(self, N: int, n_max: int, k: int, oversample: int = 10, seed: int = 0,
                 dtype: torch.dtype = torch.float32, mode: str = "single_pass",
                 prec: str = "f32", probe_rows: int = 10, rank_tol: float = 0.0,
                 sp_rcond: float = 0.0, corange_rows: int = -1, coarse: RowSet | None = None,
                 ctx: Context | None = None, probe_tol: float = 0.0):
        self.ctx = ctx or default_context()
        self.N, self.k, self.dtype = N, k, dtype
        self.mode = mode
        self.coarse = coarse  # kept alive with the stream
        p = _params(k, oversample, seed, coarse, mode, prec, probe_rows, rank_tol, sp_rcond,
                    corange_rows, probe_tol=probe_tol)
        h = ctypes.c_void_p()
        code = SID_F64 if dtype == torch.float64 else SID_F32
        self.ctx.check(self.ctx._lib.sid_stream_begin(self.ctx.handle, code, N, n_max,
                                                      ctypes.byref(p), ctypes.byref(h)))
        self._h = h

    def push(self, block: torch.Tensor):
        """block: N x c (any strides; copied to column-major if needed)."""
        B, ld = _colmajor(block.to(self.dtype))
        if B.shape[0] != self.N:
            raise ValueError("block must have N rows")
        self.ctx.check(self.ctx._lib.sid_stream_push(self._h, _ptr(B), B.shape[1], ld))
        # the library reads B on the context's stream; keep it alive until then
        self._last = B

    def save(self) -> bytes:
        nb = ctypes.c_size_t(0)
        self.ctx.check(self.ctx._lib.sid_stream_save(self._h, None, ctypes.byref(nb)))
        buf = ctypes.create_string_buffer(nb.value)
        self.ctx.check(self.ctx._lib.sid_stream_save(self._h, buf, ctypes.byref(nb)))
        return buf.raw[:nb.value]

    def info(self) -> dict:
        N, cols, k = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64()
        dt, md = ctypes.c_int(), ctypes.c_int()
        self.ctx.check(self.ctx._lib.sid_stream_info(self._h, ctypes.byref(N), ctypes.byref(cols),
                                                     ctypes.byref(k), ctypes.byref(dt),
                                                     ctypes.byref(md)))
        return dict(N=N.value, cols=cols.value, k=k.value,
                    dtype=torch.float64 if dt.value == SID_F64 else torch.float32,
                    mode={v: kk for kk, v in MODES.items()}[md.value])

    @classmethod
    def restore(cls, state: bytes, ctx: Context | None = None) -> "Stream":
        ctx = ctx or default_context()
        h = ctypes.c_void_p()
        buf = ctypes.create_string_buffer(state, len(state))
        ctx.check(ctx._lib.sid_stream_restore(ctx.handle, buf, len(state), ctypes.byref(h)))
        obj = cls.__new__(cls)
        obj.ctx, obj._h, obj.coarse = ctx, h, None
        inf = obj.info()
        obj.N, obj.k, obj.dtype, obj.mode = inf["N"], inf["k"], inf["dtype"], inf["mode"]
        return obj

    def finish(self, want_skeleton: bool = True) -> Compressed:
        dev = torch.device("cuda", self.ctx.device)
        k, N = self.k, self.N
        n = self.info()["cols"]
        J = torch.empty(k, dtype=torch.int64, device=dev)
        P = torch.empty((n, k), dtype=self.dtype, device=dev).T
        AJ = (torch.empty((k, N), dtype=self.dtype, device=dev).T
              if want_skeleton and self.mode == "single_pass" else None)
        err = torch.empty(2, dtype=torch.float64, device=dev)
        keff = torch.empty(1, dtype=torch.int64, device=dev)
        h, self._h = self._h, None
        self.ctx.check(self.ctx._lib.sid_stream_finish(
            h, _ptr(J), _ptr(P), P.stride(1), _ptr(AJ), AJ.stride(1) if AJ is not None else 1,
            _ptr(err), _ptr(keff)))
        return Compressed(J, P, AJ, err, keff)

    def close(self):
        if getattr(self, "_h", None):
            self.ctx._lib.sid_stream_abort(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class _BorrowedRowSet:
    """A row set owned by another object (an Interp's coarse rows)."""

    def __init__(self, h, count: int, N: int, owner):
        self._h, self.count, self.N, self._owner = h, count, N, owner


class Interp:
    """Structured grid and coarse subset for the single-pass ID with
    interpolation (Alg. 6): the trilinear coarse-to-fine operator Mf and the
    coarse row set S (``rowset``, for compress(..., coarse=...)).

    ``mesh`` has attributes ncomp, n (3 sizes), coords (3 arrays or None),
    coarse (3 index arrays) and period (3 floats, 0 = bounded)."""

    def __init__(self, mesh, ctx: Context | None = None):
        import numpy as np
        self.ctx = ctx or default_context()
        m = _Mesh()
        m.ncomp = int(mesh.ncomp)
        m.reserved = 0
        keep = []
        for d in range(3):
            m.n[d] = int(mesh.n[d])
            c = np.ascontiguousarray(np.asarray(mesh.coarse[d], dtype=np.int64))
            keep.append(c)
            m.coarse[d] = c.ctypes.data
            m.ncoarse[d] = c.size
            x = mesh.coords[d] if mesh.coords is not None else None
            if x is None:
                m.coord[d] = None
            else:
                xa = np.ascontiguousarray(np.asarray(x, dtype=np.float64))
                keep.append(xa)
                m.coord[d] = xa.ctypes.data
            m.period[d] = float(mesh.period[d]) if mesh.period is not None else 0.0
        h = ctypes.c_void_p()
        self.ctx.check(self.ctx._lib.sid_interp_create(self.ctx.handle, ctypes.byref(m),
                                                       ctypes.byref(h)))
        self._h = h
        N, Nc = ctypes.c_int64(), ctypes.c_int64()
        self.ctx.check(self.ctx._lib.sid_interp_info(h, ctypes.byref(N), ctypes.byref(Nc)))
        self.N, self.Nc = N.value, Nc.value
        self.rowset = _BorrowedRowSet(ctypes.c_void_p(self.ctx._lib.sid_interp_rowset(h)),
                                      self.Nc, self.N, self)

    def close(self):
        if getattr(self, "_h", None):
            self.ctx._lib.sid_interp_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def interp_reconstruct(ip: Interp, ACJ: torch.Tensor, P: torch.Tensor,
                       out: torch.Tensor | None = None, ctx: Context | None = None) -> torch.Tensor:
    """Ahat = Mf ACJ P (N x n) from the coarse skeleton ACJ (Nc x k)."""
    ctx = ctx or ip.ctx
    ACJ, ldc = _colmajor(ACJ)
    P, ldp = _colmajor(P.to(ACJ.dtype))
    k = ACJ.shape[1]
    n = P.shape[1]
    if out is None:
        out = torch.empty((n, ip.N), dtype=ACJ.dtype, device=ACJ.device).T
    ctx.check(ctx._lib.sid_interp_reconstruct(ctx.handle, ip._h, _ptr(ACJ), ldc, _ptr(P), ldp,
                                              _dtype_code(ACJ), k, n, _ptr(out), out.stride(1)))
    return out


def interp_error_norms(ip: Interp, A: torch.Tensor, ACJ: torch.Tensor, P: torch.Tensor,
                       ctx: Context | None = None) -> dict:
    """Errors of Mf ACJ P against A without forming it (as error_norms)."""
    ctx = ctx or ip.ctx
    A, lda = _colmajor(A)
    ACJ, ldc = _colmajor(ACJ.to(A.dtype))
    P, ldp = _colmajor(P.to(A.dtype))
    k = ACJ.shape[1]
    n = A.shape[1]
    out = (ctypes.c_double * 4)()
    ctx.check(ctx._lib.sid_interp_error_norms(ctx.handle, ip._h, _ptr(A), lda, _ptr(ACJ), ldc,
                                              _ptr(P), ldp, _dtype_code(A), k, n, out))
    fe, fa = out[0], out[1]
    return dict(fro_err=fe, fro_a=fa, rel_fro=fe / fa if fa > 0 else 0.0, rel_max=out[2],
                max_abs=out[3])


@dataclass
class SVD:
    U: torch.Tensor   # n x k temporal factor
    S: torch.Tensor   # k singular values (float64), descending
    V: torch.Tensor   # N x k spatial factor (A ~ V diag(S) U^T)
    rank: int         # rows of B formed (k + oversample unless A has lower rank)


def _svd_params(ctx: Context, k: int, oversample: int, block: int, seed: int,
                prec: str) -> "_SvdParams":
    p = _SvdParams()
    ctx._lib.sid_svd_params_init(ctypes.byref(p), int(k))
    p.oversample, p.block, p.seed, p.prec = int(oversample), int(block), int(seed), PRECISIONS[prec]
    return p


class SvdStream:
    """SBR-SVD over column blocks pushed in arrival order (Alg. 2's single
    pass; sid_svd_stream_begin, sid_stream_push, sid_svd_stream_finish)."""

    def __init__(self, N: int, n_max: int, k: int, oversample: int = 10, block: int = 10,
                 seed: int = 0, prec: str = "f64", dtype: torch.dtype = torch.float32,
                 ctx: Context | None = None):
        self.ctx = ctx or default_context()
        self.N, self.k, self.dtype = N, k, dtype
        p = _svd_params(self.ctx, k, oversample, block, seed, prec)
        h = ctypes.c_void_p()
        code = SID_F64 if dtype == torch.float64 else SID_F32
        self.ctx.check(self.ctx._lib.sid_svd_stream_begin(self.ctx.handle, code, N, n_max,
                                                          ctypes.byref(p), ctypes.byref(h)))
        self._h = h
        self._keep = []

    def push(self, block: torch.Tensor):
        """block: N x c (any strides; copied to column-major if needed)."""
        B, ld = _colmajor(block.to(self.dtype))
        if B.shape[0] != self.N:
            raise ValueError("block must have N rows")
        self.ctx.check(self.ctx._lib.sid_stream_push(self._h, _ptr(B), B.shape[1], ld))
        self._keep.append(B)  # read on the context's stream; kept until finish

    def cols(self) -> int:
        c = ctypes.c_int64()
        self.ctx.check(self.ctx._lib.sid_stream_info(self._h, None, ctypes.byref(c), None, None,
                                                     None))
        return c.value

    def finish(self) -> SVD:
        dev = torch.device("cuda", self.ctx.device)
        k, N, n = self.k, self.N, self.cols()
        S = torch.empty(k, dtype=torch.float64, device=dev)
        U = torch.empty((k, n), dtype=self.dtype, device=dev).T
        V = torch.empty((k, N), dtype=self.dtype, device=dev).T
        rank = ctypes.c_int64(0)
        h, self._h = self._h, None
        self.ctx.check(self.ctx._lib.sid_svd_stream_finish(h, _ptr(S), _ptr(U), U.stride(1),
                                                           _ptr(V), V.stride(1),
                                                           ctypes.byref(rank)))
        self._keep = []
        return SVD(U=U, S=S, V=V, rank=int(rank.value))

    def close(self):
        if getattr(self, "_h", None):
            self.ctx._lib.sid_stream_abort(self._h)
            self._h = None
        self._keep = []

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def sbr_svd(A: torch.Tensor, k: int, oversample: int = 10, block: int = 10, seed: int = 0,
            prec: str = "f64", ctx: Context | None = None) -> SVD:
    """Single-pass blocked randomized SVD (Alg. 2) of A (N x n, snapshots as
    columns): A ~ V diag(S) U^T (sid_sbr_svd).  `prec` is the arithmetic of
    the pass forming G; H and the block loop are FP64 whatever it is."""
    ctx = ctx or default_context(A.device)
    A, lda = _colmajor(A)
    N, n = A.shape
    p = _svd_params(ctx, k, oversample, block, seed, prec)
    dev = A.device
    S = torch.empty(k, dtype=torch.float64, device=dev)
    U = torch.empty((k, n), dtype=A.dtype, device=dev).T
    V = torch.empty((k, N), dtype=A.dtype, device=dev).T
    rank = ctypes.c_int64(0)
    ctx.check(ctx._lib.sid_sbr_svd(ctx.handle, _ptr(A), _dtype_code(A), N, n, lda, ctypes.byref(p),
                                   _ptr(S), _ptr(U), U.stride(1), _ptr(V), V.stride(1),
                                   ctypes.byref(rank)))
    return SVD(U=U, S=S, V=V, rank=int(rank.value))
