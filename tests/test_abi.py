"""C ABI checks that need no GPU: the library loads, exports every function
include/sid.h declares, and rejects bad arguments with the documented status
codes (through a validation-only context, device -1)."""
import ctypes
import os
import re

import numpy as np
import pytest

import paper_1905_13257_amd as sid
from paper_1905_13257_amd import _native

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
EINVAL, ENOMEM, EDEVICE, ESTATE = -1, -2, -3, -4


def declared_functions():
    text = open(os.path.join(ROOT, "include", "sid.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(sid_[a-z0-9_]+)\s*\(", text)))


def test_exports_match_header():
    L = sid.load()
    names = declared_functions()
    assert len(names) >= 14
    for name in names:
        assert hasattr(L, name), name
    assert set(names) == set(_native.EXPORTS)


@pytest.fixture()
def vctx():
    L = sid.load()
    h = ctypes.c_void_p()
    assert L.sid_create(ctypes.byref(h), -1, None) == 0
    yield L, h
    assert L.sid_destroy(h) == 0


def _params(L, k=5, **kw):
    p = _native._Params()
    L.sid_params_init(ctypes.byref(p), k)
    for key, v in kw.items():
        setattr(p, key, v)
    return p


def _compress(L, h, N=100, n=20, lda=100, p=None, A=1, dtype=1, J=None, P=None, ldp=5, AJ=None,
              ldaj=100):
    vp = ctypes.c_void_p
    return L.sid_compress(h, vp(A), dtype, N, n, lda, ctypes.byref(p), vp(J), vp(P), ldp,
                          vp(AJ), ldaj, vp(0), vp(0))


def test_defaults(vctx):
    L, h = vctx
    p = _params(L, 7)
    assert (p.k, p.oversample, p.seed, p.mode, p.prec, p.probe_rows, p.corange_rows) == \
        (7, 10, 0, 0, 1, 10, -1)
    assert p.rank_tol == 0.0 and p.sp_rcond == 0.0


@pytest.mark.parametrize("kw,args,code", [
    (dict(k=0), {}, EINVAL),                       # k >= 1
    (dict(k=30), dict(n=20), EINVAL),              # k <= n
    (dict(oversample=-1), {}, EINVAL),
    (dict(probe_rows=-2), {}, EINVAL),
    (dict(mode=7), {}, EINVAL),
    (dict(prec=9), {}, EINVAL),
    (dict(rank_tol=-1.0), {}, EINVAL),
    (dict(k=5, oversample=300), {}, EINVAL),       # sketch rows <= 256
    ({}, dict(N=0), EINVAL),
    ({}, dict(n=0), EINVAL),
    ({}, dict(lda=50), EINVAL),                    # lda >= N
    ({}, dict(A=0), EINVAL),                       # A non-NULL
    ({}, dict(dtype=5), EINVAL),
    ({}, dict(P=1, ldp=3), EINVAL),                # ldp >= k
    ({}, dict(AJ=1, ldaj=10), EINVAL),             # ldaj >= N
    ({}, {}, ESTATE),                              # valid -> no device to launch on
])
def test_compress_validation(vctx, kw, args, code):
    L, h = vctx
    p = _params(L, **({"k": 5} | kw))
    st = _compress(L, h, p=p, **args)
    assert st == code, L.sid_last_error(h)
    assert L.sid_last_error(h)


def test_rowset_validation(vctx):
    L, h = vctx
    out = ctypes.c_void_p()
    rows = np.array([0, 3, 3, 9], dtype=np.int64)
    assert L.sid_rowset_create(h, ctypes.c_void_p(rows.ctypes.data), 4, 10, ctypes.byref(out)) == EINVAL
    rows = np.array([0, 3, 12], dtype=np.int64)
    assert L.sid_rowset_create(h, ctypes.c_void_p(rows.ctypes.data), 3, 10, ctypes.byref(out)) == EINVAL
    rows = np.array([-1, 3], dtype=np.int64)
    assert L.sid_rowset_create(h, ctypes.c_void_p(rows.ctypes.data), 2, 10, ctypes.byref(out)) == EINVAL
    rows = np.array([1, 3, 5], dtype=np.int64)
    assert L.sid_rowset_create(h, ctypes.c_void_p(rows.ctypes.data), 3, 10, ctypes.byref(out)) == ESTATE
    assert L.sid_rowset_create(h, None, 3, 10, ctypes.byref(out)) == EINVAL


def test_other_calls_validate(vctx):
    L, h = vctx
    vp = ctypes.c_void_p
    assert L.sid_reconstruct(h, vp(0), 10, vp(1), 3, 1, 10, 3, 5, vp(1), 10) == EINVAL
    assert L.sid_reconstruct(h, vp(1), 5, vp(1), 3, 1, 10, 3, 5, vp(1), 10) == EINVAL
    assert L.sid_reconstruct(h, vp(1), 10, vp(1), 3, 1, 10, 3, 5, vp(1), 10) == ESTATE
    out = (ctypes.c_double * 4)()
    assert L.sid_error_norms(h, vp(1), 10, vp(1), 10, vp(1), 3, 1, 10, 3, 5, None) == EINVAL
    assert L.sid_error_norms(h, vp(1), 10, vp(1), 10, vp(1), 3, 1, 10, 3, 5, out) == ESTATE
    assert L.sid_fill_gaussian(h, 0, -1, 0, 4, 0, 4, vp(1)) == EINVAL
    assert L.sid_fill_gaussian(h, 0, 0, 0, 4, 0, 4, vp(1)) == ESTATE
    p = _params(L, 5)
    assert L.sid_reserve(h, 100, 20, ctypes.byref(p)) == ESTATE
    assert L.sid_reserve(h, 100, 2, ctypes.byref(p)) == EINVAL
    assert L.sid_sketch(h, vp(1), 1, 100, 20, 100, ctypes.byref(p), vp(0), vp(0)) == EINVAL
    assert L.sid_set_workspace_limit(h, 1 << 20) == 0
    assert L.sid_workspace_bytes(h) == 0
    assert L.sid_create(None, 0, None) == EINVAL


def test_stream_calls_validate(vctx):
    """Streaming entry points: parameters are checked before any device
    work; a NULL stream and a buffer that is not a saved state are rejected."""
    L, h = vctx
    vp = ctypes.c_void_p
    p = _params(L, 5)
    out = vp()
    assert L.sid_stream_begin(h, 1, 100, 20, ctypes.byref(p), ctypes.byref(out)) == ESTATE
    assert L.sid_stream_begin(h, 1, 100, 2, ctypes.byref(p), ctypes.byref(out)) == EINVAL   # k > n_max
    assert L.sid_stream_begin(h, 7, 100, 20, ctypes.byref(p), ctypes.byref(out)) == EINVAL  # dtype
    assert L.sid_stream_begin(h, 1, 100, 20, ctypes.byref(p), None) == EINVAL
    assert L.sid_stream_push(None, vp(1), 3, 100) == EINVAL
    assert L.sid_stream_finish(None, None, None, 1, None, 1, None, None) == EINVAL
    assert L.sid_stream_abort(None) == EINVAL
    assert L.sid_stream_info(None, None, None, None, None, None) == EINVAL
    nb = ctypes.c_size_t(0)
    assert L.sid_stream_save(None, None, ctypes.byref(nb)) == EINVAL
    junk = ctypes.create_string_buffer(b"not a stream state" * 10)
    assert L.sid_stream_restore(h, junk, 180, ctypes.byref(out)) == EINVAL
    assert L.sid_stream_restore(h, junk, 4, ctypes.byref(out)) == EINVAL


def test_problem_struct_layout(tmp_path):
    """The binding's sid_problem / sid_params mirror the C layout (sizes and
    field offsets from a C compiler)."""
    import shutil
    import subprocess
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no C compiler")
    src = tmp_path / "lay.c"
    src.write_text('#include <stddef.h>\n#include <stdio.h>\n#include "sid.h"\nint main(void){\n'
                   'printf("%zu %zu %zu %zu %zu %zu\\n", sizeof(sid_params), sizeof(sid_problem),'
                   ' offsetof(sid_problem, params), offsetof(sid_problem, J),'
                   ' offsetof(sid_problem, ldaj), offsetof(sid_problem, k_eff));\nreturn 0;}\n')
    exe = tmp_path / "lay"
    subprocess.check_call([cc, "-I", os.path.join(ROOT, "include"), "-o", str(exe), str(src)])
    got = [int(v) for v in subprocess.check_output([str(exe)]).split()]
    P = _native._Problem
    assert got == [ctypes.sizeof(_native._Params), ctypes.sizeof(P), P.params.offset, P.J.offset,
                   P.ldaj.offset, P.k_eff.offset]


def test_batched_validates_every_problem_first(vctx):
    L, h = vctx
    probs = (_native._Problem * 3)()
    for b in range(3):
        L.sid_params_init(ctypes.byref(probs[b].params), 5)
        probs[b].A, probs[b].N, probs[b].n, probs[b].lda = 1, 100, 20, 100
    assert L.sid_compress_batched(h, probs, 3, 1) == ESTATE
    assert L.sid_compress_batched(h, probs, 0, 1) == 0
    assert L.sid_compress_batched(h, None, 3, 1) == EINVAL
    probs[2].n = 3                      # k = 5 > n
    assert L.sid_compress_batched(h, probs, 3, 1) == EINVAL
    assert b"problem 2" in L.sid_last_error(h)
    probs[2].n = 20
    probs[1].lda = 50                   # lda < N
    assert L.sid_compress_batched(h, probs, 3, 1) == EINVAL
    assert b"problem 1" in L.sid_last_error(h)


def test_refine_validation(vctx):
    L, h = vctx
    vp = ctypes.c_void_p
    p = _params(L, 5)
    p.refine = 2
    assert L.sid_reserve(h, 100, 20, ctypes.byref(p)) == EINVAL
    p.refine, p.refine_prec = 1, 9
    assert L.sid_reserve(h, 100, 20, ctypes.byref(p)) == EINVAL
    p.refine_prec = 3
    assert L.sid_reserve(h, 100, 20, ctypes.byref(p)) == ESTATE
    out = vp()
    assert L.sid_stream_begin(h, 1, 100, 20, ctypes.byref(p), ctypes.byref(out)) == EINVAL
    q = _params(L, 5)
    assert q.refine == 0 and q.refine_prec == 3


def test_literal_select_validation(vctx):
    """Literal (Alg. 5) selection: needs a coarse set, two-pass, F64/F32, at
    most 4096 coarse rows, no refinement, no stream; unknown select rejected."""
    L, h = vctx
    p = _params(L, 5)
    assert p.select == 0
    p.select = 1
    assert L.sid_reserve(h, 100, 20, ctypes.byref(p)) == EINVAL       # no coarse set
    assert b"coarse" in L.sid_last_error(h)
    p.select = 7
    assert L.sid_reserve(h, 100, 20, ctypes.byref(p)) == EINVAL
    out = ctypes.c_void_p()
    p.select = 1
    assert L.sid_stream_begin(h, 1, 100, 20, ctypes.byref(p), ctypes.byref(out)) == EINVAL


def _mesh(n=(6, 5, 4), coarse=((0, 2, 4), (0, 2, 4), (0, 3)), coords=(None, None, None),
          period=(0.0, 0.0, 0.0), ncomp=2):
    m = _native._Mesh()
    m.ncomp = ncomp
    keep = []
    for d in range(3):
        m.n[d] = n[d]
        c = np.asarray(coarse[d], dtype=np.int64)
        keep.append(c)
        m.coarse[d] = c.ctypes.data
        m.ncoarse[d] = c.size
        if coords[d] is not None:
            x = np.asarray(coords[d], dtype=np.float64)
            keep.append(x)
            m.coord[d] = x.ctypes.data
        m.period[d] = period[d]
    return m, keep


@pytest.mark.parametrize("kw,code", [
    ({}, ESTATE),                                                   # valid: no device
    (dict(ncomp=0), EINVAL),
    (dict(coarse=((0, 2, 2), (0, 2, 4), (0, 3))), EINVAL),          # not increasing
    (dict(coarse=((0, 2, 6), (0, 2, 4), (0, 3))), EINVAL),          # out of range
    (dict(coarse=((), (0, 2, 4), (0, 3))), EINVAL),                 # empty
    (dict(coords=((0, 1, 2, 2, 4, 5), None, None)), EINVAL),        # coordinates not increasing
    (dict(period=(4.0, 0.0, 0.0)), EINVAL),                         # coarse span 4 >= period
    (dict(period=(4.5, 0.0, -1.0)), EINVAL),                        # negative period
    (dict(period=(4.5, 0.0, 0.0)), ESTATE),                         # periodic x, valid
    (dict(n=(1 << 20, 1 << 10, 4), coarse=((0,), (0,), (0,))), EINVAL),  # N >= 2^31
])
def test_interp_mesh_validation(vctx, kw, code):
    """The structured grid of Alg. 6 is checked on the host before anything
    touches a device."""
    L, h = vctx
    m, keep = _mesh(**kw)
    out = ctypes.c_void_p()
    assert L.sid_interp_create(h, ctypes.byref(m), ctypes.byref(out)) == code, L.sid_last_error(h)
    m.reserved = 1
    assert L.sid_interp_create(h, ctypes.byref(m), ctypes.byref(out)) == EINVAL


def test_interp_calls_validate(vctx):
    L, h = vctx
    vp = ctypes.c_void_p
    out4 = (ctypes.c_double * 4)()
    assert L.sid_interp_reconstruct(h, None, vp(1), 10, vp(1), 3, 1, 3, 5, vp(1), 10) == EINVAL
    assert L.sid_interp_error_norms(h, None, vp(1), 10, vp(1), 10, vp(1), 3, 1, 3, 5,
                                    out4) == EINVAL
    assert L.sid_interp_destroy(None) == EINVAL
    assert L.sid_interp_info(None, None, None) == EINVAL
    assert L.sid_interp_rowset(None) is None
    assert L.sid_interp_create(h, None, ctypes.byref(vp())) == EINVAL


def test_coarse_skeleton_mode_validation(vctx):
    """Alg. 6 mode: needs a coarse row set and is not streamed."""
    L, h = vctx
    p = _params(L, 5)
    p.mode = 2
    assert L.sid_reserve(h, 100, 20, ctypes.byref(p)) == EINVAL
    assert b"coarse" in L.sid_last_error(h)
    out = ctypes.c_void_p()
    assert L.sid_stream_begin(h, 1, 100, 20, ctypes.byref(p), ctypes.byref(out)) == EINVAL
    p.mode = 3
    assert L.sid_reserve(h, 100, 20, ctypes.byref(p)) == EINVAL


def test_mesh_struct_layout(tmp_path):
    import shutil
    import subprocess
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no C compiler")
    src = tmp_path / "mesh.c"
    src.write_text('#include <stddef.h>\n#include <stdio.h>\n#include "sid.h"\nint main(void){\n'
                   'printf("%zu %zu %zu %zu %zu %zu\\n", sizeof(sid_mesh), offsetof(sid_mesh, n),'
                   ' offsetof(sid_mesh, coord), offsetof(sid_mesh, coarse),'
                   ' offsetof(sid_mesh, ncoarse), offsetof(sid_mesh, period));\nreturn 0;}\n')
    exe = tmp_path / "mesh"
    subprocess.check_call([cc, "-I", os.path.join(ROOT, "include"), "-o", str(exe), str(src)])
    got = [int(v) for v in subprocess.check_output([str(exe)]).split()]
    M = _native._Mesh
    assert got == [ctypes.sizeof(M), M.n.offset, M.coord.offset, M.coarse.offset,
                   M.ncoarse.offset, M.period.offset]


def test_probe_tol_validation(vctx):
    """Adaptive rank: probe_tol finite and >= 0; > 0 needs probe rows and
    the Gaussian selection."""
    L, h = vctx
    p = _params(L, 5)
    assert p.probe_tol == 0.0
    for bad in (-1e-3, float("nan"), float("inf")):
        p.probe_tol = bad
        assert L.sid_reserve(h, 100, 20, ctypes.byref(p)) == EINVAL
    p.probe_tol = 1e-3
    assert L.sid_reserve(h, 100, 20, ctypes.byref(p)) == ESTATE
    p.probe_rows = 0
    assert L.sid_reserve(h, 100, 20, ctypes.byref(p)) == EINVAL
    assert b"probe" in L.sid_last_error(h)


def test_sbr_svd_validation(vctx, tmp_path):
    """SBR-SVD arguments are checked before any device work; the parameter
    struct mirrors the C layout."""
    L, h = vctx
    vp = ctypes.c_void_p
    p = _native._SvdParams()
    L.sid_svd_params_init(ctypes.byref(p), 20)
    assert (p.k, p.oversample, p.block, p.seed, p.prec) == (20, 10, 10, 0, 0)
    r = ctypes.c_int64()
    call = lambda N=1000, n=200, lda=1000, A=1: L.sid_sbr_svd(
        h, vp(A), 1, N, n, lda, ctypes.byref(p), vp(1), vp(1), n, vp(1), N, ctypes.byref(r))
    assert call() == ESTATE
    assert call(A=0) == EINVAL
    assert call(lda=10) == EINVAL
    assert call(n=25) == EINVAL                 # l = 30 > n
    p.block = 7
    assert call() == EINVAL                     # l % block
    p.block, p.oversample = 10, 250
    assert call() == EINVAL                     # l > 256
    # the streamed form checks the same rules against n_max
    p.oversample = 10
    out = vp()
    begin = lambda N=1000, n_max=200, dt=1: L.sid_svd_stream_begin(h, dt, N, n_max,
                                                                   ctypes.byref(p),
                                                                   ctypes.byref(out))
    assert begin() == ESTATE
    assert begin(n_max=25) == EINVAL            # l = 30 > n_max
    assert begin(dt=7) == EINVAL
    assert L.sid_svd_stream_begin(h, 1, 1000, 200, ctypes.byref(p), None) == EINVAL
    assert L.sid_svd_stream_finish(None, vp(1), vp(1), 1, vp(1), 1, None) == EINVAL
    import shutil
    import subprocess
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        return
    src = tmp_path / "svdp.c"
    src.write_text('#include <stddef.h>\n#include <stdio.h>\n#include "sid.h"\nint main(void){\n'
                   'printf("%zu %zu %zu\\n", sizeof(sid_svd_params), offsetof(sid_svd_params, seed),'
                   ' offsetof(sid_svd_params, prec));\nreturn 0;}\n')
    exe = tmp_path / "svdp"
    subprocess.check_call([cc, "-I", os.path.join(ROOT, "include"), "-o", str(exe), str(src)])
    got = [int(v) for v in subprocess.check_output([str(exe)]).split()]
    S = _native._SvdParams
    assert got == [ctypes.sizeof(S), S.seed.offset, S.prec.offset]
