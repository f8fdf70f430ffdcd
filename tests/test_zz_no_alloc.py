"""The allocation-free sketch (sid_sketch_noalloc) through the C ABI against
sid_sketch on the same inputs: W and Y bit for bit, on calls in a row (each
later one with a smaller input than the one before it on its pass: the C2
shape, then a narrow one; the k = 150, p = 30 shape on the workgroup-pair
pass, then a smaller one), with the context's workspace and torch's device
memory unchanged by the calls.  Marked gpu."""
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


def _matrix(N, n, seed):
    g = torch.Generator(device="cuda").manual_seed(seed)
    A = torch.randn((n, N), dtype=torch.float32, device="cuda", generator=g).T
    return synth.as_colmajor(A * torch.exp(-torch.arange(n, device="cuda") / 40.0))


@pytest.mark.parametrize("prec", ["bf16x2", "fp8"])
def test_sketch_noalloc_equals_sketch(sid, prec):
    ctx = sid.Context()
    cases = [(200000, 500, 100, 20, 10, True), (70004, 130, 24, 8, 4, True),
             (50000, 300, 40, 10, 6, False), (60000, 384, 150, 30, 10, True),
             (30000, 200, 150, 30, 10, True)]
    for N, n, k, p, q, want_y in cases:
        say("noalloc", prec, N, n, k, p, q, want_y)
        A = _matrix(N, n, N + n)
        l = k + p
        lw = l + (p if want_y else 0) + q
        # reference: the allocating entry point
        Wr, Yr = sid.sketch(A, k, p, seed=3, prec=prec, probe_rows=q, want_y=want_y, ctx=ctx)
        torch.cuda.synchronize()
        W = torch.full((n, lw), float("nan"), dtype=torch.float64, device="cuda").T
        Y = torch.full((N, l), float("nan"), dtype=torch.float32, device="cuda") if want_y else None
        torch.cuda.synchronize()
        held = ctx.workspace_bytes()
        mem = torch.cuda.memory_allocated()
        sid.sketch_noalloc(A, k, W, Y, oversample=p, seed=3, prec=prec, probe_rows=q, ctx=ctx)
        ctx.sync()
        assert ctx.workspace_bytes() == held
        assert torch.cuda.memory_allocated() == mem
        assert torch.equal(W, Wr), (prec, N, n)
        if want_y:
            assert torch.equal(Y, Yr), (prec, N, n)
    ctx.close()


def test_sketch_noalloc_rejects(sid):
    ctx = sid.Context()
    A = _matrix(4096, 64, 1)
    W = torch.empty((64, 30), dtype=torch.float64, device="cuda").T
    with pytest.raises(sid.SidError):   # FP32 sketch form: not an allocation-free path
        sid.sketch_noalloc(A, 10, W, None, oversample=10, prec="f32", probe_rows=10, ctx=ctx)
    big = synth.colmajor_empty(1 << 20, 512, device="cuda")
    Wb = torch.empty((512, 266), dtype=torch.float64, device="cuda").T
    with pytest.raises(sid.SidError):   # lw = 266 > 256 rows
        sid.sketch_noalloc(big, 200, Wb, None, oversample=56, prec="bf16", probe_rows=10, ctx=ctx)
    # l = 128, lw = 160, n = 512 on 256 workgroups: 80 MiB of partials plus
    # Omega and Omega^T exceed the static array
    Wc = torch.empty((512, 160), dtype=torch.float64, device="cuda").T
    Yc = torch.empty((1 << 20, 128), dtype=torch.float32, device="cuda")
    with pytest.raises(sid.SidError, match="static scratch"):
        sid.sketch_noalloc(big, 100, Wc, Yc, oversample=28, prec="bf16", probe_rows=10,
                           corange_rows=22, ctx=ctx)
    ctx.close()
