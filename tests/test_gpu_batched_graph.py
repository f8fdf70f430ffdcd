"""A batched call on the persistent sketch pass captured in a HIP graph:
eight matrices of the uneven batch's shapes (rows capped at 65536), after
sid_reserve_batched, replayed three times with eager work and
synchronization in between, bit for bit equal to the eager call.

Skipped: this capture (and the 64-matrix one) ended the process with a
segmentation fault inside the runtime's end of capture, right after the
eager call of the same batch had passed; no mistake in the library's
capture sequence has been found, and the library now refuses batched calls
under capture (SID_ESTATE).  Marked gpu."""
import sys

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


@pytest.mark.skip(reason="captured batched calls crashed the runtime's end of capture; "
                         "the library refuses them under capture")
@pytest.mark.parametrize("mode", ["single_pass", "two_pass"])
def test_batched_graph_capture(sid, mode):
    shapes = [(min(N, 65536), n, k) for N, n, k in synth.batched_shapes()[:8]]
    mats = [synth.batched_matrix(N, n, seed=2000 + b, device="cuda")
            for b, (N, n, _) in enumerate(shapes)]
    ks = [k for _, _, k in shapes]
    torch.cuda.synchronize()
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        ctx = sid.Context(stream=stream)
        bt = sid.Batch(mats, ks, oversample=10, seed=list(range(8)), mode=mode, prec="bf16x2",
                       probe_rows=10, ctx=ctx).reserve()
        held = ctx.workspace_bytes()
        outs = bt.run()
    ctx.sync()
    torch.cuda.synchronize()
    eager = [[t.clone() for t in (o.J, o.P, o.err, o.AJ, o.k_eff)] for o in outs]
    say("graph", mode, "streams", sid.batch_streams(ctx), "capture")
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=stream):
        bt.run()
    say("graph", mode, "captured")
    assert ctx.workspace_bytes() == held
    for rep in range(3):
        for o in outs:
            for t in (o.J, o.P, o.err, o.AJ, o.k_eff):
                t.zero_()
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        ctx.sync()
        for b, o in enumerate(outs):
            got = [o.J, o.P, o.err, o.AJ, o.k_eff]
            assert all(torch.equal(x, y) for x, y in zip(eager[b], got)), (rep, b)
        sid.compress(mats[0], 8, 10, seed=5, mode=mode, prec="bf16x2", probe_rows=10, ctx=ctx)
        ctx.sync()
        say("graph", mode, "replay", rep, "ok")
