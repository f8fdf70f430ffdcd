"""The uneven batch: 64 independent FP32 matrices (N log-uniform in
[16384, 1048576], n uniform in [64, 512], sigma_j = j^-1.5, k uniform in
[8, 64], p = 10) compressed by one sid_compress_batched call on the
persistent sketch pass.

* bit for bit equal to one sid_compress per matrix (J, P, err, AJ), single
  and two pass, bf16x2;
* the autotuner picks a stream count, cached per context;
* the oracle's pivots on the two smallest matrices up to its first
  near-tie, and their errors within 5 %.

Capturing this 64-matrix call in a HIP graph ended the process with a
segmentation fault inside the runtime's end of capture (the eager call had
just passed), for eight matrices as well; no mistake in the library's capture
sequence has been found, so the library refuses batched calls under capture
(SID_ESTATE) and the capture test is skipped.

In single pass every matrix of this workload takes the batched steps after
the sketch (mgsqr, solves and estimates as one launch per step), so the
equality below also covers those launches."""
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


def host(t):
    return t.detach().cpu().numpy()


@pytest.fixture(scope="module")
def batch():
    shapes = synth.batched_shapes()
    say("batch: synthesizing", len(shapes), "matrices,",
        sum(N * n for N, n, _ in shapes) * 4 / 1e9, "GB")
    mats = [synth.batched_matrix(N, n, seed=1000 + b, device="cuda")
            for b, (N, n, _) in enumerate(shapes)]
    torch.cuda.synchronize()
    return shapes, mats


def _outputs(outs):
    return [[t.clone() for t in (o.J, o.P, o.err, o.AJ, o.k_eff)] for o in outs]


def _same(a, b):
    return all(torch.equal(x, y) for x, y in zip(a, b))


@pytest.mark.timeout(900)
@pytest.mark.parametrize("mode", ["single_pass", "two_pass"])
def test_batched_persistent(sid, oracle_mod, batch, mode):
    shapes, mats = batch
    ks = [k for _, _, k in shapes]
    seeds = list(range(11, 11 + len(mats)))
    prec, q = "bf16x2", 10
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        ctx = sid.Context(stream=stream)
        bt = sid.Batch(mats, ks, oversample=10, seed=seeds, mode=mode, prec=prec, probe_rows=q,
                       ctx=ctx)
        bt.reserve(tune=(mode == "single_pass"))
        outs = bt.run()
    ctx.sync()
    torch.cuda.synchronize()
    say("batch", mode, "streams after reserve", sid.batch_streams(ctx))
    eager = _outputs(outs)

    say("batch", mode, ": per-matrix calls")
    for b, A in enumerate(mats):
        ref = sid.compress(A, ks[b], 10, seed=seeds[b], mode=mode, prec=prec, probe_rows=q)
        torch.cuda.synchronize()
        assert int(host(ref.k_eff)[0]) == ks[b], b
        assert _same(eager[b], [ref.J, ref.P, ref.err, ref.AJ, ref.k_eff]), b

    say("batch", mode, ": oracle pivots on the two smallest matrices")
    order = np.argsort([N * n for N, n, _ in shapes])[:2]
    for b in order.tolist():
        A64 = mats[b].double().cpu().numpy()
        orc = oracle_mod.compress(A64, ks[b], 10, seed=seeds[b], mode=mode, prec=prec,
                                  probe_rows=q)
        tie = np.nonzero(orc.cp.margins <= 1e-4)[0]
        ist = int(tie[0]) if tie.size else ks[b]
        say("batch", mode, b, shapes[b], "pivots compared", ist, "of", ks[b])
        assert host(eager[b][0])[:ist].tolist() == orc.J[:ist].tolist()
        e_g = sid.error_norms(mats[b], outs[b].AJ, outs[b].P)["rel_fro"]
        e_o = oracle_mod.error_norms(A64, orc.AJ, orc.P)["rel_fro"]
        say("batch", mode, b, "rel_fro gpu", e_g, "oracle", e_o)
        assert abs(e_g - e_o) <= 0.05 * e_o


@pytest.mark.timeout(600)
def test_batched_outputs_change_between_calls(sid, batch):
    """The batched skeleton estimate (one launch for every problem's
    AJ = Y T) follows the caller's output table from call to call: problems
    without an AJ buffer are skipped (their other outputs still written,
    the problem's previous AJ buffer untouched), and a second call with new
    AJ buffers (another row stride) writes those.  Every AJ equals the single
    call's bit for bit."""
    shapes, mats = batch
    order = np.argsort([N * n for N, n, _ in shapes])[:10].tolist()
    sub = [mats[b] for b in order]
    ks = [shapes[b][2] for b in order]
    seeds = [31 + i for i in range(len(sub))]
    kw = dict(oversample=10, mode="single_pass", prec="bf16x2", probe_rows=10)
    bt = sid.Batch(sub, ks, seed=seeds, **kw).reserve()
    refs = []
    for A, k, sd in zip(sub, ks, seeds):
        refs.append(sid.compress(A, k, kw["oversample"], seed=sd, mode=kw["mode"],
                                 prec=kw["prec"], probe_rows=kw["probe_rows"]))
    torch.cuda.synchronize()
    # first call: odd problems without AJ (their buffers hold a sentinel)
    for i, o in enumerate(bt.outs):
        o.AJ.fill_(float("nan"))
        if i % 2:
            bt.probs[i].AJ = None
    outs = bt.run()
    torch.cuda.synchronize()
    for i, (o, r) in enumerate(zip(outs, refs)):
        assert torch.equal(o.J, r.J) and torch.equal(o.P, r.P) and torch.equal(o.err, r.err), i
        if i % 2:
            assert torch.isnan(o.AJ).all(), i
        else:
            assert torch.equal(o.AJ, r.AJ), i
    # second call: new AJ buffers with a padded leading dimension
    fresh = []
    for i, (A, k) in enumerate(zip(sub, ks)):
        N = A.shape[0]
        buf = torch.full((k, N + 3), float("nan"), dtype=torch.float32, device="cuda")
        fresh.append(buf)
        bt.probs[i].AJ = buf.data_ptr()
        bt.probs[i].ldaj = N + 3
    bt.run()
    torch.cuda.synchronize()
    for i, (buf, r) in enumerate(zip(fresh, refs)):
        N = sub[i].shape[0]
        assert torch.equal(buf[:, :N].T, r.AJ), i
        assert torch.isnan(buf[:, N:]).all(), i
