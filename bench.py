#!/usr/bin/env python
"""Throughput of the single-pass ID compressor on one MI355X.

Workload: a 1,572,864 x 500 FP32 channel-like snapshot matrix (u, v, w on a
128 x 64 x 64 grid, 500 snapshots; random Fourier modes with a k^-5/3
spectrum, wall-damped profiles, slowly drifting phases -- see synth), the
stand-in for the paper's DNS snapshot data.  One step = one single-pass
compression at k = 100, oversampling 20, 10 probe rows: the sketch pass
(W = Psi A and Y = A Omega in one read of A), the FP64 pivoted QR and
coefficients, the probe estimate, and the skeleton estimate AJ = Y T.
The data are resident in HBM before timing starts.

Prints one JSON line: snapshot GB/s (bytes of A per second) for the chosen
sketch precision (default bf16x2), with the FP32-plain form on the same GPU,
the relative Frobenius error of each, the sketch kernel's HBM roofline
fraction, and the CPU oracle's throughput on a bounded row sample.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "snapshot GB/s compressed (single-pass ID, k=100) vs FP32 plain; rel. Frob. error"
HBM_PEAK_GBS = 8000.0
PROFILE_DIR = os.path.join(ROOT, "profiles")


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    for f in ("sid_kernels.hip", "sid_sketch_mfma.hip", "sid_cpqr.hip", "sid_device.hpp"):
        with open(os.path.join(ROOT, "paper_1905_13257_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(kernel_hash: str):
    """HBM bytes per sketch launch from the committed rocprofv3 counter
    summary, if it was taken on the current kernel sources."""
    path = os.path.join(PROFILE_DIR, "sketch_c2_traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        rec = json.load(fh)
    if rec.get("kernel_source_hash") != kernel_hash:
        return None
    return rec.get("hbm_bytes_per_launch")


def time_steps(fn, steps: int, warmup: int, torch) -> float:
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    start = torch.cuda.Event(enable_timing=True)
    end = torch.cuda.Event(enable_timing=True)
    start.record()
    for _ in range(steps):
        fn()
    end.record()
    torch.cuda.synchronize()
    return start.elapsed_time(end) / steps


def _oracle_single_thread(sample_path: str, k: int, p: int, q: int) -> float:
    """Seconds of the oracle on the saved sample with one OpenMP thread (a
    child process that touches no GPU)."""
    import subprocess
    code = ("import sys, time, numpy as np; sys.path.insert(0, %r); import oracle; "
            "A = np.load(%r); t = time.perf_counter(); "
            "oracle.compress(A, %d, %d, seed=0, mode='single_pass', prec='f64', probe_rows=%d); "
            "print(time.perf_counter() - t)" % (ROOT, sample_path, k, p, q))
    env = dict(os.environ, OMP_NUM_THREADS="1")
    res = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, env=env,
                         timeout=600)
    return float(res.stdout.strip().splitlines()[-1])


def cpu_baseline(A, k, p, q, rows: int, st_rows: int):
    """The oracle (FP64, plain loops, OpenMP) on the first `rows` rows, with
    its per-phase times and the relative Frobenius error of its result, and
    the same oracle on one thread on the first `st_rows` rows."""
    import tempfile
    import numpy as np
    import oracle
    oracle.build()
    sample = A[:rows].cpu().numpy().astype(np.float64)
    phases = {}
    t0 = time.perf_counter()
    res = oracle.compress(sample, k, p, seed=0, mode="single_pass", prec="f64", probe_rows=q,
                          timings=phases)
    dt = time.perf_counter() - t0
    t1 = time.perf_counter()
    err = oracle.error_norms(sample, res.AJ, res.P)
    t_err = time.perf_counter() - t1
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    st = None
    if st_rows > 0:
        with tempfile.TemporaryDirectory() as d:
            path = os.path.join(d, "sample.npy")
            np.save(path, np.ascontiguousarray(sample[:st_rows]))
            del res
            st_s = _oracle_single_thread(path, k, p, q)
        st = {"value": st_rows * A.shape[1] * 4 / st_s / 1e9, "unit": "GB/s", "cores": 1,
              "sample": f"first {st_rows} rows x {A.shape[1]} snapshots, same call; {st_s:.1f} s"}
    return {"value": rows * A.shape[1] * 4 / dt / 1e9, "unit": "GB/s", "cores": threads,
            "kind": "oracle",
            "sample": f"first {rows} of {A.shape[0]} rows x {A.shape[1]} snapshots, single-pass "
                      f"k={k} p={p} q={q}, FP64; {dt:.1f} s",
            "phase_s": {kk: round(v, 3) for kk, v in phases.items()},
            "rel_fro_error": err["rel_fro"], "error_norms_s": round(t_err, 2),
            "single_thread": st}


def batched_main(args, torch, sid, synth) -> int:
    """The uneven batch: 64 independent FP32 matrices, N log-uniform in
    [16384, 1048576], n uniform in [64, 512], k uniform in [8, 64],
    sigma_j = j^-1.5 (device-generated), single pass, p = 10, one
    sid_compress_batched call (persistent sketch pass, autotuned stream count)
    against one call per matrix."""
    import numpy as np
    shapes = synth.batched_shapes()
    mats = [synth.batched_matrix(N, n, seed=1000 + b, device="cuda")
            for b, (N, n, _) in enumerate(shapes)]
    ks = [k for _, _, k in shapes]
    seeds = list(range(11, 11 + len(mats)))
    torch.cuda.synchronize()
    total = sum(N * n * 4 for N, n, _ in shapes)
    kw = dict(oversample=10, mode="single_pass", prec=args.prec, probe_rows=10)
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        ctx = sid.Context(stream=stream)
        bt = sid.Batch(mats, ks, seed=seeds, ctx=ctx, **kw).reserve(tune=True)
        streams = sid.batch_streams(ctx)
        ms_b = time_steps(bt.run, args.steps, args.warmup, torch)
    ctx.sync()
    outs = bt.outs
    ms_s = time_steps(lambda: [sid.compress(A, k, seed=sd, **kw) for A, k, sd in zip(mats, ks, seeds)],
                      max(3, args.steps // 2), 1, torch)
    errs = [sid.error_norms(A, o.AJ, o.P)["rel_fro"] for A, o in zip(mats, outs)]
    line = {
        "metric": "batched snapshot GB/s (single-pass ID of 64 matrices)",
        "value": round(total / (ms_b * 1e-3) / 1e9, 2),
        "unit": "GB/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(ms_b, 4), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": args.prec, "data": "synthetic",
        "config": {"workload": "64 FP32 matrices, N log-uniform in [16384, 1048576], n in [64, 512], "
                               "k in [8, 64], p = 10, q = 10, sigma_j = j^-1.5, one batched call",
                   "total_bytes": total, "factor_streams": streams,
                   "sequential_ms": round(ms_s, 4),
                   "sequential_value": round(total / (ms_s * 1e-3) / 1e9, 2),
                   "rel_fro_error_max": max(errs), "rel_fro_error_median": float(np.median(errs))},
    }
    print(json.dumps(line), flush=True)
    return 0


def stream_main(args, torch, sid, synth) -> int:
    """The streamed workload: 1,572,864 x 2000 FP32 snapshots pushed in blocks
    of 32 columns (62 of 32 and one of 16), single pass, k = 150, p = 30,
    q = 10; the FP8 sketch (the form the in-situ setting is after), with
    bf16x2 beside it.  A step = begin, every push, finish; the blocks are
    resident in HBM."""
    import numpy as np
    A = synth.spectral_snapshots(synth.streaming_config(), device="cuda")
    torch.cuda.synchronize()
    N, n = A.shape
    k, p, q = 150, 30, 10
    total = N * n * 4

    def run(prec):
        kw = dict(seed=0, mode="single_pass", prec=prec, probe_rows=q)

        def step():
            st = sid.Stream(N, n, k, p, dtype=torch.float32, **kw)
            for c0 in range(0, n, 32):
                st.push(A[:, c0:c0 + 32])
            return st.finish()

        out = step()
        ms = time_steps(step, max(2, args.steps // 4), 1, torch)
        err = sid.error_norms(A, out.AJ, out.P)["rel_fro"]
        return ms, err

    ms8, e8 = run("fp8")
    msb, eb = run("bf16x2")
    line = {
        "metric": "streamed snapshot GB/s (single-pass ID, FP8 sketch, k=150)",
        "value": round(total / (ms8 * 1e-3) / 1e9, 2), "unit": "GB/s", "n_gpus": 1,
        "steps": max(2, args.steps // 4), "warmup": 1, "ms_per_step": round(ms8, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "fp8",
        "data": "synthetic",
        "config": {"workload": "channel-like snapshots 1572864 x 2000 fp32 streamed in 32-column "
                               "blocks, single-pass ID k=150 p=30 q=10",
                   "rel_fro_error": e8,
                   "bf16x2": {"ms_per_step": round(msb, 4),
                              "value": round(total / (msb * 1e-3) / 1e9, 2),
                              "rel_fro_error": eb}},
    }
    print(json.dumps(line), flush=True)
    return 0


def probes_main(args, torch, sid, synth) -> int:
    """Ceilings the kernels' design rests on, measured with the library's
    probe kernels (sid_probe): a streaming read and two store patterns of
    HBM, and the issue rate of the two bfloat16 matrix instructions."""
    ncu = torch.cuda.get_device_properties(0).multi_processor_count
    stream = torch.cuda.current_stream()
    ctx = sid.Context(stream=stream)
    out = {}

    def timed(fn, reps=5):
        fn()
        torch.cuda.synchronize()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(stream)
        for _ in range(reps):
            fn()
        b.record(stream)
        torch.cuda.synchronize()
        return a.elapsed_time(b) / reps

    big = torch.empty((256, 1 << 22), dtype=torch.float32, device="cuda").T   # 4 GiB
    ms = timed(lambda: sid.probe("read", big, ctx=ctx))
    out["read_GBs"] = round(big.numel() * 4 / (ms * 1e-3) / 1e9, 1)
    del big
    c2 = torch.empty((500, 1572864), dtype=torch.float32, device="cuda").T
    ms = timed(lambda: sid.probe("store_columns", c2, ctx=ctx))
    out["store_columns_GBs"] = round(c2.numel() * 4 / (ms * 1e-3) / 1e9, 1)
    ms = timed(lambda: sid.probe("store_sequential", c2, ctx=ctx))
    out["store_sequential_GBs"] = round(c2.numel() * 4 / (ms * 1e-3) / 1e9, 1)
    del c2
    rounds = 20000
    for name, flops in (("mfma_16x16x32", 2 * 16 * 16 * 32), ("mfma_32x32x16", 2 * 32 * 32 * 16)):
        ms = timed(lambda: sid.probe(name, None, rounds, ctx=ctx), reps=3)
        total = ncu * 8 * 4 * 8 * rounds * flops
        out[name + "_TFLOPs"] = round(total / (ms * 1e-3) / 1e12, 1)
    ctx.sync()
    line = {"metric": "probe ceilings", "config": {"compute_units": ncu,
            "read": "4 GiB, 16-byte loads", "store_columns": "1572864 x 500 FP32, 4 columns x "
            "256 bytes per wave instruction", "mfma": "8 independent chains per wave, "
            f"{rounds} rounds, 8 workgroups of 4 waves per compute unit"}, **out}
    print(json.dumps(line), flush=True)
    return 0


def coarse_main(args, torch, sid, synth) -> int:
    """Sub-sampled ID (Alg. 5 with the Gaussian sketch of the coarse rows) on
    the fine 256 x 128 x 128 channel-like grid, error on the fine grid."""
    # drift calibrated for this grid and length as for the headline matrix: the
    # two-pass ID error at k = 100 lies in [1e-3, 1e-2] (0.0095 -> 3.1e-3 on the
    # fine grid from the coarse rows; the C2 value 0.0385 gives 0.65 here)
    cfg = synth.SpectralConfig(nx=256, ny=128, nz=128, n_snapshots=1000, seed=1002, drift=0.0095)
    A = synth.spectral_snapshots(cfg, device="cuda")
    torch.cuda.synchronize()
    N, n = A.shape
    S = synth.coarse_rows_every_other(cfg.nx, cfg.ny, cfg.nz)
    rs = sid.RowSet(S, N)
    k, p, q = 100, 20, 10
    kw = dict(seed=0, coarse=rs, mode="two_pass", prec=args.prec, probe_rows=q)
    out = sid.compress(A, k, p, **kw)
    ms = time_steps(lambda: sid.compress(A, k, p, out=out, **kw), args.steps, args.warmup, torch)
    ms_sk = time_steps(lambda: sid.sketch(A, k, p, coarse=rs, prec=args.prec, probe_rows=q,
                                          want_y=False), max(3, args.steps // 2), 1, torch)
    err = sid.error_norms(A, out.AJ, out.P)
    line = {
        "metric": "fine-grid snapshot GB/s (sub-sampled ID, two-pass, k=100)",
        "value": round(N * n * 4 / (ms * 1e-3) / 1e9, 2), "unit": "GB/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": args.prec,
        "data": "synthetic",
        "config": {"workload": "channel-like snapshots 12582912 x 1000 fp32 (3 x 256x128x128 grid), "
                               "coarse rows every other point (1572864), two-pass ID k=100 p=20 q=10",
                   "coarse_rows": int(S.size), "coarse_sketch_ms": round(ms_sk, 4),
                   "coarse_bytes": int(S.size) * n * 4, "rel_fro_error_fine": err["rel_fro"],
                   "probe_estimate": float(out.err[0]), "k_eff": int(out.k_eff[0])},
    }
    print(json.dumps(line), flush=True)
    return 0


def spid_main(args, torch, sid, synth) -> int:
    """Single-pass ID with interpolation (Alg. 6) on the fine 256 x 128 x 128
    channel-like grid: compression from the every-other-point coarse rows
    (coarse skeleton kept), the fused trilinear reconstruction of the whole
    fine matrix, and the fused error kernel against the fine data."""
    cfg = synth.SpectralConfig(nx=256, ny=128, nz=128, n_snapshots=1000, seed=1002, drift=0.0095)
    A = synth.spectral_snapshots(cfg, device="cuda")
    mesh = synth.channel_mesh(cfg, (2, 2, 2))
    ip = sid.Interp(mesh)
    torch.cuda.synchronize()
    N, n = A.shape
    k, p, q = 100, 20, 10
    kw = dict(seed=0, coarse=ip.rowset, mode="coarse_skeleton", prec=args.prec, probe_rows=q)
    c = sid.compress(A, k, p, **kw)
    ms_c = time_steps(lambda: sid.compress(A, k, p, out=c, **kw), args.steps, args.warmup, torch)
    Ahat = torch.empty((n, N), dtype=torch.float32, device="cuda").T
    rec = lambda: sid.interp_reconstruct(ip, c.AJ, c.P, out=Ahat)
    ms_r = time_steps(rec, args.steps, args.warmup, torch)
    ms_e = time_steps(lambda: sid.interp_error_norms(ip, A, c.AJ, c.P), max(3, args.steps // 2), 1,
                      torch)
    err = sid.interp_error_norms(ip, A, c.AJ, c.P)
    # the sub-sampled ID with the fine skeleton (second pass) on the same J, P
    b = sid.compress(A, k, p, seed=0, coarse=ip.rowset, mode="two_pass", prec=args.prec,
                     probe_rows=q)
    err_sub = sid.error_norms(A, b.AJ, b.P)
    del Ahat
    # algorithmic bytes of one reconstruction: write Ahat, read ACJ and P once
    rbytes = N * n * 4 + ip.Nc * k * 4 + k * n * 4
    gbs_r = rbytes / (ms_r * 1e-3) / 1e9
    line = {
        "metric": "fine-grid snapshot GB/s (single-pass ID with interpolation, Alg. 6, k=100)",
        "value": round(N * n * 4 / (ms_c * 1e-3) / 1e9, 2), "unit": "GB/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms_c, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": args.prec,
        "data": "synthetic",
        "config": {"workload": "channel-like snapshots 12582912 x 1000 fp32 (3 x 256x128x128 grid), "
                               "coarse rows every other point (1572864), coarse skeleton kept, "
                               "trilinear reconstruction; k=100 p=20 q=10",
                   "coarse_rows": int(ip.Nc),
                   "reconstruct_ms": round(ms_r, 4),
                   "reconstruct_roofline": {"bound": "hbm", "achieved": round(gbs_r, 1),
                                            "peak": HBM_PEAK_GBS, "unit": "GB/s",
                                            "frac": round(gbs_r / HBM_PEAK_GBS, 4),
                                            "bytes": rbytes,
                                            "timed": "whole call: operand packing + fused kernel"},
                   "error_kernel_ms": round(ms_e, 4),
                   "rel_fro_error_fine": err["rel_fro"], "max_abs_error_fine": err["max_abs"],
                   "rel_fro_error_subsampled_two_pass": err_sub["rel_fro"],
                   "probe_estimate_coarse": float(c.err[0]), "k_eff": int(c.k_eff[0])},
    }
    print(json.dumps(line), flush=True)
    return 0


def adaptive_main(args, torch, sid, synth) -> int:
    """Tolerance-driven rank (Remark 2.2, probe estimator as the stopping
    test) on the headline matrix: single pass at k <= 100, p = 20, q = 10,
    for a few tolerances; the step includes the prefix-error pass."""
    cfg = synth.SpectralConfig()
    k, p, q = 100, 20, 10
    A = synth.spectral_snapshots(cfg, device="cuda")
    torch.cuda.synchronize()
    N, n = A.shape
    kw = dict(seed=0, mode="single_pass", prec=args.prec, probe_rows=q)
    base = sid.compress(A, k, p, **kw)
    ms_fixed = time_steps(lambda: sid.compress(A, k, p, out=base, **kw), args.steps, args.warmup,
                          torch)
    rows = []
    for tol in (3e-2, 1e-2, 5e-3):
        out = sid.compress(A, k, p, probe_tol=tol, **kw)
        ms = time_steps(lambda: sid.compress(A, k, p, out=out, probe_tol=tol, **kw), args.steps,
                        args.warmup, torch)
        ke = int(out.k_eff[0])
        err = sid.error_norms(A, out.AJ[:, :ke], out.P[:ke])
        rows.append({"probe_tol": tol, "k_eff": ke, "ms_per_step": round(ms, 4),
                     "probe_estimate": float(out.err[0]), "rel_fro_error": err["rel_fro"]})
    first = rows[0]
    line = {
        "metric": "snapshot GB/s compressed (single-pass ID, rank chosen by probe_tol)",
        "value": round(N * n * 4 / (first["ms_per_step"] * 1e-3) / 1e9, 2), "unit": "GB/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": first["ms_per_step"], "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": args.prec, "data": "synthetic",
        "config": {"workload": "channel-like snapshots 1572864 x 500 fp32, single-pass ID, "
                               "k <= 100 p=20 q=10, probe_tol 3e-2 (value) / 1e-2 / 5e-3",
                   "tolerances": rows, "fixed_k100_ms": round(ms_fixed, 4)},
    }
    print(json.dumps(line), flush=True)
    return 0


def sweep_main(args, torch, sid, synth) -> int:
    """Error against the sub-sampling factor (the paper's Fig. 4, right): a
    channel-like field resolved on coarse grids (at most 1.5 wavelengths per
    extent) on 3 x 257 x 33 x 257 points x 200 snapshots, x and z sub-sampled
    by s = 1, 2, 4, 8, 16 (factor s^2), at rank 100 (above the field's 80
    components: the interpolation error dominates) and rank 20 (the
    truncation dominates): the single-pass ID with interpolation (Alg. 6),
    the sub-sampled ID with the fine skeleton (Alg. 5), and the interpolation
    error ||A - Mf A(S, :)|| itself."""
    cfg = synth.SpectralConfig(nx=257, ny=33, nz=257, n_snapshots=200, n_modes=40, drift=0.3,
                               seed=77, kmax=1.5)
    A = synth.spectral_snapshots(cfg, device="cuda")
    torch.cuda.synchronize()
    N, n = A.shape
    q = 10
    rows = []
    for (k, p), st in [((k_, p_), st_) for (k_, p_) in ((100, 20), (20, 10))
                       for st_ in (1, 2, 4, 8, 16)]:
        mesh = synth.channel_mesh(cfg, (st, 1, st), keep_last=True)
        ip = sid.Interp(mesh)
        kw = dict(seed=1, coarse=ip.rowset, prec=args.prec, probe_rows=q)
        c = sid.compress(A, k, p, mode="coarse_skeleton", **kw)
        ms = time_steps(lambda: sid.compress(A, k, p, mode="coarse_skeleton", out=c, **kw),
                        args.steps, args.warmup, torch)
        e_spid = sid.interp_error_norms(ip, A, c.AJ, c.P)["rel_fro"]
        b = sid.compress(A, k, p, mode="two_pass", **kw)
        e_sub = sid.error_norms(A, b.AJ, b.P)["rel_fro"]
        S = torch.from_numpy(mesh.coarse_rows).cuda()
        AS = A[S]
        eye = torch.eye(n, dtype=torch.float32, device="cuda")
        e_int = sid.interp_error_norms(ip, A, AS, eye)["rel_fro"]
        rows.append({"k": k, "stride_xz": st, "factor": st * st, "coarse_rows": int(ip.Nc),
                     "rel_fro_single_pass_interp": e_spid, "rel_fro_subsampled": e_sub,
                     "rel_fro_interpolation": e_int, "compress_ms": round(ms, 4)})
        del AS, ip
    at16 = next(r for r in rows if r["factor"] == 16 and r["k"] == 100)
    line = {
        "metric": "rel. Frobenius error of the single-pass ID with interpolation vs sub-sampling "
                  "factor (value: factor 16, k=100)",
        "value": at16["rel_fro_single_pass_interp"], "unit": "relative error", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": at16["compress_ms"],
        "higher_is_better": False, "scaling": "weak", "vs_baseline": None, "dtype": args.prec,
        "data": "synthetic",
        "config": {"workload": "channel-like snapshots 6539622 x 200 fp32 (3 x 257x33x257 grid, "
                               "at most 1.5 wavelengths per extent), x and z sub-sampled by "
                               "1/2/4/8/16, k=100 p=20 and k=20 p=10, q=10", "sweep": rows},
    }
    print(json.dumps(line), flush=True)
    return 0


def svd_main(args, torch, sid, synth) -> int:
    """SBR-SVD (Alg. 2) on the headline matrix: k = 100, p = 20, block 20,
    one pass for G = (Psi A)^T, H = A G and the block loop in FP64.  The
    line is the FP64-sketch run; the FP32 and BF16x2 sketches are timed
    beside it, with the error ||A - V S U^T||_F / ||A||_F of each and the
    single-pass ID's on the same matrix."""
    cfg = synth.SpectralConfig()
    A = synth.spectral_snapshots(cfg, device="cuda")
    torch.cuda.synchronize()
    N, n = A.shape
    k, p, b = 100, 20, 20
    runs = {}
    for prec in ("f64", "f32", "bf16x2"):
        out = sid.sbr_svd(A, k, p, b, seed=0, prec=prec)
        ms = time_steps(lambda: sid.sbr_svd(A, k, p, b, seed=0, prec=prec), args.steps,
                        args.warmup, torch)
        err = sid.error_norms(A, out.V * out.S.float()[None, :], out.U.T.contiguous())
        runs[prec] = (ms, err["rel_fro"], out)
        print(f"# sbr_svd prec={prec}: {ms:.3f} ms, rel_fro {err['rel_fro']:.4e}, "
              f"rank {out.rank}", file=sys.stderr, flush=True)
    ide = sid.compress(A, k, p, seed=0, mode="single_pass", prec="bf16x2", probe_rows=10)
    err_id = sid.error_norms(A, ide.AJ, ide.P)
    # the optimal rank-k error (Eckart-Young) from the eigenvalues of A^T A in FP64
    import numpy as np
    lam = np.linalg.eigvalsh((A.double().T @ A.double()).cpu().numpy())[::-1].clip(min=0)
    opt = float(np.sqrt(lam[k:].sum() / lam.sum()))
    ms, rel, out = runs["f64"]
    line = {
        "metric": "snapshot GB/s compressed (SBR-SVD, Alg. 2, k=100)",
        "value": round(N * n * 4 / (ms * 1e-3) / 1e9, 2), "unit": "GB/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "channel-like snapshots 1572864 x 500 fp32, SBR-SVD k=100 p=20 "
                               "block 20",
                   "rel_fro_error": rel, "rank": out.rank,
                   "sigma_1": float(out.S[0]), "sigma_k": float(out.S[k - 1]),
                   "by_sketch_prec": {q: {"ms_per_step": round(v[0], 4), "rel_fro_error": v[1]}
                                      for q, v in runs.items()},
                   "rel_fro_error_optimal_rank_k": opt,
                   "rel_fro_error_single_pass_id_bf16x2": err_id["rel_fro"]},
    }
    print(json.dumps(line), flush=True)
    return 0


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--prec", default="bf16x2", choices=["bf16x2", "bf16", "fp8", "f32", "f64"])
    ap.add_argument("--also", default="bf16,fp8",
                    help="further sketch precisions timed beside the main one (comma list, '' for none)")
    ap.add_argument("--cpu-st-rows", type=int, default=49152,
                    help="rows of the single-thread oracle sample (0: skip)")
    ap.add_argument("--cpu-rows", type=int, default=1572864,
                    help="rows of the matrix the oracle baseline compresses (default: all)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-compare", action="store_true", help="skip the FP32-plain run")
    ap.add_argument("--probes", action="store_true",
                    help="the measured ceilings: HBM read and store rates, bf16 matrix-"
                         "instruction issue rates (sid_probe)")
    ap.add_argument("--stream", action="store_true",
                    help="auxiliary measurement instead of the headline: the 1,572,864 x 2000 "
                         "field streamed in 32-column blocks, FP8 sketch, k = 150, p = 30")
    ap.add_argument("--batched", action="store_true",
                    help="auxiliary measurement instead of the headline: 64 independent matrices "
                         "(N log-uniform in [2^14, 2^20], n in [64, 512], k in [8, 64], spectrum "
                         "j^-1.5) compressed by sid_compress_batched, and by one sid_compress per "
                         "matrix")
    ap.add_argument("--coarse", action="store_true",
                    help="auxiliary measurement instead of the headline: the sub-sampled ID on the "
                         "256 x 128 x 128 grid (12,582,912 x 1000 FP32), two-pass, coarse rows = "
                         "every other grid point (1,572,864 rows), k=100 p=20")
    ap.add_argument("--spid", action="store_true",
                    help="auxiliary measurement instead of the headline: the single-pass ID with "
                         "interpolation (Alg. 6) on the 256 x 128 x 128 grid (12,582,912 x 1000 "
                         "FP32), coarse rows = every other grid point, k=100 p=20: compression, "
                         "trilinear reconstruction of the fine matrix, and its error")
    ap.add_argument("--adaptive", action="store_true",
                    help="auxiliary measurement instead of the headline: the rank chosen by the "
                         "held-out probe estimate (probe_tol 3e-2, 1e-2, 5e-3) on the headline "
                         "matrix, single pass, k <= 100")
    ap.add_argument("--sweep", action="store_true",
                    help="auxiliary measurement instead of the headline: error of the single-pass "
                         "ID with interpolation and of the sub-sampled ID against the sub-sampling "
                         "factor on a field resolved on coarse grids")
    ap.add_argument("--svd", action="store_true",
                    help="auxiliary measurement instead of the headline: SBR-SVD (Alg. 2) of the "
                         "headline matrix at k=100, p=20, block 20")
    ap.add_argument("--sketch-only", action="store_true",
                    help="profiling aid for hardware counters: a plain 1 GiB device copy (the "
                         "calibration kernel for FETCH_SIZE / WRITE_SIZE) and three sketch passes")
    args = ap.parse_args()

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU only: the compressor's hot path runs on a single "
              "MI355X (sharding the rows across GPUs is described, not implemented); "
              f"--gpus {args.gpus} is not supported.", file=sys.stderr)
        return 2

    import torch
    import paper_1905_13257_amd as sid
    import synth

    torch.cuda.set_device(0)
    if args.probes:
        return probes_main(args, torch, sid, synth)
    if args.stream:
        return stream_main(args, torch, sid, synth)
    if args.batched:
        return batched_main(args, torch, sid, synth)
    if args.coarse:
        return coarse_main(args, torch, sid, synth)
    if args.spid:
        return spid_main(args, torch, sid, synth)
    if args.adaptive:
        return adaptive_main(args, torch, sid, synth)
    if args.sweep:
        return sweep_main(args, torch, sid, synth)
    if args.svd:
        return svd_main(args, torch, sid, synth)
    cfg = synth.SpectralConfig()
    k, p, q = 100, 20, 10
    A = synth.spectral_snapshots(cfg, device="cuda")
    torch.cuda.synchronize()
    N, n = A.shape
    if args.sketch_only:
        src = torch.ones(1 << 28, dtype=torch.float32, device="cuda")  # 1 GiB
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        for _ in range(3):
            sid.sketch(A, k, p, seed=0, prec=args.prec, probe_rows=q, want_y=True)
        torch.cuda.synchronize()
        print(json.dumps({"sketch_only": True, "copy_bytes_read": 1 << 30, "copy_bytes_written": 1 << 30,
                          "A_bytes": N * n * 4, "Y_bytes": N * (k + p) * 4, "prec": args.prec}), flush=True)
        return 0
    bytes_a = N * n * 4
    l = k + p

    def run_mode(prec: str, steps: int, warmup: int):
        kw = dict(seed=0, mode="single_pass", prec=prec, probe_rows=q)
        out = sid.compress(A, k, p, **kw)
        # eager: one sid_compress call per step
        ms_eager = time_steps(lambda: sid.compress(A, k, p, out=out, **kw), steps, warmup, torch)
        # the same call captured once into a HIP graph (after sid_reserve, so
        # the call allocates nothing) and replayed: every kernel of the step
        # runs at every replay, only the host's launch work is saved
        stream = torch.cuda.Stream()
        with torch.cuda.stream(stream):
            ctx = sid.Context(stream=stream)
            sid.reserve(N, n, k, p, mode="single_pass", prec=prec, probe_rows=q, ctx=ctx)
            sid.compress(A, k, p, ctx=ctx, out=out, **kw)
        ctx.sync()
        torch.cuda.synchronize()
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g, stream=stream):
            sid.compress(A, k, p, ctx=ctx, out=out, **kw)
        ms = time_steps(g.replay, steps, warmup, torch)
        ctx.sync()  # raises if a device-side wait of the replays failed
        del g
        ctx.close()
        err = sid.error_norms(A, out.AJ, out.P)
        sk = lambda: sid.sketch(A, k, p, seed=0, prec=prec, probe_rows=q, want_y=True)
        sketch_ms = time_steps(sk, max(3, steps // 2), 1, torch)
        return dict(ms=ms, ms_eager=ms_eager, gbs=bytes_a / (ms * 1e-3) / 1e9,
                    rel_fro=err["rel_fro"], max_abs=err["max_abs"], est=float(out.err[0]),
                    sketch_ms=sketch_ms, k_eff=int(out.k_eff[0]))

    main_r = run_mode(args.prec, args.steps, args.warmup)
    cmp_r = None
    if not args.no_compare and args.prec != "f32":
        cmp_r = run_mode("f32", max(3, args.steps // 2), 1)
    also = {}
    for pr in [x for x in args.also.split(",") if x and x != args.prec]:
        also[pr] = run_mode(pr, max(3, args.steps // 2), 1)

    # roofline of the sketch pass: algorithmic bytes = read A once + write Y
    alg_bytes = bytes_a + N * l * 4
    achieved = alg_bytes / (main_r["sketch_ms"] * 1e-3) / 1e9
    khash = kernel_source_hash()
    roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                "traffic": measured_traffic(khash), "kernel": "sketch pass (W = Psi A, Y = A Omega)",
                "algorithmic_bytes_per_launch": alg_bytes, "launch_ms": round(main_r["sketch_ms"], 4)}

    # the reconstruction Ahat = AJ P (eq. (ID); a posteriori, outside the
    # step): HBM-bound on writing Ahat, algorithmic bytes = write N n + read
    # AJ (N k) in FP32
    o = sid.compress(A, k, p, seed=0, mode="single_pass", prec=args.prec, probe_rows=q)
    Ahat = torch.empty((n, N), dtype=torch.float32, device="cuda").T
    rec_ms = time_steps(lambda: sid.reconstruct(o.AJ, o.P, out=Ahat), 5, 1, torch)
    rec_bytes = N * n * 4 + N * k * 4
    reconstruct = {"kernel": "reconstruction Ahat = AJ P (matrix cores)", "ms": round(rec_ms, 4),
                   "algorithmic_bytes": rec_bytes,
                   "achieved_GBs": round(rec_bytes / (rec_ms * 1e-3) / 1e9, 1),
                   "frac": round(rec_bytes / (rec_ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)}
    del Ahat, o

    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(A, k, p, q, min(args.cpu_rows, N), min(args.cpu_st_rows, N))

    config = {
        "workload": "channel-like snapshots 1572864 x 500 fp32 (3 x 128x64x64 grid), single-pass "
                    "ID k=100 p=20 q=10",
        "N": N, "n": n, "k": k, "oversample": p, "probe_rows": q, "corange_rows": p,
        "sketch_precision": args.prec, "rel_fro_error": main_r["rel_fro"],
        "max_abs_error": main_r["max_abs"], "probe_estimate": main_r["est"],
        "k_eff": main_r["k_eff"], "sketch_ms": round(main_r["sketch_ms"], 4),
        "timing": "HIP graph replays of the captured call; eager_ms_per_step: one sid_compress "
                  "call per step",
        "eager_ms_per_step": round(main_r["ms_eager"], 4),
        "reconstruct": reconstruct,
    }
    if cpu is not None and min(args.cpu_rows, N) == N:
        # the oracle's own FP64 compression of the same matrix, beside the GPU's
        config["oracle_rel_fro_error"] = cpu["rel_fro_error"]
    if cmp_r is not None:
        config["fp32_plain"] = {"value": round(cmp_r["gbs"], 2), "ms_per_step": round(cmp_r["ms"], 4),
                                "eager_ms_per_step": round(cmp_r["ms_eager"], 4),
                                "rel_fro_error": cmp_r["rel_fro"], "sketch_ms": round(cmp_r["sketch_ms"], 4)}
    for pr, r in also.items():
        config[pr] = {"value": round(r["gbs"], 2), "ms_per_step": round(r["ms"], 4),
                      "eager_ms_per_step": round(r["ms_eager"], 4),
                      "rel_fro_error": r["rel_fro"], "probe_estimate": r["est"],
                      "sketch_ms": round(r["sketch_ms"], 4)}
    line = {
        "metric": METRIC, "value": round(main_r["gbs"], 2), "unit": "GB/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(main_r["ms"], 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": args.prec,
        "data": "synthetic", "config": config, "roofline": roofline, "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
