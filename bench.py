#!/usr/bin/env python3
"""Benchmark of dtANS-fused sparse matrix-vector multiplication on one MI355X.

Default workload: the 27-point stencil on a 128^3 grid in FP64 (2,097,152
rows, 55,742,968 nonzeros, 216 distinct values), y = A x, synthetic seeded
data.  A step is one multiplication: decode of every compressed stream fused
with the multiply-accumulate and the write of y.

Inputs are resident in device memory before the timed region.  The timed loop
cycles through several copies of the encoded matrix and of x / y so that
consecutive steps never find their data in the 256 MB memory-side cache
(MALL): every step streams its compressed matrix from HBM.  The same
multiplication on a single copy, back to back ("warm"), and the plain HIP CSR
kernel on the same GPU are reported alongside, as is the CPU oracle on the
host cores.

Other workloads (--workload): band (4096 x 4096, FP64 SpMV), rmat (scale 22,
FP32 SpMV), pruned1 / pruned8 / pruned32 (11008 x 4096 BF16-valued FP32
weight, SpMV / SpMM with k = 8 / 32), batch (64 banded FP32 matrices in one
persistent launch, against one CSR launch per matrix), autograd (forward
SpMM and backward transposed product with batch 16 on the pruned weight) and
encode (host arrays to container: the host encoder against the one whose
stream base/digit passes and word interleave run on the GPU, on the stencil
and the pruned weight) and sym (a symmetric 27-point stencil multiplied
through its strict upper triangle and diagonal, against the whole matrix).

Prints one JSON line (see the keys below).
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "SpMV GFLOP/s + compressed HBM GB/s, dtANS-CSR vs plain CSR, same MI355X"
HBM_PEAK_GBPS = 8000.0
MALL_BYTES = 256 << 20


def log(msg):
    print("[bench] " + msg, file=sys.stderr, flush=True)


def make_workload(name):
    import workloads

    if name == "stencil":
        rp, ci, v = workloads.stencil27(128)
        return dict(name="stencil27 128^3 fp64 spmv", rp=rp, ci=ci, v=v, n=128 ** 3, k=1, cfg=2)
    if name == "band":
        rp, ci, v = workloads.band()
        return dict(name="band 4096x4096 16/row fp64 spmv", rp=rp, ci=ci, v=v, n=4096, k=1, cfg=1)
    if name == "rmat":
        rp, ci, v = workloads.rmat(22)
        return dict(name="rmat scale22 ef16 fp32 spmv", rp=rp, ci=ci, v=v, n=1 << 22, k=1, cfg=3)
    if name == "skewed":
        rp, ci, v = workloads.skewed_rows()
        return dict(name="skewed rows 2^21 fp64 spmv", rp=rp, ci=ci, v=v, n=1 << 21, k=1, cfg=6)
    if name.startswith("pruned"):
        k = int(name[len("pruned"):] or 1)
        rp, ci, v = workloads.pruned_weight()
        return dict(name="pruned 11008x4096 bf16-valued fp32 spmm k=%d" % k, rp=rp, ci=ci, v=v,
                    n=4096, k=k, cfg=4)
    raise SystemExit("unknown workload " + name)


def kernel_source_hash():
    import hashlib

    h = hashlib.sha256()
    for name in ("kernels.hip", "dtans_core.hpp", "kernels.hpp"):
        with open(os.path.join(ROOT, "paper_2603_01915_amd", "csrc", name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def profile_values(name, info):
    """Key: value lines of the committed summary profiles/<name>.txt, if it was
    taken on the current kernel sources and the same encoded size; else None."""
    path = os.path.join(ROOT, "profiles", "%s.txt" % name)
    if not os.path.exists(path):
        return None
    kv = {}
    with open(path) as f:
        for line in f:
            if ":" in line and not line.startswith("#") and not line.startswith(" "):
                k, v = line.split(":", 1)
                kv[k.strip()] = v.strip()
    if kv.get("kernel_source_hash") != kernel_source_hash():
        return None
    if int(kv.get("dtans_total_bytes", -1)) != info["total_bytes"]:
        return None
    return kv


def measured_traffic(workload, info):
    """HBM bytes per launch of the decode kernel from the committed counter
    summary (profiles/<workload>_traffic.txt)."""
    kv = profile_values("%s_traffic" % workload, info)
    return None if kv is None else int(kv["hbm_bytes_per_launch"])


def co_roofs(workload, info):
    """Utilisation of the decode kernel's other units (VALU issue, the vector
    memory address unit, LDS bandwidth) from the committed SQ/TA counter
    summary (profiles/<workload>_decode_sq_counters.txt)."""
    kv = profile_values("%s_decode_sq_counters" % workload, info)
    if kv is None:
        return None
    return {k: float(kv[k]) for k in ("valu_busy", "ta_busy", "lds_bandwidth_frac", "waves_waiting_frac")
            if k in kv} | {"source": "profiles/%s_decode_sq_counters.txt" % workload}


def time_steps(torch, fn, steps, warmup):
    for i in range(warmup):
        fn(i)
    torch.cuda.synchronize()
    start = torch.cuda.Event(enable_timing=True)
    end = torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    start.record()
    for i in range(steps):
        fn(i)
    end.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    return start.elapsed_time(end) / steps, wall


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def host_threads():
    """Threads the all-cores oracle run uses: the CPUs this process may run
    on (the box's share, not every core of the host)."""
    try:
        return len(os.sched_getaffinity(0))
    except AttributeError:
        return os.cpu_count() or 1


def cpu_baseline(W, seconds):
    """The oracle (plain FP64 CSR SpMV / SpMM in C, rows split over OpenMP
    threads) on the same matrix: one thread, then every CPU this process may
    use, each repeated for about seconds / 2."""
    import oracle

    rp, ci, v = W["rp"], W["ci"], W["v"]
    x = np.random.default_rng(0).uniform(-1, 1, W["n"])
    if W["k"] == 1:
        fn = lambda: oracle.spmv(rp, ci, v, x)  # noqa: E731
        flops = 2.0 * len(ci)
    else:
        X = np.random.default_rng(0).uniform(-1, 1, (W["n"], W["k"]))
        fn = lambda: oracle.spmm(rp, ci, v, X)  # noqa: E731
        flops = 2.0 * len(ci) * W["k"]

    def run(threads):
        oracle.set_threads(threads)
        fn()
        reps, t0 = 0, time.perf_counter()
        while True:
            fn()
            reps += 1
            el = time.perf_counter() - t0
            if el >= seconds / 2:
                break
        return flops * reps / el / 1e9, reps, el

    one = run(1)
    threads = host_threads()
    many = run(threads)
    oracle.set_threads(1)
    kind = "SpMV" if W["k"] == 1 else "SpMM k=%d" % W["k"]
    return {"value": many[0], "unit": "GFLOP/s", "cores": threads, "kind": "oracle",
            "sample": "oracle FP64 CSR %s over the whole matrix: %d repetitions in %.1f s on %d threads, "
                      "%d in %.1f s on one" % (kind, many[1], many[2], threads, one[1], one[2]),
            "single_core": {"value": one[0], "cores": 1},
            "cpu_count": os.cpu_count(), "cpu_model": cpu_model()}


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--workload", default="stencil",
                    help="stencil, band, rmat, skewed, pruned1, pruned8, pruned32, batch, batch8, "
                         "autograd, encode or sym")
    ap.add_argument("--layout", default="auto")
    ap.add_argument("--lane-nnz", type=int, default=0)
    ap.add_argument("--waves-per-wg", type=int, default=0)
    ap.add_argument("--wg-per-cu", type=int, default=0)
    ap.add_argument("--stream-stage", type=int, default=0,
                    help="SpMV: 0 auto, 1 direct word reads, 2 LDS ring")
    ap.add_argument("--first-delta-column", action="store_true",
                    help="first delta of a row is its column (the paper's form) instead of "
                         "column - row + 2^29")
    ap.add_argument("--max-mult", type=int, default=0,
                    help="multiplicity cap of the alphabet fit (0: the library's 255; 256 is the paper's M)")
    ap.add_argument("--escape-in-stream", action="store_true",
                    help="escaped symbols inside the word stream instead of separate regions")
    ap.add_argument("--sort-window", type=int, default=0,
                    help="row layout: encode rows sorted by length within windows of this many rows")
    ap.add_argument("--copies", type=int, default=0, help="0: enough to exceed twice the MALL")
    ap.add_argument("--cpu-seconds", type=float, default=10.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-csr", action="store_true")
    ap.add_argument("--no-paper-form", action="store_true",
                    help="stencil: skip the extra timing of the paper's own format")
    ap.add_argument("--no-warm", action="store_true", help="skip the single-copy (warm) timing")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="first run a plain device copy of MIB MiB three times (counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path "
              "(--gpus %d requested)" % args.gpus, file=sys.stderr)
        return 2

    import torch

    import paper_2603_01915_amd as P

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        return 2
    torch.cuda.set_device(0)
    if args.calibrate_copy:
        # a kernel that reads and writes exactly MIB MiB each: the HBM byte
        # counters of a profiled run are scaled by what they report for it
        src = torch.ones(args.calibrate_copy << 18, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            torch.mul(src, 1.0, out=dst)
        torch.cuda.synchronize()
        del src, dst
    if args.workload.startswith("batch"):
        return bench_batch(args, torch, P, int(args.workload[len("batch"):] or 1))
    if args.workload == "autograd":
        return bench_autograd(args, torch, P)
    if args.workload == "encode":
        return bench_encode(args, torch, P)
    if args.workload == "sym":
        return bench_sym(args, torch, P)
    log("generating workload %s" % args.workload)
    W = make_workload(args.workload)
    rp, ci, v, n, k = W["rp"], W["ci"], W["v"], W["n"], W["k"]
    m, nnz = len(rp) - 1, len(ci)
    is64 = v.dtype == np.float64
    vb = 8 if is64 else 4
    tdt = torch.float64 if is64 else torch.float32
    log("encoding %d x %d, %d nonzeros" % (m, n, nnz))
    t0 = time.perf_counter()
    A0 = P.Matrix.from_csr(rp, ci, v, n, layout=args.layout, lane_nnz=args.lane_nnz,
                           waves_per_wg=args.waves_per_wg, wg_per_cu=args.wg_per_cu,
                           stream_stage=args.stream_stage, first_delta_column=args.first_delta_column,
                           max_mult=args.max_mult, escape_in_stream=args.escape_in_stream,
                           sort_window=args.sort_window)
    enc_s = time.perf_counter() - t0
    info = A0.info()
    log("encoded in %.1f s: %.2f bits/nnz, %d bytes (CSR %d)" % (enc_s, info["bits_per_nnz"],
                                                                 info["total_bytes"], info["csr_bytes"]))
    vec_bytes = (n + m) * k * vb
    per_copy = info["total_bytes"] + vec_bytes
    copies = args.copies or max(1, math.ceil(2 * MALL_BYTES / per_copy))
    mats = [A0]
    if copies > 1:  # further copies come from the saved container (load verifies it)
        import tempfile

        with tempfile.TemporaryDirectory() as td:
            path = os.path.join(td, "a.dtans")
            A0.save(path)
            for _ in range(copies - 1):
                B = P.Matrix.load(path)
                B.set_launch(args.waves_per_wg, args.wg_per_cu, args.stream_stage)
                mats.append(B)
    for A in mats:  # upload and size each copy's scratch before any timing
        A.to_device().reserve(k)
    gen = torch.Generator(device="cuda").manual_seed(2000 + W["cfg"])
    shape_x = (n,) if k == 1 else (n, k)
    shape_y = (m,) if k == 1 else (m, k)
    xs = [torch.rand(shape_x, dtype=tdt, device="cuda", generator=gen) * 2 - 1 for _ in range(copies)]
    ys = [torch.empty(shape_y, dtype=tdt, device="cuda") for _ in range(copies)]

    def step(i):
        j = i % copies
        if k == 1:
            mats[j].spmv(xs[j], ys[j])
        else:
            mats[j].spmm(xs[j], ys[j])

    log("timing %d steps over %d copies" % (args.steps, copies))
    ms, wall = time_steps(torch, step, args.steps, args.warmup)
    warm_ms = None if args.no_warm else time_steps(torch, lambda i: step(0), args.steps, args.warmup)[0]
    flops = 2.0 * nnz * k
    alg_bytes = info["total_bytes"] + vec_bytes
    gflops = flops / (ms * 1e-3) / 1e9
    achieved = alg_bytes / (ms * 1e-3) / 1e9
    res = {
        "metric": METRIC, "value": round(gflops, 3), "unit": "GFLOP/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms, 6),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64" if is64 else "f32", "data": "synthetic (seeded generator)",
        "config": {"workload": W["name"], "rows": m, "cols": n, "nnz": nnz, "k": k,
                   "layout": {1: "row", 2: "nnz"}[info["layout"]], "lane_nnz": info["lane_nnz"],
                   "waves_per_wg": info["waves_per_wg"],
                   "stream_stage": {1: "direct", 2: "lds_ring"}[info["stream_stage"]],
                   "first_delta": "column" if info["first_delta_column"] else "column - row + 2^29",
                   "max_mult": args.max_mult or 255, "direct_table": bool(info["direct_table"]),
                   "escapes": "in stream" if info["escape_in_stream"] else "separate regions",
                   "sort_window": info["sort_window"],
                   "copies_rotated": copies},
        "compressed_GBps": round(achieved, 2),
        "roofline": {"bound": "hbm", "achieved": round(achieved, 2), "peak": HBM_PEAK_GBPS,
                     "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBPS, 4), "traffic": None,
                     "algorithmic_bytes_per_launch": alg_bytes},
        "compression": {"dtans_bytes": info["total_bytes"], "stream_bytes": info["stream_bytes"],
                        "csr_bytes": info["csr_bytes"], "coo_bytes": info["coo_bytes"],
                        "sell32_bytes": info["sell_bytes"], "bits_per_nnz": round(info["bits_per_nnz"], 3),
                        "ratio_vs_csr": round(info["csr_bytes"] / info["total_bytes"], 3),
                        "ratio_vs_smallest": round(min(info["csr_bytes"], info["coo_bytes"],
                                                       info["sell_bytes"]) / info["total_bytes"], 3),
                        "escaped_deltas": info["esc_delta"], "escaped_values": info["esc_value"]},
        "warm": None if warm_ms is None else {
            "ms": round(warm_ms, 6), "GFLOP/s": round(flops / (warm_ms * 1e-3) / 1e9, 3),
            "GB/s": round(alg_bytes / (warm_ms * 1e-3) / 1e9, 2)},
        "encode_seconds": round(enc_s, 2),
    }
    res["roofline"]["traffic"] = measured_traffic(args.workload, info)
    res["roofline"]["co_roofs"] = co_roofs(args.workload, info)
    if not args.no_csr:
        log("plain CSR baseline")
        B = P.CsrBaseline(rp, ci, v, n)
        csr_copies = max(1, math.ceil(2 * MALL_BYTES / (B.bytes + vec_bytes)))
        Bs = [B] + [P.CsrBaseline(rp, ci, v, n) for _ in range(csr_copies - 1)]
        bx = [torch.rand(shape_x, dtype=tdt, device="cuda", generator=gen) * 2 - 1 for _ in range(csr_copies)]
        by = [torch.empty(shape_y, dtype=tdt, device="cuda") for _ in range(csr_copies)]

        def cstep(i):
            j = i % csr_copies
            if k == 1:
                Bs[j].spmv(bx[j], by[j])
            else:
                Bs[j].spmm(bx[j], by[j])

        cms, _ = time_steps(torch, cstep, args.steps, args.warmup)
        cb = B.bytes + vec_bytes
        res["csr_baseline"] = {"ms": round(cms, 6), "GFLOP/s": round(flops / (cms * 1e-3) / 1e9, 3),
                               "GB/s": round(cb / (cms * 1e-3) / 1e9, 2),
                               "frac": round(cb / (cms * 1e-3) / 1e9 / HBM_PEAK_GBPS, 4),
                               "copies_rotated": csr_copies}
        res["speedup_vs_csr"] = round(cms / ms, 3)
        log("rocSPARSE baseline")
        R = P.RocsparseBaseline(rp, ci, v, n)
        Rs = [R] + [P.RocsparseBaseline(rp, ci, v, n) for _ in range(csr_copies - 1)]

        def rstep(i):
            j = i % csr_copies
            if k == 1:
                Rs[j].spmv(bx[j], by[j])
            else:
                Rs[j].spmm(bx[j], by[j])

        rms, _ = time_steps(torch, rstep, args.steps, args.warmup)
        res["rocsparse_baseline"] = {"ms": round(rms, 6), "GFLOP/s": round(flops / (rms * 1e-3) / 1e9, 3),
                                     "GB/s": round(cb / (rms * 1e-3) / 1e9, 2),
                                     "frac": round(cb / (rms * 1e-3) / 1e9 / HBM_PEAK_GBPS, 4),
                                     "alg": "csr_adaptive" if k == 1 else "spmm default (csr)",
                                     "copies_rotated": csr_copies}
        res["speedup_vs_rocsparse"] = round(rms / ms, 3)
        for B_ in Rs:
            B_.close()
    if args.workload == "stencil" and not args.no_paper_form and not args.first_delta_column and not args.max_mult:
        # the same product in the paper's own format: first delta = column,
        # multiplicity cap M = 256 (general tables)
        log("paper-form encoding")
        A1 = P.Matrix.from_csr(rp, ci, v, n, layout=args.layout, lane_nnz=args.lane_nnz,
                               first_delta_column=True, max_mult=256)
        inf1 = A1.info()
        per1 = inf1["total_bytes"] + vec_bytes
        c1 = max(1, math.ceil(2 * MALL_BYTES / per1))
        ms1 = [A1]
        if c1 > 1:
            import tempfile

            with tempfile.TemporaryDirectory() as td:
                path = os.path.join(td, "p.dtans")
                A1.save(path)
                ms1 += [P.Matrix.load(path) for _ in range(c1 - 1)]
        for M_ in ms1:
            M_.to_device().reserve(k)
        x1 = [xs[i % copies] for i in range(c1)]
        y1 = [torch.empty(shape_y, dtype=tdt, device="cuda") for _ in range(c1)]
        pms, _ = time_steps(torch, lambda i: ms1[i % c1].spmv(x1[i % c1], y1[i % c1]), args.steps, args.warmup)
        ab1 = inf1["total_bytes"] + vec_bytes
        res["paper_form"] = {"ms": round(pms, 6), "GFLOP/s": round(flops / (pms * 1e-3) / 1e9, 3),
                             "frac": round(ab1 / (pms * 1e-3) / 1e9 / HBM_PEAK_GBPS, 4),
                             "bits_per_nnz": round(inf1["bits_per_nnz"], 3),
                             "escaped_deltas": inf1["esc_delta"], "direct_table": bool(inf1["direct_table"]),
                             "first_delta": "column", "max_mult": 256, "copies_rotated": c1}
        if "csr_baseline" in res:
            res["paper_form"]["speedup_vs_csr"] = round(res["csr_baseline"]["ms"] / pms, 3)
    if not args.no_cpu_baseline:
        log("CPU oracle baseline")
        res["cpu_baseline"] = cpu_baseline(W, args.cpu_seconds)
    print(json.dumps(res), flush=True)
    return 0


def bench_autograd(args, torch, P):
    """The differentiable product on the pruned 11008 x 4096 weight with a
    batch of 16: one step is the forward Y = A X and the backward
    dX = A^T dY through DtansLinearFn.  The headline keeps an encoded A^T
    beside A (the backward is a product on it); the decode-and-scatter
    backward over A's own streams (A stored once) is timed too.  The plain
    CSR baseline runs the forward on A and the backward on an explicitly
    transposed CSR copy of A."""
    import scipy.sparse as sp

    from paper_2603_01915_amd.autograd import DtansLinearFn, transpose_csr
    import workloads

    rp, ci, v = workloads.pruned_weight()
    m, n, k, nnz = len(rp) - 1, 4096, 16, len(ci)
    log("encoding %d x %d, %d nonzeros, and its transpose" % (m, n, nnz))
    t0 = time.perf_counter()
    A0 = P.Matrix.from_csr(rp, ci, v, n)
    At0 = P.Matrix.from_csr(*transpose_csr(rp, ci, v, n), m)
    enc_s = time.perf_counter() - t0
    info, info_t = A0.info(), At0.info()
    vec_bytes = 2 * (n + m) * k * 4
    copies = args.copies or max(1, math.ceil(2 * MALL_BYTES / (info["total_bytes"] + info_t["total_bytes"]
                                                             + vec_bytes)))

    def replicate(M0):
        mats = [M0]
        if copies > 1:
            import tempfile

            with tempfile.TemporaryDirectory() as td:
                path = os.path.join(td, "a.dtans")
                M0.save(path)
                mats += [P.Matrix.load(path) for _ in range(copies - 1)]
        for M in mats:  # upload and size each copy's scratch before any timing
            M.to_device().reserve(k)
        return mats

    mats, mats_t = replicate(A0), replicate(At0)
    gen = torch.Generator(device="cuda").manual_seed(2005)
    Xs = [(torch.rand((n, k), dtype=torch.float32, device="cuda", generator=gen) * 2 - 1).requires_grad_()
          for _ in range(copies)]
    dYs = [torch.rand((m, k), dtype=torch.float32, device="cuda", generator=gen) * 2 - 1 for _ in range(copies)]

    def step(i):
        j = i % copies
        Y = DtansLinearFn.apply(mats[j], Xs[j], mats_t[j])
        Y.backward(dYs[j])

    def step_scatter(i):
        j = i % copies
        Y = DtansLinearFn.apply(mats[j], Xs[j])
        Y.backward(dYs[j])

    log("timing %d steps over %d copies (encoded transpose)" % (args.steps, copies))
    ms, _ = time_steps(torch, step, args.steps, args.warmup)
    log("timing %d steps over %d copies (decode-and-scatter)" % (args.steps, copies))
    sms, _ = time_steps(torch, step_scatter, args.steps, args.warmup)
    flops = 2 * 2.0 * nnz * k
    alg = info["total_bytes"] + info_t["total_bytes"] + vec_bytes
    salg = 2 * info["total_bytes"] + vec_bytes
    res = {
        "metric": METRIC, "value": round(flops / (ms * 1e-3) / 1e9, 3), "unit": "GFLOP/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms, 6),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic (seeded generator)",
        "config": {"workload": "autograd pruned 11008x4096 fp32, batch 16, forward + backward "
                               "(backward on an encoded transpose)",
                   "rows": m, "cols": n, "nnz": nnz, "k": k, "layout": {1: "row", 2: "nnz"}[info["layout"]],
                   "layout_transpose": {1: "row", 2: "nnz"}[info_t["layout"]],
                   "lane_nnz": info["lane_nnz"], "copies_rotated": copies},
        "compressed_GBps": round(alg / (ms * 1e-3) / 1e9, 2),
        "roofline": {"bound": "hbm", "achieved": round(alg / (ms * 1e-3) / 1e9, 2), "peak": HBM_PEAK_GBPS,
                     "unit": "GB/s", "frac": round(alg / (ms * 1e-3) / 1e9 / HBM_PEAK_GBPS, 4),
                     "traffic": None, "algorithmic_bytes_per_launch": alg},
        "compression": {"dtans_bytes": info["total_bytes"], "dtans_transpose_bytes": info_t["total_bytes"],
                        "csr_bytes": info["csr_bytes"],
                        "ratio_vs_csr": round(info["csr_bytes"] / info["total_bytes"], 3)},
        "scatter_backward": {"ms": round(sms, 6), "GFLOP/s": round(flops / (sms * 1e-3) / 1e9, 3),
                             "GBps": round(salg / (sms * 1e-3) / 1e9, 2),
                             "note": "backward by decode-and-scatter over A (A stored once)"},
        "encode_seconds": round(enc_s, 2),
    }
    if not args.no_csr:
        log("plain CSR baseline: forward on A, backward on A^T")
        At = sp.csr_matrix((v, ci, rp), shape=(m, n)).T.tocsr()
        At.sort_indices()
        rpt, cit, vt = At.indptr.astype(np.int32), At.indices.astype(np.int32), At.data.astype(np.float32)
        B, Bt = P.CsrBaseline(rp, ci, v, n), P.CsrBaseline(rpt, cit, vt, m)
        ccopies = max(1, math.ceil(2 * MALL_BYTES / (2 * B.bytes + vec_bytes)))
        pairs = [(B, Bt)] + [(P.CsrBaseline(rp, ci, v, n), P.CsrBaseline(rpt, cit, vt, m))
                             for _ in range(ccopies - 1)]
        cX = [torch.rand((n, k), dtype=torch.float32, device="cuda", generator=gen) for _ in range(ccopies)]
        cdY = [torch.rand((m, k), dtype=torch.float32, device="cuda", generator=gen) for _ in range(ccopies)]
        cY = [torch.empty((m, k), dtype=torch.float32, device="cuda") for _ in range(ccopies)]
        cdX = [torch.empty((n, k), dtype=torch.float32, device="cuda") for _ in range(ccopies)]

        def cstep(i):
            j = i % ccopies
            pairs[j][0].spmm(cX[j], cY[j])
            pairs[j][1].spmm(cdY[j], cdX[j])

        cms, _ = time_steps(torch, cstep, args.steps, args.warmup)
        res["csr_baseline"] = {"ms": round(cms, 6), "GFLOP/s": round(flops / (cms * 1e-3) / 1e9, 3),
                               "copies_rotated": ccopies}
        res["speedup_vs_csr"] = round(cms / ms, 3)
    print(json.dumps(res), flush=True)
    return 0


def bench_encode(args, torch, P):
    """Encoding throughput (nonzeros per second, CSR arrays in, host
    container out) of dtans_encode_csr and dtans_encode_csr_gpu (host arrays)
    and dtans_encode_csr_device (arrays already in device memory), whose
    containers are identical; each is the best of `steps` (at most 5) calls.
    The GPU calls include their uploads and downloads."""
    import workloads

    steps = max(1, min(args.steps, 5))
    cases = []
    rp, ci, v = workloads.stencil27(128)
    cases.append(("stencil27 128^3 fp64, row layout", rp, ci, v, 128 ** 3, "row"))
    rp, ci, v = workloads.pruned_weight()
    cases.append(("pruned 11008x4096 fp32, nnz layout", rp, ci, v, 4096, "auto"))
    out = []
    for name, rp, ci, v, n, layout in cases:
        drp = torch.from_numpy(np.ascontiguousarray(rp, np.int32)).cuda()
        dci = torch.from_numpy(np.ascontiguousarray(ci, np.int32)).cuda()
        dv = torch.from_numpy(np.ascontiguousarray(v)).cuda()
        times = {}
        for mode in ("host", "gpu", "device"):
            best = None
            for _ in range(steps + (0 if mode == "host" else 1)):  # one untimed GPU call first
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                if mode == "device":
                    A = P.Matrix.from_csr_device(drp, dci, dv, n, layout=layout)
                else:
                    A = P.Matrix.from_csr(rp, ci, v, n, layout=layout, gpu_encode=mode == "gpu")
                dt = time.perf_counter() - t0
                A.close()
                best = dt if best is None else min(best, dt)
            times[mode] = best
            log("%s: %s encoder %.3f s" % (name, mode, best))
        del drp, dci, dv
        out.append({"workload": name, "nnz": len(ci), "host_s": round(times["host"], 4),
                    "gpu_s": round(times["gpu"], 4), "gpu_device_inputs_s": round(times["device"], 4),
                    "host_Mnnz_per_s": round(len(ci) / times["host"] / 1e6, 1),
                    "gpu_Mnnz_per_s": round(len(ci) / times["gpu"] / 1e6, 1),
                    "gpu_device_inputs_Mnnz_per_s": round(len(ci) / times["device"] / 1e6, 1),
                    "speedup": round(times["host"] / times["gpu"], 3)})
    res = {"metric": "encode throughput (host CSR arrays to container)", "value": out[0]["gpu_Mnnz_per_s"],
           "unit": "Mnnz/s", "n_gpus": 1, "steps": steps, "warmup": 1,
           "ms_per_step": round(out[0]["gpu_s"] * 1e3, 3), "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": "u32", "data": "synthetic (seeded generator)",
           "config": {"workload": "encode " + out[0]["workload"]}, "cases": out,
           "host_threads": min(os.cpu_count() or 4, 32), "roofline": None,
           "note": "word-pass kernel times are in the rocprofv3 kernel trace; the rest of either call "
                   "(keys, alphabet fit, tables, symbol lookup, escapes) runs on the host"}
    print(json.dumps(res), flush=True)
    return 0


def bench_sym(args, torch, P):
    """A symmetric 128^3 27-point stencil in FP64 (the upper triangle of the
    stencil mirrored, so the 216-value pool is kept): SpMV through the strict
    upper triangle and the diagonal (dtans_spmv_sym, half storage) against the
    ordinary SpMV on the whole encoded matrix; both rotate copies past the
    MALL."""
    import scipy.sparse as sp

    import workloads

    rp, ci, v = workloads.stencil27(128)
    n = 128 ** 3
    A = sp.csr_matrix((v, ci, rp), shape=(n, n))
    U = sp.triu(A, k=1).tocsr()
    S = (sp.triu(A) + U.T).tocsr()
    S.sort_indices()
    rps, cis, vs = S.indptr.astype(np.int32), S.indices.astype(np.int32), S.data
    rpu, ciu, vu, d = P.symmetric_split(rps, cis, vs)
    log("encoding the whole matrix (%d nonzeros) and its strict upper triangle (%d)" % (len(cis), len(ciu)))
    F0 = P.Matrix.from_csr(rps, cis, vs, n)
    H0 = P.Matrix.from_csr(rpu, ciu, vu, n)
    fi, hi = F0.info(), H0.info()

    def copies_of(M0, extra):
        c = args.copies or max(1, math.ceil(2 * MALL_BYTES / (M0.info()["total_bytes"] + extra)))
        mats = [M0]
        if c > 1:
            import tempfile

            with tempfile.TemporaryDirectory() as td:
                path = os.path.join(td, "a.dtans")
                M0.save(path)
                mats += [P.Matrix.load(path) for _ in range(c - 1)]
        for M in mats:
            M.to_device()
        return mats

    vec = 2 * n * 8
    full, half = copies_of(F0, vec), copies_of(H0, vec + n * 8)
    gen = torch.Generator(device="cuda").manual_seed(7)
    nc = max(len(full), len(half))
    xs = [torch.rand(n, dtype=torch.float64, device="cuda", generator=gen) * 2 - 1 for _ in range(nc)]
    ys = [torch.empty(n, dtype=torch.float64, device="cuda") for _ in range(nc)]
    ds = [torch.from_numpy(d).cuda() for _ in range(len(half))]
    fms, _ = time_steps(torch, lambda i: full[i % len(full)].spmv(xs[i % nc], ys[i % nc]), args.steps,
                        args.warmup)
    hms, _ = time_steps(torch, lambda i: half[i % len(half)].spmv_sym(xs[i % nc], ds[i % len(half)], ys[i % nc]),
                        args.steps, args.warmup)
    flops = 2.0 * len(cis)
    res = {"metric": METRIC, "value": round(flops / (hms * 1e-3) / 1e9, 3), "unit": "GFLOP/s", "n_gpus": 1,
           "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(hms, 6), "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic (seeded generator)",
           "config": {"workload": "symmetric stencil27 128^3 fp64 spmv through its strict upper triangle",
                      "rows": n, "nnz_whole": len(cis), "nnz_triangle": len(ciu),
                      "copies_rotated": [len(full), len(half)]},
           "roofline": None,
           "whole_matrix": {"ms": round(fms, 6), "GFLOP/s": round(flops / (fms * 1e-3) / 1e9, 3),
                            "dtans_bytes": fi["total_bytes"], "bits_per_nnz": round(fi["bits_per_nnz"], 3)},
           "half_storage": {"ms": round(hms, 6), "dtans_bytes": hi["total_bytes"] + n * 8,
                            "bits_per_nnz_triangle": round(hi["bits_per_nnz"], 3),
                            "transpose_path": "global atomics" if n * 8 > 64 * 1024 else "LDS copies"},
           "note": "the transposed half scatters into y with atomic adds; GFLOP/s counts the whole matrix"}
    print(json.dumps(res), flush=True)
    return 0


def bench_batch(args, torch, P, k=1):
    """64 banded FP32 matrices of 1k-64k rows (8-64 nonzeros per row) in one
    persistent launch (k right-hand sides per matrix: one launch per column
    chunk), against the plain CSR kernel launched per matrix."""
    import workloads

    log("generating 64 uneven matrices")
    mats_csr = workloads.batch()
    total_nnz = sum(len(c[1]) for _, c in mats_csr)
    log("encoding %d matrices, %d nonzeros" % (len(mats_csr), total_nnz))
    t0 = time.perf_counter()
    enc = [P.Matrix.from_csr(c[0], c[1], c[2], m, layout="row", sort_window=args.sort_window) for m, c in mats_csr]
    enc_s = time.perf_counter() - t0
    dt_bytes = sum(A.info()["total_bytes"] for A in enc)
    csr_bytes = sum(A.info()["csr_bytes"] for A in enc)
    vec_bytes = sum(2 * m * 4 * k for m, _ in mats_csr)
    copies = args.copies or max(1, math.ceil(2 * MALL_BYTES / (dt_bytes + vec_bytes)))
    sets = [enc]
    if copies > 1:
        import tempfile

        with tempfile.TemporaryDirectory() as td:
            paths = []
            for i, A in enumerate(enc):
                paths.append(os.path.join(td, "a%d.dtans" % i))
                A.save(paths[-1])
            for _ in range(copies - 1):
                sets.append([P.Matrix.load(q) for q in paths])
    for S in sets:
        for A in S:
            A.to_device()
    batches = [P.Batch(S) for S in sets]
    gen = torch.Generator(device="cuda").manual_seed(2005)
    shp = (lambda m: (m,)) if k == 1 else (lambda m: (m, k))
    xs = [[torch.rand(shp(m), dtype=torch.float32, device="cuda", generator=gen) * 2 - 1 for m, _ in mats_csr]
          for _ in range(copies)]
    ys = [[torch.empty(shp(m), dtype=torch.float32, device="cuda") for m, _ in mats_csr] for _ in range(copies)]

    def step(i):
        j = i % copies
        if k == 1:
            batches[j].spmv(xs[j], ys[j])
        else:
            batches[j].spmm(xs[j], ys[j])

    log("timing %d steps over %d copies" % (args.steps, copies))
    ms, _ = time_steps(torch, step, args.steps, args.warmup)
    flops = 2.0 * total_nnz * k
    alg = dt_bytes + vec_bytes
    res = {
        "metric": METRIC, "value": round(flops / (ms * 1e-3) / 1e9, 3), "unit": "GFLOP/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms, 6),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic (seeded generator)",
        "config": {"workload": "batch of 64 banded fp32 matrices, 1k-64k rows, 8-64 nnz/row, one launch"
                               + ("" if k == 1 else " per column chunk, k=%d" % k),
                   "matrices": len(mats_csr), "nnz": total_nnz, "k": k, "layout": "row",
                   "copies_rotated": copies},
        "compressed_GBps": round(alg / (ms * 1e-3) / 1e9, 2),
        "roofline": {"bound": "hbm", "achieved": round(alg / (ms * 1e-3) / 1e9, 2), "peak": HBM_PEAK_GBPS,
                     "unit": "GB/s", "frac": round(alg / (ms * 1e-3) / 1e9 / HBM_PEAK_GBPS, 4),
                     "traffic": None, "algorithmic_bytes_per_launch": alg},
        "compression": {"dtans_bytes": dt_bytes, "csr_bytes": csr_bytes,
                        "ratio_vs_csr": round(csr_bytes / dt_bytes, 3)},
        "encode_seconds": round(enc_s, 2),
    }
    if not args.no_csr:
        log("plain CSR baseline, one launch per matrix")
        ccopies = max(1, math.ceil(2 * MALL_BYTES / (csr_bytes + vec_bytes)))
        cs = [[P.CsrBaseline(c[0], c[1], c[2], m) for m, c in mats_csr] for _ in range(ccopies)]
        cx = [[torch.rand(shp(m), dtype=torch.float32, device="cuda", generator=gen) * 2 - 1 for m, _ in mats_csr]
              for _ in range(ccopies)]
        cy = [[torch.empty(shp(m), dtype=torch.float32, device="cuda") for m, _ in mats_csr] for _ in range(ccopies)]

        def cstep(i):
            j = i % ccopies
            for B, x, y in zip(cs[j], cx[j], cy[j]):
                if k == 1:
                    B.spmv(x, y)
                else:
                    B.spmm(x, y)

        cms, _ = time_steps(torch, cstep, args.steps, args.warmup)
        res["csr_baseline"] = {"ms": round(cms, 6), "GFLOP/s": round(flops / (cms * 1e-3) / 1e9, 3),
                               "copies_rotated": ccopies, "launches_per_step": len(mats_csr)}
        res["speedup_vs_csr"] = round(cms / ms, 3)
        del cs, cx, cy
        # one launch for all matrices: the block-diagonal CSR matrix of the
        # batch (rows and columns of matrix i offset by those before it), x
        # and y the matrices' vectors laid end to end
        log("plain CSR baseline, one launch (block diagonal)")
        import numpy as np

        offs = np.cumsum([0] + [m for m, _ in mats_csr])
        lens = np.concatenate([np.diff(c[0]) for _, c in mats_csr])
        rp_all = np.zeros(len(lens) + 1, np.int64)
        np.cumsum(lens, out=rp_all[1:])
        ci_all = np.concatenate([c[1].astype(np.int64) + offs[i] for i, (_, c) in enumerate(mats_csr)])
        v_all = np.concatenate([c[2] for _, c in mats_csr])
        ntot = int(offs[-1])
        one = [P.CsrBaseline(rp_all.astype(np.int32), ci_all.astype(np.int32), v_all, ntot)
               for _ in range(ccopies)]
        ox = [torch.rand(shp(ntot), dtype=torch.float32, device="cuda", generator=gen) * 2 - 1
              for _ in range(ccopies)]
        oy = [torch.empty(shp(ntot), dtype=torch.float32, device="cuda") for _ in range(ccopies)]

        def ostep(i):
            j = i % ccopies
            if k == 1:
                one[j].spmv(ox[j], oy[j])
            else:
                one[j].spmm(ox[j], oy[j])

        oms, _ = time_steps(torch, ostep, args.steps, args.warmup)
        res["csr_one_launch_baseline"] = {"ms": round(oms, 6), "GFLOP/s": round(flops / (oms * 1e-3) / 1e9, 3),
                                          "copies_rotated": ccopies,
                                          "note": "block-diagonal CSR of the 64 matrices, one launch"}
        res["speedup_vs_csr_one_launch"] = round(oms / ms, 3)
    print(json.dumps(res), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
