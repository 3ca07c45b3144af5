#!/usr/bin/env python3
"""Benchmark of the M2L translation (Sec. 4.1) on one MI355X.

A step is one M2L + fused reduction over every box of levels 2..depth (the
whole interaction-list schedule, contraction and reduction), on expansions
already resident in HBM; the operator bank is generated once per p before
timing, as the operators depend only on p.  The default workload is N = 2^20
uniform points, quadtree depth 8, p = 12, FP32.

Prints one JSON line with translations/s (exact, boundary-truncated count),
the 8p^2-flop Gop/s, the roofline of the M2L kernel measured with HIP events
on the stream it runs on, the adjoint's time, and the FP64 oracle's rate on
the host cores.
"""
from __future__ import annotations

import argparse
import ctypes
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

# name -> (points, depth, p, point set, precision)
WORKLOADS = {
    "m2l_uniform_n1M_d8_p12": (1 << 20, 8, 12, "uniform", "f32"),
    "m2l_mixed_n4M_d9_p16": (1 << 22, 9, 16, "mixed", "f32"),
    "m2l_mixed_n16M_d10_p20": (1 << 24, 10, 20, "mixed", "f32"),
    "m2l_uniform_n4k_d4_p8": (4096, 4, 8, "uniform", "f32"),
}
DEFAULT = "m2l_uniform_n1M_d8_p12"
PEAK_FP32_MFMA_TFLOPS = 157.3   # MI355X dense FP32 matrix peak
PEAK_HBM_GBS = 8000.0
PAPER_P12_TRANS_PER_S = 80.05e6  # Tesla C1060, p = 12, depth-8 tree (Table tab:m2ltesla)


def m2l_kernel_sources(precision="f32"):
    """Source files whose text decides the M2L kernel's memory traffic."""
    c = os.path.join(ROOT, "paper_1009_3457_amd", "csrc")
    names = ["m2l_f32.hip", "m2l_bank.h", "m2l_common.h", "fmm2d_internal.h"]
    if precision != "f32":
        names = ["m2l_mixed.hip", "m2l_mixed_bank.h", "m2l_common.h", "fmm2d_internal.h"]
    return [os.path.join(c, n) for n in names]


def source_digest(paths):
    import hashlib
    h = hashlib.sha256()
    for pth in paths:
        with open(pth, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def recorded_traffic(workload, precision):
    """HBM bytes per launch from the committed FETCH_SIZE / WRITE_SIZE summary,
    or None when it is absent or was taken on different kernel sources."""
    tpath = os.path.join(ROOT, "profiles", f"traffic_{workload}_{precision}.json")
    if not os.path.exists(tpath):
        return None
    with open(tpath) as fh:
        rec = json.load(fh)
    if rec.get("source_sha256") != source_digest(m2l_kernel_sources(precision)):
        return None
    return rec.get("bytes_per_launch")


def _points(kind, n, seed):
    import synthetic as sy
    return sy.uniform(n, seed) if kind == "uniform" else sy.mixed(n, seed)


def cpu_baseline(Ms_np, depth, p, budget_s=12.0, max_runs=200):
    """The FP64 oracle's M2L (operator built per translation from Eq.
    (eq:M2Lmat)) over all levels 2..depth, timed on the host cores; repeated
    while the time budget allows (at least once), median reported."""
    import numpy as np

    import oracle
    M = oracle.unscale_multipoles(Ms_np.astype(np.complex128), depth)
    ntrans = None
    times = []
    t_start = time.perf_counter()
    while len(times) < max_runs:
        t0 = time.perf_counter()
        oracle.m2l(M, depth, p)
        times.append(time.perf_counter() - t0)
        if time.perf_counter() - t_start + times[-1] > budget_s:
            break
    import paper_1009_3457_amd as P
    ntrans = P.translation_count(2, depth)
    med = sorted(times)[len(times) // 2]
    return {"value": ntrans / med, "unit": "translations/s", "cores": oracle.num_threads(),
            "kind": "oracle",
            "sample": f"full M2L, levels 2..{depth}, p={p}, {ntrans} translations, FP64, "
                      f"median of {len(times)} runs ({med:.3f} s each)"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--workload", default=DEFAULT, choices=sorted(WORKLOADS))
    ap.add_argument("--precision", default=None, choices=["f32", "bf16x3", "f16x3"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--seed", type=int, default=1)
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="only run a plain 256 MiB device-to-device copy, 4 times (reference for "
                         "scaling the FETCH_SIZE / WRITE_SIZE counters)")
    args = ap.parse_args()

    if args.calibrate_copy:
        import torch
        src = torch.ones(64 << 20, dtype=torch.float32, device="cuda:0")
        dst = torch.empty_like(src)
        for _ in range(4):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_each_way": src.numel() * 4, "copies": 4}))
        return

    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on exactly one GPU; the M2L of one "
                                   "device's share is measured at --gpus 1"}))
        sys.exit(2)

    import numpy as np
    import torch

    import paper_1009_3457_amd as P
    import synthetic as sy
    from paper_1009_3457_amd import _binding as B

    n, depth, p, kind, prec_name = WORKLOADS[args.workload]
    prec_name = args.precision or prec_name
    prec = B.PRECISIONS[prec_name]
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)

    # inputs resident in HBM: points -> tree -> P2M -> M2M on the GPU
    xy = torch.from_numpy(_points(kind, n, args.seed)).to(dev)
    q = torch.from_numpy(sy.charges(n, args.seed + 1)).to(dev)
    perm, ls = P.build_tree(xy, depth)
    xs, qs = P.gather(xy, perm), P.gather(q, perm)
    M = P.m2m(P.p2m(xs, qs, ls, depth, p), depth, p)
    ops = P.m2l_operators(p, prec, dev)
    nb = P.num_boxes(depth)
    L = torch.zeros(nb, p, dtype=torch.complex64, device=dev)
    b = torch.zeros(nb, dtype=torch.complex64, device=dev)
    gM = torch.zeros(nb, p, dtype=torch.complex64, device=dev)
    torch.cuda.synchronize(dev)

    lib = B.load()
    stream = torch.cuda.current_stream(dev)
    sp = ctypes.c_void_p(stream.cuda_stream)
    vp = ctypes.c_void_p
    fwd_args = (vp(M.data_ptr()), vp(L.data_ptr()), vp(b.data_ptr()), depth, p, 2, depth, prec,
                vp(ops.data_ptr()), ops.numel(), sp)
    bwd_args = (vp(L.data_ptr()), vp(b.data_ptr()), vp(gM.data_ptr()), depth, p, 2, depth, prec,
                vp(ops.data_ptr()), ops.numel(), sp)
    fwd, bwd = lib.fmm2d_m2l, lib.fmm2d_m2l_backward

    def timed(fn, fargs, steps, warmup):
        for _ in range(warmup):
            if fn(*fargs) != 0:
                raise RuntimeError(lib.fmm2d_last_error().decode())
        torch.cuda.synchronize(dev)
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        rc = 0
        for _ in range(steps):
            rc |= fn(*fargs)
        e1.record(stream)
        torch.cuda.synchronize(dev)
        if rc != 0:
            raise RuntimeError(lib.fmm2d_last_error().decode())
        return e0.elapsed_time(e1) / steps  # ms per launch

    # the timed region: K forward M2L steps, bracketed by synchronisation
    ms_fwd = timed(fwd, fwd_args, args.steps, args.warmup)
    ms_bwd = timed(bwd, bwd_args, max(args.steps // 2, 1), max(args.warmup // 2, 1))

    ntrans = P.translation_count(2, depth)
    padded = 27 * sum(4 ** l for l in range(2, depth + 1))
    flops = 8.0 * p * p * ntrans
    tflops = flops / (ms_fwd * 1e-3) / 1e12
    boxes = sum(4 ** l for l in range(2, depth + 1))
    alg_bytes = boxes * p * 8 * 2 + boxes * 8  # read M~, write L~ and b (complex64)
    value = ntrans / (ms_fwd * 1e-3)

    traffic = recorded_traffic(args.workload, prec_name)

    out = {
        "metric": "M2L Gop/s & translations/s (N=2^20, p=12), % of roofline; mixed vs FP32 at tol",
        "value": value,
        "unit": "translations/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_fwd,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": value / PAPER_P12_TRANS_PER_S if (depth, p) == (8, 12) else None,
        "dtype": "f32" if prec_name == "f32" else prec_name,
        "data": "synthetic",
        "config": {"workload": args.workload, "points": n, "point_set": kind, "depth": depth,
                   "p": p, "levels": f"2..{depth}", "precision": prec_name,
                   "translations": ntrans, "padded_translations": padded},
        "gop_s": flops / (ms_fwd * 1e-3) / 1e9,
        "roofline": {"bound": "mfma", "achieved": tflops, "peak": PEAK_FP32_MFMA_TFLOPS,
                     "unit": "TFLOP/s", "frac": tflops / PEAK_FP32_MFMA_TFLOPS,
                     "traffic": traffic,
                     "algorithmic_bytes": alg_bytes,
                     "hbm_frac": alg_bytes / (ms_fwd * 1e-3) / 1e9 / PEAK_HBM_GBS},
        "adjoint_ms": ms_bwd,
        "adjoint_translations_per_s": ntrans / (ms_bwd * 1e-3),
        "paper_context": {"translations_per_s": PAPER_P12_TRANS_PER_S, "gop_s": 511.06,
                          "hardware": "Tesla C1060, FP32, p=12, 2,359,152 translations"},
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(M.cpu().numpy(), depth, p)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
