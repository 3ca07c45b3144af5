#!/usr/bin/env python3
"""Benchmark of the M2L translation (Sec. 4.1) on one MI355X.

A step is one M2L with its fused reduction over every box of levels 2..depth:
the whole interaction-list schedule, contraction and reduction, run on
expansions already resident in HBM. The operator bank is generated once per
(p, precision) before timing, because the operators depend only on p.

The default workload is N = 2^20 uniform points, quadtree depth 8, p = 12,
FP32 in the Pascal form of the operator (A~ = D1 B D2 with the constant
binomial matrix B), with b (the log-potential constant, carried in spare MFMA
rows).

Prints one JSON line with:
  * translations/s, using the exact, boundary-truncated count;
  * Gop/s, at 8p^2 flops per translation;
  * the roofline of the M2L kernel, timed with HIP events on its stream
    (mean over the timed launches; the default 2000 untimed launches before
    them, about 50 ms of load, let the shader clock settle, which takes tens
    of milliseconds from an idle GPU), priced at the flops the launched form
    performs (Pascal form 4p^2 + 14p, +4p + 8 with b; Gauss form 6p^2 + p,
    +6p + 2; split precision 24p^2, +24p), and as `effective_frac` at the
    dense operator's 8p^2 (+8p);
  * launch times one by one after the timed region: warm p10/p50/p90, and
    cold (caches flushed by a 512 MiB fill before each launch) p50;
  * the adjoint's time and roofline;
  * the relative error per level against the FP64 oracle's M2L of the same
    FP32 inputs, for every precision, on the 2^20- and 2^22-point workloads
    (computed after the timed region, by the oracle run that the CPU baseline
    times);
  * split precision against FP32: the same step in BF16x3 and FP16x3 on this
    workload and on the 2^22-point, depth-9, p = 16 one;
  * the 2^24-point, depth-10, p = 20 workload: forward and adjoint M2L in
    every precision, and the whole FMM's forward and reverse stage times;
  * the gradient of sum (Re phi)^2 at 4096 targets for 2^20 sources (forward
    plus backward through the whole FMM);
  * the FP64 oracle's M2L rate on the host cores, at all threads and at one,
    with the CPU model;
  * the whole FMM's stage times on the default workload;
  * the fast Gauss transform's Hermite evaluation (Sec. 4.2) at 6,553,600
    targets, p = 12 (or --fgt W): targets/s, its ALU roofline and the FP64
    oracle on a sample.
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

# name -> (points, depth, p, point set, default precision, outputs)
# outputs "Lb": the local expansions and b; "L": the local expansions only (the
# M2L of Eq. (eq:M2Lmat); at p = 16 b needs a separate pass)
WORKLOADS = {
    "m2l_uniform_n1M_d8_p12": (1 << 20, 8, 12, "uniform", "f32_pascal", "Lb"),
    "m2l_mixed_n4M_d9_p16": (1 << 22, 9, 16, "mixed", "f32_pascal", "L"),
    "m2l_mixed_n16M_d10_p20": (1 << 24, 10, 20, "mixed", "f32_pascal", "L"),
    "m2l_uniform_n4k_d4_p8": (4096, 4, 8, "uniform", "f32", "Lb"),
}
DEFAULT = "m2l_uniform_n1M_d8_p12"
MIXED_COMPARE = ["m2l_uniform_n1M_d8_p12", "m2l_mixed_n4M_d9_p16"]
# MI355X peaks: dense MFMA for the matrix-core forms; FP64 vector arithmetic
# for the Hankel form, which runs on the vector ALUs
PEAK_TFLOPS = {"f32": 157.3, "f32_pascal": 157.3, "bf16x3": 2500.0, "f16x3": 2500.0, "f64_hankel": 78.6}
PEAK_HBM_GBS = 8000.0
TOLERANCE_VS_FP64 = {"f32": 1e-5, "f32_pascal": 1e-5, "bf16x3": 1e-4, "f16x3": 1e-4, "f64_hankel": 1e-5}
PAPER_P12_TRANS_PER_S = 80.05e6  # Tesla C1060, p = 12, depth-8 tree (Table tab:m2ltesla)

# Fast Gauss transform, Hermite evaluation: name -> (depth, p, K).  Sources and
# targets are 100 * 4^depth uniform points each (100 per box, as in the
# paper's runs: its N are 100 * 4^k), sigma = sqrt(2) 2^-depth (box width
# r sqrt(2) sigma with r = 1/2), K = 8 boxes each way (cutoff exp(-16)).
FGT_WORKLOADS = {
    "fgt_hermite_n6.5M_d8_p12_K8": (8, 12, 8),
    "fgt_hermite_n6.5M_d8_p9_K8": (8, 9, 8),
    "fgt_hermite_n6.5M_d8_p5_K8": (8, 5, 8),
    "fgt_hermite_n25k_d4_p12_K8": (4, 12, 8),
}
FGT_DEFAULT = "fgt_hermite_n6.5M_d8_p12_K8"
PEAK_FP32_VECTOR_TFLOPS = 157.3
PAPER_FGT_PPS = {5: 2.78e7, 9: 6.48e6, 12: 3.27e6}  # Fermi C2050, N = 6,553,600 (Table tab:fgt_results_yeager)


def m2l_kernel_sources(precision="f32"):
    """Source files whose text decides the M2L kernel's memory traffic."""
    c = os.path.join(ROOT, "paper_1009_3457_amd", "csrc")
    names = ["m2l_f32.hip", "m2l_stage.h", "m2l_bank.h", "m2l_common.h", "fmm2d_internal.h"]
    if precision == "f32_pascal":
        names = ["m2l_pascal.hip", "m2l_pascal_bank.h", "m2l_stage.h", "m2l_bank.h", "m2l_common.h",
                 "fmm2d_internal.h"]
    elif precision == "f64_hankel":
        names = ["m2l_hankel.hip", "m2l_hankel_bank.h", "m2l_logrow.hip", "m2l_bank.h", "m2l_common.h",
                 "fmm2d_internal.h"]
    elif precision != "f32":
        names = ["m2l_mixed.hip", "m2l_mixed_bank.h", "m2l_bank.h", "m2l_common.h", "fmm2d_internal.h"]
    return [os.path.join(c, n) for n in names]


def source_digest(paths):
    import hashlib
    h = hashlib.sha256()
    for pth in paths:
        with open(pth, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def fgt_kernel_sources():
    """Source files of the Hermite evaluation kernel."""
    return [os.path.join(ROOT, "paper_1009_3457_amd", "csrc", "fgt.hip"), os.path.join(ROOT, "include", "fgt2d.h"),
            os.path.join(ROOT, "paper_1009_3457_amd", "csrc", "fmm2d_internal.h")]


def recorded_traffic(workload, precision, sources=None):
    """HBM bytes per launch from the committed FETCH_SIZE / WRITE_SIZE summary,
    or None when it is absent or was taken on different kernel sources."""
    tpath = os.path.join(ROOT, "profiles", f"traffic_{workload}_{precision}.json")
    if not os.path.exists(tpath):
        return None
    with open(tpath) as fh:
        rec = json.load(fh)
    if rec.get("source_sha256") != source_digest(sources or m2l_kernel_sources(precision)):
        return None
    return rec.get("bytes_per_launch")


def _points(kind, n, seed):
    import synthetic as sy
    return sy.uniform(n, seed) if kind == "uniform" else sy.mixed(n, seed)


def cpu_model():
    """The host CPU's model name (from /proc/cpuinfo)."""
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def cpu_baseline(w, budget_s=12.0, max_runs=200, single_thread=True):
    """The FP64 oracle's M2L over all levels 2..depth of the workload's own
    multipole expansions, timed on the host cores.

    The oracle builds the operator per translation from Eq. (eq:M2Lmat). The
    run is repeated at all threads while the time budget allows (at least
    once) and the median is reported; with `single_thread` it is also timed
    once on one thread.  Returns (record, reference): the reference is the
    oracle's result in the scaled basis the GPU stores, (L~, b or None), from
    which the per-level errors of the GPU results are computed."""
    import numpy as np

    import oracle
    with_b = w.outputs == "Lb"
    M = oracle.unscale_multipoles(w.M.cpu().numpy().astype(np.complex128), w.depth)
    times = []
    t_start = time.perf_counter()
    while len(times) < max_runs:
        t0 = time.perf_counter()
        Lr, br = oracle.m2l(M, w.depth, w.p, with_b=with_b)
        times.append(time.perf_counter() - t0)
        if time.perf_counter() - t_start + times[-1] > budget_s:
            break
    med = sorted(times)[len(times) // 2]
    rec = {"value": w.ntrans / med, "unit": "translations/s", "cores": oracle.num_threads(),
           "kind": "oracle", "cpu_model": cpu_model(),
           "sample": f"full M2L, levels 2..{w.depth}, p={w.p}, {w.ntrans} translations, FP64"
                     f"{' with b' if with_b else ''}, median of {len(times)} runs ({med:.3f} s each)"}
    if single_thread:
        n_all = oracle.num_threads()
        oracle.set_num_threads(1)
        try:
            t0 = time.perf_counter()
            oracle.m2l(M, w.depth, w.p, with_b=with_b)
            t1 = time.perf_counter() - t0
        finally:
            oracle.set_num_threads(n_all)
        rec["single_thread"] = {"value": w.ntrans / t1, "unit": "translations/s", "cores": 1,
                                "sample": f"the same M2L once on one thread ({t1:.3f} s)"}
    return rec, (oracle.scale_locals(Lr, w.depth), br)


class Workload:
    """Points -> tree -> P2M -> M2M on the GPU; the multipole expansions stay
    resident in HBM for the timed M2L launches."""

    def __init__(self, name, seed, dev):
        import torch

        import paper_1009_3457_amd as P
        import synthetic as sy
        self.name = name
        self.n, self.depth, self.p, self.kind, self.default_prec, self.outputs = WORKLOADS[name]
        xy = torch.from_numpy(_points(self.kind, self.n, seed)).to(dev)
        q = torch.from_numpy(sy.charges(self.n, seed + 1)).to(dev)
        perm, ls = P.build_tree(xy, self.depth)
        xs, qs = P.gather(xy, perm), P.gather(q, perm)
        self.M = P.m2m(P.p2m(xs, qs, ls, self.depth, self.p), self.depth, self.p)
        nb = P.num_boxes(self.depth)
        self.L = torch.zeros(nb, self.p, dtype=torch.complex64, device=dev)
        self.b = torch.zeros(nb, dtype=torch.complex64, device=dev) if self.outputs == "Lb" else None
        self.gM = torch.zeros(nb, self.p, dtype=torch.complex64, device=dev)
        self.gb = torch.zeros(nb, dtype=torch.complex64, device=dev) if self.outputs == "Lb" else None
        self.dev = dev
        self.ntrans = P.translation_count(2, self.depth)
        torch.cuda.synchronize(dev)

    def time_m2l(self, prec_name, steps, warmup):
        """(forward ms, adjoint ms) per launch: HIP events recorded on the
        stream the kernels are launched on, around `steps` back-to-back calls
        of the C ABI."""
        import torch

        import paper_1009_3457_amd as P
        from paper_1009_3457_amd import _binding as B
        prec = B.PRECISIONS[prec_name]
        ops = P.m2l_operators(self.p, prec, self.dev)
        lib = B.load()
        stream = torch.cuda.current_stream(self.dev)
        sp, vp = ctypes.c_void_p(stream.cuda_stream), ctypes.c_void_p
        ptr = lambda t: vp(t.data_ptr()) if t is not None else None  # noqa: E731
        fwd_args = (ptr(self.M), ptr(self.L), ptr(self.b), self.depth, self.p, 2, self.depth, prec,
                    ptr(ops), ops.numel(), sp)
        bwd_args = (ptr(self.L), ptr(self.gb), ptr(self.gM), self.depth, self.p, 2, self.depth, prec,
                    ptr(ops), ops.numel(), sp)

        def timed(fn, fargs, k, w):
            for _ in range(w):
                if fn(*fargs) != 0:
                    raise RuntimeError(lib.fmm2d_last_error().decode())
            torch.cuda.synchronize(self.dev)
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            rc = 0
            for _ in range(k):
                rc |= fn(*fargs)
            e1.record(stream)
            torch.cuda.synchronize(self.dev)
            if rc != 0:
                raise RuntimeError(lib.fmm2d_last_error().decode())
            return e0.elapsed_time(e1) / k

        ms_fwd = timed(lib.fmm2d_m2l, fwd_args, steps, warmup)
        ms_bwd = timed(lib.fmm2d_m2l_backward, bwd_args, max(steps // 2, 1), max(warmup // 2, 1))
        self._launch = (lib, fwd_args, stream)
        return ms_fwd, ms_bwd

    def launch_spread(self, reps=50, cold_reps=10, flush_bytes=512 << 20):
        """Forward M2L launch times one by one, after the timed region:
        warm (back-to-back, operands resident in L2/MALL) as p10/p50/p90, and
        cold (a 512 MiB fill between launches evicts every cache) as p50."""
        import torch
        lib, fwd_args, stream = self._launch

        def one():
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            rc = lib.fmm2d_m2l(*fwd_args)
            e1.record(stream)
            if rc != 0:
                raise RuntimeError(lib.fmm2d_last_error().decode())
            return e0, e1

        pairs = [one() for _ in range(reps)]
        torch.cuda.synchronize(self.dev)
        warm = sorted(a.elapsed_time(b) for a, b in pairs)
        flush = torch.empty(flush_bytes // 4, dtype=torch.float32, device=self.dev)
        cold = []
        for i in range(cold_reps):
            flush.fill_(float(i))
            a, b = one()
            torch.cuda.synchronize(self.dev)
            cold.append(a.elapsed_time(b))
        del flush
        cold.sort()
        q = lambda v, f: v[min(len(v) - 1, int(f * len(v)))]  # noqa: E731
        return {"warm_p10": q(warm, 0.1), "warm_p50": q(warm, 0.5), "warm_p90": q(warm, 0.9),
                "cold_p50": q(cold, 0.5), "warm_reps": reps, "cold_reps": cold_reps}

    def error_vs_fp64(self, ref):
        """Relative Frobenius error per level of the last launch's L~ (and b)
        against the FP64 oracle's result `ref` = (L~, b or None) of the same
        FP32 inputs: {"L": [e_2, ..., e_depth], "b": [...], "max": ...}."""
        import numpy as np

        import paper_1009_3457_amd as P
        if ref is None:
            return None
        Lr, br = ref
        L = self.L.cpu().numpy()
        b = self.b.cpu().numpy() if (self.b is not None and br is not None) else None
        out = {"levels": list(range(2, self.depth + 1)), "L": [], "b": [] if b is not None else None}
        for l in range(2, self.depth + 1):
            lo, hi = P.level_offset(l), P.level_offset(l + 1)
            den = np.linalg.norm(Lr[lo:hi])
            out["L"].append(float(np.linalg.norm(L[lo:hi] - Lr[lo:hi]) / den) if den > 0 else 0.0)
            if b is not None:
                den = np.linalg.norm(br[lo:hi])
                out["b"].append(float(np.linalg.norm(b[lo:hi] - br[lo:hi]) / den) if den > 0 else 0.0)
        out["max"] = max(out["L"] + (out["b"] or []))
        return out


def dense_flops_per_translation(p, outputs):
    """The dense operator's count for one translation: the p x p complex
    mat-vec, 8p^2 (4 multiplies and 4 adds per complex multiply-add), plus 8p
    for the log row when b is produced."""
    return 8 * p * p + (8 * p if outputs == "Lb" else 0)


def own_flops_per_translation(p, prec_name, outputs):
    """Flops one translation costs in the form that is launched.

    * Pascal form (A~ = D1 B D2): the scaling by D2 (6p), the two real
      products with B (4p^2) and the scaled accumulation by D1 (8p); the log
      row adds 4p + 8.
    * Gauss form: three real p x p products (Ar Xr, Ai Xi, (Ar+Ai)(Xr+Xi)),
      6p^2, and the p additions forming Xr + Xi; the log row is one more row
      of the three products (6p) plus the M~_0 sum for the log(h) term (2).
    * Split precision (BF16x3, FP16x3): three real products with the 2p x 2p
      real embedding, 24p^2, and 24p for the log row's two real rows.
    * Hankel form (FP64): counted per target and divided by its 27
      translations: the source transforms (144 records per 64 targets, each
      N = 2p frequencies by p - 1 complex multiply-adds, plus the scaling),
      27 N complex multiply-adds of spectra, and the p inverse-transform
      outputs (N - 1 complex multiply-adds each, plus the scaling); the log
      row, in its own pass, adds 8p + 2."""
    with_b = outputs == "Lb"
    if prec_name == "f64_hankel":
        n = 2 * p
        per_target = (144 / 64) * (n * (p - 1) * 8 + 2 * p) + 27 * n * 8 + p * (n - 1) * 8 + 2 * p
        return per_target / 27 + (8 * p + 2 if with_b else 0)
    if prec_name == "f32_pascal":
        return 4 * p * p + 14 * p + (4 * p + 8 if with_b else 0)
    if prec_name == "f32":
        return 6 * p * p + p + (6 * p + 2 if with_b else 0)
    return 24 * p * p + (24 * p if with_b else 0)


def roofline(w, prec_name, ms):
    """The M2L kernel against the MFMA peak of its dtype: `achieved` and
    `frac` at the flops the launched form performs, `effective_frac` at the
    dense operator's count."""
    own = own_flops_per_translation(w.p, prec_name, w.outputs)
    dense = dense_flops_per_translation(w.p, w.outputs)
    tflops = float(own) * w.ntrans / (ms * 1e-3) / 1e12
    eff = float(dense) * w.ntrans / (ms * 1e-3) / 1e12
    boxes = sum(4 ** l for l in range(2, w.depth + 1))
    alg_bytes = boxes * w.p * 8 * 2 + (boxes * 8 if w.outputs == "Lb" else 0)
    peak = PEAK_TFLOPS[prec_name]
    return {"bound": "alu" if prec_name == "f64_hankel" else "mfma", "achieved": tflops, "peak": peak, "unit": "TFLOP/s", "frac": tflops / peak,
            "flops_per_translation": own,
            "effective_frac": eff / peak, "dense_flops_per_translation": dense,
            "traffic": recorded_traffic(w.name, prec_name),
            "algorithmic_bytes": alg_bytes,
            "hbm_frac": alg_bytes / (ms * 1e-3) / 1e9 / PEAK_HBM_GBS}


def precision_block(w, prec, steps, warmup, ref, best=None):
    """One precision on one workload: forward and adjoint time per launch,
    rooflines, error per level against FP64, and the speedup over `best` =
    (forward ms, adjoint ms) of the faster FP32 form."""
    ms, bwd = w.time_m2l(prec, steps, warmup)
    err = w.error_vs_fp64(ref)
    rf, rb = roofline(w, prec, ms), roofline(w, prec, bwd)
    rec = {"ms": ms, "adjoint_ms": bwd, "translations_per_s": w.ntrans / (ms * 1e-3),
           "roofline_frac": rf["frac"], "effective_frac": rf["effective_frac"],
           "adjoint_roofline_frac": rb["frac"], "achieved_tflops": rf["achieved"],
           "error_vs_fp64": err, "tolerance_vs_fp64": TOLERANCE_VS_FP64[prec]}
    if err is not None:
        rec["within_tolerance"] = err["max"] <= TOLERANCE_VS_FP64[prec]
    if best is not None:
        rec["speedup_vs_f32"] = best[0] / ms
        rec["adjoint_speedup_vs_f32"] = best[1] / bwd
    return rec


def mixed_comparison(seed, dev, steps, warmup, main=None, main_ref=None, cpu=True):
    """The FP32 forms (Gauss and Pascal) against BF16x3, FP16x3 and the FP64
    Hankel form on the same inputs: time per launch, rooflines, speedup over the faster FP32 form and
    the error per level against the FP64 oracle (whose M2L of the same inputs
    is timed as that workload's CPU baseline)."""
    out = {}
    for name in MIXED_COMPARE:
        if main is not None and main.name == name:
            w, ref, base = main, main_ref, None
        else:
            w = Workload(name, seed, dev)
            base, ref = cpu_baseline(w, budget_s=4.0, max_runs=5, single_thread=False) if cpu else (None, None)
        rec = {"outputs": w.outputs, "translations": w.ntrans}
        rec["f32"] = precision_block(w, "f32", steps, warmup, ref)
        rec["f32_pascal"] = precision_block(w, "f32_pascal", steps, warmup, ref)
        best = (min(rec["f32"]["ms"], rec["f32_pascal"]["ms"]),
                min(rec["f32"]["adjoint_ms"], rec["f32_pascal"]["adjoint_ms"]))
        for prec in ("bf16x3", "f16x3", "f64_hankel"):
            rec[prec] = precision_block(w, prec, steps, warmup, ref, best)
        if base is not None:
            rec["cpu_baseline"] = base
        out[name] = rec
    out["speedup_reference"] = "the faster FP32 form on the same workload"
    return out


def large_workload(seed, dev, steps, warmup):
    """The 2^24-point mixed set, depth 10, p = 20: forward and adjoint M2L in
    every form (the FP64 Hankel form included) (time, roofline; the error against FP64 is checked by the
    parity tests), and the whole FMM's forward and reverse stage times in the
    Pascal form and in BF16x3."""
    name = "m2l_mixed_n16M_d10_p20"
    w = Workload(name, seed, dev)
    out = {"workload": name, "translations": w.ntrans}
    pa = precision_block(w, "f32_pascal", steps, warmup, None)
    ga = precision_block(w, "f32", steps, warmup, None)
    out["f32_pascal"], out["f32"] = pa, ga
    best = (min(pa["ms"], ga["ms"]), min(pa["adjoint_ms"], ga["adjoint_ms"]))
    for prec in ("bf16x3", "f16x3", "f64_hankel"):
        out[prec] = precision_block(w, prec, steps, warmup, None, best)
    del w
    out["fmm_stages_ms"] = {prec: fmm_stage_times(name, prec, seed, dev, reps=3) for prec in ("f32_pascal", "bf16x3")}
    return out


def gradient_timing(seed, dev, reps=5):
    """Forward plus backward of the loss sum_t (Re phi(z_t))^2 at 4096 uniform
    targets for 2^20 uniform sources (depth 8, p = 12, FP32 Pascal-form M2L)
    through the autograd layer: host-clock medians (the tree build
    synchronises with the host), gradients with respect to charges and
    positions."""
    import torch

    import paper_1009_3457_amd as P
    import synthetic as sy
    n, depth, p = 1 << 20, 8, 12
    xy = torch.from_numpy(sy.uniform(n, seed)).to(dev)
    q = torch.from_numpy(sy.charges(n, seed + 1)).to(dev)
    t = torch.from_numpy(sy.uniform(4096, seed + 3)).to(dev)
    fw, bw = [], []
    for _ in range(reps + 1):
        xg = xy.clone().requires_grad_(True)
        qg = q.clone().requires_grad_(True)
        torch.cuda.synchronize(dev)
        t0 = time.perf_counter()
        phi, _ = P.potential(xg, qg, t, depth=depth, p=p, precision="f32_pascal")
        loss = (phi.real ** 2).sum()
        torch.cuda.synchronize(dev)
        t1 = time.perf_counter()
        loss.backward()
        torch.cuda.synchronize(dev)
        t2 = time.perf_counter()
        fw.append((t1 - t0) * 1e3)
        bw.append((t2 - t1) * 1e3)
    fw, bw = sorted(fw[1:]), sorted(bw[1:])
    return {"workload": "2^20 uniform sources, 4096 uniform targets, depth 8, p 12, f32_pascal",
            "forward_ms": fw[len(fw) // 2], "backward_ms": bw[len(bw) // 2],
            "total_ms": fw[len(fw) // 2] + bw[len(bw) // 2], "reps": reps}


def fgt_pairs(txy, depth, K):
    """Exact number of (target, box) pairs: each target takes the boxes within
    K of its own box in both directions, clipped to the grid."""
    import numpy as np
    side = 1 << depth
    b = np.clip(np.floor(txy.astype(np.float64) * side), 0, side - 1).astype(np.int64)
    w = np.minimum(b + K, side - 1) - np.maximum(b - K, 0) + 1
    return int(np.sum(w[:, 0] * w[:, 1]))


def fgt_bench(name, seed, dev, steps, warmup, cpu=True, cpu_budget_s=12.0):
    """The Hermite evaluation of the fast Gauss transform (Sec. 4.2): targets/s
    over `steps` launches (HIP events on the launch stream, coefficients and
    sorted targets resident), its ALU roofline, and the FP64 oracle on a
    sample of the same targets."""
    import math

    import numpy as np
    import torch

    import paper_1009_3457_amd as P
    import synthetic as sy
    depth, p, K = FGT_WORKLOADS[name]
    n = 100 * 4 ** depth
    sigma = float(np.float32(math.sqrt(2.0) * 2.0 ** -depth))
    xy = torch.from_numpy(sy.uniform(n, seed + 10)).to(dev)
    q = torch.from_numpy(sy.charges(n, seed + 11)).to(dev)
    t = torch.from_numpy(sy.uniform(n, seed + 12)).to(dev)
    perm, ls = P.build_tree(xy, depth)
    xs, qs = P.gather(xy, perm), P.gather(q, perm)
    tperm, _ = P.build_tree(t, depth)
    ts = P.gather(t, tperm)
    stream = torch.cuda.current_stream(dev)
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(4)]
    A = P.fgt_hermite_coeffs(xs, qs, ls, depth, p, sigma)  # first call loads the code object
    ev[0].record(stream)
    A = P.fgt_hermite_coeffs(xs, qs, ls, depth, p, sigma)
    ev[1].record(stream)
    G = P.fgt_hermite_eval(ts, depth, p, sigma, K, A)
    for _ in range(warmup):
        P.fgt_hermite_eval(ts, depth, p, sigma, K, A, G)
    torch.cuda.synchronize(dev)
    ev[2].record(stream)
    for _ in range(steps):
        P.fgt_hermite_eval(ts, depth, p, sigma, K, A, G)
    ev[3].record(stream)
    torch.cuda.synchronize(dev)
    ms = ev[2].elapsed_time(ev[3]) / steps
    ts_np = ts.cpu().numpy()
    pairs = fgt_pairs(ts_np, depth, K)
    flops = pairs * (2.0 * p * p + 2.0 * p)
    tflops = flops / (ms * 1e-3) / 1e12
    alg_bytes = n * 8 + n * 4 + (1 << (2 * depth)) * p * p * 4
    out = {
        "workload": name, "targets": n, "sources": n, "depth": depth, "boxes": 1 << (2 * depth), "p": p, "K": K,
        "sigma": sigma, "r": 0.5, "pairs": pairs, "ms_per_eval": ms, "targets_per_s": n / (ms * 1e-3),
        "gflop_s": flops / (ms * 1e-3) / 1e9, "coeffs_ms": ev[0].elapsed_time(ev[1]),
        "roofline": {"bound": "alu", "achieved": tflops, "peak": PEAK_FP32_VECTOR_TFLOPS, "unit": "TFLOP/s",
                     "frac": tflops / PEAK_FP32_VECTOR_TFLOPS,
                     "traffic": recorded_traffic(name, "f32", fgt_kernel_sources()),
                     "algorithmic_bytes": alg_bytes},
        "flops_per_pair": f"2p^2 + 2p = {2 * p * p + 2 * p}",
        "paper_context": {"targets_per_s": PAPER_FGT_PPS.get(p), "hardware": "Fermi C2050, N = 6,553,600"},
    }
    if cpu:
        import oracle
        from oracle import fgt as ofgt
        xs_np, qs_np, ls_np = xs.cpu().numpy(), qs.cpu().numpy(), ls.cpu().numpy()
        Ar = ofgt.hermite_coeffs(xs_np.astype(np.float64), qs_np.astype(np.float64), ls_np, depth, p, sigma)
        m, spent = 512, 0.0
        while True:  # grow the sample until one evaluation takes a few seconds
            sample = ts_np[:: max(n // m, 1)][:m].astype(np.float64)
            t0 = time.perf_counter()
            ofgt.hermite_eval(sample, depth, p, sigma, K, Ar)
            spent = time.perf_counter() - t0
            if spent > cpu_budget_s / 4 or m >= n:
                break
            m = min(n, int(m * max(2.0, (cpu_budget_s / 4) / max(spent, 1e-3))))
        out["cpu_baseline"] = {"value": len(sample) / spent, "unit": "targets/s", "cores": oracle.num_threads(),
                               "kind": "oracle",
                               "sample": f"{len(sample)} of the {n} targets in box order (stride {max(n // m, 1)}), "
                                         f"FP64 Hermite evaluation with the oracle's coefficients, p={p}, K={K}, "
                                         f"{spent:.2f} s"}
    return out


def near_field_pairs(leaf_start, depth):
    """Ordered source-target pairs (i != j) the near field evaluates: every
    point of a leaf against every other point of the leaf and its 8
    neighbours.  leaf_start holds the Morton-ordered leaf offsets (host)."""
    import numpy as np
    counts = np.diff(np.asarray(leaf_start, np.int64))
    m = np.arange(counts.size, dtype=np.int64)
    x = np.zeros_like(m)
    y = np.zeros_like(m)
    for bit in range(depth):
        x |= ((m >> (2 * bit)) & 1) << bit
        y |= ((m >> (2 * bit + 1)) & 1) << bit
    side = 1 << depth
    grid = np.zeros((side + 2, side + 2), np.int64)
    grid[y + 1, x + 1] = counts
    near = sum(grid[1 + dy:side + 1 + dy, 1 + dx:side + 1 + dx] for dy in (-1, 0, 1) for dx in (-1, 0, 1))
    c = grid[1:side + 1, 1:side + 1]
    return int(np.sum(c * near) - np.sum(c))


def fmm_stage_times(name, prec_name, seed, dev, reps=5):
    """Per-stage times (ms, median of `reps`) of the whole FMM with every point
    as both source and target: tree build (with the sorted gathers), P2M, M2M,
    M2L, L2L, L2P, P2P, then the reverse pass for seeded cotangents of a
    loss on Re phi and the field (a real cotangent of phi, a complex one of
    the field): L2P^T, L2L^T, M2L^T, M2M^T, P2M^T, P2P^T.  HIP events on the
    stream; the tree build leaves its domain check on the device, which is
    read after the pass."""
    import torch

    import paper_1009_3457_amd as P
    from paper_1009_3457_amd import _binding as B
    import synthetic as sy
    n, depth, p, kind, _, _ = WORKLOADS[name]
    prec = B.PRECISIONS[prec_name]
    xy = torch.from_numpy(_points(kind, n, seed)).to(dev)
    q = torch.from_numpy(sy.charges(n, seed + 1)).to(dev)
    P.m2l_operators(p, prec, dev)
    stream = torch.cuda.current_stream(dev)
    # cotangents of a loss on the physical quantities: Re phi (a real
    # cotangent of phi) and the field (complex)
    gen = torch.Generator().manual_seed(seed + 2)
    cot = torch.randn(2, n, dtype=torch.complex64, generator=gen)
    cot[0] = cot[0].real.to(torch.complex64)
    cot = cot.to(dev)
    rows = []
    for _ in range(reps + 1):
        torch.cuda.synchronize(dev)
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(14)]
        ev[0].record(stream)
        perm, ls, flag = B.build_tree(xy, depth, check=False)
        xs, qs = P.gather(xy, perm), P.gather(q, perm)
        ev[1].record(stream)
        M = B.p2m(xs, qs, ls, depth, p)
        ev[2].record(stream)
        B.m2m(M, depth, p)
        ev[3].record(stream)
        Lm, bm = B.m2l(M, depth, p, 2, depth, prec)
        ev[4].record(stream)
        L, b = B.l2l(Lm, bm, depth, p)
        ev[5].record(stream)
        phi, field = B.l2p(xs, ls, L, b, depth, p)
        ev[6].record(stream)
        B.p2p(xs, qs, ls, xs, ls, depth, phi, field)
        ev[7].record(stream)
        cphi, cfield = cot[0], cot[1]
        gL, gb = B.l2p_backward(xs, ls, cphi, cfield, depth, p)
        ev[8].record(stream)
        gLm, gbm = B.l2l_backward(gL, gb, depth, p)
        ev[9].record(stream)
        gM = B.m2l_backward(gLm, gbm, depth, p, 2, depth, prec)
        ev[10].record(stream)
        B.m2m_backward(gM, depth, p)
        ev[11].record(stream)
        gq, G = B.p2m_backward(xs, qs, ls, depth, p, gM)
        ev[12].record(stream)
        B.p2p_backward(xs, qs, ls, xs, ls, depth, cphi, cfield, gq, G)
        ev[13].record(stream)
        torch.cuda.synchronize(dev)
        B.check_domain(flag)
        rows.append([ev[i].elapsed_time(ev[i + 1]) for i in range(13)])
    rows = sorted(rows[1:], key=lambda r: sum(r))  # drop the first (warm-up) pass
    med = rows[len(rows) // 2]
    names = ["tree_build_and_gather", "p2m", "m2m", "m2l", "l2l", "l2p", "p2p",
             "l2p_T", "l2l_T", "m2l_T", "m2m_T", "p2m_T", "p2p_T"]
    out = {k: v for k, v in zip(names, med)}
    out["forward_total"] = sum(med[:7])
    out["backward_total"] = sum(med[7:])
    pairs = near_field_pairs(ls.cpu().numpy(), depth)
    out["p2p_pairs"] = pairs
    out["p2p_pairs_per_s"] = pairs / (out["p2p"] * 1e-3)
    out["p2p_T_pairs_per_s"] = pairs / (out["p2p_T"] * 1e-3)
    out["workload"] = name
    out["precision"] = prec_name
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--warmup", type=int, default=2000)
    ap.add_argument("--workload", default=DEFAULT, choices=sorted(WORKLOADS))
    ap.add_argument("--precision", default=None, choices=["f32", "f32_pascal", "bf16x3", "f16x3", "f64_hankel"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-mixed", action="store_true", help="skip the split-precision comparison")
    ap.add_argument("--no-large", action="store_true",
                    help="skip the 2^24-point workload and the gradient timing")
    ap.add_argument("--fmm", action="store_true",
                    help="also time every stage of the whole FMM (all points as sources and targets)")
    ap.add_argument("--fgt", default=None, choices=sorted(FGT_WORKLOADS),
                    help="time the fast Gauss transform's Hermite evaluation on this workload "
                         f"(the default run times {FGT_DEFAULT})")
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

    import torch
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)

    w = Workload(args.workload, args.seed, dev)
    prec_name = args.precision or w.default_prec
    # the timed region: K forward M2L launches, bracketed by synchronisation
    ms_fwd, ms_bwd = w.time_m2l(prec_name, args.steps, args.warmup)
    value = w.ntrans / (ms_fwd * 1e-3)
    launch = w.launch_spread()
    padded = 27 * sum(4 ** l for l in range(2, w.depth + 1))
    default_run = args.workload == DEFAULT and args.precision is None

    # after the timed region: the oracle's M2L of the same inputs, timed on
    # the host cores, is also the FP64 reference for the error per level
    base, ref = (None, None)
    if not args.no_cpu_baseline:
        base, ref = cpu_baseline(w)
    err = w.error_vs_fp64(ref)  # w.L still holds the headline launch's result

    rf = roofline(w, prec_name, ms_fwd)
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
        # the paper's p = 12 figure on the same tree (another machine: context, not the target)
        "vs_baseline": (value / PAPER_P12_TRANS_PER_S
                        if (w.depth, w.p) == (8, 12) and prec_name in ("f32", "f32_pascal") else None),
        "dtype": "f32" if prec_name.startswith("f32") else prec_name,
        "data": "synthetic",
        "config": {"workload": args.workload, "points": w.n, "point_set": w.kind, "depth": w.depth,
                   "p": w.p, "levels": f"2..{w.depth}", "precision": prec_name, "outputs": w.outputs,
                   "translations": w.ntrans, "padded_translations": padded, "seed": args.seed},
        "gop_s": 8.0 * w.p * w.p * w.ntrans / (ms_fwd * 1e-3) / 1e9,
        "roofline": rf,
        "error_vs_fp64": err,
        "tolerance_vs_fp64": TOLERANCE_VS_FP64[prec_name],
        "m2l_launch_ms": launch,
        "adjoint_ms": ms_bwd,
        "adjoint_translations_per_s": w.ntrans / (ms_bwd * 1e-3),
        "adjoint_roofline_frac": roofline(w, prec_name, ms_bwd)["frac"],
        "paper_context": {"translations_per_s": PAPER_P12_TRANS_PER_S, "gop_s": 511.06,
                          "hardware": "Tesla C1060, FP32, p=12, 2,359,152 translations"},
    }
    if err is not None:
        out["within_tolerance"] = err["max"] <= TOLERANCE_VS_FP64[prec_name]
    if default_run and not args.no_mixed:
        out["mixed_vs_f32"] = mixed_comparison(args.seed, dev, max(args.steps // 2, 10),
                                               max(args.warmup // 2, 2), main=w, main_ref=ref,
                                               cpu=not args.no_cpu_baseline)
    if args.fmm or default_run:
        out["fmm_stages_ms"] = fmm_stage_times(args.workload, prec_name, args.seed, dev)
    if default_run and not args.no_large:
        out["large_n16M_d10_p20"] = large_workload(args.seed, dev, max(args.steps // 4, 5),
                                                   max(args.warmup // 4, 2))
        out["gradient_n1M_4096_targets"] = gradient_timing(args.seed, dev)
    fgt_name = args.fgt or (FGT_DEFAULT if default_run else None)
    if fgt_name:
        out["fgt_hermite"] = fgt_bench(fgt_name, args.seed, dev, max(args.steps // 10, 5),
                                       max(args.warmup // 10, 2), cpu=not args.no_cpu_baseline)
    if base is not None:
        out["cpu_baseline"] = base
    print(json.dumps(out))


if __name__ == "__main__":
    main()
