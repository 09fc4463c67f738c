#!/usr/bin/env python3
"""Benchmark of the randomized LU hot path (Algorithm 4.1 of Shabat et al.,
arXiv 1310.7202) on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload NAME]

A step is one complete rlu_factor call (Steps 1-8: Gaussian sketch matrix,
sketch GEMM, pivoted LU of Y, Gram matrix and its inverse, projection GEMM,
pivoted LU of B^T, assembly of L and U) on a device-resident input; for the
batched workload a step is one rlu_factor_batched call over 256 problems.
Prints one JSON line: the main workload (default: 8192 x 8192 FP64) plus,
under "forms", the same matrix through the FP32 path and with one power
iteration (Section 5.2), least squares on its factors (Algorithm 4.3),
the 512 x 512 configuration's p50/p99 latency, the 16384 x 16384
mixed-precision configuration beside the FP64 path on the same matrix, the
256-problem batch, and the served request stream (throughput with p50/p99
latency; disable the extra measurements with --forms none).  Only one GPU is used; --gpus N with
N > 1 exits with a message.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "rank-k LU/s + %MFMA/HBM peak, mixed vs FP64 at equal error; p50/p99 latency"
PEAK = {"f64": 78.6e12, "f32": 157.3e12, "bf16": 2.5e15, "hbm": 8.0e12}

WORKLOADS = {
    # name: (m, n, k, l, spectrum, data seed, sketch seed, precision, description)
    "exp8192": (8192, 8192, 200, 210, "exp50", 102, 7204, "fp64",
                "8192x8192, U and V Haar, sigma_i = exp(-i/50), k=200, l=210, FP64"),
    "exp8192_fp32": (8192, 8192, 200, 210, "exp50", 102, 7204, "fp32",
                     "8192x8192, U and V Haar, sigma_i = exp(-i/50), k=200, l=210, FP32"),
    "small512": (512, 512, 10, 15, "lowrank10", 101, 7203, "fp64",
                 "512x512, X Y^T + 1e-9 N(0,1), X, Y 512x10, k=10, l=15, FP64"),
}
MIXED = ("mixed16384", 16384, 16384, 500, 520, 103, 7205,
         "16384x16384, U and V Haar, sigma_i = i^-2, k=500, l=520; A stored FP32, BF16 MFMA "
         "products with FP32 accumulation, FP64 pivoted LUs and Gram inverse; the same matrix "
         "in FP64 through the FP64 path for the equal-error comparison")
BATCH = ("batch256", 256, 104, 7204,
         "256 FP32 problems per call, m, n ~ U[256, 4096], A = X Y^T + 1e-6 N(0,1) with "
         "rank r ~ U[8, 64], k = r, l = r + 8")


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def make_input(name, torch, kind="spectral"):
    import numpy as np
    import workloads

    m, n, k, l, spec, dseed, sseed, prec, _ = WORKLOADS[name]
    dt = torch.float32 if prec == "fp32" else torch.float64
    if kind == "gaussian":
        # same shape, i.i.d. N(0,1) values (counter runs: traffic does not depend on values)
        g = torch.Generator(device="cuda")
        g.manual_seed(dseed)
        return torch.randn(n, m, generator=g, device="cuda", dtype=dt).t(), k, l, sseed
    if spec == "exp50":
        A = workloads.spectral_matrix_torch(m, n, workloads.exp_decay(min(m, n), 50.0), dseed,
                                            device="cuda", dtype=torch.float64)
        A = A.t().contiguous().t().to(dt)       # column-major
    else:
        Ah, _, _ = workloads.config_small(dseed)
        A = torch.from_numpy(np.ascontiguousarray(Ah.T)).cuda().t().to(dt)
    return A, k, l, sseed


def power_residual(A, L, U, p, q, iters=30):
    """||L U - P A Q||_2 / ||A||_2 by power iterations (validation only)."""
    import torch
    gen = torch.Generator(device=A.device)
    gen.manual_seed(1)
    n = A.shape[1]
    qinv = torch.empty_like(q); qinv[q] = torch.arange(q.numel(), device=q.device)
    pinv = torch.empty_like(p); pinv[p] = torch.arange(p.numel(), device=p.device)

    def op(x):
        return L @ (U @ x) - (A @ x[qinv])[p]

    def opt(y):
        return U.t() @ (L.t() @ y) - (A.t() @ y[pinv])[q]

    x = torch.randn(n, generator=gen, device=A.device, dtype=A.dtype)
    x /= x.norm()
    r = 0.0
    for _ in range(iters):
        z = opt(op(x)); nz = z.norm()
        if nz == 0:
            break
        r = math.sqrt(float(nz)); x = z / nz
    x = torch.randn(n, generator=gen, device=A.device, dtype=A.dtype)
    x /= x.norm()
    a = 0.0
    for _ in range(iters):
        z = A.t() @ (A @ x); nz = z.norm()
        a = math.sqrt(float(nz)); x = z / nz
    return r / a


def traffic_from_profiles(kernel_src):
    """HBM bytes per launch of the dominant kernel from the committed
    rocprofv3 counter summary, if it was taken on the current kernel source."""
    path = os.path.join(ROOT, "profiles", "traffic_sketch_gemm_exp8192.md")
    if not os.path.exists(path):
        return None
    txt = open(path).read()
    m_b = re.search(r"traffic_bytes_per_launch:\s*([0-9.eE+]+)", txt)
    m_h = re.search(r"source_sha256:\s*([0-9a-f]{64})", txt)
    if not (m_b and m_h):
        return None
    h = hashlib.sha256(open(kernel_src, "rb").read()).hexdigest()
    return float(m_b.group(1)) if h == m_h.group(1) else None


def cpu_baseline(A_host, k, l, seed, budget_s):
    import numpy as np
    from oracle import philox, rlu as orl
    try:
        from threadpoolctl import threadpool_info
        cores = max([i.get("num_threads", 1) for i in threadpool_info()] or [1])
    except Exception:
        cores = os.cpu_count() or 1
    m, n = A_host.shape
    G = philox.gaussian_matrix(n, l, seed)
    runs, t0 = 0, time.perf_counter()
    out = None
    while True:
        out = orl.randomized_lu(A_host, k, l, G)
        runs += 1
        el = time.perf_counter() - t0
        log(f"oracle run {runs}: {el:.1f} s")
        if el >= budget_s or runs >= 50:
            break
    return {"value": runs / el, "unit": "factorizations/s", "cores": int(cores), "kind": "oracle",
            "sample": f"{runs} full factorization(s) of the same input by the FP64 NumPy oracle "
                      f"in {el:.1f} s"}, out, G


def phase_work(m, n, k, l, s_a, s_out):
    """Algorithmic flops and HBM bytes of each timed phase for one problem
    (what the method must do: dense products counted at 2 flops per
    multiply-add, operands read once, results written once)."""
    return {
        "sketch_gemm": (2.0 * m * n * l, s_a * m * n + s_a * n * l + 8.0 * m * l),
        "panel_lu_y": (m * l * l - l ** 3 / 3.0, 16.0 * m * l),
        "gram_gemm": (2.0 * m * k * k, 8.0 * m * k),
        "gram_inverse": (2.0 * k ** 3, 16.0 * k * k),
        "project_gemm": (2.0 * m * n * k, s_a * m * n + 8.0 * m * k + 8.0 * k * n),
        "solve_gemm": (2.0 * k * k * n, 16.0 * k * n + 8.0 * k * k),
        "panel_lu_bt": (n * k * k - k ** 3 / 3.0, 16.0 * k * n),
        "form_l_gemm": (2.0 * m * k * k, 8.0 * m * k + s_out * m * k),
    }


def kernel_table(phase_ms, works, mfma_peak):
    """Per-phase achieved rates against the roofline of that phase: bound =
    whichever of MFMA time and HBM time is larger; the two pivoted LUs are
    chains of l (or k) dependent steps and are reported as latency-bound."""
    out = {}
    for name, (fl, by) in works.items():
        t = phase_ms.get(name, 0.0) * 1e-3
        if t <= 0:
            continue
        t_f, t_b = fl / mfma_peak, by / PEAK["hbm"]
        if name.startswith("panel") or name == "gram_inverse":
            bound = "latency"
        else:
            bound = "mfma" if t_f >= t_b else "hbm"
        out[name] = {"ms": phase_ms[name], "tflops": fl / t / 1e12, "gbs": by / t / 1e9,
                     "bound": bound, "roofline_frac": max(t_f, t_b) / t}
    return out


def sum_works(shapes, s_a, s_out):
    tot = {}
    for (m, n, k, l) in shapes:
        for key, (f, b) in phase_work(m, n, k, l, s_a, s_out).items():
            a = tot.get(key, (0.0, 0.0))
            tot[key] = (a[0] + f, a[1] + b)
    return tot


def step_roofline(works, mfma_peak, ms_per_step):
    """T_roof = max(GEMM flops / MFMA peak, GEMM bytes / HBM) + small-kernel
    flops at the same peak, against the measured step time."""
    gem = [k for k in works if k.endswith("gemm")]
    f = sum(works[k][0] for k in gem)
    b = sum(works[k][1] for k in gem)
    tail = sum(v[0] for k, v in works.items() if k not in gem)
    t_roof = max(f / mfma_peak, b / PEAK["hbm"]) + tail / PEAK["f64"]
    return {"t_roof_ms": t_roof * 1e3, "frac": t_roof * 1e3 / ms_per_step}


def run_single(rlu, torch, np, name, steps, warmup, input_kind="spectral", check=True):
    m, n, k, l = WORKLOADS[name][:4]
    prec = WORKLOADS[name][7]
    log(f"generating {WORKLOADS[name][8]}")
    A, k, l, sseed = make_input(name, torch, input_kind)
    torch.cuda.synchronize()
    log("input ready")
    h = rlu.Handle(0)
    # the timed region carries one event pair per call, around the sketch
    # product (the roofline kernel); every phase is timed in a pass after it
    h.set_timing(2)
    out = rlu.Factors(torch.empty((k, m), dtype=A.dtype, device="cuda").t(),
                      torch.empty((n, k), dtype=A.dtype, device="cuda").t(),
                      torch.empty(m, dtype=torch.int64, device="cuda"),
                      torch.empty(n, dtype=torch.int64, device="cuda"),
                      torch.empty(3, dtype=torch.int32, device="cuda"))
    stream = torch.cuda.current_stream()
    for _ in range(warmup):
        rlu.factor(A, k, l, seed=sseed, handle=h, out=out, stream=stream)
    torch.cuda.synchronize()
    log(f"warmup {warmup} done")
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
           for _ in range(steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(steps):
        evs[i][0].record(stream)
        rlu.factor(A, k, l, seed=sseed, handle=h, out=out, stream=stream)
        evs[i][1].record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    log(f"{name}: timed {steps} steps in {wall * 1e3:.1f} ms")
    lat = np.array([a.elapsed_time(b) for a, b in evs])
    sketch_timed = float(np.mean([h.phase_times(back)["sketch_gemm"] for back in range(steps)]))
    # every phase, in a separate pass (its events add ~0.1 ms per call)
    h.set_timing(True)
    nph = min(steps, 10)
    for _ in range(nph):
        rlu.factor(A, k, l, seed=sseed, handle=h, out=out, stream=stream)
    torch.cuda.synchronize()
    phases = [h.phase_times(back) for back in range(nph)]
    ph = {key: float(np.mean([p[key] for p in phases])) for key in phases[0]}
    ph["sketch_gemm"] = sketch_timed  # the timed region's own measurement
    h.set_timing(False)
    s_a = 4.0 if prec == "fp32" else 8.0
    peak = PEAK["f32"] if prec == "fp32" else PEAK["f64"]
    works = phase_work(m, n, k, l, s_a, s_a)
    res = {
        "value": steps / wall, "ms_per_step": wall * 1e3 / steps,
        "latency_ms": {"p50": float(np.percentile(lat, 50)), "p99": float(np.percentile(lat, 99)),
                       "mean": float(lat.mean())},
        "phase_ms": ph,
        "kernels": kernel_table(ph, works, peak),
        "step_roofline": step_roofline(works, peak, wall * 1e3 / steps),
        "info": out.info.cpu().tolist(),
    }
    if check:
        res["rel_residual"] = power_residual(A.double() if prec == "fp32" else A,
                                             out.L.double(), out.U.double(), out.p, out.q)
        log(f"{name}: relative residual {res['rel_residual']:.3e}")
    return res, A, out, (m, n, k, l, sseed, prec, s_a, peak, works)


def timed_calls(rlu, torch, np, A, k, l, sseed, precision, steps, warmup, power_iters=0):
    h = rlu.Handle(0)
    h.set_timing(2)  # one event pair per call in the timed region (the sketch product)
    st = torch.cuda.current_stream()
    out = None
    for _ in range(warmup):
        out = rlu.factor(A, k, l, seed=sseed, precision=precision, handle=h, stream=st,
                         power_iters=power_iters)
    torch.cuda.synchronize()
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
           for _ in range(steps)]
    t0 = time.perf_counter()
    for i in range(steps):
        evs[i][0].record(st)
        out = rlu.factor(A, k, l, seed=sseed, precision=precision, handle=h, stream=st,
                         power_iters=power_iters)
        evs[i][1].record(st)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    lat = np.array([a.elapsed_time(b) for a, b in evs])
    sk = float(np.mean([h.phase_times(b)["sketch_gemm"] for b in range(steps)]))
    h.set_timing(True)  # every phase, in a pass after the timed region
    nph = min(steps, 5)
    for _ in range(nph):
        out = rlu.factor(A, k, l, seed=sseed, precision=precision, handle=h, stream=st, out=out,
                         power_iters=power_iters)
    torch.cuda.synchronize()
    ph = [h.phase_times(b) for b in range(nph)]
    ph = {key: float(np.mean([p[key] for p in ph])) for key in ph[0]}
    ph["sketch_gemm"] = sk
    return out, steps / wall, wall * 1e3 / steps, lat, ph


def run_small(rlu, torch, np, calls=1000, warm=50):
    """The 512 x 512 configuration (rank-10 + 1e-9 noise, k = 10, l = 15):
    a latency-bound call; p50/p99 over `calls` calls after `warm` warm-up
    calls (events around each call), plus the throughput of the sequence."""
    A, k, l, sseed = make_input("small512", torch)
    h = rlu.Handle(0)
    st = torch.cuda.current_stream()
    out = None
    for _ in range(warm):
        out = rlu.factor(A, k, l, seed=sseed, handle=h, stream=st, out=out)
    torch.cuda.synchronize()
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
           for _ in range(calls)]
    t0 = time.perf_counter()
    for e0, e1 in evs:
        e0.record(st)
        rlu.factor(A, k, l, seed=sseed, handle=h, stream=st, out=out)
        e1.record(st)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    lat = np.array([e0.elapsed_time(e1) for e0, e1 in evs])
    rel = power_residual(A, out.L, out.U, out.p, out.q)
    log(f"small512: p50 {np.percentile(lat, 50) * 1e3:.1f} us, p99 "
        f"{np.percentile(lat, 99) * 1e3:.1f} us, residual {rel:.3e}")
    return {"workload": WORKLOADS["small512"][8], "value": calls / wall,
            "unit": "factorizations/s", "calls": calls, "warmup": warm,
            "latency_ms": {"p50": float(np.percentile(lat, 50)),
                           "p99": float(np.percentile(lat, 99))},
            "rel_residual": rel, "info": out.info.cpu().tolist()}


def run_lstsq(rlu, torch, np, A, f, k, steps=20):
    """Algorithm 4.3 (Section 4.4) on the factors of the timed run: solve
    A x ~ b for b = A x0 (x0 Gaussian, fixed seed) with 1 and 64 right-hand
    sides; per-call time from events around each call, relative residual
    ||A x - b|| / ||b||."""
    m, n = A.shape
    h = rlu.Handle(0)
    st = torch.cuda.current_stream()
    gen = torch.Generator(device="cuda")
    gen.manual_seed(7206)
    res = {"workload": "rank-deficient least squares (Algorithm 4.3) on the 8192x8192 "
                       f"FP64 factors, k={k}, b = A x0"}
    for r in (1, 64):
        x0 = torch.randn(r, n, dtype=A.dtype, device="cuda", generator=gen).t()
        b = (A @ x0).t().contiguous().t()
        x = rlu.lstsq(f, b, handle=h, stream=st)
        for _ in range(3):
            rlu.lstsq(f, b, handle=h, stream=st, x=x)
        torch.cuda.synchronize()
        evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
               for _ in range(steps)]
        for e0, e1 in evs:
            e0.record(st)
            rlu.lstsq(f, b, handle=h, stream=st, x=x)
            e1.record(st)
        torch.cuda.synchronize()
        ms = np.array([e0.elapsed_time(e1) for e0, e1 in evs])
        rel = float(torch.linalg.norm(A @ x - b) / torch.linalg.norm(b))
        # bytes the solve must move: L (m k) and b (m r) read, x (n r) written
        byts = 8.0 * (m * k + m * r + n * r)
        res[f"rhs{r}"] = {"ms_per_call": float(np.median(ms)), "p99_ms": float(np.percentile(ms, 99)),
                          "rel_residual": rel,
                          "hbm_gbs": byts / (float(np.median(ms)) * 1e-3) / 1e9}
        log(f"lstsq form, {r} rhs: {np.median(ms):.3f} ms, residual {rel:.3e}")
    return res


def run_mixed(rlu, torch, np, steps):
    import workloads

    name, m, n, k, l, dseed, sseed, desc = MIXED
    log(f"generating {name}")
    A64 = workloads.spectral_matrix_torch(m, n, workloads.inv_square(min(m, n)), dseed,
                                          device="cuda", dtype=torch.float64)
    A64 = A64.t().contiguous().t()
    A32 = A64.float().t().contiguous().t()
    torch.cuda.synchronize()
    o16, v16, ms16, lat16, ph16 = timed_calls(rlu, torch, np, A32, k, l, sseed,
                                              rlu.PREC_MIXED_BF16, steps, 2)
    r16 = power_residual(A64, o16.L.double(), o16.U.double(), o16.p, o16.q)
    log(f"mixed bf16: {v16:.1f}/s residual {r16:.3e}")
    del o16
    o64, v64, ms64, lat64, ph64 = timed_calls(rlu, torch, np, A64, k, l, sseed,
                                              rlu.PREC_FP64, max(3, steps // 2), 1)
    r64 = power_residual(A64, o64.L, o64.U, o64.p, o64.q)
    log(f"fp64 path: {v64:.1f}/s residual {r64:.3e}")
    info64 = o64.info.cpu().tolist()
    del o64
    works16 = phase_work(m, n, k, l, 4.0, 4.0)
    works64 = phase_work(m, n, k, l, 8.0, 8.0)
    f_sk, b_sk = works16["sketch_gemm"]
    t_sk = ph16["sketch_gemm"] * 1e-3
    hbm_bound = b_sk / PEAK["hbm"] >= f_sk / PEAK["bf16"]
    roof = ({"bound": "hbm", "achieved": b_sk / t_sk / 1e9, "peak": PEAK["hbm"] / 1e9,
             "unit": "GB/s", "frac": b_sk / t_sk / PEAK["hbm"]} if hbm_bound else
            {"bound": "mfma", "achieved": f_sk / t_sk / 1e12, "peak": PEAK["bf16"] / 1e12,
             "unit": "TFLOP/s", "frac": f_sk / t_sk / PEAK["bf16"]})
    roof.update({"traffic": None, "kernel": "sketch GEMM (Step 2), BF16 MFMA 16x16x32, FP32 A",
                 "algorithmic_flops_per_launch": f_sk, "algorithmic_bytes_per_launch": b_sk})
    del A32, A64
    torch.cuda.empty_cache()
    return {
        "workload": desc, "value": v16, "unit": "factorizations/s", "ms_per_step": ms16,
        "latency_ms": {"p50": float(np.percentile(lat16, 50)),
                       "p99": float(np.percentile(lat16, 99))},
        "phase_ms": ph16,
        "kernels": kernel_table(ph16, works16, PEAK["bf16"]),
        "step_roofline": step_roofline(works16, PEAK["bf16"], ms16),
        "roofline": roof,
        "rel_residual": r16,
        "fp64_path": {"value": v64, "ms_per_step": ms64, "rel_residual": r64, "phase_ms": ph64,
                      "kernels": kernel_table(ph64, works64, PEAK["f64"]), "info": info64},
        "speedup_vs_fp64": v16 / v64,
        "residual_excess_vs_fp64": r16 - r64,
        "equal_error": bool(r16 <= r64 + 1e-3),
    }


SERVE = ("serve", 64, 105, 7206,
         "request stream: m log-uniform [512, 32768], n log-uniform [512, 8192], "
         "k ~ U{16..256}, l = k + 10, A = U_R diag(exp(-i/k)) V_R^T with R = min(m, n, 24 k), "
         "FP32 storage, BF16 products with FP32 accumulation; Poisson arrivals at 0.7 x the "
         "closed-loop saturation rate")


def make_serve_pool(torch, count, seed):
    """Device-resident request matrices of the serving workload (Haar-like
    thin factors from an FP32 QR of Gaussian matrices)."""
    import workloads

    shapes = workloads.serve_stream(count, seed=seed)
    pool = []
    gen = torch.Generator(device="cuda")
    for i, (m, n, k, l, s) in enumerate(shapes):
        gen.manual_seed(s % (2 ** 63))
        R = min(m, n, 24 * k)
        U, _ = torch.linalg.qr(torch.randn(m, R, generator=gen, device="cuda"))
        V, _ = torch.linalg.qr(torch.randn(n, R, generator=gen, device="cuda"))
        sig = torch.exp(-torch.arange(1, R + 1, device="cuda", dtype=torch.float32) / k)
        At = (V * sig) @ U.t()          # n x m = A^T, so A is column-major
        pool.append((At.t(), k, l))
        del U, V
    torch.cuda.synchronize()
    return pool


def run_serve(rlu, torch, np, n_req=2048, warm=256):
    name, pool_n, dseed, sseed, desc = SERVE
    log(f"generating serving pool of {pool_n} matrices")
    pool = make_serve_pool(torch, pool_n, dseed)
    srv = rlu.Server(0)
    order = np.random.default_rng(dseed).integers(0, pool_n, size=warm + n_req + 512)

    def submit(i):
        A, k, l = pool[order[i]]
        return srv.submit(A, k, l, seed=sseed + i, precision=rlu.PREC_MIXED_BF16)

    # closed loop: everything submitted at once
    t0 = time.perf_counter()
    ts = [submit(i) for i in range(512)]
    sat_status = {}
    for i, t in enumerate(ts):
        st = srv.wait(t)
        sat_status[st] = sat_status.get(st, 0) + 1
        if st != 0 and sat_status[st] == 1:
            A, k, l = pool[order[i]]
            _, r = srv.poll(t)
            log(f"serve: request {i} ({A.shape[0]}x{A.shape[1]}, k={k}, l={l}) status {st} "
                f"info {list(r.info)}")
    sat = 512 / (time.perf_counter() - t0)
    for t in ts:
        srv.release(t)
    log(f"serve: closed-loop saturation {sat:.0f} requests/s")
    # open loop, Poisson arrivals at 0.7 x saturation
    lam = 0.7 * sat
    gaps = np.random.default_rng(dseed + 1).exponential(1.0 / lam, size=warm + n_req)
    arrive = np.cumsum(gaps)
    outstanding = {}
    lat = []
    done_t = []
    statuses = {}
    start = time.perf_counter()
    i = 0
    total = warm + n_req
    while i < total or outstanding:
        now = time.perf_counter() - start
        while i < total and arrive[i] <= now:
            outstanding[submit(512 + i)] = i
            i += 1
        for t in list(outstanding):
            st, r = srv.poll(t)
            if st == 1:
                continue
            idx = outstanding.pop(t)
            statuses[st] = statuses.get(st, 0) + 1
            if idx >= warm:
                lat.append((r.t_done_us - r.t_submit_us) * 1e-3)
                done_t.append(time.perf_counter() - start)
            srv.release(t)
        if i < total:
            wait = arrive[i] - (time.perf_counter() - start)
            if wait > 2e-4:
                time.sleep(min(wait, 1e-3))
    span = max(done_t) - arrive[warm] if done_t else float("nan")
    srv.close()
    lat = np.array(lat)
    fp = [rlu.serve_footprint(A.shape[0], A.shape[1], k, l, rlu.F32, rlu.PREC_MIXED_BF16)
          for A, k, l in pool]
    del pool
    torch.cuda.empty_cache()
    return {
        "workload": desc, "value": len(lat) / span, "unit": "requests/s",
        "offered_rate": lam, "closed_loop_saturation": sat,
        "latency_ms": {"p50": float(np.percentile(lat, 50)), "p99": float(np.percentile(lat, 99)),
                       "mean": float(lat.mean()), "max": float(lat.max())},
        "requests": {"measured": int(len(lat)), "warmup": warm, "pool": pool_n,
                     "statuses": {str(k): v for k, v in statuses.items()},
                     "closed_loop_statuses": {str(k): v for k, v in sat_status.items()}},
        "footprint_mb": {"mean": float(np.mean(fp) / 1e6), "max": float(np.max(fp) / 1e6)},
    }


def run_batch(rlu, torch, np, steps, warmup):
    import workloads

    name, count, dseed, sseed, desc = BATCH
    shapes = workloads.batch_shapes(count, seed=dseed)
    log(f"generating {desc}")
    As = [workloads.low_rank_plus_noise_torch(m, n, r, 1e-6, s) for m, n, r, s in shapes]
    items = [(A, r, r + 8, sseed + i) for i, (A, (m, n, r, s)) in enumerate(zip(As, shapes))]
    torch.cuda.synchronize()
    h = rlu.Handle(0)
    batch = rlu.Batch(items, precision=rlu.PREC_FP32)
    stream = torch.cuda.current_stream()
    for _ in range(max(1, warmup)):
        batch.run(h, stream)           # first call records the graph
    torch.cuda.synchronize()
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
           for _ in range(steps)]
    t0 = time.perf_counter()
    for i in range(steps):
        evs[i][0].record(stream)
        batch.run(h, stream)           # graph replay
        evs[i][1].record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    lat = np.array([a.elapsed_time(b) for a, b in evs])
    infos = torch.stack([f.info for f in batch.outs]).cpu().numpy()
    log(f"batch: {steps} calls of {count} in {wall * 1e3:.1f} ms")
    # phase breakdown from one eager (timed) call of the same batch
    ht = rlu.Handle(0)
    ht.set_timing(True)
    rlu.Batch(items, precision=rlu.PREC_FP32).run(ht, stream)
    torch.cuda.synchronize()
    ph = ht.phase_times(0)
    # the same problems as sequential rlu_factor calls
    hs = rlu.Handle(0)
    for (A, k, l, sd) in items[:8]:
        rlu.factor(A, k, l, seed=sd, handle=hs, stream=stream)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    for (A, k, l, sd) in items:
        rlu.factor(A, k, l, seed=sd, handle=hs, stream=stream)
    torch.cuda.synchronize()
    seq = time.perf_counter() - t1
    dims = [(m, n, r, r + 8) for (m, n, r, s) in shapes]
    works = sum_works(dims, 4.0, 4.0)
    ms = wall * 1e3 / steps
    # dominant kernel of the batch: the grouped sketch GEMM
    f_sk, b_sk = works["sketch_gemm"]
    t_sk = ph["sketch_gemm"] * 1e-3
    hbm_bound = b_sk / PEAK["hbm"] >= f_sk / PEAK["f32"]
    roof = ({"bound": "hbm", "achieved": b_sk / t_sk / 1e9, "peak": PEAK["hbm"] / 1e9,
             "unit": "GB/s", "frac": b_sk / t_sk / PEAK["hbm"]} if hbm_bound else
            {"bound": "mfma", "achieved": f_sk / t_sk / 1e12, "peak": PEAK["f32"] / 1e12,
             "unit": "TFLOP/s", "frac": f_sk / t_sk / PEAK["f32"]})
    roof.update({"traffic": None, "kernel": "grouped sketch GEMM (Step 2), FP32 MFMA 16x16x4",
                 "algorithmic_flops_per_launch": f_sk, "algorithmic_bytes_per_launch": b_sk})
    return {
        "workload": desc, "value": count * steps / wall, "unit": "factorizations/s",
        "ms_per_call": ms, "steps": steps,
        "latency_ms": {"p50": float(np.percentile(lat, 50)), "p99": float(np.percentile(lat, 99))},
        "phase_ms_eager": ph,
        "kernels": kernel_table(ph, works, PEAK["f32"]),
        "step_roofline": step_roofline(works, PEAK["f32"], ms),
        "roofline": roof,
        "sequential_rlu_factor": {"factorizations_per_s": count / seq, "ms_total": seq * 1e3},
        "exchange_failures": int((infos[:, 2] != 0).sum()),
        "graph": "one captured HIP graph per batch, replayed",
    }


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=30)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default="exp8192", choices=sorted(WORKLOADS))
    ap.add_argument("--forms", default="fp32,power,lstsq,small,batch,mixed,serve",
                    help="extra measurements in the same line: comma list of fp32, power, lstsq, small, batch, "
                         "mixed, serve, or none")
    ap.add_argument("--input", default="spectral", choices=["spectral", "gaussian"],
                    help="gaussian: i.i.d. values of the same shape (hardware-counter runs)")
    ap.add_argument("--no-check", action="store_true",
                    help="skip the residual check after the timed steps")
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="after the timed steps, copy a 256 MiB buffer once (a plain copy "
                         "kernel of known traffic, to scale hardware byte counters)")
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU: the randomized LU path here runs on a single "
              "MI355X (multi-GPU sharding is design-only); run with --gpus 1", file=sys.stderr)
        sys.exit(2)
    if args.steps < 1 or args.steps > 64:
        print("--steps must be in [1, 64]", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    import paper_1310_7202_amd as rlu

    if not os.path.exists(rlu.LIB_PATH):
        from paper_1310_7202_amd import build
        build.build()
    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(2)

    name = args.workload
    res, A, out, (m, n, k, l, sseed, prec, s_a, peak, works) = run_single(
        rlu, torch, np, name, args.steps, args.warmup, args.input, not args.no_check)

    flops_sketch = works["sketch_gemm"][0]
    t_sketch = res["phase_ms"]["sketch_gemm"] * 1e-3
    achieved = flops_sketch / t_sketch
    kernel_src = os.path.join(ROOT, "paper_1310_7202_amd", "csrc", "gemm.hip")
    roofline = {"bound": "mfma", "achieved": achieved / 1e12, "peak": peak / 1e12,
                "unit": "TFLOP/s", "frac": achieved / peak,
                "traffic": traffic_from_profiles(kernel_src) if name == "exp8192" else None,
                "kernel": "sketch GEMM Y = A G (Step 2), "
                          + ("FP32" if prec == "fp32" else "FP64") + " MFMA 16x16x4",
                "algorithmic_flops_per_launch": flops_sketch,
                "algorithmic_bytes_per_launch": works["sketch_gemm"][1]}

    if args.calibrate_copy:
        src = torch.empty(32 << 20, dtype=torch.float64, device="cuda").fill_(1.0)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        log("copy calibration: 256 MiB read + 256 MiB written")
        del src, dst

    flops_total = sum(v[0] for v in works.values())
    result = {
        "metric": METRIC,
        "value": res["value"],
        "unit": "factorizations/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": res["ms_per_step"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32" if prec == "fp32" else "f64", "data": "synthetic",
        "config": {"workload": WORKLOADS[name][8], "m": m, "n": n, "k": k, "l": l,
                   "precision": prec, "sketch": "Philox4x32-10 Gaussian on device",
                   "input": args.input},
        "latency_ms": res["latency_ms"],
        "phase_ms": res["phase_ms"],
        "tflops_effective": flops_total / (res["ms_per_step"] * 1e-3) / 1e12,
        "roofline": roofline,
        "kernels": res["kernels"],
        "step_roofline": res["step_roofline"],
        "check": {"rel_residual": res.get("rel_residual"), "info": res["info"]},
    }

    forms = [f for f in args.forms.split(",") if f and f != "none"]
    result["forms"] = {}
    if "fp32" in forms and name == "exp8192":
        A32 = A.float()
        A32 = A32.t().contiguous().t()
        h32 = rlu.Handle(0)
        h32.set_timing(2)
        st = torch.cuda.current_stream()
        o32 = None
        for _ in range(3):
            o32 = rlu.factor(A32, k, l, seed=sseed, handle=h32, stream=st, out=o32)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        n32 = max(5, args.steps // 2)
        for _ in range(n32):
            o32 = rlu.factor(A32, k, l, seed=sseed, handle=h32, stream=st, out=o32)
        torch.cuda.synchronize()
        w32 = time.perf_counter() - t0
        sk32 = float(np.mean([h32.phase_times(b)["sketch_gemm"] for b in range(n32)]))
        h32.set_timing(True)  # every phase, in a pass after the timed region
        for _ in range(5):
            o32 = rlu.factor(A32, k, l, seed=sseed, handle=h32, stream=st, out=o32)
        torch.cuda.synchronize()
        ph32 = [h32.phase_times(b) for b in range(5)]
        ph32 = {key: float(np.mean([p[key] for p in ph32])) for key in ph32[0]}
        ph32["sketch_gemm"] = sk32
        works32 = phase_work(m, n, k, l, 4.0, 4.0)
        r32 = power_residual(A, o32.L.double(), o32.U.double(), o32.p, o32.q)
        result["forms"]["fp32"] = {
            "workload": WORKLOADS["exp8192_fp32"][8], "value": n32 / w32,
            "unit": "factorizations/s", "ms_per_step": w32 * 1e3 / n32, "phase_ms": ph32,
            "kernels": kernel_table(ph32, works32, PEAK["f32"]),
            "step_roofline": step_roofline(works32, PEAK["f32"], w32 * 1e3 / n32),
            "rel_residual": r32,
            "rel_residual_fp64_path": res.get("rel_residual"),
            "speedup_vs_fp64": (n32 / w32) / res["value"]}
        log(f"fp32 form: {n32 / w32:.1f}/s residual {r32:.3e}")
        del A32, o32
    if "power" in forms and name == "exp8192":
        # Section 5.2: one power iteration, Y = (A A^T) A G with the LU
        # normalization, on the same matrix and sketch seed
        outp, vp, msp, latp, php = timed_calls(rlu, torch, np, A, k, l, sseed, None,
                                               max(5, args.steps // 3), 2, power_iters=1)
        rp = power_residual(A, outp.L, outp.U, outp.p, outp.q)
        r0 = res.get("rel_residual")
        result["forms"]["power_q1"] = {
            "workload": WORKLOADS["exp8192"][8] + ", q = 1 power iteration",
            "value": vp, "unit": "factorizations/s", "ms_per_step": msp,
            "latency_ms": {"p50": float(np.percentile(latp, 50)),
                           "p99": float(np.percentile(latp, 99))},
            "phase_ms": php, "rel_residual": rp, "rel_residual_q0": r0,
            "error_ratio_vs_q0": rp / r0 if r0 else None,
            "info": outp.info.cpu().tolist()}
        log(f"power form: {vp:.1f}/s ({msp:.2f} ms), residual {rp:.3e} against {r0}")
        del outp
    if "small" in forms:
        result["forms"]["small512"] = run_small(rlu, torch, np)
    if "lstsq" in forms and name == "exp8192":
        result["forms"]["lstsq"] = run_lstsq(rlu, torch, np, A, out, k)
    if "mixed" in forms:
        result["forms"]["mixed16384"] = run_mixed(rlu, torch, np, 8)
    if "batch" in forms:
        result["forms"]["batch256"] = run_batch(rlu, torch, np, max(5, args.steps // 2), 2)
        log(f"batch form: {result['forms']['batch256']['value']:.0f} factorizations/s")
    if "serve" in forms:
        result["forms"]["serve"] = run_serve(rlu, torch, np)
        sv = result["forms"]["serve"]
        log(f"serve form: {sv['value']:.0f} requests/s, p50 {sv['latency_ms']['p50']:.2f} ms, "
            f"p99 {sv['latency_ms']['p99']:.2f} ms")

    if not args.no_cpu_baseline:
        A_host = A.double().cpu().numpy() if prec == "fp32" else A.cpu().numpy()
        base, o, G = cpu_baseline(A_host, k, l, sseed, args.cpu_seconds)
        result["cpu_baseline"] = base
        # parity at full size: same G up to libm rounding on the two sides
        L, U = out.L.double().cpu().numpy(), out.U.double().cpu().numpy()
        p, q = out.p.cpu().numpy(), out.q.cpu().numpy()
        Lu = np.empty_like(L); Lu[p] = L
        Lo = np.empty_like(o["L"]); Lo[o["p"]] = o["L"]
        Uu = np.empty_like(U); Uu[:, q] = U
        Uo = np.empty_like(o["U"]); Uo[:, o["q"]] = o["U"]
        result["check"]["max_rel_diff_vs_oracle"] = {
            "L_unpermuted": float(np.abs(Lu - Lo).max() / np.abs(Lo).max()),
            "U_unpermuted": float(np.abs(Uu - Uo).max() / np.abs(Uo).max()),
            "q_equal": bool(np.array_equal(q, o["q"])),
            "p_equal": bool(np.array_equal(p, o["p"]))}
    else:
        result["cpu_baseline"] = None
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
