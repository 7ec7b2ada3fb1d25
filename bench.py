"""Benchmark: Greek-path throughput of the QMC-CPW hot path on one MI355X.

One step = one call of the whole hot path (Sobol points + shifts, inverse
normal, Brownian-bridge path, exponentials and sums, breakpoint, Phi tails,
price/delta/vega/gamma, reduction over points and replications) over the
workload "three products at d = 64": arithmetic Asian, binary Asian and
lookback calls x K {90, 100, 110} x sigma {0.1, 0.3}, S0 = 100, r = 0.05,
T = 1, 2^20 Sobol points x 32 random shifts each (18 options, 6.04e8
Greek-paths, 3.8e10 path-dates), FP32-mixed arithmetic.  Inputs are
synthetic option parameters (no dataset) and stay on the device.

Prints one JSON line.  Extra legs (each its own timed loop, outside the
headline value): the same workload in plain FP64, and the oracle on the
host cores (cpu_baseline, a bounded sample).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# Algorithmic work (op-count model of the method, independent of the kernel):
# per path-date (one conditioned coordinate of one path) the inverse normal
# (log + degree-9 polynomial + argument and sign: 24), the bridge step (5), the
# exponential (1) and the running sums (5) make about 35 FP32 flops (36 with
# the uint->float conversion); per path the breakpoint (log), two Phi tails,
# the density, the four Greeks and the compensated sums make about 200 FP64
# flops.
F32_PER_PATH_DATE = 36.0
F64_PER_PATH = 200.0
PEAK_F32 = 157.3e12       # MI355X vector FP32 (packed), 256 CU x 2.4 GHz x 256 flop/clk
PEAK_F64 = 78.6e12        # MI355X vector FP64

# HBM bytes per launch of the fused kernel on this workload, from rocprofv3
# FETCH_SIZE and WRITE_SIZE scaled by a 1 GiB copy (profiles/
# paths_kernel_fp32_bridge_three_products_d64.md), valid only for the kernel
# sources they were taken on (sha256 prefix of their concatenation).
TRAFFIC_SOURCES = ("kernels.hip", "device_math.h", "qcpw_internal.h", "ninv_table.inc")
TRAFFIC_SHA = "058e69e34590da59"
TRAFFIC_BYTES = {"fetch": 0.925e6, "write": 15.729e6}


def kernel_sources_sha() -> str:
    import hashlib
    h = hashlib.sha256()
    for f in TRAFFIC_SOURCES:
        with open(os.path.join(ROOT, "paper_2209_11337_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


# The paper's own timings (Sec. 6.1; Tesla T4, CUDA 11.2, FP32 path arithmetic, CPU model not
# stated): context only, other hardware and a single option per kernel run.
PAPER_CONTEXT = {
    "hardware": "NVIDIA Tesla T4 (paper), serial CPU of unstated model",
    "qmc_bb_cpw_kernel_ms": {"2^15 paths": 0.8, "2^19 paths": 12.5},
    "other_cpw_kernel_ms": {"2^15 paths": 0.2, "2^19 paths": 3.0},
    "serial_cpu_ms_2^15_paths": 150.0,
    "speedup_vs_serial_cpu": {"qmc_bb_cpw": "about 200x", "other methods": "over 500x (d=64), 900x (d=256)"},
    "derived_greek_paths_per_s_qmc_bb_cpw": 4.2e7,
}


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=10)
    p.add_argument("--warmup", type=int, default=2)
    p.add_argument("--precision", choices=["fp32", "fp64"], default="fp32")
    p.add_argument("--no-extras", action="store_true", help="skip the FP64 and CPU legs")
    p.add_argument("--cpu-points", type=int, default=1 << 19)
    p.add_argument("--no-portfolio", action="store_true", help="skip the uneven-portfolio leg")
    p.add_argument("--no-serve", action="store_true", help="skip the serving leg")
    p.add_argument("--pca-only", action="store_true",
                   help="run only the principal-component leg (one timed call per GEMM) and print it")
    p.add_argument("--copy-mib", type=int, default=0,
                   help="after the timed loop, run one plain device copy of this many MiB "
                        "(reference kernel for HBM byte counters)")
    return p.parse_args()


def main():
    a = parse()
    if a.gpus != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path (its work units "
              "would shard across GPUs by option, replication and point range)", file=sys.stderr)
        sys.exit(2)
    import torch

    import paper_2209_11337_amd as q
    import workloads

    q.lib()  # raises if the HIP library is not built
    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    if a.pca_only:
        print(json.dumps({"pca": pca_leg(q, workloads, torch, steps=1)}), flush=True)
        return
    L = 32
    opts = workloads.three_products_grid(d=64, n_points=1 << 20)
    n_paths = workloads.total_paths(opts, L)
    n_pd = workloads.total_path_dates(opts, L)
    prec = q.FP32_MIXED if a.precision == "fp32" else q.FP64
    out = (torch.empty((len(opts), 4), dtype=torch.float64, device=dev),
           torch.empty((len(opts), 4), dtype=torch.float64, device=dev))
    stream = torch.cuda.Stream()

    def step(p):
        q.greeks(opts, L, q.PATH_BB, p, device_outputs=True, out=out, stream=stream)

    def timed(p, steps, warmup):
        for _ in range(warmup):
            step(p)
        torch.cuda.synchronize()
        stream.synchronize()
        evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(steps)]
        q.kernel_timer(q.TIMER_START)
        t0 = time.perf_counter()
        for s, e in evs:
            s.record(stream)
            step(p)
            e.record(stream)
        stream.synchronize()
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        k_ms, k_n = q.kernel_timer(q.TIMER_STOP)
        ev_ms = float(np.mean([s.elapsed_time(e) for s, e in evs]))
        return wall, ev_ms, k_ms / max(k_n, 1)

    # HIP events recorded by the library on the launch stream around the
    # fused per-path kernel alone (kernel_ms), and torch events around each
    # whole call on the same stream (call_ms)
    wall, ev_ms, kern_ms = timed(prec, a.steps, a.warmup)
    if a.copy_mib > 0:
        src = torch.ones(a.copy_mib << 18, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    print("timed %d steps: %.3f s wall, %.3f ms/call, %.3f ms/kernel (events)" % (a.steps, wall, ev_ms, kern_ms),
          file=sys.stderr, flush=True)
    value = n_paths * a.steps / wall
    g = out[0].cpu().numpy()
    e = out[1].cpu().numpy()

    f32 = F32_PER_PATH_DATE * n_pd if prec == q.FP32_MIXED else 0.0
    f64 = F64_PER_PATH * n_paths + (0.0 if prec == q.FP32_MIXED else F32_PER_PATH_DATE * n_pd)
    t_ideal = f32 / PEAK_F32 + f64 / PEAK_F64
    t_kernel = kern_ms * 1e-3
    achieved = (f32 + f64 * PEAK_F32 / PEAK_F64) / t_kernel
    same_kernel = prec == q.FP32_MIXED and kernel_sources_sha() == TRAFFIC_SHA
    traffic = TRAFFIC_BYTES["fetch"] + TRAFFIC_BYTES["write"] if same_kernel else None
    roofline = {"bound": "alu", "achieved": achieved / 1e12, "peak": PEAK_F32 / 1e12, "unit": "TFLOP/s",
                "frac": t_ideal / t_kernel, "traffic": traffic,
                "model": "FP32-equivalent flops: %.0f FP32/path-date + %.0f FP64/path (FP64 weighted x2)"
                         % (F32_PER_PATH_DATE, F64_PER_PATH),
                "kernel": "qcpw::paths_kernel", "kernel_ms": kern_ms, "call_ms": ev_ms}

    res = {"metric": "Greek-paths/sec (delta+vega+gamma) at fixed RMSE vs FP64; p99 request latency",
           "value": value, "unit": "Greek-paths/s", "n_gpus": 1, "steps": a.steps, "warmup": a.warmup,
           "ms_per_step": wall / a.steps * 1e3, "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": "f32+f64" if prec == q.FP32_MIXED else "f64",
           "data": "synthetic (Black-Scholes option parameters, seeded)",
           "config": {"workload": "three products (arith Asian, binary Asian, lookback) x K{90,100,110} x "
                                  "sigma{0.1,0.3}, d=64, Brownian bridge, 2^20 Sobol points x 32 shifts",
                      "options": len(opts), "greek_paths_per_step": n_paths, "path_dates_per_step": n_pd,
                      "precision": a.precision},
           "roofline": roofline}

    if not a.no_extras:
        # plain FP64 on the same workload, same launch path
        w64, ev64, _ = timed(q.FP64, 2, 1)
        g64 = out[0].cpu().numpy()
        res["fp64"] = {"value": n_paths * 2 / w64, "ms_per_step": w64 / 2 * 1e3, "kernel_ms": ev64}
        if prec == q.FP32_MIXED:
            rel = np.abs(g - g64) / np.maximum(np.abs(g64), 1e-300)
            res["fp32_vs_fp64_max_rel_diff"] = {k: float(rel[:, i].max()) for i, k in enumerate(q.OUTPUTS)}
            res["stderr_max_rel"] = {k: float((e[:, i] / np.maximum(np.abs(g64[:, i]), 1e-300)).max())
                                     for i, k in enumerate(q.OUTPUTS)}
        # the oracle on the host cores, a bounded sample of the same workload
        import oracle
        n_cpu = a.cpu_points
        Ls = 8
        sample = workloads.three_products_grid(d=64, n_points=n_cpu)
        threads = os.cpu_count() or 1
        t0 = time.perf_counter()
        _, _, _, used = oracle.options(sample, Ls, oracle.PATH_BB, n_threads=threads)
        tc = time.perf_counter() - t0
        res["cpu_baseline"] = {"value": workloads.total_paths(sample, Ls) / tc, "unit": "Greek-paths/s",
                               "cores": used, "kind": "oracle",
                               "sample": "the 18 options at d=64, 2^%d points x %d shifts (%.1f s)"
                                         % (int(np.log2(n_cpu)), Ls, tc),
                               "cpu_model": cpu_model()}
        # one host thread, a smaller sample of the same workload
        sample1 = workloads.three_products_grid(d=64, n_points=1 << 14)
        t0 = time.perf_counter()
        oracle.options(sample1, 2, oracle.PATH_BB, n_threads=1)
        t1c = time.perf_counter() - t0
        res["cpu_baseline"]["single_thread"] = {"value": workloads.total_paths(sample1, 2) / t1c,
                                                "sample": "the 18 options at d=64, 2^14 points x 2 shifts (%.1f s)"
                                                          % t1c}
        res["paper_context"] = PAPER_CONTEXT
    if not a.no_extras:
        # the same workload randomised by nested scrambling instead of the shift
        q.greeks(opts, L, q.PATH_BB, prec, device_outputs=True, out=out, stream=stream, owen=True)
        stream.synchronize()
        q.kernel_timer(q.TIMER_START)
        t0 = time.perf_counter()
        for _ in range(3):
            q.greeks(opts, L, q.PATH_BB, prec, device_outputs=True, out=out, stream=stream, owen=True)
        stream.synchronize()
        w_owen = (time.perf_counter() - t0) / 3
        k_ms, k_n = q.kernel_timer(q.TIMER_STOP)
        e_owen = out[1].cpu().numpy()
        res["owen"] = {"value": n_paths / w_owen, "unit": "Greek-paths/s", "kernel_ms": k_ms / max(k_n, 1),
                       "stderr_ratio_owen_over_shift": {k: float(np.median(e_owen[:, i] / e[:, i]))
                                                        for i, k in enumerate(q.OUTPUTS)}}
        res["geometric"] = geometric_leg(q, workloads, torch, prec)
        res["more_products"] = more_products_leg(q, workloads, torch, prec)
        res["small_call"] = small_call_leg(q, workloads, torch)
        res["pca"] = pca_leg(q, workloads, torch)
    if not a.no_extras and not a.no_portfolio:
        res["portfolio"] = portfolio_leg(q, workloads, torch)
    if not a.no_extras and not a.no_serve:
        # the configured stream (1..512 options, d in [4, 365], targets 1e-4 / 1e-6, which the
        # point cap of 2^22 per option decides): a short stream at a rate the GPU sustains
        res["serving"] = serving_leg(q, workloads, n_requests=12, rate=0.3, max_opts=512, d_range=(4, 365),
                                     targets=(1e-4, 1e-6), fp64_requests=3, fp64_max_opts=8)
        # a dense stream of small requests (1..32 options, d in [4, 64], targets 1e-3 / 1e-4)
        res["serving_small_requests"] = serving_leg(q, workloads)
    print(json.dumps(res), flush=True)


def geometric_leg(q, workloads, torch, prec, L=32, steps=3):
    """Six geometric Asian calls on the main workload's setting (d = 64, bridge,
    2^20 points x 32 shifts): rate, kernel time, and the distance of every
    estimate from the closed form of the discretely monitored geometric call
    in reported standard errors."""
    sys.path.insert(0, os.path.join(os.path.dirname(os.path.abspath(__file__)), "tests"))
    from closed_forms import geometric_asian_closed_form
    dev = torch.device("cuda", 0)
    opts = workloads.geometric_grid(d=64, n_points=1 << 20)
    out = (torch.empty((len(opts), 4), dtype=torch.float64, device=dev),
           torch.empty((len(opts), 4), dtype=torch.float64, device=dev))
    stream = torch.cuda.Stream()
    q.greeks(opts, L, q.PATH_BB, prec, device_outputs=True, out=out, stream=stream)
    stream.synchronize()
    q.kernel_timer(q.TIMER_START)
    t0 = time.perf_counter()
    for _ in range(steps):
        q.greeks(opts, L, q.PATH_BB, prec, device_outputs=True, out=out, stream=stream)
    stream.synchronize()
    w = (time.perf_counter() - t0) / steps
    k_ms, k_n = q.kernel_timer(q.TIMER_STOP)
    g, e = out[0].cpu().numpy(), out[1].cpu().numpy()
    exact = np.array([geometric_asian_closed_form(o["S0"], o["K"], o["r"], o["sigma"], o["T"], o["d"])
                      for o in opts])
    z = np.abs(g - exact) / e
    return {"value": workloads.total_paths(opts, L) / w, "unit": "Greek-paths/s", "kernel_ms": k_ms / max(k_n, 1),
            "max_abs_err_in_stderr": {k: float(z[:, i].max()) for i, k in enumerate(q.OUTPUTS)},
            "stderr_max_rel": {k: float((e[:, i] / np.abs(exact[:, i])).max()) for i, k in enumerate(q.OUTPUTS)}}


def more_products_leg(q, workloads, torch, prec, L=32, steps=2):
    """Puts (24 options: arithmetic, binary, geometric Asian and lookback on the
    minimum, d = 64, bridge) and baskets (8 options on 4 assets, d = 64,
    standard construction), 2^20 points x 32 shifts each: rate, kernel time
    and the largest relative standard error per Greek."""
    dev = torch.device("cuda", 0)
    out = {}
    for name, opts, path in [("puts_d64_bridge", workloads.put_grid(d=64, n_points=1 << 20), q.PATH_BB),
                             ("basket_4_assets_d64_standard",
                              workloads.basket_grid(d=64, n_assets=4, n_points=1 << 20), q.PATH_STANDARD)]:
        res = (torch.empty((len(opts), 4), dtype=torch.float64, device=dev),
               torch.empty((len(opts), 4), dtype=torch.float64, device=dev))
        stream = torch.cuda.Stream()
        q.greeks(opts, L, path, prec, device_outputs=True, out=res, stream=stream)
        stream.synchronize()
        q.kernel_timer(q.TIMER_START)
        t0 = time.perf_counter()
        for _ in range(steps):
            q.greeks(opts, L, path, prec, device_outputs=True, out=res, stream=stream)
        stream.synchronize()
        w = (time.perf_counter() - t0) / steps
        k_ms, k_n = q.kernel_timer(q.TIMER_STOP)
        g, e = res[0].cpu().numpy(), res[1].cpu().numpy()
        out[name] = {"value": workloads.total_paths(opts, L) / w, "unit": "Greek-paths/s",
                     "kernel_ms": k_ms / max(k_n, 1),
                     "stderr_max_rel": {k: float((e[:, i] / np.maximum(np.abs(g[:, i]), 1e-300)).max())
                                        for i, k in enumerate(q.OUTPUTS)}}
    return out


def small_call_leg(q, workloads, torch, calls=200):
    """Latency-bound call: one arithmetic Asian, d = 16, 2^12 points x 16
    shifts, bridge, device outputs; per-call time eager vs replayed from a
    captured HIP graph, in FP64 (eager_us, graph_us) and FP32-mixed
    (fp32_eager_us, fp32_graph_us)."""
    opts = workloads.single_asian()
    s = torch.cuda.Stream()
    out = (torch.empty((1, 4), dtype=torch.float64, device="cuda"),
           torch.empty((1, 4), dtype=torch.float64, device="cuda"))
    res = {"workload": "1 arithmetic Asian, d=16, 2^12 points x 16 shifts, bridge; FP64 (eager_us, graph_us) "
                       "and FP32-mixed (fp32_eager_us, fp32_graph_us)"}
    for prefix, prec in (("", q.FP64), ("fp32_", q.FP32_MIXED)):
        for name, graph in (("eager_us", False), ("graph_us", True)):
            for _ in range(3):
                q.greeks(opts, 16, q.PATH_BB, prec, device_outputs=True, out=out, stream=s, graph=graph)
            s.synchronize()
            t0 = time.perf_counter()
            for _ in range(calls):
                q.greeks(opts, 16, q.PATH_BB, prec, device_outputs=True, out=out, stream=s, graph=graph)
            s.synchronize()
            res[prefix + name] = (time.perf_counter() - t0) / calls * 1e6
    return res


def pca_leg(q, workloads, torch, steps=3):
    """Principal-component paths at d = 256 (255 x 255 factor padded to 256,
    a dense (256 x 256) x (256 x 64-point) product per tile on the matrix
    cores): arithmetic and binary Asian, 2^22 points x 16 shifts, FP32-mixed,
    GEMM in FP32 MFMA and in split BF16x3; kernel time from the library's
    HIP events.  gemm_frac is the product's algorithmic flops 2 n^2 per path
    over the time of the whole fused kernel, against the FP32 MFMA peak
    (157.3 TFLOP/s) or, for BF16x3 (three BF16 products per FP32 product),
    a third of the BF16 peak (2.5 PFLOP/s / 3)."""
    opts = workloads.pca_pair(d=256, n_points=1 << 22)
    L = 16
    n = 255
    paths = workloads.total_paths(opts, L)
    s = torch.cuda.Stream()
    out = (torch.empty((2, 4), dtype=torch.float64, device="cuda"),
           torch.empty((2, 4), dtype=torch.float64, device="cuda"))
    res = {"workload": "arith + binary Asian, d=256, PCA, 2^22 points x 16 shifts, FP32-mixed",
           "greek_paths": paths}
    for name, gemm, peak in (("fp32_mfma", q.GEMM_FP32, 157.3e12), ("bf16x3_mfma", q.GEMM_BF16X3, 2.5e15 / 3)):
        q.greeks(opts, L, q.PATH_PCA, q.FP32_MIXED, pca_gemm=gemm, device_outputs=True, out=out, stream=s)
        s.synchronize()
        q.kernel_timer(q.TIMER_START)
        t0 = time.perf_counter()
        for _ in range(steps):
            q.greeks(opts, L, q.PATH_PCA, q.FP32_MIXED, pca_gemm=gemm, device_outputs=True, out=out, stream=s)
        s.synchronize()
        wall = (time.perf_counter() - t0) / steps
        k_ms, k_n = q.kernel_timer(q.TIMER_STOP)
        k_ms /= max(k_n, 1)
        gflop = 2.0 * n * n * paths
        res[name] = {"value": paths / wall, "unit": "Greek-paths/s", "kernel_ms": k_ms,
                     "gemm_tflops": gflop / (k_ms * 1e-3) / 1e12,
                     "gemm_frac": gflop / (k_ms * 1e-3) / peak}
        if gemm == q.GEMM_FP32:
            se_x1 = out[1].cpu().numpy().copy()
    # the same points conditioned on the first principal component of all d
    # dates (FP64 Newton root-find per path): time, and the variance ratio of
    # each Greek against conditioning on the first date's normal
    q.greeks(opts, L, q.PATH_PCA_FULL, q.FP32_MIXED, device_outputs=True, out=out, stream=s)
    s.synchronize()
    q.kernel_timer(q.TIMER_START)
    t0 = time.perf_counter()
    for _ in range(steps):
        q.greeks(opts, L, q.PATH_PCA_FULL, q.FP32_MIXED, device_outputs=True, out=out, stream=s)
    s.synchronize()
    wall = (time.perf_counter() - t0) / steps
    k_ms, k_n = q.kernel_timer(q.TIMER_STOP)
    se_full = out[1].cpu().numpy()
    res["pca_full_fp32_mfma"] = {
        "value": paths / wall, "unit": "Greek-paths/s", "kernel_ms": k_ms / max(k_n, 1),
        "variance_ratio_vs_first_date": {k: [float((se_x1[i, j] / se_full[i, j]) ** 2) for i in range(2)]
                                         for j, k in enumerate(q.OUTPUTS)}}
    return res


def portfolio_leg(q, workloads, torch):
    """4096 options of uneven type, d, K, sigma, T, r and 2^14..2^20 points,
    16 shifts, FP32-mixed, in one persistent launch; beside it the plain
    path (FP64, one option per launch) on a fixed sample of the options."""
    opts = workloads.portfolio(4096)
    L = 16
    q.greeks(opts[:64], L, q.PATH_BB, q.FP32_MIXED)   # warm the tables / workspace
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    g, e = q.greeks(opts, L, q.PATH_BB, q.FP32_MIXED)
    t = time.perf_counter() - t0
    paths = workloads.total_paths(opts, L)
    sample = opts[::128]
    t1 = time.perf_counter()
    for o in sample:
        q.greeks([o], L, q.PATH_BB, q.FP64)
    t64 = time.perf_counter() - t1
    p64 = workloads.total_paths(sample, L)
    return {"options": len(opts), "shifts": L, "greek_paths": paths,
            "path_dates": workloads.total_path_dates(opts, L), "seconds": t, "value": paths / t,
            "unit": "Greek-paths/s", "precision": "fp32-mixed, one persistent launch",
            "fp64_one_option_per_launch": {"value": p64 / t64, "sample": "every 128th option (%d)" % len(sample),
                                           "seconds": t64}}


def serving_leg(q, workloads, n_requests=300, rate=100.0, max_opts=32, d_range=(4, 64), targets=(1e-3, 1e-4),
                fp64_requests=40, fp64_max_opts=None):
    """Poisson request stream into the continuous-batching server (FP32-mixed):
    requests of 1..max_opts options (d in d_range, otherwise drawn as the
    uneven portfolio) with a target standard error from `targets` (relative
    to max(1, |Greek|)); latency = submit to result.  Beside it the plain
    path: each option of the first fp64_requests requests (at most
    fp64_max_opts options of each) alone in FP64 at the point count the
    server reached."""
    import threading
    stream = workloads.request_stream(n_requests, rate, max_opts=max_opts, d_range=d_range, targets=targets)
    L = 16
    lat, pts, paths = [], [], 0
    done = {}
    pending = []
    lock = threading.Lock()
    finished = threading.Event()
    with q.Server(hbm_budget_bytes=8 << 30, precision=q.FP32_MIXED) as srv:

        def poller():
            # completion times are taken as soon as a result is ready
            while True:
                with lock:
                    todo = list(pending)
                for item in todo:
                    rid, ts, r = item
                    out = srv.poll(rid, len(r["options"]))
                    if out is not None:
                        done[rid] = (time.perf_counter() - ts, out[2])
                        with lock:
                            pending.remove(item)
                if finished.is_set() and not todo:
                    return
                time.sleep(0.0002)

        th = threading.Thread(target=poller)
        th.start()
        t0 = time.perf_counter()
        ids = []
        for r in stream:
            now = time.perf_counter() - t0
            if r["t_arrival"] > now:
                time.sleep(r["t_arrival"] - now)
            item = (srv.submit(r["options"], L, r["target_stderr"]), time.perf_counter(), r)
            ids.append(item)
            with lock:
                pending.append(item)
        finished.set()
        th.join()
        wall = time.perf_counter() - t0
        stats = srv.stats()
    for rid, ts, r in ids:
        l, p = done[rid]
        lat.append(l)
        pts.append(p)
        paths += len(r["options"]) * p * L
    lat = np.array(lat) * 1e3
    # plain FP64, one option per launch, same points
    base_lat, base_paths, t64 = [], 0, 0.0
    for (rid, ts, r), p in list(zip(ids, pts))[:fp64_requests]:
        sub = r["options"][:fp64_max_opts]
        t1 = time.perf_counter()
        for o in sub:
            q.greeks([dict(o, n_points=p)], L, q.PATH_BB, q.FP64)
        dt = time.perf_counter() - t1
        base_lat.append(dt * 1e3)
        t64 += dt
        base_paths += len(sub) * p * L
    return {"requests": n_requests, "rate_per_s": rate, "options_per_request": [1, max_opts],
            "d_range": list(d_range), "target_stderr": list(targets), "shifts": L,
            "p50_ms": float(np.percentile(lat, 50)),
            "p99_ms": float(np.percentile(lat, 99)), "mean_points": float(np.mean(pts)),
            "value": paths / wall, "unit": "Greek-paths/s", "launches": stats["launches"],
            "fp64_one_option_per_launch": {"value": base_paths / t64,
                                           "p50_ms_no_queueing": float(np.percentile(base_lat, 50)),
                                           "p99_ms_no_queueing": float(np.percentile(base_lat, 99)),
                                           "sample": "first %d requests%s" % (
                                               fp64_requests, "" if fp64_max_opts is None else
                                               ", first %d options of each" % fp64_max_opts)}}


if __name__ == "__main__":
    main()
