"""Benchmark: Greek-path throughput of the QMC-CPW hot path on one MI355X.

One step = one call of the whole hot path (Sobol points + shifts, inverse
normal, Brownian-bridge path, exponentials and sums, breakpoint, Phi tails,
price/delta/vega/gamma, reduction over points and replications) over the
uneven portfolio: 4096 options in one persistent launch, type uniform over
{arithmetic Asian, binary Asian, lookback} calls, d uniform in [4, 365],
K ~ U[80,120], sigma ~ U[0.1,0.5], T ~ U[0.25,2], r ~ U[0,0.08], S0 = 100,
2^k Sobol points with k uniform in [14, 20], 16 random shifts, Brownian
bridge, FP32 path arithmetic with FP64 breakpoint, tails and sums (1.95e10
Greek-paths, 3.6e12 path-dates).  Inputs are synthetic option parameters
(no dataset) and stay on the device; outputs are written on the device.

Prints one JSON line.  Extra legs (each its own timed loop, outside the
headline value): the three-product grid at d = 64 (FP32-mixed and plain
FP64), the principal-component pair at d = 256 on the matrix cores, nested
scrambling, more products, the latency-bound single call, the serving
stream, and the oracle on the host cores (cpu_baseline, a bounded sample of
the headline workload).
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
# flops.  Plain FP64 mode: about 75 FP64 flops per path-date (software exp
# and log in place of the FP32 table lookups).
F32_PER_PATH_DATE = 36.0
F64_PER_PATH_DATE_PLAIN = 75.0
F64_PER_PATH = 200.0
PEAK_F32 = 157.3e12       # MI355X vector FP32 (packed), 256 CU x 2.4 GHz x 256 flop/clk
PEAK_F64 = 78.6e12        # MI355X vector FP64
PEAK_MFMA_F32 = 157.3e12  # MI355X dense FP32 matrix
PEAK_MFMA_BF16 = 2.5e15   # MI355X dense BF16 matrix

# HBM bytes per call of the fused kernel (its launches summed), from
# rocprofv3 FETCH_SIZE and WRITE_SIZE scaled by a plain 1 GiB copy
# (profiles/), valid only for the kernel and launch-planning sources they
# were taken on (sha256 prefix of their concatenation).
TRAFFIC_SOURCES = ("paths_kernel.h", "device_math.h", "qcpw_internal.h", "ninv_table.inc", "phi_f64_coeffs.inc",
                   "kernels.hip")
TRAFFIC = {
    "portfolio": {"sha": "5c97a5a5ac6d6577", "fetch": 1169816677, "write": 1329362464},
    "three_products": {"sha": "5c97a5a5ac6d6577", "fetch": 12950537, "write": 14156128},
}


# Per-unit work the fused kernel itself executes, from the rocprofv3 counters
# of the same kernel sources (profiles/): SQ_INSTS_VALU, SQ_INSTS_VALU_FLOPS_FP32
# and _FP64 (per wave, x64 lanes, the call's launches summed) over its
# path-dates and paths.
COUNTERS = {
    "portfolio": {"sha": "5c97a5a5ac6d6577", "valu_per_path_date": 16.84, "fp32_flops_per_path_date": 15.28,
                  "fp64_flops_per_path": 178.7},
    "three_products": {"sha": "5c97a5a5ac6d6577", "valu_per_path_date": 16.46, "fp32_flops_per_path_date": 14.75,
                       "fp64_flops_per_path": 172.3},
}
CLOCK_HZ = 2.4e9
SIMDS = 1024


def counters_of(workload: str):
    c = COUNTERS[workload]
    if c["sha"] is None or c["sha"] != kernel_sources_sha():
        return None
    return c


def kernel_sources_sha() -> str:
    import hashlib
    h = hashlib.sha256()
    for f in TRAFFIC_SOURCES:
        with open(os.path.join(ROOT, "paper_2209_11337_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def traffic_of(workload: str):
    t = TRAFFIC[workload]
    if t["sha"] is None or t["sha"] != kernel_sources_sha():
        return None
    return t["fetch"] + t["write"]


def roofline(paths, path_dates, kernel_ms, fp32=True, mfma_flops=0.0, mfma_peak=PEAK_MFMA_F32,
             kernel="qcpw::paths_kernel (every launch of the call)", traffic=None, call_ms=None, counters=None):
    """Whole-kernel roofline of the op-count model: t_ideal = F32 / 157.3e12 +
    F64 / 78.6e12 (+ matrix flops / their peak); frac = t_ideal / t_kernel;
    achieved in FP32-equivalent TFLOP/s (each term weighted by 157.3e12 over
    its own peak)."""
    f32 = F32_PER_PATH_DATE * path_dates if fp32 else 0.0
    f64 = F64_PER_PATH * paths + (0.0 if fp32 else F64_PER_PATH_DATE_PLAIN * path_dates)
    t_ideal = f32 / PEAK_F32 + f64 / PEAK_F64 + mfma_flops / mfma_peak
    t_kernel = kernel_ms * 1e-3
    out = {"bound": "alu", "achieved": t_ideal * PEAK_F32 / t_kernel / 1e12, "peak": PEAK_F32 / 1e12,
           "unit": "TFLOP/s", "frac": t_ideal / t_kernel, "traffic": traffic,
           "model": "FP32-equivalent flops: %s + %.0f FP64/path%s" % (
               "%.0f FP32/path-date" % F32_PER_PATH_DATE if fp32 else
               "%.0f FP64/path-date" % F64_PER_PATH_DATE_PLAIN, F64_PER_PATH,
               " + %.3g matrix flops at %.4g TFLOP/s" % (mfma_flops, mfma_peak / 1e12) if mfma_flops else ""),
           "ideal_ms": t_ideal * 1e3, "kernel": kernel, "kernel_ms": kernel_ms}
    if call_ms is not None:
        out["call_ms"] = call_ms
    if counters is not None:
        # what the kernel executes (counters), beside the algorithmic model
        # above: FLOP/s it issues and the share of the SIMDs' VALU issue
        # slots (a wave64 VALU instruction holds a SIMD for 4 cycles) it fills
        f32c = counters["fp32_flops_per_path_date"] * path_dates
        f64c = counters["fp64_flops_per_path"] * paths
        waves = counters["valu_per_path_date"] * path_dates / 64.0
        # (valu_issue_frac counts 4 cycles per wave64 instruction; it exceeds 1
        # where transcendental and other instructions overlap in the SIMD)
        out["measured"] = {"source": "rocprofv3 counters of these kernel sources (profiles/)",
                           "fp32_tflops": f32c / t_kernel / 1e12, "fp64_tflops": f64c / t_kernel / 1e12,
                           "valu_lane_instructions_per_path_date": counters["valu_per_path_date"],
                           "valu_issue_frac": waves * 4.0 / (t_kernel * CLOCK_HZ * SIMDS)}
    return out


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


def host_threads() -> int:
    """Threads for the oracle: the host share given to this process
    (OMP_NUM_THREADS when set), at most 16."""
    try:
        n = int(os.environ.get("OMP_NUM_THREADS", "0"))
    except ValueError:
        n = 0
    if n <= 0:
        n = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else (os.cpu_count() or 1)
    return max(1, min(n, 16))


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=10)
    p.add_argument("--warmup", type=int, default=2)
    p.add_argument("--workload", choices=["portfolio", "three_products"], default="portfolio",
                   help="headline workload: the 4096-option uneven portfolio (default) or the "
                        "18-option three-product grid at d = 64")
    p.add_argument("--precision", choices=["fp32", "fp64"], default="fp32")
    p.add_argument("--no-extras", action="store_true", help="headline only: no extra legs, no CPU baseline")
    p.add_argument("--no-serve", action="store_true", help="skip the serving legs")
    p.add_argument("--pca-only", action="store_true",
                   help="run only the principal-component leg (one timed call per GEMM) and print it")
    p.add_argument("--serve-sweep", action="store_true",
                   help="run only the serving sweep (saturation rate, then arrival rates 0.25, 0.5, 0.8 "
                        "times it, FP32-mixed and plain FP64 servers) and print it")
    p.add_argument("--serve-burst", action="store_true",
                   help="run only the serving sweep's saturation burst (24 requests at once) and print its time "
                        "and the server's counts")
    p.add_argument("--serve-requests", type=int, default=300, help="requests per arrival rate in --serve-sweep")
    p.add_argument("--serve-rates", type=str, default="0.25,0.5,0.8",
                   help="arrival rates of --serve-sweep as fractions of the saturation rate")
    p.add_argument("--serve-sat", type=float, default=0.0,
                   help="saturation rate (requests/s) measured before: --serve-sweep skips its burst")
    p.add_argument("--serve-fp64-cap", type=float, default=120.0,
                   help="seconds after the first arrival at which the plain FP64 server stops taking requests")
    p.add_argument("--copy-mib", type=int, default=0,
                   help="after the timed loop, run one plain device copy of this many MiB "
                        "(reference kernel for HBM byte counters)")
    return p.parse_args()


def headline_workload(workloads, name):
    if name == "portfolio":
        opts = workloads.portfolio(4096)
        return opts, 16, ("uneven portfolio: 4096 options in one persistent launch, type uniform over "
                          "{arith Asian, binary Asian, lookback} calls, d ~ U{4..365}, K ~ U[80,120], "
                          "sigma ~ U[0.1,0.5], T ~ U[0.25,2], r ~ U[0,0.08], 2^k points k ~ U{14..20}, "
                          "16 shifts, Brownian bridge")
    opts = workloads.three_products_grid(d=64, n_points=1 << 20)
    return opts, 32, ("three products (arith Asian, binary Asian, lookback) x K{90,100,110} x "
                      "sigma{0.1,0.3}, d=64, Brownian bridge, 2^20 Sobol points x 32 shifts")


def timed_calls(q, torch, opts, L, path, prec, steps, warmup, out, stream, **kw):
    """W untimed calls, then K calls bracketed by synchronisation on both
    sides: (wall seconds of the K calls, mean per-call ms from torch events
    on the launch stream, mean fused-kernel ms from the library's HIP events
    on the same stream)."""
    for _ in range(warmup):
        q.greeks(opts, L, path, prec, device_outputs=True, out=out, stream=stream, **kw)
    torch.cuda.synchronize()
    stream.synchronize()
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(steps)]
    q.kernel_timer(q.TIMER_START)
    t0 = time.perf_counter()
    for s, e in evs:
        s.record(stream)
        q.greeks(opts, L, path, prec, device_outputs=True, out=out, stream=stream, **kw)
        e.record(stream)
    stream.synchronize()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    k_ms, k_n = q.kernel_timer(q.TIMER_STOP)
    ev_ms = float(np.mean([s.elapsed_time(e) for s, e in evs]))
    return wall, ev_ms, k_ms / max(k_n, 1)


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
    if a.serve_burst:
        sec, stats = serve_burst(q, workloads)
        print(json.dumps({"serving_burst": {"requests": 24, "seconds": sec,
                                            "saturation_requests_per_s": 24 / sec, "server": stats}}), flush=True)
        return
    if a.serve_sweep:
        print(json.dumps({"serving_sweep": serve_sweep(q, workloads, a.serve_requests,
                                                       [float(x) for x in a.serve_rates.split(",")],
                                                       fp64_cap_s=a.serve_fp64_cap, sat=a.serve_sat)}),
              flush=True)
        return
    opts, L, desc = headline_workload(workloads, a.workload)
    n_paths = workloads.total_paths(opts, L)
    n_pd = workloads.total_path_dates(opts, L)
    prec = q.FP32_MIXED if a.precision == "fp32" else q.FP64
    out = (torch.empty((len(opts), 4), dtype=torch.float64, device=dev),
           torch.empty((len(opts), 4), dtype=torch.float64, device=dev))
    stream = torch.cuda.Stream()
    print("headline: %s, %d steps after %d warmup" % (a.workload, a.steps, a.warmup), file=sys.stderr, flush=True)
    wall, ev_ms, kern_ms = timed_calls(q, torch, opts, L, q.PATH_BB, prec, a.steps, a.warmup, out, stream)
    if a.copy_mib > 0:
        src = torch.ones(a.copy_mib << 18, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    print("timed %d steps: %.3f s wall, %.3f ms/call, %.3f ms/kernel (events)" % (a.steps, wall, ev_ms, kern_ms),
          file=sys.stderr, flush=True)
    value = n_paths * a.steps / wall
    fp32 = prec == q.FP32_MIXED
    rl = roofline(n_paths, n_pd, kern_ms, fp32=fp32, traffic=traffic_of(a.workload) if fp32 else None,
                  counters=counters_of(a.workload) if fp32 else None,
                  call_ms=ev_ms)

    res = {"metric": "Greek-paths/sec (delta+vega+gamma) at fixed RMSE vs FP64; p99 request latency",
           "value": value, "unit": "Greek-paths/s", "n_gpus": 1, "steps": a.steps, "warmup": a.warmup,
           "ms_per_step": wall / a.steps * 1e3, "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": "f32+f64" if fp32 else "f64",
           "data": "synthetic (Black-Scholes option parameters, seeded)",
           "config": {"workload": desc, "options": len(opts), "shifts": L, "greek_paths_per_step": n_paths,
                      "path_dates_per_step": n_pd, "precision": a.precision},
           "roofline": rl}
    if a.no_extras:
        print(json.dumps(res), flush=True)
        return
    # the oracle on the host cores: a bounded sample of the headline workload
    res["cpu_baseline"] = cpu_baseline(workloads, opts, L, a.workload, n_pd)
    res["paper_context"] = PAPER_CONTEXT
    if a.workload == "portfolio":
        # plain FP64 on the same portfolio (one persistent launch)
        w64, ev64, k64 = timed_calls(q, torch, opts, L, q.PATH_BB, q.FP64, 1, 1, out, stream)
        res["fp64"] = {"value": n_paths / w64, "ms_per_step": w64 * 1e3, "kernel_ms": k64,
                       "roofline": roofline(n_paths, n_pd, k64, fp32=False)}
        res["three_products"] = three_products_leg(q, workloads, torch)
    else:
        res["three_products"] = None
    res["owen"] = owen_leg(q, workloads, torch)
    res["geometric"] = geometric_leg(q, workloads, torch, q.FP32_MIXED)
    res["more_products"] = more_products_leg(q, workloads, torch, q.FP32_MIXED)
    res["small_call"] = small_call_leg(q, workloads, torch)
    res["pca"] = pca_leg(q, workloads, torch)
    res["portfolio_fp64_one_option_per_launch"] = per_option_fp64_leg(q, workloads, opts, L)
    if not a.no_serve:
        # the configured stream (1..512 options, d in [4, 365], targets 1e-4 / 1e-6, which the
        # point cap of 2^22 per option decides): a short stream at a rate the GPU sustains
        res["serving"] = serving_leg(q, workloads, n_requests=12, rate=0.3, max_opts=512, d_range=(4, 365),
                                     targets=(1e-4, 1e-6), fp64_requests=3, fp64_max_opts=8)
        # a dense stream of small requests (1..32 options, d in [4, 64], targets 1e-3 / 1e-4)
        res["serving_small_requests"] = serving_leg(q, workloads)
    print(json.dumps(res), flush=True)


def cpu_baseline(workloads, opts, L, workload, n_pd_full):
    """The oracle (plain FP64 C, OpenMP over option x shift) on the host
    cores, on a bounded sample of the headline workload: every 64th option
    of the portfolio at its first 2^14 points and all shifts (or, for the
    three-product grid, all 18 options at 2^19 points x 8 shifts), plus one
    host thread on a smaller sample.  A reported baseline, not a target."""
    import oracle
    threads = host_threads()
    if workload == "portfolio":
        sample = [dict(o, n_points=min(o["n_points"], 1 << 14)) for o in opts[::64]]
        Ls, what = L, "every 64th option of the portfolio (%d), first 2^14 points, %d shifts" % (len(opts[::64]), L)
        sample1 = [dict(o, n_points=1 << 12) for o in opts[::256]]
        L1, what1 = 2, "every 256th option (%d), first 2^12 points, 2 shifts" % len(opts[::256])
    else:
        sample = [dict(o, n_points=1 << 19) for o in opts]
        Ls, what = 8, "the 18 options at d=64, 2^19 points x 8 shifts"
        sample1 = [dict(o, n_points=1 << 14) for o in opts]
        L1, what1 = 2, "the 18 options at d=64, 2^14 points x 2 shifts"
    t0 = time.perf_counter()
    _, _, _, used = oracle.options(sample, Ls, oracle.PATH_BB, n_threads=threads)
    tc = time.perf_counter() - t0
    pd_s = workloads.total_path_dates(sample, Ls)
    res = {"value": workloads.total_paths(sample, Ls) / tc, "unit": "Greek-paths/s", "cores": used,
           "kind": "oracle", "sample": "%s (%.1f s)" % (what, tc), "cpu_model": cpu_model(),
           "path_dates_per_s": pd_s / tc,
           "extrapolated_full_workload_s": tc * n_pd_full / pd_s}
    t0 = time.perf_counter()
    oracle.options(sample1, L1, oracle.PATH_BB, n_threads=1)
    t1c = time.perf_counter() - t0
    res["single_thread"] = {"value": workloads.total_paths(sample1, L1) / t1c,
                            "path_dates_per_s": workloads.total_path_dates(sample1, L1) / t1c,
                            "sample": "%s (%.1f s)" % (what1, t1c)}
    return res


def three_products_leg(q, workloads, torch, steps=5, warmup=1):
    """The 18-option three-product grid at d = 64 (2^20 points x 32 shifts,
    bridge): FP32-mixed with its roofline, plain FP64, their differences."""
    dev = torch.device("cuda", 0)
    opts = workloads.three_products_grid(d=64, n_points=1 << 20)
    L = 32
    paths = workloads.total_paths(opts, L)
    pd = workloads.total_path_dates(opts, L)
    out = (torch.empty((len(opts), 4), dtype=torch.float64, device=dev),
           torch.empty((len(opts), 4), dtype=torch.float64, device=dev))
    stream = torch.cuda.Stream()
    wall, ev_ms, k_ms = timed_calls(q, torch, opts, L, q.PATH_BB, q.FP32_MIXED, steps, warmup, out, stream)
    g = out[0].cpu().numpy()
    e = out[1].cpu().numpy()
    res = {"value": paths * steps / wall, "unit": "Greek-paths/s", "ms_per_step": wall / steps * 1e3,
           "greek_paths": paths, "path_dates": pd,
           "roofline": roofline(paths, pd, k_ms, traffic=traffic_of("three_products"), call_ms=ev_ms,
                                counters=counters_of("three_products"))}
    w64, ev64, k64 = timed_calls(q, torch, opts, L, q.PATH_BB, q.FP64, 2, 1, out, stream)
    g64 = out[0].cpu().numpy()
    res["fp64"] = {"value": paths * 2 / w64, "ms_per_step": w64 / 2 * 1e3, "kernel_ms": k64}
    rel = np.abs(g - g64) / np.maximum(np.abs(g64), 1e-300)
    res["fp32_vs_fp64_max_rel_diff"] = {k: float(rel[:, i].max()) for i, k in enumerate(q.OUTPUTS)}
    res["stderr_max_rel"] = {k: float((e[:, i] / np.maximum(np.abs(g64[:, i]), 1e-300)).max())
                             for i, k in enumerate(q.OUTPUTS)}
    res["stderr_min_rel"] = {k: float((e[:, i] / np.maximum(np.abs(g64[:, i]), 1e-300)).min())
                             for i, k in enumerate(q.OUTPUTS)}
    # the same grid with principal-component paths (matrix cores, FP32 MFMA):
    # rate, and each Greek's variance against the bridge at the same points
    wp, evp, kp = timed_calls(q, torch, opts, L, q.PATH_PCA, q.FP32_MIXED, steps, warmup, out, stream)
    ep = out[1].cpu().numpy()
    vr = (e / np.maximum(ep, 1e-300)) ** 2
    res["pca_fp32_mfma"] = {"value": paths * steps / wp, "unit": "Greek-paths/s", "ms_per_step": wp / steps * 1e3,
                            "kernel_ms": kp,
                            "variance_ratio_bridge_over_pca": {k: [float(np.min(vr[:, i])), float(np.median(vr[:, i])),
                                                                   float(np.max(vr[:, i]))]
                                                               for i, k in enumerate(q.OUTPUTS)}}
    return res


def owen_leg(q, workloads, torch, steps=3):
    """The three-product grid randomised by nested scrambling instead of the
    digital shift: rate, kernel time, standard errors against the shift."""
    dev = torch.device("cuda", 0)
    opts = workloads.three_products_grid(d=64, n_points=1 << 20)
    L = 32
    out = (torch.empty((len(opts), 4), dtype=torch.float64, device=dev),
           torch.empty((len(opts), 4), dtype=torch.float64, device=dev))
    stream = torch.cuda.Stream()
    timed_calls(q, torch, opts, L, q.PATH_BB, q.FP32_MIXED, 1, 0, out, stream)
    e = out[1].cpu().numpy()
    wall, ev_ms, k_ms = timed_calls(q, torch, opts, L, q.PATH_BB, q.FP32_MIXED, steps, 1, out, stream, owen=True)
    e_owen = out[1].cpu().numpy()
    return {"value": workloads.total_paths(opts, L) * steps / wall, "unit": "Greek-paths/s", "kernel_ms": k_ms,
            "stderr_ratio_owen_over_shift": {k: float(np.median(e_owen[:, i] / e[:, i]))
                                             for i, k in enumerate(q.OUTPUTS)}}


def per_option_fp64_leg(q, workloads, opts, L):
    """The plain path beside the persistent launch: FP64, one option per
    launch, on every 128th option of the portfolio."""
    sample = opts[::128]
    t1 = time.perf_counter()
    for o in sample:
        q.greeks([o], L, q.PATH_BB, q.FP64)
    t64 = time.perf_counter() - t1
    p64 = workloads.total_paths(sample, L)
    return {"value": p64 / t64, "unit": "Greek-paths/s", "sample": "every 128th option (%d)" % len(sample),
            "seconds": t64}


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
    cores): arithmetic and binary Asian on the same paths (one seed), 2^22
    points x 16 shifts, FP32-mixed, GEMM in FP32 MFMA and in split BF16x3;
    kernel time from the library's HIP events.  The two options share one
    product and one epilogue per tile, as the configuration states (one
    256 x 256 by 256 x 2^22 GEMM per shift, both payoffs' Greeks in its
    epilogue), so the whole-kernel roofline counts: the product's 2 n^2
    flops per point and shift once, at the FP32 matrix peak (BF16x3: three
    BF16 products at the BF16 matrix peak), 36 FP32 flops per path-date of
    the one path set, and 200 FP64 flops per path of each option."""
    opts = workloads.pca_pair(d=256, n_points=1 << 22)
    L = 16
    n = 255
    paths = workloads.total_paths(opts, L)          # Greek-paths: both options
    pd = workloads.total_path_dates(opts[:1], L)    # one shared path set
    s = torch.cuda.Stream()
    out = (torch.empty((2, 4), dtype=torch.float64, device="cuda"),
           torch.empty((2, 4), dtype=torch.float64, device="cuda"))
    res = {"workload": "arith + binary Asian, d=256, PCA, 2^22 points x 16 shifts, FP32-mixed",
           "greek_paths": paths}
    gflop = 2.0 * n * n * workloads.total_paths(opts[:1], L)   # one product per point and shift
    for name, gemm, mf, peak in (("fp32_mfma", q.GEMM_FP32, gflop, PEAK_MFMA_F32),
                                 ("bf16x3_mfma", q.GEMM_BF16X3, 3 * gflop, PEAK_MFMA_BF16)):
        wall, ev_ms, k_ms = timed_calls(q, torch, opts, L, q.PATH_PCA, q.FP32_MIXED, steps, 1, out, s,
                                        pca_gemm=gemm)
        res[name] = {"value": paths * steps / wall, "unit": "Greek-paths/s", "kernel_ms": k_ms,
                     "roofline": roofline(paths, pd, k_ms, mfma_flops=mf, mfma_peak=peak,
                                          kernel="qcpw::pca_f32_kernel"),
                     "gemm_only_frac": mf / peak / (k_ms * 1e-3)}
        if gemm == q.GEMM_FP32:
            se_x1 = out[1].cpu().numpy().copy()
    # the same points conditioned on the first principal component of all d
    # dates (FP64 Newton root-find per path): time, and the variance ratio of
    # each Greek against conditioning on the first date's normal
    wall, ev_ms, k_ms = timed_calls(q, torch, opts, L, q.PATH_PCA_FULL, q.FP32_MIXED, steps, 1, out, s)
    se_full = out[1].cpu().numpy()
    res["pca_full_fp32_mfma"] = {
        "value": paths * steps / wall, "unit": "Greek-paths/s", "kernel_ms": k_ms,
        "variance_ratio_vs_first_date": {k: [float((se_x1[i, j] / se_full[i, j]) ** 2) for i in range(2)]
                                         for j, k in enumerate(q.OUTPUTS)}}
    return res


class Progress:
    """A line on stderr at most every `every` seconds while work completes."""

    def __init__(self, what, total, every=20.0):
        self.what, self.total, self.every = what, total, every
        self.t_last = time.perf_counter()

    def step(self, k):
        now = time.perf_counter()
        if now - self.t_last >= self.every or k == self.total:
            self.t_last = now
            print("%s: %d / %d" % (self.what, k, self.total), file=sys.stderr, flush=True)


def run_stream(q, srv, stream, L=16, what="served"):
    """Submit a request stream at its arrival times into server srv, poll for
    results from a second thread; returns (latency seconds per request,
    points reached per request, wall seconds)."""
    import threading
    done = {}
    pending = []
    lock = threading.Lock()
    finished = threading.Event()
    prog = Progress(what, len(stream))

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
                    prog.step(len(done))
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
        item = (srv.submit(r["options"], L, r["target_stderr"]), t0 + r["t_arrival"], r)
        ids.append(item)
        with lock:
            pending.append(item)
    finished.set()
    th.join()
    wall = time.perf_counter() - t0
    lat = np.array([done[rid][0] for rid, _, _ in ids])
    pts = [done[rid][1] for rid, _, _ in ids]
    return lat, pts, wall


def plain_fp64_stream(q, stream, pts, L=16, cap_s=120.0):
    """The plain method under the same arrivals: one worker takes requests in
    arrival order and prices each option alone (FP64, one option per launch)
    at the points the mixed-precision server reached for that request (so
    both sides have the same RMSE).  Stops taking requests cap_s seconds
    after the first arrival; a request not finished by then counts with its
    waiting time so far (a lower bound on its latency)."""
    lat, finished, paths = [], 0, 0
    prog = Progress("fp64 one option per launch", len(stream))
    t0 = time.perf_counter()
    for r, p in zip(stream, pts):
        now = time.perf_counter() - t0
        if now > cap_s:
            break
        if r["t_arrival"] > now:
            time.sleep(r["t_arrival"] - now)
        for o in r["options"]:
            q.greeks([dict(o, n_points=p)], L, q.PATH_BB, q.FP64)
            prog.step(finished)
        lat.append(time.perf_counter() - t0 - r["t_arrival"])
        finished += 1
        paths += len(r["options"]) * p * L
    busy = time.perf_counter() - t0
    t_end = time.perf_counter() - t0
    censored = [t_end - r["t_arrival"] for r in stream[finished:] if r["t_arrival"] < t_end]
    all_lat = np.array(lat + censored) * 1e3
    return {"requests_finished": finished, "requests_arrived_unfinished": len(censored),
            "value": paths / busy if busy > 0 else 0.0, "unit": "Greek-paths/s",
            "p50_ms": float(np.percentile(all_lat, 50)) if len(all_lat) else None,
            "p99_ms": float(np.percentile(all_lat, 99)) if len(all_lat) else None,
            "latency_is_lower_bound": bool(censored), "cap_s": cap_s}


def serve_burst(q, workloads, n_burst=24, max_opts=512, d_range=(4, 365), targets=(1e-4, 1e-6), L=16):
    """n_burst requests of the serving stream submitted at once to a
    FP32-mixed server: seconds until the last result, and the server's
    counts."""
    burst = workloads.request_stream(n_burst, 1e9, seed=5150, max_opts=max_opts, d_range=d_range,
                                     targets=targets)
    for r in burst:
        r["t_arrival"] = 0.0
    with q.Server(hbm_budget_bytes=8 << 30, precision=q.FP32_MIXED) as srv:
        lat, pts, wall = run_stream(q, srv, burst, L, what="burst")
        stats = srv.stats()
    return float(lat.max()), stats


def serve_sweep(q, workloads, n_requests, fracs, max_opts=512, d_range=(4, 365), targets=(1e-4, 1e-6),
                n_burst=24, L=16, fp64_cap_s=120.0, sat=0.0):
    """The configured serving stream (Poisson arrivals of 1..max_opts-option
    portfolios drawn as the uneven portfolio, target standard error 1e-4 or
    1e-6 relative): the saturation rate of the mixed-precision server (a
    burst of n_burst requests submitted at once, over the time to finish
    them), then n_requests requests at each rate frac x saturation with
    p50/p99 latency and throughput; beside each, the plain FP64
    one-option-per-launch method under the same arrivals.  sat > 0: the
    saturation rate measured before (the burst is skipped)."""
    if sat <= 0.0:
        sec, _ = serve_burst(q, workloads, n_burst, max_opts, d_range, targets, L)
        sat = n_burst / sec
        print("serve sweep: saturation %.3f requests/s" % sat, file=sys.stderr, flush=True)
    res = {"stream": {"options_per_request": [1, max_opts], "d_range": list(d_range),
                      "target_stderr": list(targets), "shifts": L},
           "saturation_requests_per_s": sat, "rates": []}
    for frac in fracs:
        rate = frac * sat
        stream = workloads.request_stream(n_requests, rate, seed=22091 + int(frac * 1000), max_opts=max_opts,
                                          d_range=d_range, targets=targets)
        with q.Server(hbm_budget_bytes=8 << 30, precision=q.FP32_MIXED) as srv:
            lat, pts, wall = run_stream(q, srv, stream, L)
            stats = srv.stats()
        paths = sum(len(r["options"]) * p * L for r, p in zip(stream, pts))
        lat_ms = lat * 1e3
        entry = {"fraction_of_saturation": frac, "rate_per_s": rate, "requests": n_requests,
                 "p50_ms": float(np.percentile(lat_ms, 50)), "p99_ms": float(np.percentile(lat_ms, 99)),
                 "max_ms": float(lat_ms.max()), "value": paths / wall, "unit": "Greek-paths/s",
                 "launches": stats["launches"], "mean_points": float(np.mean(pts))}
        print("serve sweep: %.2f x saturation: p50 %.1f ms, p99 %.1f ms" % (frac, entry["p50_ms"], entry["p99_ms"]),
              file=sys.stderr, flush=True)
        entry["fp64_one_option_per_launch"] = plain_fp64_stream(q, stream, pts, L, cap_s=fp64_cap_s)
        res["rates"].append(entry)
        print(json.dumps({"serving_rate": entry}), flush=True)
    return res


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
