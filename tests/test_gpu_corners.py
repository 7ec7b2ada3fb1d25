"""GPU parity at the corners: the FP32-mixed bound where the breakpoint
amplifies path rounding most, the principal-component workload at its full
shape against the oracle, served requests against the oracle, and the
spread of single replications (the sigma of Sec. 5)."""
import concurrent.futures as cf
import sys

import numpy as np
import pytest

import oracle
import paper_2209_11337_amd as q
import workloads

pytestmark = pytest.mark.gpu

TOL64 = 1e-10
FP32_TOL = np.array([2e-5, 2e-5, 1e-4, 2e-4])
BF16X3_TOL = np.array([2e-4, 2e-4, 1e-3, 2e-3])


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def scaled_err(got, ref, scale):
    """|got - ref| / max(|ref|, scale), the summand-scale reading of "1e-10
    relative".  A zero scale means every summand was zero (a Gaussian density
    that underflows far from the money): then the two must be equal, so 0/0
    counts as 0 and any difference as infinite."""
    diff = np.abs(got - ref)
    den = np.maximum(np.abs(ref), scale)
    with np.errstate(divide="ignore", invalid="ignore"):
        return np.where(diff == 0, 0.0, diff / den)


def oracle_range(o, l, path, N, parts=16):
    """Replication l of option o over points 0..N-1, from `parts` equal point
    ranges run side by side on the host cores (each a plain oracle call)."""
    step = N // parts
    with cf.ThreadPoolExecutor(parts) as ex:
        means = list(ex.map(lambda i: oracle.replication(o, l, path, k0=i * step, N=step), range(parts)))
    return np.mean(np.array(means), axis=0)


def scale_of(o, path, N=512):
    return oracle.option(o["type"], o["d"], o["S0"], o["K"], o["r"], o["sigma"], o["T"], o["seed"], N, 1,
                         path)["abs_mean"]


# ------------------------------------------------------------------------
# FP32 bound at its worst corner: short maturity, low volatility, many
# dates.  s1 = sigma sqrt(T/d) = 0.0026, so the breakpoint multiplies the
# relative rounding of the path statistic by 1/s1 ~ 380.
# ------------------------------------------------------------------------
CORNER = dict(S0=100.0, r=0.05, sigma=0.1, T=0.25, d=365)
# Relative FP32 rounding of the path statistic X (a few ulps of the sum of d
# exponentials), which the breakpoint turns into delta psi = EPS_PATH / s1.
EPS_PATH = 2e-7


def fp32_bound(o, k):
    """FP32-mixed bound for Greek k of call o, relative to the summand scale.
    A summand moves by |d ln F / d psi| delta psi ~ |psi| EPS_PATH / s1 when
    the FP32 path shifts the breakpoint: at the money that stays inside
    FP32_TOL, far out of the money (psi >> 1 at the forward, prices below
    1e-60 here) the relative error grows with psi while the absolute error
    is negligible."""
    s1 = o["sigma"] * np.sqrt(o["T"] / o["d"])
    psi_f = max(0.0, (np.log(o["K"] / o["S0"]) - o["r"] * o["T"]) / s1)
    return FP32_TOL[k] + EPS_PATH * psi_f / s1


@pytest.mark.parametrize("K", [70.0, 80.0, 97.0, 100.0, 103.0, 120.0, 130.0])
def test_fp32_corner_short_low_vol_many_dates(K):
    opts = [dict(CORNER, type=t, K=K, seed=0xC0 + t + int(K), n_points=4096 + 77)
            for t in (q.ARITH_ASIAN, q.BINARY_ASIAN, q.LOOKBACK)]
    say("fp32 corner", K)
    g, e, ps = q.greeks(opts, 2, q.PATH_BB, q.FP32_MIXED, per_shift=True)
    ref = [oracle.option(o["type"], o["d"], o["S0"], o["K"], o["r"], o["sigma"], o["T"], o["seed"],
                         o["n_points"], 2, oracle.PATH_BB) for o in opts]
    Cl = np.array([r["C_l"] for r in ref])
    am = np.array([r["abs_mean"] for r in ref])
    err = scaled_err(ps, Cl, am[:, None, :])
    say("corner K=%g scaled error per type:" % K, err.max(axis=1))
    for i, o in enumerate(opts):
        for k in range(4):
            assert err[i, :, k].max() <= fp32_bound(o, k), (K, i, k, err[i, :, k].max(), fp32_bound(o, k))


def test_fp32_lookback_near_ties():
    """A lookback whose dates sit a hair apart (sigma = 0.005, d = 365): the
    largest and second largest of the path are often within a few FP32 ulps,
    so the FP32 argmax may pick the neighbour.  The vega term moves by one
    path increment then, which the bound covers."""
    opts = [dict(CORNER, type=q.LOOKBACK, sigma=0.005, K=K, seed=0x7E + i, n_points=8192 + 13)
            for i, K in enumerate((99.0, 100.5, 102.0))]
    say("fp32 near ties")
    g, e, ps = q.greeks(opts, 2, q.PATH_BB, q.FP32_MIXED, per_shift=True)
    ref = [oracle.option(o["type"], o["d"], o["S0"], o["K"], o["r"], o["sigma"], o["T"], o["seed"],
                         o["n_points"], 2, oracle.PATH_BB) for o in opts]
    Cl = np.array([r["C_l"] for r in ref])
    am = np.array([r["abs_mean"] for r in ref])
    err = scaled_err(ps, Cl, am[:, None, :])
    say("near-tie scaled error:", err.max(axis=(0, 1)))
    for i, o in enumerate(opts):
        for k in range(4):
            assert err[i, :, k].max() <= fp32_bound(o, k), (i, k, err[i, :, k].max(), fp32_bound(o, k))


# ------------------------------------------------------------------------
# principal components at the full shape: d = 256 (a 256 x 256 factor), 16
# replications of 2^18 points, in the benchmark's launch configuration;
# replication 5 of each option is recomputed by the oracle over all 2^18
# points.
# ------------------------------------------------------------------------
@pytest.mark.parametrize("gemm,tol", [(q.GEMM_FP32, FP32_TOL), (q.GEMM_BF16X3, BF16X3_TOL)])
def test_pca_d256_replication_against_oracle(gemm, tol):
    N, L, l = 1 << 18, 16, 5
    opts = workloads.pca_pair(d=256, n_points=N)
    say("pca d256 oracle replication", gemm)
    g, e, ps = q.greeks(opts, L, q.PATH_PCA, q.FP32_MIXED, pca_gemm=gemm, per_shift=True)
    for i, o in enumerate(opts):
        ref = oracle_range(o, l, oracle.PATH_PCA, N)
        sc = scale_of(o, oracle.PATH_PCA)
        err = scaled_err(ps[i, l], ref, sc)
        say("pca d256 option %d scaled error" % i, err)
        assert (err <= tol).all(), err
    se = ps.std(axis=1, ddof=1) / np.sqrt(L)
    assert np.allclose(se, e, rtol=1e-9, atol=1e-300)


# ------------------------------------------------------------------------
# served requests against the oracle at the points they reached
# ------------------------------------------------------------------------
@pytest.mark.parametrize("prec,tol", [(q.FP64, None), (q.FP32_MIXED, FP32_TOL)])
def test_served_request_matches_oracle(prec, tol):
    opts = workloads.portfolio(3, seed=4242, d_range=(8, 120), log2_points=(14, 14))
    L = 4
    say("served vs oracle", prec)
    with q.Server(hbm_budget_bytes=1 << 28, precision=prec) as srv:
        rid = srv.submit(opts, L, target_stderr=1e-1)
        g, e, pts = srv.wait(rid, len(opts))
    assert pts == 1 << 14   # a loose target stops after the first round
    for i, o in enumerate(opts):
        ref = oracle.option(o["type"], o["d"], o["S0"], o["K"], o["r"], o["sigma"], o["T"], o["seed"], pts, L,
                            oracle.PATH_BB)
        err = scaled_err(g[i], ref["mean"], ref["abs_mean"])
        say("served option %d scaled error" % i, err)
        assert (err <= (TOL64 if tol is None else tol)).all(), err
        if prec == q.FP64:
            assert np.allclose(e[i], ref["stderr"], rtol=1e-6, atol=1e-10 * ref["abs_mean"].max())


# ------------------------------------------------------------------------
# the spread of single replications (Sec. 5's sigma)
# ------------------------------------------------------------------------
def test_paper_sigma_is_spread_of_replications():
    opts = workloads.three_products_grid(d=16, n_points=4096)[::3]
    L = 8
    g, e, ps, sg = q.greeks(opts, L, q.PATH_BB, q.FP32_MIXED, per_shift=True, paper_sigma=True)
    spread = np.sqrt(((ps - g[:, None, :]) ** 2).mean(axis=1))
    assert np.allclose(sg, spread, rtol=1e-9, atol=1e-300)
    assert np.allclose(sg, e * np.sqrt(L - 1), rtol=1e-12, atol=1e-300)
    import torch
    out = q.greeks(opts, L, q.PATH_BB, q.FP32_MIXED, device_outputs=True, paper_sigma=True)
    torch.cuda.synchronize()
    assert np.array_equal(out[2].cpu().numpy(), sg)
    _, _, sg1 = q.greeks(opts[:1], 1, q.PATH_BB, q.FP64, paper_sigma=True)
    assert np.all(np.isnan(sg1))
