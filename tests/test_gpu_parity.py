"""GPU parity: the HIP path through the C ABI against the FP64 oracle.

Sobol integers (with shifts) must be bit-exact.  FP64 Greeks must agree to
1e-10, measured against the scale of the summands: |g - o| <=
1e-10 * max(|o|, mean |F|), since some means (binary gamma, deep
in-the-money gammas) sit near zero while the per-path values do not.  The
FP32-mixed path is held to the bound stated in FP32_TOL below.
"""
import os
import sys

import numpy as np
import pytest

import oracle
import paper_2209_11337_amd as q
import workloads

pytestmark = pytest.mark.gpu

TOL64 = 1e-10
# FP32-mixed bound (relative to the summand scale, per output price, delta,
# vega, gamma); the derivation is in the design notes: FP32 rounding of the
# path enters psi amplified by 1/(sigma sqrt(t_1)).
FP32_TOL = np.array([2e-5, 2e-5, 1e-4, 2e-4])


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _oracle_one(o, L, path, rand=oracle.RAND_SHIFT):
    if o["type"] in (oracle.BASKET_ASIAN, oracle.BASKET_ASIAN_PUT):
        return oracle.basket_option(o["type"], o["d"], o["n_assets"], o["rho"], o["S0"], o["K"], o["r"],
                                    o["sigma"], o["T"], o["seed"], o["n_points"], L, rand)
    return oracle.option(o["type"], o["d"], o["S0"], o["K"], o["r"], o["sigma"], o["T"], o["seed"],
                         o["n_points"], L, path, rand)


def oracle_many(opts, L, path):
    out = [_oracle_one(o, L, path) for o in opts]
    return (np.array([r["mean"] for r in out]), np.array([r["stderr"] for r in out]),
            np.array([r["abs_mean"] for r in out]), np.array([r["C_l"] for r in out]))


def scaled_err(got, ref, scale):
    """|got - ref| / max(|ref|, scale); a zero scale means every summand was
    zero (a density that underflows far from the money), so the two must be
    equal: 0/0 counts as 0, any difference as infinite."""
    diff = np.abs(np.asarray(got) - np.asarray(ref))
    den = np.maximum(np.abs(ref), scale)
    with np.errstate(divide="ignore", invalid="ignore"):
        return np.where(diff == 0, 0.0, diff / den)


def assert_scaled(g, o, scale, tol, what=""):
    g, o, scale = np.asarray(g), np.asarray(o), np.asarray(scale)
    bound = tol * np.maximum(np.abs(o), scale)
    bad = np.abs(g - o) > bound
    assert not bad.any(), "%s: max scaled error %.3g at %s" % (
        what, (np.abs(g - o) / np.maximum(np.abs(o), scale)).max(), np.argwhere(bad)[:4].tolist())


# ------------------------------------------------------------------------
# Sobol points
# ------------------------------------------------------------------------
@pytest.mark.parametrize("n_dims,k0,count,shift", [(16, 0, 4096, 0), (65, 0, 3000, 3), (365, 1000, 700, 7),
                                                   (130, (1 << 20) - 50, 300, 31), (1024, 123457, 65, 2),
                                                   (3, (1 << 32) - 70, 70, 65535)])
def test_sobol_points_bit_exact(n_dims, k0, count, shift):
    say("sobol", n_dims, k0, count, shift)
    seed = 0x220911337 + n_dims
    got = q.sobol_points(seed, shift, n_dims, k0, count)
    ref = oracle.sobol_points(n_dims, k0, count)
    s = oracle.shifts(seed, shift + 1, n_dims)[shift].copy()
    s[0] = 0
    assert np.array_equal(got, ref ^ s[None, :])


# ------------------------------------------------------------------------
# FP64 parity
# ------------------------------------------------------------------------
def test_fp64_single_asian_bridge():
    """One arithmetic Asian call, d = 16, 2^12 points x 16 shifts, bridge."""
    opts = workloads.single_asian()
    say("single asian fp64")
    g, e, ps = q.greeks(opts, 16, q.PATH_BB, q.FP64, per_shift=True)
    m, se, am, Cl = oracle_many(opts, 16, oracle.PATH_BB)
    assert_scaled(g, m, am, TOL64, "mean")
    assert_scaled(ps, Cl, am[:, None, :], TOL64, "per shift")
    assert np.allclose(e, se, rtol=1e-6, atol=1e-10 * am.max())
    # the plain entry point is the same computation
    g2, e2 = q.greeks_plain(opts, 16, q.PATH_BB)
    assert np.array_equal(g, g2) and np.array_equal(e, e2)


@pytest.mark.parametrize("path", [q.PATH_BB, q.PATH_STANDARD])
@pytest.mark.parametrize("d", [2, 5, 64, 100])
def test_fp64_three_products_ragged(path, d):
    """All three products, several K and sigma, a point count spanning three
    work units with a ragged tail (2 * 8192 + 77)."""
    opts = workloads.three_products_grid(d=d, n_points=2 * 8192 + 77)[::5]
    say("fp64 ragged", path, d, len(opts))
    g, e, ps = q.greeks(opts, 3, path, q.FP64, per_shift=True)
    m, se, am, Cl = oracle_many(opts, 3, path)
    assert_scaled(g, m, am, TOL64, "mean")
    assert_scaled(ps, Cl, am[:, None, :], TOL64, "per shift")


def test_fp64_one_date_is_exact_black_scholes():
    from scipy.stats import norm
    S0, K, r, sig, T = 100.0, 95.0, 0.05, 0.25, 1.3
    opts = [dict(type=t, d=1, S0=S0, K=K, r=r, sigma=sig, T=T, seed=5, n_points=100) for t in range(3)]
    g, e = q.greeks(opts, 4, q.PATH_BB, q.FP64)
    d1 = (np.log(S0 / K) + (r + sig**2 / 2) * T) / (sig * np.sqrt(T))
    d2 = d1 - sig * np.sqrt(T)
    call = [S0 * norm.cdf(d1) - K * np.exp(-r * T) * norm.cdf(d2), norm.cdf(d1), S0 * norm.pdf(d1) * np.sqrt(T),
            norm.pdf(d1) / (S0 * sig * np.sqrt(T))]
    D = np.exp(-r * T)
    dig = [D * norm.cdf(d2), D * norm.pdf(d2) / (S0 * sig * np.sqrt(T)), -D * norm.pdf(d2) * d1 / sig,
           -D * norm.pdf(d2) * d1 / (S0**2 * sig**2 * T)]
    assert np.allclose(g[0], call, rtol=1e-13) and np.allclose(g[2], call, rtol=1e-13)
    assert np.allclose(g[1], dig, rtol=1e-13)
    assert np.all(e == 0)


def test_fp64_edge_counts_and_largest_d():
    opts = [dict(type=0, d=385, S0=100, K=100, r=0.03, sigma=0.3, T=2.0, seed=1, n_points=130),
            dict(type=2, d=385, S0=100, K=90, r=0.03, sigma=0.3, T=2.0, seed=2, n_points=64),
            dict(type=1, d=7, S0=100, K=100, r=0.03, sigma=0.3, T=2.0, seed=3, n_points=1),
            dict(type=0, d=3, S0=100, K=105, r=0.0, sigma=0.1, T=0.25, seed=4, n_points=63)]
    for path in (q.PATH_BB, q.PATH_STANDARD):
        say("edge", path)
        g, e, ps = q.greeks(opts, 2, path, q.FP64, per_shift=True)
        m, se, am, Cl = oracle_many(opts, 2, path)
        assert_scaled(ps, Cl, am[:, None, :], TOL64, "per shift")


@pytest.mark.parametrize("units", [1, 7, 9, 17])
def test_fp64_every_unit_once(units):
    # fewer, and not a multiple of, the work queues of the fused kernel: one
    # option of 256-point units, so the launch holds exactly `units` units
    o = dict(type=0, d=5, S0=100, K=100, r=0.03, sigma=0.3, T=1.0, seed=11 + units, n_points=256 * units)
    say("units", units)
    g, e, ps = q.greeks([o], 1, q.PATH_BB, q.FP64, per_shift=True)
    m, se, am, Cl = oracle_many([o], 1, q.PATH_BB)
    assert_scaled(ps, Cl, am[:, None, :], TOL64, "per shift")


def test_single_shift_gives_nan_stderr():
    g, e = q.greeks(workloads.single_asian(n_points=256), 1, q.PATH_BB, q.FP64)
    assert np.all(np.isnan(e)) and np.all(np.isfinite(g))


# ------------------------------------------------------------------------
# FP32-mixed bound
# ------------------------------------------------------------------------
@pytest.mark.parametrize("path", [q.PATH_BB, q.PATH_STANDARD])
def test_fp32_mixed_within_bound(path):
    opts = workloads.three_products_grid(d=64, n_points=8192 + 300)
    say("fp32 bound", path)
    g, e, ps = q.greeks(opts, 2, path, q.FP32_MIXED, per_shift=True)
    m, se, am, Cl = oracle_many(opts, 2, path)
    err = scaled_err(ps, Cl, am[:, None, :])
    say("fp32 scaled error per output (max over options, shifts):", err.max(axis=(0, 1)))
    for k in range(4):
        assert err[..., k].max() <= FP32_TOL[k], (k, err[..., k].max())


@pytest.mark.parametrize("d", [16, 32, 128, 256])
def test_fp32_bridge_across_d(d):
    # compile-time bridges (n = 15, 31, 127) and the plan walker (n = 255)
    opts = workloads.three_products_grid(d=d, n_points=4096 + 77)[::4]
    say("fp32 bridge", d)
    g, e, ps = q.greeks(opts, 2, q.PATH_BB, q.FP32_MIXED, per_shift=True)
    m, se, am, Cl = oracle_many(opts, 2, oracle.PATH_BB)
    err = scaled_err(ps, Cl, am[:, None, :])
    for k in range(4):
        assert err[..., k].max() <= FP32_TOL[k], (d, k, err[..., k].max())


def test_fp32_mixed_portfolio_within_bound():
    opts = workloads.portfolio(24, seed=99, log2_points=(10, 12))
    say("fp32 portfolio")
    g, e, ps = q.greeks(opts, 2, q.PATH_BB, q.FP32_MIXED, per_shift=True)
    m, se, am, Cl = oracle_many(opts, 2, oracle.PATH_BB)
    err = scaled_err(ps, Cl, am[:, None, :])
    say("portfolio fp32 scaled error:", err.max(axis=(0, 1)))
    for k in range(4):
        assert err[..., k].max() <= FP32_TOL[k], (k, err[..., k].max())


# ------------------------------------------------------------------------
# batching
# ------------------------------------------------------------------------
@pytest.mark.parametrize("typ", [q.ARITH_ASIAN, q.BINARY_ASIAN, q.LOOKBACK])
def test_same_bits_in_narrow_and_wide_launches(typ):
    """An option gives the same bits alone (a launch whose lane rows fit
    several workgroups per CU) and beside a d = 365 option (the 128-VGPR
    kernel instances): d = 16, 32, 64, 128 are walked by the compile-time
    bridges in one and by the split bridge in the other, d = 8 by the plan
    walker, d = 40 and 200 by the split bridge in both."""
    ds = (8, 16, 32, 40, 64, 128, 200)
    opts = [dict(type=typ, d=d, S0=100.0, K=95.0 + 2 * i, r=0.05, sigma=0.25, T=1.0,
                 seed=1000 + d, n_points=1 << 12) for i, d in enumerate(ds)]
    big = dict(type=q.ARITH_ASIAN, d=365, S0=100.0, K=100.0, r=0.05, sigma=0.2, T=1.0,
               seed=5, n_points=1 << 10)
    say("narrow/wide invariance", typ)
    g_mix, e_mix = q.greeks(opts + [big], 4, q.PATH_BB, q.FP32_MIXED)
    for i, o in enumerate(opts):
        g1, e1 = q.greeks([o], 4, q.PATH_BB, q.FP32_MIXED)
        assert np.array_equal(g1[0], g_mix[i]) and np.array_equal(e1[0], e_mix[i]), (o["d"], g1[0], g_mix[i])


def test_same_bits_in_a_split_launch():
    """A call whose longest options need the 128-VGPR instances and whose
    others hold most of the work runs as two launches (d = 8, walked by the
    plan walker with its stack, and d = 365 in one; d = 16, 64, 200, 250 in
    the 80-VGPR one at 768 threads): 6 options x 1024 units x 64
    replications, 262144 units and 59 % of the path-dates in the second
    launch.  Every option gives
    the bits it gives alone (where d = 8, 200 and 250 run the 80-VGPR
    instances, d = 365 the 128-VGPR ones)."""
    ds = (365, 16, 64, 8, 200, 250)
    L = 64
    opts = [dict(type=(q.ARITH_ASIAN, q.BINARY_ASIAN, q.LOOKBACK)[i % 3], d=d, S0=100.0, K=97.0 + 2 * i, r=0.04,
                 sigma=0.3, T=1.2, seed=7000 + d, n_points=1 << 22) for i, d in enumerate(ds)]
    say("split launch invariance")
    g_mix, e_mix = q.greeks(opts, L, q.PATH_BB, q.FP32_MIXED)
    for i, o in enumerate(opts):
        g1, e1 = q.greeks([o], L, q.PATH_BB, q.FP32_MIXED)
        assert np.array_equal(g1[0], g_mix[i]) and np.array_equal(e1[0], e_mix[i]), (o["d"], g1[0], g_mix[i])
    # and the FP32-mixed results stay those of the FP64 kernel within the FP32 bound
    g64, _ = q.greeks(opts, L, q.PATH_BB, q.FP64)
    scale = np.maximum(np.abs(g64), 1e-3 * np.abs(g64).max(axis=0))
    assert (np.abs(g_mix - g64) / scale).max() <= 1e-3


@pytest.mark.parametrize("prec", [q.FP64, q.FP32_MIXED])
def test_each_option_same_alone_and_in_a_mix(prec):
    mix = workloads.portfolio(40, seed=7, log2_points=(10, 14))
    pick = [3, 17, 31]
    say("batch invariance", prec)
    g_mix, e_mix = q.greeks(mix, 4, q.PATH_BB, prec, block_threads=512)
    for i in pick:
        g1, e1 = q.greeks([mix[i]], 4, q.PATH_BB, prec, block_threads=512)
        assert np.array_equal(g1[0], g_mix[i]) and np.array_equal(e1[0], e_mix[i])
    # work units belong to waves and depend on the option alone, so the
    # workgroup shape does not change a single bit
    for bd in (256, 640, 1024):
        g_other, e_other = q.greeks(mix, 4, q.PATH_BB, prec, block_threads=bd)
        assert np.array_equal(g_other, g_mix) and np.array_equal(e_other, e_mix)


def test_device_outputs_on_torch_stream():
    import torch
    opts = workloads.three_products_grid(d=16, n_points=4096)
    ref_g, ref_e = q.greeks(opts, 4, q.PATH_BB, q.FP32_MIXED)
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        out = q.greeks(opts, 4, q.PATH_BB, q.FP32_MIXED, device_outputs=True, stream=s)
    s.synchronize()
    assert np.array_equal(out[0].cpu().numpy(), ref_g)
    assert np.array_equal(out[1].cpu().numpy(), ref_e)


def test_kernel_timer_counts_eager_launches():
    import torch
    opts = workloads.three_products_grid(d=16, n_points=1 << 14)
    s = torch.cuda.Stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    q.kernel_timer(q.TIMER_START)
    e0.record(s)
    for _ in range(3):
        q.greeks(opts, 8, q.PATH_BB, q.FP32_MIXED, device_outputs=True, stream=s)
    e1.record(s)
    s.synchronize()
    ms, n = q.kernel_timer(q.TIMER_READ)
    assert n == 3 and 0.0 < ms <= e0.elapsed_time(e1) * 1.01 + 0.01
    q.greeks(opts, 8, q.PATH_BB, q.FP32_MIXED, device_outputs=True, stream=s, graph=True)   # not timed
    ms2, n2 = q.kernel_timer(q.TIMER_STOP)
    assert n2 == 3 and ms2 == ms
    q.greeks(opts, 8, q.PATH_BB, q.FP32_MIXED)
    assert q.kernel_timer(q.TIMER_READ)[1] == 3   # stopped


# ------------------------------------------------------------------------
# full size: the benchmark's workload, sampled
# ------------------------------------------------------------------------
@pytest.mark.parametrize("prec", [q.FP32_MIXED, q.FP64])
def test_full_size_three_products_sampled(prec):
    """18 options x 2^20 points x 32 shifts, d = 64 (the benchmark workload),
    in the launch configuration the benchmark times; two (option, shift)
    replication means are recomputed by the oracle over all 2^20 points."""
    opts = workloads.three_products_grid(d=64, n_points=1 << 20)
    say("full size", prec)
    g, e, ps = q.greeks(opts, 32, q.PATH_BB, prec, per_shift=True)
    assert np.all(np.isfinite(g)) and np.all(np.isfinite(e))
    for (i, l) in [(4, 31), (15, 0)]:
        ref = oracle.replication(opts[i], l, oracle.PATH_BB)
        o1 = oracle.option(opts[i]["type"], 64, opts[i]["S0"], opts[i]["K"], opts[i]["r"], opts[i]["sigma"],
                           opts[i]["T"], opts[i]["seed"], 4096, 1)
        scale = o1["abs_mean"]
        tol = TOL64 if prec == q.FP64 else FP32_TOL
        assert_scaled(ps[i, l], ref, scale, tol, "option %d shift %d" % (i, l))
    # replications are exchangeable: the spread of C_l is the reported stderr
    se = ps.std(axis=1, ddof=1) / np.sqrt(32)
    assert np.allclose(se, e, rtol=1e-9, atol=1e-300)


# ------------------------------------------------------------------------
# principal components on the matrix cores
# ------------------------------------------------------------------------
# FP32 MFMA keeps the FP32 bound; the BF16x3 split carries ~2^-17 relative
# error per product into W~, which psi amplifies like any other path error.
BF16X3_TOL = np.array([2e-4, 2e-4, 1e-3, 2e-3])


@pytest.mark.parametrize("d", [2, 17, 64, 100, 257])
def test_fp64_pca_parity(d):
    opts = workloads.three_products_grid(d=d, n_points=8192 + 150)[::4]
    say("pca fp64", d)
    g, e, ps = q.greeks(opts, 2, q.PATH_PCA, q.FP64, per_shift=True)
    m, se, am, Cl = oracle_many(opts, 2, oracle.PATH_PCA)
    assert_scaled(ps, Cl, am[:, None, :], TOL64, "per shift")


@pytest.mark.parametrize("gemm,tol", [(q.GEMM_FP32, FP32_TOL), (q.GEMM_BF16X3, BF16X3_TOL)])
@pytest.mark.parametrize("d", [17, 64, 257])
def test_pca_matrix_cores_within_bound(gemm, tol, d):
    opts = workloads.three_products_grid(d=d, n_points=4096 + 100)[::3]
    say("pca mfma", gemm, d)
    g, e, ps = q.greeks(opts, 2, q.PATH_PCA, q.FP32_MIXED, pca_gemm=gemm, per_shift=True)
    m, se, am, Cl = oracle_many(opts, 2, oracle.PATH_PCA)
    err = scaled_err(ps, Cl, am[:, None, :])
    say("pca scaled error", gemm, d, err.max(axis=(0, 1)))
    for k in range(4):
        assert err[..., k].max() <= tol[k], (k, err[..., k].max())


@pytest.mark.parametrize("path", [q.PATH_PCA, q.PATH_PCA_FULL])
@pytest.mark.parametrize("gemm,tol", [(q.GEMM_FP32, FP32_TOL), (q.GEMM_BF16X3, BF16X3_TOL)])
def test_pca_shared_paths_one_product(gemm, tol, path):
    """Options with the same paths (seed, d, sigma, r, T) but other strikes
    and payoffs share one product and epilogue per tile in the matrix-core
    kernel (under either conditioning; with the first principal component
    each option still runs its own FP64 root-find): each result equals the
    option's result alone, bit for bit, and the oracle's within the bound; a
    lookback and an option of another seed in the same launch keep their own
    paths."""
    base = dict(d=65, S0=100.0, r=0.05, sigma=0.25, T=1.0, seed=0x5eed, n_points=8192 + 300)
    grp = [dict(base, type=t, K=K) for t, K in ((q.ARITH_ASIAN, 95.0), (q.BINARY_ASIAN, 95.0),
                                                 (q.ARITH_ASIAN, 108.0), (q.BINARY_ASIAN, 101.0),
                                                 (q.ARITH_ASIAN, 100.0))]   # five: a group of 4 and one more
    others = [dict(base, type=q.LOOKBACK, K=100.0), dict(base, type=q.ARITH_ASIAN, K=100.0, seed=0x5eee)]
    opts = grp + others
    say("pca shared paths", gemm, path)
    g, e, ps = q.greeks(opts, 4, path, q.FP32_MIXED, pca_gemm=gemm, per_shift=True)
    for i, o in enumerate(opts):
        g1, e1, ps1 = q.greeks([o], 4, path, q.FP32_MIXED, pca_gemm=gemm, per_shift=True)
        assert np.array_equal(ps[i], ps1[0]), i
    m, se, am, Cl = oracle_many(opts, 4, oracle.PATH_PCA if path == q.PATH_PCA else oracle.PATH_PCA_FULL)
    err = scaled_err(ps, Cl, am[:, None, :])
    say("pca shared scaled error", gemm, err.max(axis=(0, 1)))
    for k in range(4):
        assert err[..., k].max() <= tol[k], (k, err[..., k].max())


def test_pca_full_size_properties():
    """The d = 256 PCA workload at full size (2 options x 2^22 points x 16
    shifts): the matrix-core results agree with the FP64 path at the same
    points within their bounds, and the standard errors match the spread of
    the replications."""
    opts = workloads.pca_pair(d=256, n_points=1 << 22)
    say("pca full fp64")
    g64, e64, p64 = q.greeks(opts, 16, q.PATH_PCA, q.FP64, per_shift=True)
    for gemm, tol in [(q.GEMM_FP32, FP32_TOL), (q.GEMM_BF16X3, BF16X3_TOL)]:
        say("pca full", gemm)
        g, e, ps = q.greeks(opts, 16, q.PATH_PCA, q.FP32_MIXED, pca_gemm=gemm, per_shift=True)
        o1 = [oracle.option(o["type"], o["d"], o["S0"], o["K"], o["r"], o["sigma"], o["T"], o["seed"], 512, 1,
                            oracle.PATH_PCA)["abs_mean"] for o in opts]
        scale = np.array(o1)[:, None, :]
        err = scaled_err(ps, p64, scale)
        say("full pca scaled diff", gemm, err.max(axis=(0, 1)))
        for k in range(4):
            assert err[..., k].max() <= tol[k]
        se = ps.std(axis=1, ddof=1) / 4.0
        assert np.allclose(se, e, rtol=1e-9, atol=1e-300)


# ------------------------------------------------------------------------
# conditioning on the first principal component of all d dates
# ------------------------------------------------------------------------
@pytest.mark.parametrize("d,pts,step", [(1, 8192 + 150, 3), (2, 8192 + 150, 3), (16, 8192 + 150, 3),
                                        (63, 8192 + 150, 3), (256, 4096 + 100, 6)])
def test_fp64_pca_full_parity(d, pts, step):
    opts = workloads.three_products_grid(d=d, n_points=pts)[::step]   # arithmetic, binary, lookback
    say("pca_full fp64", d, len(opts))
    g, e, ps = q.greeks(opts, 2, q.PATH_PCA_FULL, q.FP64, per_shift=True)
    m, se, am, Cl = oracle_many(opts, 2, oracle.PATH_PCA_FULL)
    assert_scaled(ps, Cl, am[:, None, :], TOL64, "per shift")
    assert_scaled(g, m, am, TOL64, "mean")


@pytest.mark.parametrize("gemm,tol", [(q.GEMM_FP32, FP32_TOL), (q.GEMM_BF16X3, BF16X3_TOL)])
@pytest.mark.parametrize("d", [17, 64, 256])
def test_pca_full_matrix_cores_within_bound(gemm, tol, d):
    opts = workloads.three_products_grid(d=d, n_points=4096 + 100)[::3 if d < 256 else 6]
    say("pca_full mfma", gemm, d)
    g, e, ps = q.greeks(opts, 2, q.PATH_PCA_FULL, q.FP32_MIXED, pca_gemm=gemm, per_shift=True)
    m, se, am, Cl = oracle_many(opts, 2, oracle.PATH_PCA_FULL)
    err = scaled_err(ps, Cl, am[:, None, :])
    say("pca_full scaled error", gemm, d, err.max(axis=(0, 1)))
    for k in range(4):
        assert err[..., k].max() <= tol[k], (k, err[..., k].max())


def test_pca_full_large_properties():
    """d = 256, 2^20 points x 8 shifts: the matrix-core results agree with
    the FP64 path at the same points within their bounds and the standard
    errors match the spread of the replications; one replication of 2^16
    points (eight work units) is recomputed by the oracle."""
    opts = workloads.pca_pair(d=256, n_points=1 << 20)
    say("pca_full large fp64")
    g64, e64, p64 = q.greeks(opts, 8, q.PATH_PCA_FULL, q.FP64, per_shift=True)
    o1 = [oracle.option(o["type"], o["d"], o["S0"], o["K"], o["r"], o["sigma"], o["T"], o["seed"], 512, 1,
                        oracle.PATH_PCA_FULL)["abs_mean"] for o in opts]
    scale = np.array(o1)
    mid = dict(opts[1], n_points=1 << 16)
    _, _, pm = q.greeks([mid], 8, q.PATH_PCA_FULL, q.FP64, per_shift=True)
    ref = oracle.replication(mid, 5, oracle.PATH_PCA_FULL)
    assert_scaled(pm[0, 5], ref, scale[1], TOL64, "replication 5 of the binary Asian, 2^16 points")
    for gemm, tol in [(q.GEMM_FP32, FP32_TOL), (q.GEMM_BF16X3, BF16X3_TOL)]:
        say("pca_full large", gemm)
        g, e, ps = q.greeks(opts, 8, q.PATH_PCA_FULL, q.FP32_MIXED, pca_gemm=gemm, per_shift=True)
        err = scaled_err(ps, p64, scale[:, None, :])
        say("pca_full large scaled diff", gemm, err.max(axis=(0, 1)))
        for k in range(4):
            assert err[..., k].max() <= tol[k]
        se = ps.std(axis=1, ddof=1) / np.sqrt(8)
        assert np.allclose(se, e, rtol=1e-9, atol=1e-300)


# ------------------------------------------------------------------------
# nested (Owen) scrambling instead of the digital shift
# ------------------------------------------------------------------------
@pytest.mark.parametrize("n_dims,k0,count,shift", [(16, 0, 4096, 0), (65, 0, 3000, 3), (365, 1000, 700, 7),
                                                   (130, (1 << 20) - 50, 300, 31)])
def test_scrambled_points_bit_exact(n_dims, k0, count, shift):
    say("owen points", n_dims, k0, count, shift)
    seed = 0x5C4A + n_dims
    got = q.sobol_points(seed, shift, n_dims, k0, count, owen=True)
    raw = oracle.sobol_points(n_dims, k0, count)
    keys = oracle.shifts(seed, shift + 1, n_dims)[shift]
    ref = raw.copy()
    for j in range(1, n_dims):
        ref[:, j] = [oracle.owen(int(y), int(keys[j])) for y in raw[:, j]]
    assert np.array_equal(got, ref)


@pytest.mark.parametrize("path,d", [(q.PATH_BB, 16), (q.PATH_BB, 65), (q.PATH_STANDARD, 33), (q.PATH_PCA, 17),
                                    (q.PATH_PCA, 64), (q.PATH_PCA_FULL, 16), (q.PATH_PCA_FULL, 63)])
def test_fp64_owen_parity(path, d):
    opts = workloads.three_products_grid(d=d, n_points=4096 + 77)[::4]
    say("owen fp64", path, d)
    g, e, ps = q.greeks(opts, 3, path, q.FP64, per_shift=True, owen=True)
    m, se, am, Cl = oracle_many_rand(opts, 3, path, oracle.RAND_OWEN)
    assert_scaled(ps, Cl, am[:, None, :], TOL64, "per shift")


@pytest.mark.parametrize("path,d", [(q.PATH_BB, 64), (q.PATH_BB, 65), (q.PATH_STANDARD, 17), (q.PATH_PCA, 64),
                                    (q.PATH_PCA, 257), (q.PATH_PCA_FULL, 17)])
def test_fp32_owen_within_bound(path, d):
    opts = workloads.three_products_grid(d=d, n_points=4096 + 77)[::3]
    say("owen fp32", path, d)
    g, e, ps = q.greeks(opts, 3, path, q.FP32_MIXED, per_shift=True, owen=True)
    m, se, am, Cl = oracle_many_rand(opts, 3, path, oracle.RAND_OWEN)
    err = scaled_err(ps, Cl, am[:, None, :])
    for k in range(4):
        assert err[..., k].max() <= FP32_TOL[k], (k, err[..., k].max())


def oracle_many_rand(opts, L, path, rand):
    out = [_oracle_one(o, L, path, rand) for o in opts]
    return (np.array([r["mean"] for r in out]), np.array([r["stderr"] for r in out]),
            np.array([r["abs_mean"] for r in out]), np.array([r["C_l"] for r in out]))


# ------------------------------------------------------------------------
# geometric Asian call: the same template with another average
# ------------------------------------------------------------------------
@pytest.mark.parametrize("path", [q.PATH_BB, q.PATH_STANDARD, q.PATH_PCA])
@pytest.mark.parametrize("d", [2, 64, 100])
def test_fp64_geometric_parity(path, d):
    opts = workloads.geometric_grid(d=d, n_points=2 * 8192 + 77)
    say("geometric fp64", path, d)
    g, e, ps = q.greeks(opts, 3, path, q.FP64, per_shift=True)
    m, se, am, Cl = oracle_many(opts, 3, path)
    assert_scaled(ps, Cl, am[:, None, :], TOL64, "per shift")
    assert_scaled(g, m, am, TOL64, "mean")


@pytest.mark.parametrize("path,d,gemm", [(q.PATH_BB, 64, 0), (q.PATH_BB, 65, 0), (q.PATH_STANDARD, 64, 0),
                                         (q.PATH_PCA, 64, q.GEMM_FP32), (q.PATH_PCA, 64, q.GEMM_BF16X3)])
def test_fp32_geometric_within_bound(path, d, gemm):
    opts = workloads.geometric_grid(d=d, n_points=8192 + 300)
    say("geometric fp32", path, d, gemm)
    g, e, ps = q.greeks(opts, 2, path, q.FP32_MIXED, pca_gemm=gemm, per_shift=True)
    m, se, am, Cl = oracle_many(opts, 2, path)
    err = scaled_err(ps, Cl, am[:, None, :])
    say("geometric fp32 scaled error", err.max(axis=(0, 1)))
    tol = BF16X3_TOL if (path == q.PATH_PCA and gemm == q.GEMM_BF16X3) else FP32_TOL
    for k in range(4):
        assert err[..., k].max() <= tol[k], (k, err[..., k].max())


@pytest.mark.parametrize("path,prec", [(q.PATH_BB, q.FP32_MIXED), (q.PATH_BB, q.FP64),
                                       (q.PATH_STANDARD, q.FP32_MIXED), (q.PATH_PCA, q.FP32_MIXED)])
def test_geometric_full_size_matches_closed_form(path, prec):
    """6 geometric calls, d = 64, 2^20 points x 32 shifts: every Greek lies
    within 5 reported standard errors of the exact discrete-monitoring value
    (plus the FP32 bound where the path runs in FP32), and the standard
    errors are the spread of the replications."""
    from closed_forms import geometric_asian_closed_form
    opts = workloads.geometric_grid(d=64, n_points=1 << 20)
    say("geometric full size", path, prec)
    g, e, ps = q.greeks(opts, 32, path, prec, per_shift=True)
    exact = np.array([geometric_asian_closed_form(o["S0"], o["K"], o["r"], o["sigma"], o["T"], o["d"])
                      for o in opts])
    slack = 0.0 if prec == q.FP64 else 1.0
    z = np.abs(g - exact) / (5 * e + slack * FP32_TOL[None, :] * np.abs(exact))
    say("geometric |g - exact| / allowed:", z.max(axis=0), "stderr / |exact|:", (e / np.abs(exact)).max(axis=0))
    assert (z <= 1).all(), z
    se = ps.std(axis=1, ddof=1) / np.sqrt(32)
    assert np.allclose(se, e, rtol=1e-9, atol=1e-300)


# ------------------------------------------------------------------------
# puts (average, binary, geometric, lookback on the minimum)
# ------------------------------------------------------------------------
@pytest.mark.parametrize("path", [q.PATH_BB, q.PATH_STANDARD, q.PATH_PCA])
@pytest.mark.parametrize("d", [2, 64, 100])
def test_fp64_puts_parity(path, d):
    opts = workloads.put_grid(d=d, n_points=8192 + 77)[::2]
    say("puts fp64", path, d)
    g, e, ps = q.greeks(opts, 3, path, q.FP64, per_shift=True)
    m, se, am, Cl = oracle_many(opts, 3, path)
    assert_scaled(ps, Cl, am[:, None, :], TOL64, "per shift")
    assert_scaled(g, m, am, TOL64, "mean")


@pytest.mark.parametrize("path,d,gemm", [(q.PATH_BB, 64, 0), (q.PATH_BB, 65, 0), (q.PATH_STANDARD, 64, 0),
                                         (q.PATH_PCA, 64, q.GEMM_FP32), (q.PATH_PCA, 64, q.GEMM_BF16X3)])
def test_fp32_puts_within_bound(path, d, gemm):
    opts = workloads.put_grid(d=d, n_points=8192 + 300)
    say("puts fp32", path, d, gemm)
    g, e, ps = q.greeks(opts, 2, path, q.FP32_MIXED, pca_gemm=gemm, per_shift=True)
    m, se, am, Cl = oracle_many(opts, 2, path)
    err = scaled_err(ps, Cl, am[:, None, :])
    say("puts fp32 scaled error", err.max(axis=(0, 1)))
    tol = BF16X3_TOL if (path == q.PATH_PCA and gemm == q.GEMM_BF16X3) else FP32_TOL
    for k in range(4):
        assert err[..., k].max() <= tol[k], (k, err[..., k].max())


def test_geometric_put_full_size_matches_closed_form():
    """6 geometric puts, d = 64, 2^20 points x 32 shifts, FP32-mixed bridge:
    every Greek within 5 reported standard errors (plus the FP32 bound) of
    the closed form obtained from the call's by put-call parity."""
    from closed_forms import geometric_asian_closed_form
    opts = [o for o in workloads.put_grid(d=64, n_points=1 << 20) if o["type"] == q.GEOMETRIC_ASIAN_PUT]
    g, e = q.greeks(opts, 32, q.PATH_BB, q.FP32_MIXED)
    ref = []
    for o in opts:
        S0, K, r, sig, T, d = o["S0"], o["K"], o["r"], o["sigma"], o["T"], o["d"]
        c = geometric_asian_closed_form(S0, K, r, sig, T, d)
        dt = T / d
        tbar = dt * (d + 1) / 2
        cv = dt * (d + 1) * (2 * d + 1) / (6 * d)
        F = np.exp(np.log(S0) + (r - sig**2 / 2) * tbar + sig**2 * cv / 2)
        D = np.exp(-r * T)
        ref.append(c - np.array([D * (F - K), D * F / S0, D * F * sig * (cv - tbar), 0.0]))
    ref = np.array(ref)
    z = np.abs(g - ref) / (5 * e + FP32_TOL[None, :] * np.abs(ref))
    say("geometric put |g - exact| / allowed:", z.max(axis=0))
    assert (z <= 1).all(), z


# ------------------------------------------------------------------------
# basket of M assets (one-factor model, standard construction)
# ------------------------------------------------------------------------
@pytest.mark.parametrize("d,M", [(1, 3), (16, 1), (16, 4), (40, 8)])
def test_fp64_basket_parity(d, M):
    opts = workloads.basket_grid(d=d, n_assets=M, n_points=8192 + 77)
    say("basket fp64", d, M)
    g, e, ps = q.greeks(opts, 3, q.PATH_STANDARD, q.FP64, per_shift=True)
    m, se, am, Cl = oracle_many(opts, 3, q.PATH_STANDARD)
    assert_scaled(ps, Cl, am[:, None, :], TOL64, "per shift")
    assert_scaled(g, m, am, TOL64, "mean")


@pytest.mark.parametrize("d,M", [(16, 4), (40, 8)])
def test_fp32_basket_within_bound(d, M):
    opts = workloads.basket_grid(d=d, n_assets=M, n_points=8192 + 300)
    say("basket fp32", d, M)
    g, e, ps = q.greeks(opts, 2, q.PATH_STANDARD, q.FP32_MIXED, per_shift=True)
    m, se, am, Cl = oracle_many(opts, 2, q.PATH_STANDARD)
    err = scaled_err(ps, Cl, am[:, None, :])
    say("basket fp32 scaled error", err.max(axis=(0, 1)))
    for k in range(4):
        assert err[..., k].max() <= FP32_TOL[k], (k, err[..., k].max())


def test_fp64_basket_owen_parity():
    opts = workloads.basket_grid(d=12, n_assets=3, n_points=4096 + 77)[::2]
    g, e, ps = q.greeks(opts, 3, q.PATH_STANDARD, q.FP64, per_shift=True, owen=True)
    m, se, am, Cl = oracle_many_rand(opts, 3, q.PATH_STANDARD, oracle.RAND_OWEN)
    assert_scaled(ps, Cl, am[:, None, :], TOL64, "per shift")


# ------------------------------------------------------------------------
# serving: continuous batching
# ------------------------------------------------------------------------
def test_server_results_match_direct_calls_and_overlap():
    """Requests submitted while others run are admitted into later launches;
    each result equals a direct call on the same options at the number of
    points the request reached (same points, same shifts)."""
    import time
    reqs = [workloads.portfolio(n, seed=100 + i, d_range=(8, 96)) for i, n in enumerate([3, 40, 1, 17, 64, 5])]
    with q.Server(hbm_budget_bytes=1 << 30, precision=q.FP32_MIXED) as srv:
        ids = []
        for i, opts in enumerate(reqs):
            ids.append(srv.submit(opts, 8, target_stderr=1e-4))
            if i == 2:
                time.sleep(0.01)   # later requests arrive while earlier ones run
        results = [srv.wait(rid, len(opts)) for rid, opts in zip(ids, reqs)]
        st = srv.stats()
    say("server stats", st)
    assert st["completed"] == len(reqs) and st["bytes_in_use"] == 0
    for opts, (g, e, pts) in zip(reqs, results):
        assert pts >= 1 << 14 and pts <= 1 << 22
        gd, ed = q.greeks([dict(o, n_points=pts) for o in opts], 8, q.PATH_BB, q.FP32_MIXED)
        scale = np.maximum(np.abs(gd), 1e-12)
        assert np.all(np.abs(g - gd) <= 1e-12 * scale + 1e-15), np.abs(g - gd).max()
        met = (e[:, 1:] <= 1e-4 * np.maximum(1.0, np.abs(g[:, 1:]))).all()
        assert met or pts == 1 << 22


def test_server_admission_budget_and_cancel():
    # each request holds 20 options x 16 shifts: a slice of 2^21 points would
    # take 10.5 MB, so under a 12 MB budget (6 MB per launch slot) the rounds
    # ride in slices of 2^20 points, one request per launch
    small = workloads.portfolio(20, seed=1, d_range=(8, 32))
    budget = 12 << 20
    with q.Server(hbm_budget_bytes=budget, precision=q.FP32_MIXED) as srv:
        with pytest.raises(q.QcpwError):
            srv.submit(workloads.portfolio(200, seed=2), 16, 1e-6)      # smallest slice exceeds a slot
        ids = [srv.submit(small, 16, 1e-9) for _ in range(6)]           # unmet target: run to the cap
        srv.cancel(ids[-1])
        out = [srv.wait(i, len(small)) if i != ids[-1] else None for i in ids]
        with pytest.raises(q.QcpwError):
            srv.wait(ids[-1], len(small))
        st = srv.stats()
    say("admission stats", st)
    assert st["peak_bytes"] <= budget
    assert st["workspace_bytes"] <= budget          # what the slots actually hold on the device
    assert st["bytes_in_use"] == 0
    assert st["cancelled"] >= 1
    assert all(o[2] == 1 << 22 for o in out if o is not None)


def test_server_destroy_returns_promptly():
    """Destroying a server with long requests queued and running stops taking
    work at once: it waits only for the (bounded) launches in flight."""
    import time
    heavy = workloads.portfolio(64, seed=9, d_range=(300, 365))
    srv = q.Server(hbm_budget_bytes=8 << 30, precision=q.FP32_MIXED)
    for _ in range(8):
        srv.submit(heavy, 16, 1e-12)        # each would run to 2^22 points: seconds of work
    time.sleep(0.2)
    t0 = time.perf_counter()
    srv.close()
    dt = time.perf_counter() - t0
    say("destroy took %.3f s" % dt)
    assert dt < 1.0


# ------------------------------------------------------------------------
# HIP graph capture / replay
# ------------------------------------------------------------------------
@pytest.mark.parametrize("prec", [q.FP64, q.FP32_MIXED])
def test_graph_replays_match_eager(prec):
    """A captured launch replayed several times, with other eager launches,
    host synchronisations and a cleared output in between, gives the eager
    result every time."""
    import torch
    opts = workloads.three_products_grid(d=16, n_points=3 * 8192 + 5)
    ref_g, ref_e = q.greeks(opts, 8, q.PATH_BB, prec)
    s = torch.cuda.Stream()
    out = (torch.empty((len(opts), 4), dtype=torch.float64, device="cuda"),
           torch.empty((len(opts), 4), dtype=torch.float64, device="cuda"))
    other = workloads.portfolio(6, seed=3, log2_points=(10, 12))
    for rep in range(4):
        with torch.cuda.stream(s):
            out[0].zero_()
            out[1].zero_()
        q.greeks(opts, 8, q.PATH_BB, prec, device_outputs=True, out=out, stream=s, graph=True)
        s.synchronize()
        assert np.array_equal(out[0].cpu().numpy(), ref_g), rep
        assert np.array_equal(out[1].cpu().numpy(), ref_e), rep
        q.greeks(other, 4, q.PATH_BB, prec)                 # unrelated eager work in between
        torch.cuda.synchronize()


def test_graph_flag_requires_device_outputs():
    with pytest.raises(q.QcpwError):
        q.greeks(workloads.single_asian(n_points=64), 2, q.PATH_BB, q.FP64, graph=True)
