"""Seeded synthetic workloads for QMC-CPW Greeks (arXiv 2209.11337).

This module only draws option parameters, seeds and arrival times.  It holds
none of the estimator's arithmetic and is the one module that both the HIP
path's callers and the oracle's callers read inputs from.  Every draw comes
from ``numpy.random.Generator(PCG64(seed))`` with a fixed seed, so every run
sees the same inputs.

The paper prices with Black-Scholes parameters only (Sec. 5: S(0) = 100,
sigma = 0.2, r = 0.1, T = 1, K in {90, 100, 110}, d in {64, 256}, 2^15 paths,
500 runs); there is no dataset.  The workloads below keep that setting and
widen it where a configuration asks for more (several sigma, an uneven
portfolio, a request stream).

An option is a dict with keys type, d, S0, K, r, sigma, T, seed, n_points
(the fields of ``qcpw_option_spec``).
"""
from __future__ import annotations

import numpy as np

ARITH_ASIAN, BINARY_ASIAN, LOOKBACK, GEOMETRIC_ASIAN = 0, 1, 2, 3
ARITH_ASIAN_PUT, BINARY_ASIAN_PUT, LOOKBACK_PUT, GEOMETRIC_ASIAN_PUT = 4, 5, 6, 7
BASKET_ASIAN, BASKET_ASIAN_PUT = 8, 9
PATH_BB, PATH_PCA, PATH_STANDARD = 0, 1, 2
TYPE_NAMES = {ARITH_ASIAN: "arith_asian", BINARY_ASIAN: "binary_asian", LOOKBACK: "lookback",
              GEOMETRIC_ASIAN: "geometric_asian", ARITH_ASIAN_PUT: "arith_asian_put",
              BINARY_ASIAN_PUT: "binary_asian_put", LOOKBACK_PUT: "lookback_put",
              GEOMETRIC_ASIAN_PUT: "geometric_asian_put", BASKET_ASIAN: "basket_asian",
              BASKET_ASIAN_PUT: "basket_asian_put"}

BASE_SEED = 0x220911337


def _rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def _seeds(n: int, seed: int) -> list[int]:
    return [int(x) for x in _rng(seed).integers(0, 2**63, size=n, dtype=np.int64)]


def single_asian(d: int = 16, n_points: int = 1 << 12) -> list[dict]:
    """One arithmetic Asian call: S0 = K = 100, r = 0.05, sigma = 0.2, T = 1,
    d equally spaced dates (default 16), 2^12 points; Brownian bridge, 16 shifts."""
    return [dict(type=ARITH_ASIAN, d=d, S0=100.0, K=100.0, r=0.05, sigma=0.2, T=1.0,
                 seed=BASE_SEED, n_points=n_points)]


def three_products_grid(d: int = 64, n_points: int = 1 << 20) -> list[dict]:
    """18 options: {arith Asian, binary Asian, lookback} x K {90,100,110} x
    sigma {0.1, 0.3}; S0 = 100, r = 0.05, T = 1, d dates (default 64)."""
    out = []
    for typ in (ARITH_ASIAN, BINARY_ASIAN, LOOKBACK):
        for K in (90.0, 100.0, 110.0):
            for sig in (0.1, 0.3):
                out.append(dict(type=typ, d=d, S0=100.0, K=K, r=0.05, sigma=sig, T=1.0,
                                n_points=n_points))
    for o, s in zip(out, _seeds(len(out), BASE_SEED)):
        o["seed"] = s
    return out


def paper_grid(d: int = 64, n_points: int = 1 << 15) -> list[dict]:
    """The paper's Sec. 5 setting: 3 products x K {90,100,110}; S0 = 100,
    sigma = 0.2, r = 0.1, T = 1; d in {64, 256}; 2^15 points."""
    out = []
    for typ in (ARITH_ASIAN, BINARY_ASIAN, LOOKBACK):
        for K in (90.0, 100.0, 110.0):
            out.append(dict(type=typ, d=d, S0=100.0, K=K, r=0.1, sigma=0.2, T=1.0,
                            n_points=n_points))
    for o, s in zip(out, _seeds(len(out), BASE_SEED + 1)):
        o["seed"] = s
    return out


def geometric_grid(d: int = 64, n_points: int = 1 << 20) -> list[dict]:
    """6 geometric Asian calls: K {90,100,110} x sigma {0.1, 0.3}; S0 = 100,
    r = 0.05, T = 1, d dates (default 64) -- the three-product grid's setting
    for the one product whose expectation has a closed form."""
    out = [dict(type=GEOMETRIC_ASIAN, d=d, S0=100.0, K=K, r=0.05, sigma=sig, T=1.0, n_points=n_points)
           for K in (90.0, 100.0, 110.0) for sig in (0.1, 0.3)]
    for o, s in zip(out, _seeds(len(out), BASE_SEED + 3)):
        o["seed"] = s
    return out


def put_grid(d: int = 64, n_points: int = 1 << 20) -> list[dict]:
    """24 puts: {arith, binary, geometric Asian, fixed-strike lookback on the
    minimum} x K {90,100,110} x sigma {0.1, 0.3}; S0 = 100, r = 0.05, T = 1."""
    out = [dict(type=t, d=d, S0=100.0, K=K, r=0.05, sigma=sig, T=1.0, n_points=n_points)
           for t in (ARITH_ASIAN_PUT, BINARY_ASIAN_PUT, LOOKBACK_PUT, GEOMETRIC_ASIAN_PUT)
           for K in (90.0, 100.0, 110.0) for sig in (0.1, 0.3)]
    for o, s in zip(out, _seeds(len(out), BASE_SEED + 4)):
        o["seed"] = s
    return out


def basket_grid(d: int = 16, n_assets: int = 4, n_points: int = 1 << 20) -> list[dict]:
    """8 basket options on n_assets assets (one-factor model): {call, put} x
    K {95, 105} x rho {0.3, 0.8}; S0 = 100, sigma = 0.25, r = 0.05, T = 1."""
    out = [dict(type=t, d=d, S0=100.0, K=K, r=0.05, sigma=0.25, T=1.0, n_points=n_points,
                n_assets=n_assets, rho=rho)
           for t in (BASKET_ASIAN, BASKET_ASIAN_PUT) for K in (95.0, 105.0) for rho in (0.3, 0.8)]
    for o, s in zip(out, _seeds(len(out), BASE_SEED + 5)):
        o["seed"] = s
    return out


def pca_pair(d: int = 256, n_points: int = 1 << 22, shared: bool = True) -> list[dict]:
    """Arithmetic and binary Asian, S0 = K = 100, r = 0.05, sigma = 0.2, T = 1,
    d = 256 (255 conditioned coordinates, padded to a 256 x 256 factor).
    shared: one seed for both, so that they price the same paths (one
    product per shift, both payoffs in its epilogue); else a seed each."""
    out = [dict(type=t, d=d, S0=100.0, K=100.0, r=0.05, sigma=0.2, T=1.0, n_points=n_points)
           for t in (ARITH_ASIAN, BINARY_ASIAN)]
    seeds = _seeds(2, BASE_SEED + 2)
    for o, s in zip(out, seeds[:1] * 2 if shared else seeds):
        o["seed"] = s
    return out


def portfolio(n_opts: int = 4096, seed: int = 220911337, d_range=(4, 365),
              log2_points=(14, 20)) -> list[dict]:
    """Uneven portfolio: type uniform over 3, d uniform integer in d_range,
    K ~ U[80,120], sigma ~ U[0.1,0.5], T ~ U[0.25,2], r ~ U[0,0.08], S0 = 100,
    points 2^k with k uniform integer in log2_points (inclusive)."""
    g = _rng(seed)
    typ = g.integers(0, 3, size=n_opts)
    d = g.integers(d_range[0], d_range[1] + 1, size=n_opts)
    K = g.uniform(80.0, 120.0, size=n_opts)
    sig = g.uniform(0.1, 0.5, size=n_opts)
    T = g.uniform(0.25, 2.0, size=n_opts)
    r = g.uniform(0.0, 0.08, size=n_opts)
    k = g.integers(log2_points[0], log2_points[1] + 1, size=n_opts)
    seeds = g.integers(0, 2**63, size=n_opts, dtype=np.int64)
    return [dict(type=int(typ[i]), d=int(d[i]), S0=100.0, K=float(K[i]), r=float(r[i]),
                 sigma=float(sig[i]), T=float(T[i]), seed=int(seeds[i]), n_points=1 << int(k[i]))
            for i in range(n_opts)]


def request_stream(n_requests: int, rate_per_s: float, seed: int = 22091,
                   max_opts: int = 512, d_range=(4, 365), targets=(1e-4, 1e-6)) -> list[dict]:
    """Poisson arrivals: exponential gaps at rate_per_s; each request holds
    U{1..max_opts} options drawn as in ``portfolio`` and a target standard
    error drawn from ``targets`` (equal odds; 1e-4 or 1e-6 by default)."""
    g = _rng(seed)
    gaps = g.exponential(1.0 / rate_per_s, size=n_requests)
    t = np.cumsum(gaps) - gaps[0]
    out = []
    for i in range(n_requests):
        n = int(g.integers(1, max_opts + 1))
        opts = portfolio(n, seed=int(g.integers(0, 2**31)), d_range=d_range)
        out.append(dict(t_arrival=float(t[i]), options=opts,
                        target_stderr=float(g.choice(list(targets)))))
    return out


def total_paths(opts: list[dict], n_shifts: int) -> int:
    return int(sum(o["n_points"] for o in opts)) * n_shifts


def total_path_dates(opts: list[dict], n_shifts: int) -> int:
    return int(sum(o["n_points"] * max(o["d"] - 1, 0) for o in opts)) * n_shifts
