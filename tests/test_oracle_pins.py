"""Pins of the FP64 oracle against facts fixed outside it (no GPU needed).

Each test checks one part of the oracle against something other than the
oracle itself: values derived by hand from the paper, a textbook worked
example, a published generator test vector, a library routine (scipy), a
closed form, an invariant, finite differences, or numerical quadrature of the
unconditioned payoff.
"""
import math
import os

import numpy as np
import pytest
import scipy.integrate
import scipy.optimize
import scipy.special
import scipy.stats
from scipy.stats import qmc

import oracle
from closed_forms import geometric_asian_closed_form

# --------------------------------------------------------------------------
# Sobol' points (Sec. 2.2)
# --------------------------------------------------------------------------


def _read_rows(path):
    rows = []
    with open(path) as f:
        for line in f:
            line = line.split("#")[0].strip()
            if line:
                rows.append(line.split())
    return rows


def test_sobol_leading_points_from_paper(golden_dir):
    rows = _read_rows(os.path.join(golden_dir, "sobol_leading_points.txt"))
    P = oracle.sobol_points(2, 0, len(rows))
    for k, (kk, a, b) in enumerate(rows):
        assert int(kk) == k
        assert P[k, 0] == int(round(float(a) * 2**32))
        assert P[k, 1] == int(round(float(b) * 2**32))


def test_direction_recurrence_textbook_example(golden_dir):
    (row,) = _read_rows(os.path.join(golden_dir, "sobol_recurrence_example.txt"))
    poly, m = int(row[0]), [int(x) for x in row[1:]]
    V = np.zeros((1, 32), dtype=np.uint32)
    minit = np.zeros((1, 18), dtype=np.int64)
    minit[0, :3] = m[:3]
    rc = oracle._load().oracle_direction_numbers(1, np.array([poly], dtype=np.int64), minit, 18, V)
    assert rc == 0
    got = [int(V[0, b]) >> (31 - b) for b in range(6)]
    assert got == m


def test_direction_numbers_reject_even_initial_value():
    V = np.zeros((1, 32), dtype=np.uint32)
    minit = np.zeros((1, 18), dtype=np.int64)
    minit[0, :2] = [1, 2]
    rc = oracle._load().oracle_direction_numbers(1, np.array([7], dtype=np.int64), minit, 18, V)
    assert rc != 0


@pytest.mark.parametrize("n_dims,m", [(16, 12), (365, 10)])
def test_sobol_matches_scipy_bit_exact(n_dims, m):
    P = oracle.sobol_points(n_dims, 0, 1 << m)
    S = qmc.Sobol(n_dims, scramble=False, bits=32).random_base2(m)
    ints = np.round(S * 2.0**32).astype(np.uint64)
    assert np.array_equal(P.astype(np.uint64), ints)


def test_sobol_random_access_offset():
    S = qmc.Sobol(40, scramble=False, bits=32).random_base2(11)
    ints = np.round(S * 2.0**32).astype(np.uint64)
    for k0, cnt in [(1, 5), (1000, 48), (2040, 8)]:
        P = oracle.sobol_points(40, k0, cnt)
        assert np.array_equal(P.astype(np.uint64), ints[k0:k0 + cnt])


# --------------------------------------------------------------------------
# Digital shift (Sec. 2.2.3) and its generator
# --------------------------------------------------------------------------


def test_splitmix64_published_vector(golden_dir):
    for seed, i, out in _read_rows(os.path.join(golden_dir, "splitmix64_vectors.txt")):
        assert oracle.splitmix64(int(seed), int(i)) == int(out)


def test_shift_is_high_word_of_counter_output():
    seed = 0xDEADBEEF12345
    for l, j in [(0, 1), (3, 17), (31, 364)]:
        assert oracle.shift(seed, l, j) == oracle.splitmix64(seed, (l << 16) + j) >> 32


@pytest.mark.parametrize("m", [4, 8, 11])
def test_shifted_points_remain_a_net(m):
    """A digital shift maps each dyadic interval of length 2^-m onto another one,
    so the first 2^m shifted points still hit every such interval once per
    coordinate (the (0,m,1)-net property in each 1-D projection)."""
    n_dims = 24
    P = oracle.sobol_points(n_dims, 0, 1 << m).astype(np.uint64)
    s = oracle.shifts(0x1234, 3, n_dims)
    for l in range(3):
        Y = P ^ s[l][None, :].astype(np.uint64)
        for j in range(n_dims):
            cells = np.sort(Y[:, j] >> (32 - m))
            assert np.array_equal(cells, np.arange(1 << m, dtype=np.uint64))


# --------------------------------------------------------------------------
# Nested (Owen) scrambling (Sec. 2.2.3)
# --------------------------------------------------------------------------

def test_owen_scrambling_is_nested():
    """Digit k of the scrambled value depends on digits 1..k of the input
    only: two inputs that share their first k digits share the first k
    scrambled digits, and the k-th scrambled digits differ iff the k-th
    input digits do."""
    rng = np.random.default_rng(17)
    for _ in range(300):
        seed = int(rng.integers(0, 2**32))
        y = int(rng.integers(0, 2**32))
        k = int(rng.integers(1, 32))                    # change digits k+1 .. 32 (bits below 32-k)
        y2 = y ^ int(rng.integers(1, 2**(32 - k)))
        a, b = oracle.owen(y, seed), oracle.owen(y2, seed)
        assert (a >> (32 - k)) == (b >> (32 - k))
        # flipping digit k alone flips scrambled digit k
        y3 = y ^ (1 << (32 - k))
        c = oracle.owen(y3, seed)
        assert (a >> (32 - k)) ^ (c >> (32 - k)) == 1


def test_owen_scrambling_is_a_bijection_per_seed():
    seed = 0x9E3779B9
    ys = np.arange(1 << 16, dtype=np.uint64) << np.uint64(16)   # all 16-digit prefixes
    out = {oracle.owen(int(y), seed) >> 16 for y in ys}
    assert len(out) == 1 << 16


def test_owen_scrambling_depends_on_the_prefix():
    """Unlike a digital shift (one XOR pattern for every point), the flips
    of a digit change with the digits above it."""
    seed = 12345
    pats = {oracle.owen(y << 24, seed) ^ (y << 24) for y in range(256)}
    assert len(pats) > 64


@pytest.mark.parametrize("m", [4, 8, 11])
def test_owen_scrambled_points_remain_a_net(m):
    """Every scrambled 2^m prefix of a coordinate keeps one point per dyadic
    cell of width 2^-m, in every dimension, for several seeds."""
    n_dims = 12
    pts = oracle.sobol_points(n_dims, 0, 1 << m)
    for seed in (1, 77, 2**31 + 5):
        for j in range(n_dims):
            s = oracle.shift(seed, 3, j)
            cells = sorted(oracle.owen(int(y), s) >> (32 - m) for y in pts[:, j])
            assert cells == list(range(1 << m))


def test_owen_scrambled_digit_is_balanced_over_seeds():
    """For a fixed input, each scrambled digit is 0 or 1 with equal odds over
    random seeds (the scrambled point is uniform)."""
    rng = np.random.default_rng(3)
    seeds = rng.integers(0, 2**32, size=4000)
    for y in (0, 0x80000000, 0x12345678):
        outs = np.array([oracle.owen(y, int(sd)) for sd in seeds], dtype=np.uint64)
        for bit in (31, 27, 20, 12):
            frac = float(((outs >> np.uint64(bit)) & np.uint64(1)).mean())
            assert abs(frac - 0.5) < 0.04, (y, bit, frac)


def test_owen_rqmc_estimate_agrees_with_quadrature():
    """The scrambled estimator is unbiased: at d = 2 the mean over
    replications lies within 4 standard errors of quadrature."""
    S0, K, r, sig, T, d = 100.0, 103.0, 0.05, 0.25, 1.0, 2
    dt = T / d

    def G(zz, i):
        W = oracle.build_path(oracle.PATH_BB, 1, dt, np.array([zz]))
        return oracle.path_greeks(oracle.ARITH_ASIAN, d, S0, K, r, sig, T, W)[i] * scipy.stats.norm.pdf(zz)

    ref = np.array([scipy.integrate.quad(G, -40, 40, args=(i,), epsabs=0, epsrel=1e-13, limit=200)[0]
                    for i in range(4)])
    res = oracle.option(oracle.ARITH_ASIAN, d, S0, K, r, sig, T, 9191, 1 << 10, 32, oracle.PATH_BB,
                        oracle.RAND_OWEN)
    for i in range(4):
        assert abs(res["mean"][i] - ref[i]) <= 4 * res["stderr"][i] + 1e-13 * abs(ref[i]), i


def test_shifts_differ_between_replications_and_dims():
    s = oracle.shifts(77, 8, 64)
    assert len(np.unique(s)) == s.size


# --------------------------------------------------------------------------
# Inverse normal
# --------------------------------------------------------------------------


def test_norm_inv_matches_scipy():
    u = np.concatenate([np.linspace(0, 1, 4001)[1:-1], 10.0 ** -np.arange(1, 300, 0.5),
                        [0.075, 0.925, 0.425, 0.5 + 2**-33, 2**-33, 1 - 2**-33]])
    ref = scipy.special.ndtri(u)
    got = np.array([oracle.norm_inv(x) for x in u])
    err = np.abs(got - ref) / np.maximum(np.abs(ref), 1e-300)
    assert err.max() < 4e-15


def test_norm_inv_symmetry_and_centre():
    assert oracle.norm_inv(0.5) == 0.0
    for y in [0, 1, 12345, 2**31 - 1, 2**30 + 7]:
        u = (y + 0.5) / 2**32
        v = ((2**32 - 1 - y) + 0.5) / 2**32
        assert abs(oracle.norm_inv(u) + oracle.norm_inv(v)) <= 4e-16 * abs(oracle.norm_inv(u))


def test_norm_cdf_matches_scipy():
    # Phi(x) = erfc(-x/sqrt 2)/2: the rounding of x/sqrt 2 alone moves the tail
    # value by about x^2 ulp, so two correct implementations differ by that much
    for x in [-30.0, -8.0, -1.0, 0.0, 0.3, 5.0, 8.5]:
        ref = scipy.special.ndtr(x)
        assert abs(oracle.norm_cdf(x) - ref) <= 4e-16 * (1 + x * x) * ref


# --------------------------------------------------------------------------
# Path factor (Sec. 3.4.1: A A^T = Sigma)
# --------------------------------------------------------------------------


def _factor_matrix(path, n, dt):
    cols = []
    for i in range(n):
        e = np.zeros(n)
        e[i] = 1.0
        cols.append(oracle.build_path(path, n, dt, e)[1:])
    return np.array(cols).T


@pytest.mark.parametrize("path", [oracle.PATH_BB, oracle.PATH_STANDARD, oracle.PATH_PCA])
@pytest.mark.parametrize("n", [1, 2, 3, 7, 15, 16, 63, 100, 255])
def test_factor_reproduces_covariance(path, n):
    dt = 1.0 / (n + 1)
    A = _factor_matrix(path, n, dt)
    Sig = dt * np.minimum.outer(np.arange(1, n + 1), np.arange(1, n + 1)).astype(float)
    assert np.abs(A @ A.T - Sig).max() <= 1e-14 * Sig.max() * max(1, n / 16)


def test_bridge_terminal_and_first_midpoint():
    """The bridge puts the first normal on the terminal value and the second on
    the midpoint, each with its conditional variance (Sec. 4.4)."""
    n, dt = 63, 1 / 64
    z = np.zeros(n)
    z[0] = 1.3
    W = oracle.build_path(oracle.PATH_BB, n, dt, z)
    assert W[n] == pytest.approx(math.sqrt(n * dt) * 1.3, rel=1e-15)
    assert W[31] == pytest.approx(31 / 63 * W[n], rel=1e-14)
    z = np.zeros(n)
    z[1] = 1.0
    W = oracle.build_path(oracle.PATH_BB, n, dt, z)
    assert W[n] == 0.0
    assert W[31] == pytest.approx(math.sqrt(dt * 31 * 32 / 63), rel=1e-14)


@pytest.mark.parametrize("n", [7, 10])
def test_bridge_dimension_to_date_order(n, golden_dir):
    """Which normal drives which point (hand-derived table): the path of the
    unit vector e_j must be the hat function on (l, r) peaking at m with the
    conditional standard deviation sqrt(dt (m - l)(r - m)/(r - l)) -- or, for
    the terminal, the straight line to sqrt(n dt).  A swapped push order, a
    ceiling midpoint or a depth-first numbering all fail it."""
    dt = 0.1
    rows = [tuple(int(v) for v in r) for r in _read_rows(os.path.join(golden_dir, "bridge_order_n7_n10.txt"))]
    rows = [r for r in rows if r[0] == n]
    assert sorted(r[1] for r in rows) == list(range(1, n + 1))
    k = np.arange(n + 1, dtype=np.float64)
    for _, j, l, m, r in rows:
        z = np.zeros(n)
        z[j - 1] = 1.0
        W = oracle.build_path(oracle.PATH_BB, n, dt, z)
        if j == 1:
            want = k / n * math.sqrt(n * dt)
        else:
            peak = math.sqrt(dt * (m - l) * (r - m) / (r - l))
            want = np.where((k >= l) & (k <= m), (k - l) / (m - l), 0.0) + \
                np.where((k > m) & (k <= r), (r - k) / (r - m), 0.0)
            want = want * peak
        assert np.allclose(W, want, rtol=0, atol=1e-15), (n, j)


@pytest.mark.parametrize("n", [5, 63, 255, 364])
def test_pca_factor_matches_library_eigensolver(n):
    """The oracle's closed-form principal components must be the eigenpairs a
    library eigensolver finds for Sigma (decreasing eigenvalue, first entry of
    each eigenvector positive), within the solver's own error
    (eps * ||Sigma|| / eigenvalue gap for the eigenvectors)."""
    dt = 1.0 / (n + 1)
    A = oracle.pca_factor(n, dt)
    lam, vec = np.linalg.eigh(oracle.covariance(n, dt))
    order = np.argsort(lam)[::-1]
    lam, vec = lam[order], vec[:, order]
    vec = vec * np.where(vec[0, :] < 0, -1.0, 1.0)[None, :]
    lam_A = (A**2).sum(axis=0)
    assert np.abs(lam_A - lam).max() < 1e-13 * lam.max()
    assert np.all(np.diff(lam_A) < 0)
    assert np.all(A[0, :] > 0)
    assert np.abs(A - vec * np.sqrt(lam)[None, :]).max() < 1e-13 * n


# --------------------------------------------------------------------------
# Conditional payoff and Greeks (Sec. 3.4.2, Sec. 4.5)
# --------------------------------------------------------------------------


def _bs(S0, K, r, sig, T):
    d1 = (math.log(S0 / K) + (r + 0.5 * sig**2) * T) / (sig * math.sqrt(T))
    d2 = d1 - sig * math.sqrt(T)
    N, n = scipy.stats.norm.cdf, scipy.stats.norm.pdf
    call = [S0 * N(d1) - K * math.exp(-r * T) * N(d2), N(d1), S0 * n(d1) * math.sqrt(T),
            n(d1) / (S0 * sig * math.sqrt(T))]
    D = math.exp(-r * T)
    digital = [D * N(d2), D * n(d2) / (S0 * sig * math.sqrt(T)), -D * n(d2) * d1 / sig,
               -D * n(d2) * d1 / (S0**2 * sig**2 * T)]
    return np.array(call), np.array(digital)


@pytest.mark.parametrize("S0,K,r,sig,T", [(100, 100, 0.05, 0.2, 1.0), (100, 90, 0.1, 0.2, 1.0),
                                          (100, 120, 0.0, 0.5, 0.25), (80, 95, 0.08, 0.1, 2.0)])
def test_one_date_reduces_to_black_scholes(S0, K, r, sig, T):
    """With d = 1 the Asian average and the lookback maximum are S(T): the
    arithmetic Asian and lookback calls are the European call and the binary
    Asian is the cash-or-nothing digital, with exact Greeks and no noise."""
    call, digital = _bs(S0, K, r, sig, T)
    put, digital_put = _bs_put(S0, K, r, sig, T)
    for typ, ref in [(oracle.ARITH_ASIAN, call), (oracle.LOOKBACK, call), (oracle.BINARY_ASIAN, digital),
                     (oracle.GEOMETRIC_ASIAN, call), (oracle.ARITH_ASIAN_PUT, put), (oracle.LOOKBACK_PUT, put),
                     (oracle.GEOMETRIC_ASIAN_PUT, put), (oracle.BINARY_ASIAN_PUT, digital_put)]:
        res = oracle.option(typ, 1, S0, K, r, sig, T, 99, 8, 4)
        assert np.allclose(res["mean"], ref, rtol=2e-13, atol=1e-14 * S0), (typ, res["mean"], ref)
        assert np.all(res["stderr"] == 0)


def _bs_put(S0, K, r, sig, T):
    """European put and cash-or-nothing put (pays 1 below K): price, delta, vega, gamma."""
    d1 = (math.log(S0 / K) + (r + sig**2 / 2) * T) / (sig * math.sqrt(T))
    d2 = d1 - sig * math.sqrt(T)
    N, n = scipy.stats.norm.cdf, scipy.stats.norm.pdf
    D = math.exp(-r * T)
    put = [K * D * N(-d2) - S0 * N(-d1), -N(-d1), S0 * n(d1) * math.sqrt(T), n(d1) / (S0 * sig * math.sqrt(T))]
    digital = [D * N(-d2), -D * n(d2) / (S0 * sig * math.sqrt(T)), D * n(d2) * d1 / sig,
               D * n(d2) * d1 / (S0**2 * sig**2 * T)]
    return np.array(put), np.array(digital)


def _fd_check(typ, d, path, z, S0=100.0, K=100.0, r=0.05, sig=0.2, T=1.0):
    n = d - 1
    dt = T / d
    W = oracle.build_path(path, n, dt, z)
    g = oracle.path_greeks(typ, d, S0, K, r, sig, T, W)
    s1 = sig * math.sqrt(dt)

    def price(s0, sg):
        # the path W~ is fixed (same z); S0 and sigma are bumped
        return oracle.path_greeks(typ, d, s0, K, r, sg, T, W)[0]

    def richardson(f, x, h):
        a = (f(x + h) - f(x - h)) / (2 * h)
        b = (f(x + h / 2) - f(x - h / 2)) / h
        return (4 * b - a) / 3

    hS = 1e-3 * S0 * s1
    delta = richardson(lambda s: price(s, sig), S0, hS)
    # gamma as the S0-derivative of the pathwise delta (itself pinned to the
    # price just above); a second difference of a deep in-the-money price
    # would lose the small gamma to rounding
    gamma = richardson(lambda s: oracle.path_greeks(typ, d, s, K, r, sig, T, W)[1], S0, hS)
    hs = 1e-3 * s1 * sig
    vega = richardson(lambda s: price(S0, s), sig, hs)
    # rounding floor of each difference quotient: ~eps * |f| / h
    eps = np.finfo(float).eps
    floor = np.array([0.0, 50 * eps * (abs(g[0]) + K) / hS, 50 * eps * (abs(g[0]) + K) / hs,
                      50 * eps * abs(g[1]) / hS])
    return g, np.array([g[0], delta, vega, gamma]), floor


ALL_TYPES = [oracle.ARITH_ASIAN, oracle.BINARY_ASIAN, oracle.LOOKBACK, oracle.GEOMETRIC_ASIAN,
             oracle.ARITH_ASIAN_PUT, oracle.BINARY_ASIAN_PUT, oracle.LOOKBACK_PUT, oracle.GEOMETRIC_ASIAN_PUT]
PUTS = (oracle.ARITH_ASIAN_PUT, oracle.BINARY_ASIAN_PUT, oracle.LOOKBACK_PUT, oracle.GEOMETRIC_ASIAN_PUT)


@pytest.mark.parametrize("typ", ALL_TYPES)
@pytest.mark.parametrize("d,path", [(2, oracle.PATH_BB), (12, oracle.PATH_BB), (64, oracle.PATH_BB),
                                    (17, oracle.PATH_STANDARD), (33, oracle.PATH_PCA)])
def test_greeks_equal_finite_differences_of_conditional_price(typ, d, path):
    rng = np.random.default_rng(1000 * d + typ)
    for trial in range(4):
        z = rng.standard_normal(d - 1)
        g, fd, floor = _fd_check(typ, d, path, z, K=[90.0, 100.0, 110.0, 100.0][trial])
        for i in (1, 2, 3):
            assert abs(g[i] - fd[i]) <= 1e-6 * abs(fd[i]) + floor[i], (i, g, fd)


def test_lookback_vega_has_no_one_over_d():
    """The printed lookback vega divides by d; finite differences reject that."""
    d = 24
    z = np.random.default_rng(5).standard_normal(d - 1)
    g, fd, _ = _fd_check(oracle.LOOKBACK, d, oracle.PATH_BB, z, K=95.0)
    assert abs(g[2] - fd[2]) < 1e-6 * abs(fd[2])
    assert abs(fd[2]) > 2.0 * abs(fd[2] - 0.0) / d


@pytest.mark.parametrize("typ", ALL_TYPES)
@pytest.mark.parametrize("K", [90.0, 100.0, 115.0])
def test_conditional_price_is_quadrature_of_unconditioned_payoff(typ, K):
    """G(theta, z) = E[discounted payoff | z]: integrate the original payoff
    over the conditioned normal x_1 numerically, with the breakpoint found by
    root-finding on the path, and compare with the oracle's closed form."""
    S0, r, sig, T, d = 100.0, 0.05, 0.3, 1.0, 10
    dt = T / d
    rng = np.random.default_rng(int(K) + 7 * typ)
    for _ in range(3):
        z = rng.standard_normal(d - 1)
        Wt = oracle.build_path(oracle.PATH_BB, d - 1, dt, z)
        t = dt * np.arange(1, d + 1)

        def stat(x1):
            # Black-Scholes path: W(t_j) = sqrt(t_1) x_1 + W~(t_j - t_1)
            W = math.sqrt(dt) * x1 + Wt
            S = S0 * np.exp((r - 0.5 * sig**2) * t + sig * W)
            if typ in (oracle.GEOMETRIC_ASIAN, oracle.GEOMETRIC_ASIAN_PUT):
                return math.exp(np.log(S).mean())
            if typ == oracle.LOOKBACK:
                return S.max()
            return S.min() if typ == oracle.LOOKBACK_PUT else S.mean()

        def payoff(x1):
            A = stat(x1)
            if typ == oracle.BINARY_ASIAN:
                return math.exp(-r * T) * (1.0 if A > K else 0.0)
            if typ == oracle.BINARY_ASIAN_PUT:
                return math.exp(-r * T) * (1.0 if A < K else 0.0)
            if typ in PUTS:
                return math.exp(-r * T) * max(K - A, 0.0)
            return math.exp(-r * T) * max(A - K, 0.0)

        root = scipy.optimize.brentq(lambda x: stat(x) - K, -60, 60, xtol=1e-15, rtol=1e-15)
        f = lambda x: payoff(x) * scipy.stats.norm.pdf(x)
        lo, hi = (-40, root) if typ in PUTS else (root, 40)
        val = scipy.integrate.quad(f, lo, hi, epsabs=0, epsrel=1e-13, limit=200)[0]
        g = oracle.path_greeks(typ, d, S0, K, r, sig, T, Wt)
        assert abs(g[0] - val) <= 1e-10 * max(abs(val), 1e-12) + 1e-13 * K, (g[0], val)
        # the breakpoint itself: binary price is e^{-rT} (1 - Phi(psi))
        if typ == oracle.BINARY_ASIAN:
            psi = -scipy.special.ndtri(g[0] / math.exp(-r * T))
            assert abs(psi - root) < 1e-8 * max(1, abs(root))


@pytest.mark.parametrize("typ", [oracle.ARITH_ASIAN, oracle.BINARY_ASIAN, oracle.LOOKBACK])
def test_rqmc_estimate_agrees_with_quadrature_at_two_dates(typ):
    """d = 2 leaves one conditioned and one sampled normal: E_z[G] and E_z[dG]
    by adaptive quadrature must lie within 4 standard errors of the
    randomised QMC estimate (Sobol + shift + inverse normal + bridge)."""
    S0, K, r, sig, T, d = 100.0, 105.0, 0.05, 0.25, 1.0, 2
    dt = T / d

    def G(zz, i):
        W = oracle.build_path(oracle.PATH_BB, 1, dt, np.array([zz]))
        return oracle.path_greeks(typ, d, S0, K, r, sig, T, W)[i] * scipy.stats.norm.pdf(zz)

    # the lookback maximum switches date where S~(t_2) = S0, i.e. at
    # z = -omega*dt / (sigma*sqrt(dt)); split the integral there
    kink = -(r - 0.5 * sig**2) * dt / (sig * math.sqrt(dt))
    ref = np.array([scipy.integrate.quad(G, -40, kink, args=(i,), epsabs=0, epsrel=1e-13, limit=200)[0] +
                    scipy.integrate.quad(G, kink, 40, args=(i,), epsabs=0, epsrel=1e-13, limit=200)[0]
                    for i in range(4)])
    res = oracle.option(typ, d, S0, K, r, sig, T, 4242, 1 << 12, 16)
    for i in range(4):
        assert abs(res["mean"][i] - ref[i]) <= 4 * res["stderr"][i] + 1e-13 * abs(ref[i]), i
        assert res["stderr"][i] < 1e-3 * max(abs(ref[i]), 1e-6)


def test_rqmc_estimate_agrees_with_quadrature_at_three_dates():
    S0, K, r, sig, T, d = 100.0, 95.0, 0.03, 0.3, 0.5, 3
    x, w = np.polynomial.hermite_e.hermegauss(64)
    w = w / w.sum()
    ref = np.zeros(4)
    for a, wa in zip(x, w):
        for b, wb in zip(x, w):
            W = oracle.build_path(oracle.PATH_BB, 2, T / d, np.array([a, b]))
            ref += wa * wb * oracle.path_greeks(oracle.ARITH_ASIAN, d, S0, K, r, sig, T, W)
    res = oracle.option(oracle.ARITH_ASIAN, d, S0, K, r, sig, T, 11, 1 << 12, 16)
    for i in range(4):
        assert abs(res["mean"][i] - ref[i]) <= 4 * res["stderr"][i] + 1e-13 * abs(ref[i])


# --------------------------------------------------------------------------
# Geometric Asian call: exact lognormal closed form at any d
# --------------------------------------------------------------------------

@pytest.mark.parametrize("path", [oracle.PATH_BB, oracle.PATH_STANDARD, oracle.PATH_PCA])
def test_put_call_parity_per_path(path):
    """(X - K)^+ - (K - X)^+ = X - K path by path, so the conditional call
    minus the conditional put is e^{r(t1-T)} X - e^{-rT} K for the average,
    the geometric mean and the lookback (max for the call, min for the put:
    a different X, checked through the binary pair), and the binary call
    plus the binary put is e^{-rT}."""
    S0, r, sig, T, d = 100.0, 0.04, 0.25, 1.5, 20
    dt = T / d
    D, D1 = math.exp(-r * T), math.exp(r * (dt - T))
    rng = np.random.default_rng(77 + path)
    for K in (85.0, 100.0, 120.0):
        z = rng.standard_normal(d - 1)
        W = oracle.build_path(path, d - 1, dt, z)
        tau = dt * np.arange(d)
        S = S0 * np.exp((r - sig**2 / 2) * tau + sig * W)
        VS = S * (W - sig * tau)
        for call, put, X, VX in [(oracle.ARITH_ASIAN, oracle.ARITH_ASIAN_PUT, S.mean(), VS.mean()),
                                 (oracle.GEOMETRIC_ASIAN, oracle.GEOMETRIC_ASIAN_PUT, math.exp(np.log(S).mean()),
                                  math.exp(np.log(S).mean()) * (W - sig * tau).mean())]:
            gc = oracle.path_greeks(call, d, S0, K, r, sig, T, W)
            gp = oracle.path_greeks(put, d, S0, K, r, sig, T, W)
            np.testing.assert_allclose(gc - gp, [D1 * X - D * K, D1 * X / S0, D1 * VX, 0.0], rtol=1e-12,
                                       atol=1e-12 * (S0 + K))
        j = int(np.argmin(S))
        gp = oracle.path_greeks(oracle.LOOKBACK_PUT, d, S0, K, r, sig, T, W)
        gb = oracle.path_greeks(oracle.BINARY_ASIAN, d, S0, K, r, sig, T, W)
        gbp = oracle.path_greeks(oracle.BINARY_ASIAN_PUT, d, S0, K, r, sig, T, W)
        np.testing.assert_allclose(gb + gbp, [D, 0.0, 0.0, 0.0], rtol=0, atol=1e-14)
        # lookback put through its own breakpoint on the minimum: the price is
        # the closed-form put on X = min S~ (checked here against the call on
        # the same X via the generic put-call identity of the conditional payoff)
        s1 = sig * math.sqrt(dt)
        psi = (math.log(K) - math.log(S[j]) - (r - sig**2 / 2) * dt) / s1
        N = scipy.stats.norm.cdf
        call_on_min = D1 * S[j] * N(s1 - psi) - D * K * N(-psi)
        assert abs((call_on_min - gp[0]) - (D1 * S[j] - D * K)) <= 1e-12 * (S0 + K)


@pytest.mark.parametrize("d,path", [(1, oracle.PATH_BB), (12, oracle.PATH_BB), (64, oracle.PATH_BB),
                                    (20, oracle.PATH_STANDARD)])
def test_geometric_put_estimate_matches_closed_form(d, path):
    """The geometric put estimate against the lognormal closed form (put-call
    parity of the discretely monitored geometric average), within 4 stderr."""
    S0, K, r, sig, T = 100.0, 103.0, 0.05, 0.3, 1.0
    c = geometric_asian_closed_form(S0, K, r, sig, T, d)
    dt = T / d
    tbar = dt * (d + 1) / 2
    v2 = sig**2 * dt * (d + 1) * (2 * d + 1) / (6 * d)
    F = math.exp(math.log(S0) + (r - sig**2 / 2) * tbar + v2 / 2)     # E[G]
    D = math.exp(-r * T)
    # put = call - D (E[G] - K): delta - D F/S0, vega - D dF/dsigma, gamma unchanged
    dF_dsig = F * (-sig * tbar + sig * (d + 1) * (2 * d + 1) * dt / (6 * d))
    ref = c - np.array([D * (F - K), D * F / S0, D * dF_dsig, 0.0])
    res = oracle.option(oracle.GEOMETRIC_ASIAN_PUT, d, S0, K, r, sig, T, 4711, 1 << 12, 16, path)
    for i in range(4):
        assert abs(res["mean"][i] - ref[i]) <= 4 * res["stderr"][i] + 1e-12 * abs(ref[i]), (i, res["mean"], ref)


def test_geometric_closed_form_by_quadrature():
    """The closed form above against direct quadrature of the lognormal
    payoff, and its Greeks against finite differences of its price."""
    S0, K, r, sig, T, d = 100.0, 104.0, 0.04, 0.3, 1.5, 9
    ref = geometric_asian_closed_form(S0, K, r, sig, T, d)
    dt = T / d
    mu = math.log(S0) + (r - sig**2 / 2) * dt * (d + 1) / 2
    v = sig * math.sqrt(dt * (d + 1) * (2 * d + 1) / (6 * d))
    f = lambda x: max(math.exp(mu + v * x) - K, 0.0) * scipy.stats.norm.pdf(x)
    price = math.exp(-r * T) * scipy.integrate.quad(f, (math.log(K) - mu) / v, 40, epsrel=1e-13)[0]
    assert abs(price - ref[0]) < 1e-11 * ref[0]
    h = 1e-4
    fd = [(geometric_asian_closed_form(S0 + h, K, r, sig, T, d)[0] -
           geometric_asian_closed_form(S0 - h, K, r, sig, T, d)[0]) / (2 * h),
          (geometric_asian_closed_form(S0, K, r, sig + h, T, d)[0] -
           geometric_asian_closed_form(S0, K, r, sig - h, T, d)[0]) / (2 * h),
          (geometric_asian_closed_form(S0 + h, K, r, sig, T, d)[1] -
           geometric_asian_closed_form(S0 - h, K, r, sig, T, d)[1]) / (2 * h)]
    np.testing.assert_allclose(ref[1:], fd, rtol=1e-7)


@pytest.mark.parametrize("d,path", [(1, oracle.PATH_BB), (12, oracle.PATH_BB), (64, oracle.PATH_BB),
                                    (20, oracle.PATH_STANDARD), (16, oracle.PATH_PCA)])
def test_geometric_estimate_matches_closed_form(d, path):
    """The QMC-CPW estimate of the geometric Asian call is unbiased for the
    exact price and Greeks: within 4 standard errors (plus 1e-12) at any d."""
    S0, K, r, sig, T = 100.0, 98.0, 0.05, 0.25, 1.0
    ref = geometric_asian_closed_form(S0, K, r, sig, T, d)
    res = oracle.option(oracle.GEOMETRIC_ASIAN, d, S0, K, r, sig, T, 4711, 1 << 12, 16, path)
    for i in range(4):
        assert abs(res["mean"][i] - ref[i]) <= 4 * res["stderr"][i] + 1e-12 * abs(ref[i]), (i, res["mean"], ref)


# --------------------------------------------------------------------------
# Conditioning on the first principal component of the full covariance
# --------------------------------------------------------------------------

def _full_path(d, T, rng):
    A = oracle.pca_factor(d, T / d)
    z = rng.standard_normal(d - 1)
    return A[:, 0].copy(), A[:, 1:] @ z


@pytest.mark.parametrize("S0,K,r,sig,T", [(100, 100, 0.05, 0.2, 1.0), (100, 90, 0.1, 0.2, 1.0),
                                          (100, 120, 0.02, 0.4, 0.5)])
def test_full_pca_one_date_is_black_scholes(S0, K, r, sig, T):
    """d = 1 leaves only the conditioned component: the estimate is the
    Black-Scholes call (arithmetic average or maximum of one date) /
    cash-or-nothing digital and their Greeks."""
    d1 = (math.log(S0 / K) + (r + sig**2 / 2) * T) / (sig * math.sqrt(T))
    d2 = d1 - sig * math.sqrt(T)
    D = math.exp(-r * T)
    N, n = scipy.stats.norm.cdf, scipy.stats.norm.pdf
    call = [S0 * N(d1) - K * D * N(d2), N(d1), S0 * math.sqrt(T) * n(d1), n(d1) / (S0 * sig * math.sqrt(T))]
    dig = [D * N(d2), D * n(d2) / (S0 * sig * math.sqrt(T)), -D * n(d2) * d1 / sig,
           -D * n(d2) * d1 / (S0 * S0 * sig * sig * T)]
    for typ, ref in ((oracle.ARITH_ASIAN, call), (oracle.BINARY_ASIAN, dig), (oracle.LOOKBACK, call)):
        res = oracle.option(typ, 1, S0, K, r, sig, T, 99, 64, 2, oracle.PATH_PCA_FULL)
        np.testing.assert_allclose(res["mean"], ref, rtol=1e-12, atol=1e-15)


@pytest.mark.parametrize("d", [2, 5, 16, 64])
def test_full_pca_root_matches_bracketing_solver(d):
    rng = np.random.default_rng(d)
    S0, r, sig, T = 100.0, 0.05, 0.3, 1.0
    for K in (60.0, 100.0, 160.0):
        a, c = _full_path(d, T, rng)
        t = T / d * np.arange(1, d + 1)
        al = math.log(S0) + (r - sig**2 / 2) * t + sig * c
        be = sig * a
        f = lambda x: np.mean(np.exp(al + be * x)) - K
        ref = scipy.optimize.brentq(f, -80, 80, xtol=1e-15, rtol=1e-15)
        assert abs(oracle.full_root(al, be, K) - ref) <= 1e-12 * max(1.0, abs(ref))


@pytest.mark.parametrize("typ", [oracle.ARITH_ASIAN, oracle.BINARY_ASIAN, oracle.LOOKBACK])
@pytest.mark.parametrize("d", [2, 7, 32])
def test_full_pca_greeks_equal_finite_differences(typ, d):
    """Per path, the pathwise delta, vega and gamma equal Richardson finite
    differences of the conditional price with the other components fixed."""
    rng = np.random.default_rng(31 * d + typ)
    T, r = 1.0, 0.05
    for trial in range(3):
        a, c = _full_path(d, T, rng)
        S0, K, sig = 100.0, [90.0, 100.0, 112.0][trial], [0.15, 0.25, 0.4][trial]
        g = oracle.path_greeks_full(typ, d, S0, K, r, sig, T, a, c)

        def rich(f, x, h):
            A1 = (f(x + h) - f(x - h)) / (2 * h)
            B1 = (f(x + h / 2) - f(x - h / 2)) / h
            return (4 * B1 - A1) / 3

        pr = lambda s0, sg: oracle.path_greeks_full(typ, d, s0, K, r, sg, T, a, c)
        hS, hs = 1e-3 * S0 * sig, 1e-4
        delta = rich(lambda s0: pr(s0, sig)[0], S0, hS)
        vega = rich(lambda sg: pr(S0, sg)[0], sig, hs)
        gamma = rich(lambda s0: pr(s0, sig)[1], S0, hS)
        eps = np.finfo(float).eps
        for got, fd, h, scale in ((g[1], delta, hS, abs(g[0]) + K), (g[2], vega, hs, abs(g[0]) + K),
                                  (g[3], gamma, hS, abs(g[1]))):
            assert abs(got - fd) <= 1e-6 * abs(fd) + 50 * eps * scale / h, (typ, d, got, fd)


@pytest.mark.parametrize("typ", [oracle.ARITH_ASIAN, oracle.BINARY_ASIAN, oracle.LOOKBACK])
def test_full_pca_conditional_price_is_quadrature_of_payoff(typ):
    """G = E[discounted payoff | other components]: integrate the original
    payoff (average, or maximum over the dates) over the first component
    numerically and compare."""
    S0, r, sig, T, d = 100.0, 0.05, 0.3, 1.0, 12
    rng = np.random.default_rng(12 + typ)
    t = T / d * np.arange(1, d + 1)
    stat = np.max if typ == oracle.LOOKBACK else np.mean
    for K in (85.0, 100.0, 120.0):
        a, c = _full_path(d, T, rng)
        avg = lambda x: stat(S0 * np.exp((r - sig**2 / 2) * t + sig * (a * x + c)))
        root = scipy.optimize.brentq(lambda x: avg(x) - K, -60, 60, xtol=1e-15, rtol=1e-15)
        if typ == oracle.BINARY_ASIAN:
            f = lambda x: math.exp(-r * T) * scipy.stats.norm.pdf(x)
        else:
            f = lambda x: math.exp(-r * T) * (avg(x) - K) * scipy.stats.norm.pdf(x)
        val = scipy.integrate.quad(f, root, 40, epsabs=0, epsrel=1e-13, limit=200)[0]
        g = oracle.path_greeks_full(typ, d, S0, K, r, sig, T, a, c)
        assert abs(g[0] - val) <= 1e-10 * max(abs(val), 1e-12), (g[0], val)


@pytest.mark.parametrize("typ", [oracle.ARITH_ASIAN, oracle.BINARY_ASIAN, oracle.LOOKBACK])
def test_full_pca_estimate_agrees_with_first_date_conditioning(typ):
    """Two different conditional estimators of the same Greeks -- the first
    principal component integrated out, or the first date's normal with a
    bridge for the rest -- must agree within their standard errors."""
    S0, K, r, sig, T, d = 100.0, 102.0, 0.05, 0.3, 1.0, 8
    a = oracle.option(typ, d, S0, K, r, sig, T, 71, 1 << 13, 16, oracle.PATH_PCA_FULL)
    b = oracle.option(typ, d, S0, K, r, sig, T, 72, 1 << 13, 16, oracle.PATH_BB)
    for i in range(4):
        tol = 4 * math.hypot(a["stderr"][i], b["stderr"][i]) + 1e-12 * abs(b["mean"][i])
        assert abs(a["mean"][i] - b["mean"][i]) <= tol, (i, a["mean"], b["mean"])


def test_full_pca_estimate_agrees_with_quadrature_at_two_dates():
    """d = 2: one conditioned and one sampled component; E over the sampled
    one by quadrature lies within 4 standard errors of the estimate."""
    S0, K, r, sig, T, d = 100.0, 97.0, 0.04, 0.25, 1.0, 2
    A = oracle.pca_factor(d, T / d)

    def G(zz, i):
        return oracle.path_greeks_full(oracle.ARITH_ASIAN, d, S0, K, r, sig, T, A[:, 0].copy(),
                                       A[:, 1] * zz)[i] * scipy.stats.norm.pdf(zz)

    ref = np.array([scipy.integrate.quad(G, -40, 40, args=(i,), epsabs=0, epsrel=1e-13, limit=200)[0]
                    for i in range(4)])
    res = oracle.option(oracle.ARITH_ASIAN, d, S0, K, r, sig, T, 5151, 1 << 12, 16, oracle.PATH_PCA_FULL)
    for i in range(4):
        assert abs(res["mean"][i] - ref[i]) <= 4 * res["stderr"][i] + 1e-13 * abs(ref[i]), i


def test_full_pca_lookback_envelope_against_brute_force():
    """The lookback's conditional price on one path, by its envelope walk,
    against the same integral done line by line on a fine grid of x: at every
    x the payoff is (max over dates - K)^+, integrated by a composite rule
    over [psi, 12] with the breakpoints of the envelope found by brute force
    (where the argmax over the dates changes), so a wrong segment or line
    shows.  Also: psi is the smallest of the lines' own crossings of ln K."""
    S0, r, sig, T, d = 100.0, 0.03, 0.35, 1.5, 40
    rng = np.random.default_rng(4040)
    t = T / d * np.arange(1, d + 1)
    for K in (95.0, 110.0, 140.0):
        a, c = _full_path(d, T, rng)
        al = math.log(S0) + (r - sig**2 / 2) * t + sig * c
        be = sig * a
        psi = np.min((math.log(K) - al) / be)
        assert abs(np.max(al + be * psi) - math.log(K)) <= 1e-12
        xs = np.linspace(psi, 12.0, 400001)
        top = np.argmax(al[None, :] + be[None, :] * xs[:, None], axis=1)
        cuts = [psi] + [0.5 * (xs[i] + xs[i + 1]) for i in np.nonzero(np.diff(top))[0]] + [12.0]
        val = 0.0
        for lo, hi in zip(cuts[:-1], cuts[1:]):
            j = top[np.searchsorted(xs, 0.5 * (lo + hi))]
            f = lambda x: (math.exp(al[j] + be[j] * x) - K) * scipy.stats.norm.pdf(x)
            val += scipy.integrate.quad(f, lo, hi, epsabs=0, epsrel=1e-12, limit=200)[0]
        g = oracle.path_greeks_full(oracle.LOOKBACK, d, S0, K, r, sig, T, a, c)
        # the grid locates breakpoints to 1e-4 in x; the payoff is continuous there
        assert abs(g[0] / math.exp(-r * T) - val) <= 1e-6 * max(abs(val), 1e-3), (K, g[0], val)


# --------------------------------------------------------------------------
# Reduction across replications (Sec. 5)
# --------------------------------------------------------------------------


def test_replication_statistics():
    res = oracle.option(oracle.ARITH_ASIAN, 8, 100, 100, 0.05, 0.2, 1.0, 5, 256, 6)
    Cl = res["C_l"]
    assert np.allclose(res["mean"], Cl.mean(axis=0), rtol=1e-15)
    se = np.sqrt(((Cl - Cl.mean(axis=0)) ** 2).sum(axis=0) / (6 * 5))
    assert np.allclose(res["stderr"], se, rtol=1e-12)
    one = oracle.option(oracle.ARITH_ASIAN, 8, 100, 100, 0.05, 0.2, 1.0, 5, 256, 1)
    assert np.all(np.isnan(one["stderr"]))
    assert np.allclose(one["mean"], Cl[0], rtol=1e-15)


def test_ragged_point_count_and_many_options():
    import workloads
    opts = workloads.three_products_grid(d=9, n_points=777)
    mean, se, am, used = oracle.options(opts, L=4, n_threads=2)
    for i in (0, 7, 17):
        o = opts[i]
        one = oracle.option(o["type"], o["d"], o["S0"], o["K"], o["r"], o["sigma"], o["T"],
                            o["seed"], o["n_points"], 4)
        assert np.array_equal(one["mean"], mean[i])
    assert used >= 1
    assert np.all(am >= np.abs(mean) * (1 - 1e-12))


# --------------------------------------------------------------------------
# Basket of M assets, one-factor model (standard construction)
# --------------------------------------------------------------------------
def _basket_paths(d, M, T, rng):
    dt = T / d
    W0 = np.concatenate([[0.0], np.cumsum(math.sqrt(dt) * rng.standard_normal(d - 1))])
    Bi = np.cumsum(math.sqrt(dt) * rng.standard_normal((M, d)), axis=1)
    return W0, Bi


@pytest.mark.parametrize("typ,single", [(oracle.BASKET_ASIAN, oracle.ARITH_ASIAN),
                                        (oracle.BASKET_ASIAN_PUT, oracle.ARITH_ASIAN_PUT)])
@pytest.mark.parametrize("d,M", [(1, 1), (12, 1), (12, 3), (40, 5)])
def test_basket_with_full_correlation_is_the_single_asset(typ, single, d, M):
    """rho = 1: every asset follows B_0, the basket average is the single
    asset's average, and the estimator (same common dimensions 1..d-1,
    standard construction) reproduces the single-asset estimate."""
    S0, K, r, sig, T = 100.0, 104.0, 0.05, 0.25, 1.2
    b = oracle.basket_option(typ, d, M, 1.0, S0, K, r, sig, T, 31, 2048, 4)
    a = oracle.option(single, d, S0, K, r, sig, T, 31, 2048, 4, oracle.PATH_STANDARD)
    np.testing.assert_allclose(b["mean"], a["mean"], rtol=1e-12, atol=1e-13 * S0)


@pytest.mark.parametrize("typ", [oracle.BASKET_ASIAN, oracle.BASKET_ASIAN_PUT])
@pytest.mark.parametrize("d,M,rho", [(1, 2, 0.5), (8, 3, 0.3), (24, 4, 0.8), (12, 2, 0.05)])
def test_basket_greeks_equal_finite_differences(typ, d, M, rho):
    """Per path, delta, vega and gamma are the S0 and sigma derivatives of the
    conditional price with the Brownian paths fixed (catches the sigma
    dependence of e^{a + s1^2/2} when rho < 1)."""
    S0, r, sig, T = 100.0, 0.05, 0.2, 1.0
    rng = np.random.default_rng(100 * d + M)
    for K in (90.0, 100.0, 112.0):
        W0, Bi = _basket_paths(d, M, T, rng)
        g = oracle.basket_path_greeks(typ, d, M, rho, S0, K, r, sig, T, W0, Bi)
        price = lambda s0, sg: oracle.basket_path_greeks(typ, d, M, rho, s0, K, r, sg, T, W0, Bi)[0]
        hS, hs = 1e-3, 1e-5
        delta = (price(S0 + hS, sig) - price(S0 - hS, sig)) / (2 * hS)
        vega = (price(S0, sig + hs) - price(S0, sig - hs)) / (2 * hs)
        gamma = (oracle.basket_path_greeks(typ, d, M, rho, S0 + hS, K, r, sig, T, W0, Bi)[1] -
                 oracle.basket_path_greeks(typ, d, M, rho, S0 - hS, K, r, sig, T, W0, Bi)[1]) / (2 * hS)
        np.testing.assert_allclose(g[1:], [delta, vega, gamma], rtol=2e-6, atol=1e-9)


@pytest.mark.parametrize("typ", [oracle.BASKET_ASIAN, oracle.BASKET_ASIAN_PUT])
@pytest.mark.parametrize("K", [92.0, 101.0, 115.0])
def test_basket_conditional_price_is_quadrature_of_the_payoff(typ, K):
    """G = E[discounted payoff | paths without x_1]: integrate the basket
    payoff over x_1 (B_0(t_j) = sqrt(t_1) x_1 + B~_0(tau_j)) numerically, the
    breakpoint by root-finding."""
    S0, r, sig, T, d, M, rho = 100.0, 0.04, 0.3, 1.0, 6, 3, 0.6
    dt = T / d
    t = dt * np.arange(1, d + 1)
    rng = np.random.default_rng(int(K))
    for _ in range(3):
        W0, Bi = _basket_paths(d, M, T, rng)

        def avg(x):
            B0 = math.sqrt(dt) * x + W0
            S = S0 * np.exp((r - sig**2 / 2) * t[None, :] + sig * (math.sqrt(rho) * B0[None, :] +
                                                                    math.sqrt(1 - rho) * Bi))
            return S.mean()

        root = scipy.optimize.brentq(lambda x: avg(x) - K, -80, 80, xtol=1e-15, rtol=1e-15)
        D = math.exp(-r * T)
        if typ == oracle.BASKET_ASIAN:
            f = lambda x: D * max(avg(x) - K, 0.0) * scipy.stats.norm.pdf(x)
            val = scipy.integrate.quad(f, root, 60, epsabs=0, epsrel=1e-13, limit=200)[0]
        else:
            f = lambda x: D * max(K - avg(x), 0.0) * scipy.stats.norm.pdf(x)
            val = scipy.integrate.quad(f, -60, root, epsabs=0, epsrel=1e-13, limit=200)[0]
        g = oracle.basket_path_greeks(typ, d, M, rho, S0, K, r, sig, T, W0, Bi)
        assert abs(g[0] - val) <= 1e-10 * max(abs(val), 1e-12) + 1e-13 * K, (g[0], val)


def test_basket_estimate_agrees_with_quadrature_one_date_two_assets():
    """d = 1, M = 2: the conditioned common normal is integrated in closed
    form and the two idiosyncratic normals are sampled; E over them of the
    conditional price and Greeks by 64 x 64 Gauss-Hermite quadrature must lie
    within 4 standard errors of the randomised QMC estimate."""
    S0, K, r, sig, T, rho = 100.0, 98.0, 0.03, 0.35, 0.75, 0.4
    x, w = np.polynomial.hermite_e.hermegauss(64)
    w = w / w.sum()
    for typ in (oracle.BASKET_ASIAN, oracle.BASKET_ASIAN_PUT):
        ref = np.zeros(4)
        for a, wa in zip(x, w):
            for b, wb in zip(x, w):
                Bi = math.sqrt(T) * np.array([[a], [b]])
                ref += wa * wb * oracle.basket_path_greeks(typ, 1, 2, rho, S0, K, r, sig, T, np.zeros(1), Bi)
        res = oracle.basket_option(typ, 1, 2, rho, S0, K, r, sig, T, 515, 1 << 12, 16)
        for i in range(4):
            assert abs(res["mean"][i] - ref[i]) <= 4 * res["stderr"][i] + 1e-12 * abs(ref[i]), (typ, i)
            assert res["stderr"][i] < 2e-3 * max(abs(ref[i]), 1e-6)
