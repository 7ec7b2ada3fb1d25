"""FP64 CPU oracle for the QMC-CPW Greeks estimator (arXiv 2209.11337).

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the benchmark's
CPU-baseline leg are the only callers.  The product path never imports this
package, and this package never imports the product package.  It shares no
code, table or constant generator with the HIP library.

The numerical work lives in ``oracle.c`` (plain C, FP64, one path at a time in
the paper's order).  This wrapper only marshals arguments and supplies two
inputs the C code takes from outside:

* the raw Joe-Kuo primitive polynomials and initial direction numbers
  (``new-joe-kuo-6.21201``) read from scipy's data file -- the paper says only
  that the initial direction numbers must be chosen (Sec. 2.2.2); the
  recurrence that turns them into direction numbers runs in ``oracle.c``;
* nothing else: the principal-component factor of the Brownian covariance
  (Sec. 3.4.1, A A^T = Sigma) is built in ``oracle.c`` from the closed-form
  eigenpairs of Sigma; the tests pin it against a library eigensolver.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_JK_NPZ = None
_lock = threading.Lock()
_lib = None

ARITH_ASIAN, BINARY_ASIAN, LOOKBACK, GEOMETRIC_ASIAN = 0, 1, 2, 3
ARITH_ASIAN_PUT, BINARY_ASIAN_PUT, LOOKBACK_PUT, GEOMETRIC_ASIAN_PUT = 4, 5, 6, 7
BASKET_ASIAN, BASKET_ASIAN_PUT = 8, 9
PATH_BB, PATH_PCA, PATH_STANDARD, PATH_PCA_FULL = 0, 1, 2, 3
RAND_SHIFT, RAND_OWEN = 0, 1
OUTPUTS = ("price", "delta", "vega", "gamma")


def build(force: bool = False) -> str:
    """Compile oracle.c into liboracle.so with gcc (-O2, OpenMP)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-fopenmp", "-fPIC", "-shared",
                               "-D_GNU_SOURCE", _SRC, "-o", tmp, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    with _lock:
        if _lib is None:
            build()
            lib = C.CDLL(_LIB)
            u32p = np.ctypeslib.ndpointer(np.uint32, flags="C_CONTIGUOUS")
            i64p = np.ctypeslib.ndpointer(np.int64, flags="C_CONTIGUOUS")
            f64p = np.ctypeslib.ndpointer(np.float64, flags="C_CONTIGUOUS")
            lib.oracle_direction_numbers.argtypes = [C.c_int, i64p, i64p, C.c_int, u32p]
            lib.oracle_direction_numbers.restype = C.c_int
            lib.oracle_sobol_points.argtypes = [u32p, C.c_int, C.c_int64, C.c_int64, u32p]
            lib.oracle_sobol_points.restype = None
            lib.oracle_splitmix64.argtypes = [C.c_uint64, C.c_uint64]
            lib.oracle_splitmix64.restype = C.c_uint64
            lib.oracle_shift.argtypes = [C.c_uint64, C.c_int, C.c_int]
            lib.oracle_shift.restype = C.c_uint32
            lib.oracle_norm_inv.argtypes = [C.c_double]
            lib.oracle_norm_inv.restype = C.c_double
            lib.oracle_norm_cdf.argtypes = [C.c_double]
            lib.oracle_norm_cdf.restype = C.c_double
            lib.oracle_pca_factor.argtypes = [C.c_int, C.c_double, f64p]
            lib.oracle_pca_factor.restype = None
            lib.oracle_build_path.argtypes = [C.c_int, C.c_int, C.c_double, f64p, C.c_void_p, f64p]
            lib.oracle_build_path.restype = C.c_int
            lib.oracle_path_greeks.argtypes = [C.c_int, C.c_int] + [C.c_double] * 5 + [f64p, f64p]
            lib.oracle_path_greeks.restype = None
            lib.oracle_full_root.argtypes = [C.c_int, f64p, f64p, C.c_double]
            lib.oracle_full_root.restype = C.c_double
            lib.oracle_path_greeks_full.argtypes = [C.c_int, C.c_int] + [C.c_double] * 5 + [f64p, f64p, f64p]
            lib.oracle_path_greeks_full.restype = C.c_int
            lib.oracle_owen.argtypes = [C.c_uint32, C.c_uint32]
            lib.oracle_owen.restype = C.c_uint32
            lib.oracle_option.argtypes = ([C.c_int, C.c_int] + [C.c_double] * 5 +
                                          [C.c_uint64, C.c_int64, C.c_int, C.c_int, C.c_int, u32p, C.c_void_p,
                                           C.c_void_p, f64p, f64p, f64p])
            lib.oracle_option.restype = C.c_int
            lib.oracle_replication.argtypes = ([C.c_int, C.c_int] + [C.c_double] * 5 +
                                               [C.c_uint64, C.c_int64, C.c_int64, C.c_int, C.c_int, C.c_int,
                                                u32p, C.c_void_p, f64p, C.c_void_p])
            lib.oracle_replication.restype = C.c_int
            lib.oracle_options.argtypes = [C.c_int, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p,
                                           C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p,
                                           C.c_int, C.c_int, C.c_int, u32p, C.c_void_p, f64p, f64p, f64p,
                                           C.c_int]
            lib.oracle_options.restype = C.c_int
            lib.oracle_basket_path_greeks.argtypes = ([C.c_int, C.c_int, C.c_int] + [C.c_double] * 6 +
                                                      [f64p, f64p, f64p])
            lib.oracle_basket_path_greeks.restype = None
            lib.oracle_basket_option.argtypes = ([C.c_int, C.c_int, C.c_int] + [C.c_double] * 6 +
                                                 [C.c_uint64, C.c_int64, C.c_int, C.c_int, u32p, C.c_void_p,
                                                  f64p, f64p, f64p])
            lib.oracle_basket_option.restype = C.c_int
            lib.oracle_basket_replication.argtypes = ([C.c_int, C.c_int, C.c_int] + [C.c_double] * 6 +
                                                      [C.c_uint64, C.c_int64, C.c_int64, C.c_int, C.c_int, u32p,
                                                       f64p, C.c_void_p])
            lib.oracle_basket_replication.restype = C.c_int
            _lib = lib
    return _lib


# --------------------------------------------------------------------------
# inputs taken from outside the C code
# --------------------------------------------------------------------------
def joe_kuo_raw(n_dims: int):
    """Raw Joe-Kuo data for the first n_dims dimensions: (poly, minit[n_dims][18])."""
    global _JK_NPZ
    if _JK_NPZ is None:
        import scipy.stats
        path = os.path.join(os.path.dirname(scipy.stats.__file__), "_sobol_direction_numbers.npz")
        with np.load(path, allow_pickle=False) as z:
            _JK_NPZ = (np.ascontiguousarray(z["poly"], dtype=np.int64),
                       np.ascontiguousarray(z["vinit"], dtype=np.int64))
    poly, vinit = _JK_NPZ
    if n_dims > poly.shape[0]:
        raise ValueError("at most %d Sobol dimensions" % poly.shape[0])
    return poly[:n_dims].copy(), np.ascontiguousarray(vinit[:n_dims])


_V_CACHE: dict = {}


def direction_numbers(n_dims: int) -> np.ndarray:
    """V[j][b] (uint32, [n_dims][32]) built by the recurrence in oracle.c."""
    if n_dims not in _V_CACHE:
        poly, minit = joe_kuo_raw(n_dims)
        V = np.zeros((n_dims, 32), dtype=np.uint32)
        rc = _load().oracle_direction_numbers(n_dims, poly, minit, minit.shape[1], V)
        if rc != 0:
            raise ValueError("invalid initial direction numbers")
        _V_CACHE[n_dims] = V
    return _V_CACHE[n_dims]


def covariance(n: int, dt: float) -> np.ndarray:
    """Sigma_{kl} = dt * min(k, l), k, l = 1..n (Sec. 3.4.1)."""
    idx = np.arange(1, n + 1, dtype=np.float64)
    return dt * np.minimum.outer(idx, idx)


def pca_factor(n: int, dt: float) -> np.ndarray:
    """A = V diag(sqrt(lambda)), decreasing lambda, first entry of each column > 0."""
    if n == 0:
        return np.zeros((0, 0))
    A = np.zeros((n, n), dtype=np.float64)
    _load().oracle_pca_factor(n, dt, A)
    return A


# --------------------------------------------------------------------------
# wrappers
# --------------------------------------------------------------------------
def sobol_points(n_dims: int, k0: int, count: int) -> np.ndarray:
    V = direction_numbers(n_dims)
    out = np.zeros((count, n_dims), dtype=np.uint32)
    _load().oracle_sobol_points(V, n_dims, k0, count, out)
    return out


def splitmix64(seed: int, i: int) -> int:
    return int(_load().oracle_splitmix64(seed, i))


def shift(seed: int, l: int, j: int) -> int:
    return int(_load().oracle_shift(seed, l, j))


def shifts(seed: int, L: int, n_dims: int) -> np.ndarray:
    """[L][n_dims] digital shifts (dimension 0 included for completeness)."""
    lib = _load()
    return np.array([[lib.oracle_shift(seed, l, j) for j in range(n_dims)] for l in range(L)],
                    dtype=np.uint32)


def norm_inv(u: float) -> float:
    return float(_load().oracle_norm_inv(float(u)))


def norm_cdf(x: float) -> float:
    return float(_load().oracle_norm_cdf(float(x)))


def build_path(path: int, n: int, dt: float, z, A=None) -> np.ndarray:
    z = np.ascontiguousarray(z, dtype=np.float64)
    W = np.zeros(n + 1, dtype=np.float64)
    Ap = None
    if path == PATH_PCA:
        A = np.ascontiguousarray(A if A is not None else pca_factor(n, dt), dtype=np.float64)
        Ap = A.ctypes.data
    if n == 0:
        z = np.zeros(1)
    rc = _load().oracle_build_path(path, n, dt, z, Ap, W)
    if rc != 0:
        raise ValueError("bad path construction")
    return W


def path_greeks(type_: int, d: int, S0, K, r, sigma, T, W) -> np.ndarray:
    W = np.ascontiguousarray(W, dtype=np.float64)
    out = np.zeros(4)
    _load().oracle_path_greeks(type_, d, S0, K, r, sigma, T, W, out)
    return out


def full_root(alpha, beta, K) -> float:
    """Root psi of (1/d) sum_j exp(alpha_j + beta_j x) = K (full-PCA conditioning)."""
    al = np.ascontiguousarray(alpha, dtype=np.float64)
    be = np.ascontiguousarray(beta, dtype=np.float64)
    return float(_load().oracle_full_root(len(al), al, be, float(K)))


def path_greeks_full(type_: int, d: int, S0, K, r, sigma, T, a, c) -> np.ndarray:
    """{price, delta, vega, gamma} of one path conditioned on the first
    principal component: a = first column of the d x d factor, c = the other
    components' part of W(t_1..t_d)."""
    a = np.ascontiguousarray(a, dtype=np.float64)
    c = np.ascontiguousarray(c, dtype=np.float64)
    out = np.zeros(4)
    if _load().oracle_path_greeks_full(type_, d, S0, K, r, sigma, T, a, c, out) != 0:
        raise ValueError("full-PCA conditioning covers the arithmetic and binary Asian and the lookback calls")
    return out


def _factor(path: int, d: int, T: float):
    """The dense factor the oracle needs for a path construction (None if none)."""
    if path == PATH_PCA and d > 1:
        return np.ascontiguousarray(pca_factor(d - 1, T / d))
    if path == PATH_PCA_FULL:
        return np.ascontiguousarray(pca_factor(d, T / d))
    return None


def owen(y: int, seed32: int) -> int:
    """Nested (Owen) scrambling of one 32-bit coordinate with a 32-bit seed."""
    return int(_load().oracle_owen(int(y) & 0xFFFFFFFF, int(seed32) & 0xFFFFFFFF))


def option(type_: int, d: int, S0, K, r, sigma, T, seed: int, N: int, L: int, path: int = PATH_BB,
           rand: int = RAND_SHIFT):
    """One option: dict(mean[4], stderr[4], abs_mean[4], C_l[L][4])."""
    V = direction_numbers(max(d, 2))
    A = _factor(path, d, T)
    Ap = A.ctypes.data if A is not None else None
    C_l = np.zeros((L, 4))
    mean, se, am = np.zeros(4), np.zeros(4), np.zeros(4)
    rc = _load().oracle_option(type_, d, S0, K, r, sigma, T, seed & (2**64 - 1), N, L, path, rand,
                               V, Ap, C_l.ctypes.data, mean, se, am)
    if rc != 0:
        raise ValueError("oracle_option rejected its arguments")
    return {"mean": mean, "stderr": se, "abs_mean": am, "C_l": C_l}


def replication(o: dict, l: int, path: int = PATH_BB, k0: int = 0, N: int | None = None,
                rand: int = RAND_SHIFT) -> np.ndarray:
    """C_l[4] of replication l of option dict o over points k0 .. k0 + N - 1."""
    d = int(o["d"])
    N = int(o["n_points"]) if N is None else int(N)
    V = direction_numbers(max(d, 2))
    A = _factor(path, d, o["T"])
    out = np.zeros(4)
    rc = _load().oracle_replication(int(o["type"]), d, float(o["S0"]), float(o["K"]), float(o["r"]),
                                    float(o["sigma"]), float(o["T"]), int(o["seed"]) & (2**64 - 1), k0, N,
                                    l, path, rand, V, A.ctypes.data if A is not None else None, out, None)
    if rc != 0:
        raise ValueError("oracle_replication rejected its arguments")
    return out


def options(specs, L: int, path: int = PATH_BB, n_threads: int = 0, rand: int = RAND_SHIFT):
    """Many options (list of dicts with type,d,S0,K,r,sigma,T,seed,n_points).

    Returns (mean[n][4], stderr[n][4], abs_mean[n][4], threads_used)."""
    n = len(specs)
    typ = np.array([s["type"] for s in specs], dtype=np.int32)
    dd = np.array([s["d"] for s in specs], dtype=np.int32)
    f = {k: np.array([float(s[k]) for s in specs], dtype=np.float64)
         for k in ("S0", "K", "r", "sigma", "T")}
    seed = np.array([int(s["seed"]) & (2**64 - 1) for s in specs], dtype=np.uint64)
    NN = np.array([int(s["n_points"]) for s in specs], dtype=np.int64)
    V = direction_numbers(max(2, int(dd.max())))
    keep = []
    Aptr = None
    if path in (PATH_PCA, PATH_PCA_FULL):
        Aptr = (C.c_void_p * n)()
        for i, s in enumerate(specs):
            A = _factor(path, s["d"], s["T"])
            A = A if A is not None else np.zeros((1, 1))
            keep.append(A)
            Aptr[i] = A.ctypes.data
    mean, se, am = np.zeros((n, 4)), np.zeros((n, 4)), np.zeros((n, 4))
    used = _load().oracle_options(n, typ.ctypes.data, dd.ctypes.data, f["S0"].ctypes.data,
                                  f["K"].ctypes.data, f["r"].ctypes.data, f["sigma"].ctypes.data,
                                  f["T"].ctypes.data, seed.ctypes.data, NN.ctypes.data, L, path, rand, V,
                                  C.cast(Aptr, C.c_void_p) if Aptr is not None else None,
                                  mean.reshape(-1), se.reshape(-1), am.reshape(-1), n_threads)
    return mean, se, am, used


# --------------------------------------------------------------------------
# basket of M assets (one-factor model, standard construction)
# --------------------------------------------------------------------------
def basket_dims(d: int, M: int) -> int:
    """Sobol dimensions a basket path reads: 1 .. d - 1 + M d (0 is x_1)."""
    return d - 1 + M * d


def basket_path_greeks(type_: int, d: int, M: int, rho, S0, K, r, sigma, T, W0, Bi) -> np.ndarray:
    """{price, delta, vega, gamma} of one basket path: W0[d] = B~_0(tau_m),
    Bi[M][d] = B_i(t_{m+1})."""
    W0 = np.ascontiguousarray(W0, dtype=np.float64)
    Bi = np.ascontiguousarray(Bi, dtype=np.float64).reshape(-1)
    out = np.zeros(4)
    _load().oracle_basket_path_greeks(type_, d, M, rho, S0, K, r, sigma, T, W0, Bi, out)
    return out


def basket_option(type_: int, d: int, M: int, rho, S0, K, r, sigma, T, seed: int, N: int, L: int,
                  rand: int = RAND_SHIFT):
    """One basket option: dict(mean[4], stderr[4], abs_mean[4], C_l[L][4])."""
    V = direction_numbers(basket_dims(d, M) + 1)
    C_l = np.zeros((L, 4))
    mean, se, am = np.zeros(4), np.zeros(4), np.zeros(4)
    rc = _load().oracle_basket_option(type_, d, M, rho, S0, K, r, sigma, T, seed & (2**64 - 1), N, L, rand, V,
                                      C_l.ctypes.data, mean, se, am)
    if rc != 0:
        raise ValueError("oracle_basket_option rejected its arguments")
    return {"mean": mean, "stderr": se, "abs_mean": am, "C_l": C_l}


def basket_replication(o: dict, l: int, k0: int = 0, N: int | None = None, rand: int = RAND_SHIFT) -> np.ndarray:
    """C_l[4] of replication l of basket option dict o (keys as option() plus n_assets, rho)."""
    d, M = int(o["d"]), int(o["n_assets"])
    N = int(o["n_points"]) if N is None else int(N)
    V = direction_numbers(basket_dims(d, M) + 1)
    out = np.zeros(4)
    rc = _load().oracle_basket_replication(int(o["type"]), d, M, float(o["rho"]), float(o["S0"]), float(o["K"]),
                                           float(o["r"]), float(o["sigma"]), float(o["T"]),
                                           int(o["seed"]) & (2**64 - 1), k0, N, l, rand, V, out, None)
    if rc != 0:
        raise ValueError("oracle_basket_replication rejected its arguments")
    return out

