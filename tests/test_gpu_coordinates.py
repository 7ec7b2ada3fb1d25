"""Bit-exact Sobol integers of the fused per-path kernel itself.

qcpw_path_coordinates runs an instance of the per-path kernel that stores
every coordinate its walk consumes.  The integers must equal the oracle's
Gray-code Sobol points (Sec. 2.2.2, XOR form) XOR the digital shift of the
replication, or their nested scrambling (Sec. 2.2.3), bit for bit, on every
route the walk takes: the compile-time bridges (FP32, d = 16, 32, 64, 128,
whose wave-uniform parts arrive by DPP row broadcast), the plan walker
(v_readlane, FP32 and FP64), the standard construction and the basket.
"""
import sys

import numpy as np
import pytest

import oracle
import paper_2209_11337_amd as q

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def expected(seed, L, N, nd, owen=False):
    """[L][N][nd] coordinates of dimensions 1..nd from the oracle."""
    raw = oracle.sobol_points(nd + 1, 0, N)[:, 1:]
    keys = oracle.shifts(seed, L, nd + 1)[:, 1:]
    if not owen:
        return raw[None, :, :] ^ keys[:, None, :]
    out = np.empty((L, N, nd), dtype=np.uint32)
    for l in range(L):
        for j in range(nd):
            out[l, :, j] = [oracle.owen(int(y), int(keys[l, j])) for y in raw[:, j]]
    return out


def option(d, N, seed, type_=q.ARITH_ASIAN):
    return dict(type=type_, d=d, S0=100.0, K=100.0, r=0.05, sigma=0.2, T=1.0, seed=seed, n_points=N)


# d = 16, 32, 64, 128: compile-time bridges in FP32; the others walk the plan.
# 4096 + 77 points: 17 work units of 256 points with a ragged last one.
@pytest.mark.parametrize("d", [16, 32, 64, 128, 2, 5, 100, 257, 365])
def test_bridge_fp32_coordinates_bit_exact(d):
    N, L, seed = 4096 + 77, 3, 0x51ab00 + d
    say("coords bridge fp32", d, N, L)
    got = q.path_coordinates(option(d, N, seed), L, q.PATH_BB, q.FP32_MIXED)
    assert np.array_equal(got, expected(seed, L, N, d - 1))


@pytest.mark.parametrize("d", [16, 100, 385])
def test_bridge_fp64_coordinates_bit_exact(d):
    N, L, seed = 2048 + 5, 2, 0x64b00 + d
    say("coords bridge fp64", d, N, L)
    got = q.path_coordinates(option(d, N, seed, q.LOOKBACK), L, q.PATH_BB, q.FP64)
    assert np.array_equal(got, expected(seed, L, N, d - 1))


@pytest.mark.parametrize("prec", [q.FP32_MIXED, q.FP64])
def test_standard_coordinates_bit_exact(prec):
    d, N, L, seed = 50, 3000, 2, 0x5d
    say("coords standard", prec)
    got = q.path_coordinates(option(d, N, seed, q.BINARY_ASIAN), L, q.PATH_STANDARD, prec)
    assert np.array_equal(got, expected(seed, L, N, d - 1))


def test_basket_coordinates_bit_exact():
    d, M, N, L, seed = 12, 3, 1024, 2, 0xba5
    o = dict(option(d, N, seed, q.BASKET_ASIAN), n_assets=M, rho=0.5)
    say("coords basket")
    got = q.path_coordinates(o, L, q.PATH_STANDARD, q.FP32_MIXED)
    assert got.shape == (L, N, d - 1 + M * d)
    assert np.array_equal(got, expected(seed, L, N, d - 1 + M * d))


# nested scrambling: the compile-time bridge (d = 64) reads the distributed
# parts, as do the plan walker (d = 20) and the standard construction
@pytest.mark.parametrize("d,path,prec", [(64, q.PATH_BB, q.FP32_MIXED), (20, q.PATH_BB, q.FP32_MIXED),
                                         (20, q.PATH_BB, q.FP64), (20, q.PATH_STANDARD, q.FP32_MIXED)])
def test_owen_coordinates_bit_exact(d, path, prec):
    N, L, seed = 512 + 3, 2, 0x0e + d
    say("coords owen", d, path, prec)
    got = q.path_coordinates(option(d, N, seed), L, path, prec, owen=True)
    assert np.array_equal(got, expected(seed, L, N, d - 1, owen=True))


def test_coordinates_argument_checks():
    with pytest.raises(q.QcpwError):
        q.path_coordinates(option(1, 64, 1), 2, q.PATH_BB, q.FP64)   # no sampled coordinate
    with pytest.raises(q.QcpwError):
        q.path_coordinates(option(16, 64, 1), 2, q.PATH_PCA, q.FP64)
    with pytest.raises(q.QcpwError):
        q.path_coordinates(option(365, 1 << 20, 1), 2, q.PATH_BB, q.FP64)   # beyond 2^28 bytes
