"""The C ABI on the CPU: the library loads, exports every declared entry
point, keeps the ABI struct layout, checks arguments before touching a
device, and its host-built path factors agree with the oracle's."""
import ctypes as C
import os
import re

import numpy as np
import pytest

import oracle
import paper_2209_11337_amd as q

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    text = open(os.path.join(ROOT, "include", "qmc_cpw.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(q\w+)\s*\(", text)) - {"qcpw_status"})


def test_every_declared_symbol_is_exported():
    names = declared_functions()
    assert len(names) >= 13
    L = q.lib()
    missing = [n for n in names if not hasattr(L, n)]
    assert missing == []
    assert set(names) == set(q.EXPORTS)


def test_struct_layout():
    assert C.sizeof(q.OptionSpec) == 80
    assert q.OptionSpec.seed.offset == 48 and q.OptionSpec.n_points.offset == 56
    assert q.OptionSpec.n_assets.offset == 64 and q.OptionSpec.rho.offset == 72
    assert C.sizeof(q.RunConfig) == 48
    assert q.RunConfig.out_paper_sigma.offset == 40


def test_version_string():
    assert "gfx950" in q.version()


BAD = [
    (dict(type=10), "unknown type"),
    (dict(type=11), "unknown type"),
    (dict(type=-1), "unknown type"),
    (dict(d=0), "d must be"),
    (dict(d=400), "exceeds"),
    (dict(S0=-1.0), "finite and > 0"),
    (dict(sigma=0.0), "finite and > 0"),
    (dict(T=float("nan")), "finite and > 0"),
    (dict(r=float("inf")), "r finite"),
    (dict(n_points=0), "n_points"),
    (dict(n_points=(1 << 32) + 1), "n_points"),
]


@pytest.mark.parametrize("patch,msg", BAD)
def test_invalid_specs_rejected_before_any_device_work(patch, msg):
    o = dict(type=0, d=16, S0=100.0, K=100.0, r=0.05, sigma=0.2, T=1.0, seed=1, n_points=64)
    o.update(patch)
    with pytest.raises(q.QcpwError) as ei:
        q.greeks([o], 4)
    assert msg in str(ei.value)
    assert ei.value.status in (-1, -4)


def test_invalid_call_arguments():
    o = dict(type=0, d=16, S0=100.0, K=100.0, r=0.05, sigma=0.2, T=1.0, seed=1, n_points=64)
    for kw in (dict(n_shifts=0), dict(n_shifts=70000), dict(path=9), dict(precision=5),
               dict(block_threads=100), dict(block_threads=1088), dict(pca_gemm=3)):
        args = dict(n_shifts=4)
        args.update(kw)
        with pytest.raises(q.QcpwError):
            q.greeks([o], **args)
    with pytest.raises(q.QcpwError):
        q.greeks([dict(o, d=300)], 4, path=q.PATH_PCA)
    st = q.lib().qmc_cpw_greeks(None, 1, 0, 0, 2, 0, None, None)
    assert st == -1


@pytest.mark.parametrize("path", [q.PATH_BB, q.PATH_STANDARD, q.PATH_PCA])
@pytest.mark.parametrize("d", [2, 3, 16, 64, 65, 257])
def test_library_factor_matches_oracle(path, d):
    """The library's factor A (host code) against the oracle's path builder:
    the same linear map z -> W~ (bridge order, increments, principal
    components), hence the same paths for the same normals."""
    T = 1.3
    n, dt = d - 1, T / d
    A = q.path_factor(path, d, T)
    Z = np.random.default_rng(d).standard_normal((n, 5))
    for c in range(5):
        ref = oracle.build_path(path, n, dt, Z[:, c])[1:]
        assert np.abs(A @ Z[:, c] - ref).max() <= 1e-13 * max(1.0, np.abs(ref).max())
    Sig = oracle.covariance(n, dt)
    assert np.abs(A @ A.T - Sig).max() <= 1e-14 * Sig.max() * max(1, n / 16)


def test_bridge_plan_every_size():
    """Every bridge plan the kernels can be given (d = 2..385), replayed on
    the host with the kernels' stack slots, builds the oracle's bridge."""
    rng = np.random.default_rng(385)
    for d in range(2, 386):
        n, dt = d - 1, 1.0 / d
        A = q.path_factor(q.PATH_BB, d, 1.0)
        z = rng.standard_normal(n)
        ref = oracle.build_path(q.PATH_BB, n, dt, z)[1:]
        assert np.isfinite(A).all(), d
        assert np.abs(A @ z - ref).max() <= 1e-13 * max(1.0, np.abs(ref).max()), d


@pytest.mark.parametrize("d", [1, 2, 17, 64, 256])
def test_library_full_pca_factor_matches_oracle(d):
    """The d x d factor of all dates (first column = conditioned component)."""
    T = 0.8
    A = q.path_factor(q.PATH_PCA_FULL, d, T)
    ref = oracle.pca_factor(d, T / d)
    assert A.shape == (d, d)
    assert np.abs(A - ref).max() <= 1e-13 * max(1.0, np.abs(ref).max())
    assert (A[:, 0] > 0).all()


def test_full_pca_argument_checks():
    o = dict(type=0, d=16, S0=100.0, K=100.0, r=0.05, sigma=0.2, T=1.0, seed=1, n_points=64)
    for t in (3, 4, 5, 6, 7):   # geometric, puts
        with pytest.raises(q.QcpwError) as ei:
            q.greeks([dict(o, type=t)], 4, q.PATH_PCA_FULL)
        assert ei.value.status == -1 and "lookback calls" in str(ei.value)
    with pytest.raises(q.QcpwError) as ei:
        q.greeks([dict(o, d=257)], 4, q.PATH_PCA_FULL)
    assert ei.value.status == -4
    with pytest.raises(q.QcpwError):
        q.path_factor(q.PATH_PCA_FULL, 257, 1.0)


def test_basket_argument_checks():
    o = dict(type=8, d=16, S0=100.0, K=100.0, r=0.05, sigma=0.2, T=1.0, seed=1, n_points=64, n_assets=4, rho=0.5)
    for patch, path, msg in [(dict(), q.PATH_BB, "standard construction"),
                             (dict(), q.PATH_PCA, "standard construction"),
                             (dict(n_assets=0), q.PATH_STANDARD, "n_assets"),
                             (dict(n_assets=9), q.PATH_STANDARD, "n_assets"),
                             (dict(rho=0.0), q.PATH_STANDARD, "rho"),
                             (dict(rho=1.5), q.PATH_STANDARD, "rho"),
                             (dict(rho=float("nan")), q.PATH_STANDARD, "rho"),
                             (dict(d=48, n_assets=8), q.PATH_STANDARD, "exceeds")]:
        with pytest.raises(q.QcpwError) as ei:
            q.greeks([dict(o, **patch)], 4, path)
        assert msg in str(ei.value), (patch, str(ei.value))


def test_noalloc_flag_and_construction_checks():
    """The call that allocates nothing takes the bridge and standard
    constructions and no flag but QCPW_FLAG_OWEN; both are refused before
    any device work."""
    o = dict(type=0, d=16, S0=100.0, K=100.0, r=0.05, sigma=0.2, T=1.0, seed=1, n_points=64)
    for path in (q.PATH_PCA, q.PATH_PCA_FULL):
        with pytest.raises(q.QcpwError) as ei:
            q.greeks_noalloc([o], 4, path, owen=True)
        assert ei.value.status == -1 and "no-allocation" in str(ei.value)


def test_kernel_timer_argument_checks():
    for op in (0, 4, -1):
        with pytest.raises(q.QcpwError) as ei:
            q.kernel_timer(op)
        assert ei.value.status == -1


def test_library_factor_argument_checks():
    with pytest.raises(q.QcpwError):
        q.path_factor(q.PATH_PCA, 300, 1.0)
    with pytest.raises(q.QcpwError):
        q.path_factor(q.PATH_BB, 10, -1.0)
