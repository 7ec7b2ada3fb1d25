"""The FP64 elementary functions of the per-path tail (ln, exp, erfcx),
emulated on the CPU in FP64 with the kernels' argument reduction, series
lengths and coefficient tables (phi_f64_coeffs.inc): the full forms (FP64
kernels) and the shorter ones (kernels whose path statistic is an FP32 sum).
Reference: numpy's log and exp and scipy's erfcx in FP64."""
import math
import os
import re

import numpy as np
import scipy.special as sp

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
INC = os.path.join(ROOT, "paper_2209_11337_amd", "csrc", "phi_f64_coeffs.inc")

LN2_HI = 6.93147180369123816490e-01
LN2_LO = 1.90821492927058770002e-10


def load_coeffs(name):
    text = open(INC).read()
    body = re.search(name + r"\[(\d+)\] = \{([^}]*)\}", text)
    co = [float(v) for v in body.group(2).split(",") if v.strip()]
    assert len(co) == int(body.group(1))
    return co


def erfcx_emul(x, co):
    t = 3.0 / (3.0 + x)
    p = np.full_like(x, co[0])
    for a in co[1:]:
        p = p * t + a
    return t * p


def ln_emul(x, ktop):
    m, e = np.frexp(x)
    low = m < 0.70710678118654752440
    m = np.where(low, 2.0 * m, m)
    e = np.where(low, e - 1, e).astype(np.float64)
    s = (m - 1.0) / (m + 1.0)
    z = s * s
    p = np.full_like(x, 1.0 / ktop)
    for k in range(ktop - 2, 0, -2):
        p = p * z + 1.0 / k
    return e * LN2_HI + (e * LN2_LO + 2.0 * s * p)


def exp_emul(x, jtop):
    k = np.rint(x * 1.44269504088896340736)
    r = x - k * LN2_HI
    r = r - k * LN2_LO
    p = np.full_like(x, 1.0 / math.factorial(jtop))
    for j in range(jtop - 1, -1, -1):
        p = p * r + 1.0 / math.factorial(j)
    return np.ldexp(p, k.astype(np.int64))


def test_erfcx_tables_relative_error():
    x = np.concatenate([np.linspace(0.0, 6.0, 60001), np.linspace(6.0, 40.0, 20001),
                        np.geomspace(40.0, 1e8, 2001)])
    ref = sp.erfcx(x)
    full = np.abs(erfcx_emul(x, load_coeffs("QCPW_ERFCX_P")) / ref - 1.0)
    short = np.abs(erfcx_emul(x, load_coeffs("QCPW_ERFCX_S")) / ref - 1.0)
    assert full.max() <= 2e-15, full.max()
    assert short.max() <= 2e-11, short.max()
    # the short fit is a genuine approximation (not the full table cut short)
    assert short.max() >= 1e-13


def test_ln_series_lengths():
    rng = np.random.default_rng(7)
    x = np.concatenate([np.exp(rng.uniform(-40, 40, 200000)), [1.0, 0.5, 2.0, 0.70710678, 1.41421356, 1e-300, 1e300]])
    ref = np.log(x)
    scale = np.maximum(np.abs(ref), 1.0)
    full = np.abs(ln_emul(x, 23) - ref) / scale
    short = np.abs(ln_emul(x, 13) - ref) / scale
    assert full.max() <= 1e-15, full.max()
    assert short.max() <= 1.5e-12, short.max()
    # near 1 the error is relative to ln x itself
    y = 1.0 + rng.uniform(-0.29, 0.41, 100000)
    rel = np.abs(ln_emul(y, 13) / np.log(y) - 1.0)
    assert np.nanmax(rel) <= 1.5e-12


def test_exp_series_lengths():
    rng = np.random.default_rng(8)
    x = np.concatenate([rng.uniform(-700, 0, 200000), rng.uniform(-5, 5, 100000), [0.0, -0.34657359, 0.34657359]])
    ref = np.exp(x)
    full = np.abs(exp_emul(x, 13) / ref - 1.0)
    short = np.abs(exp_emul(x, 10) / ref - 1.0)
    assert full.max() <= 1e-15, full.max()
    assert short.max() <= 4e-13, short.max()
