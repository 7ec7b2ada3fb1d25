"""The FP32 inverse-normal table the kernels read (ninv_table.inc), checked
on the CPU by emulating the kernels' lookup bit for bit: q = float(int32(y)),
cell row from bits 16..31 of q masked with 0x8FF0, cubic in |q| by FP32
fused multiply-adds.  Reference: scipy's ndtri in FP64."""
import os
import re

import numpy as np
import scipy.special as sp

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
INC = os.path.join(ROOT, "paper_2209_11337_amd", "csrc", "ninv_table.inc")


def load_table():
    text = open(INC).read()
    rows = re.findall(r"\{([^{}]*)\},", text)
    tab = np.array([[float(v.strip().rstrip("f")) for v in r.split(",")] for r in rows], dtype=np.float32)
    assert tab.shape == (512, 4)
    return tab


def fma32(a, b, c):
    return (a.astype(np.float64) * b.astype(np.float64) + c.astype(np.float64)).astype(np.float32)


def emulate(tab, y):
    q = y.astype(np.uint32).view(np.int32).astype(np.float32)
    bits = q.view(np.uint32)
    off = (bits >> 16) & 0x8FF0
    row = np.where(off & 0x8000, 256, 0) + ((off & 0x0FF0) >> 4)
    c = tab[row]
    a = np.abs(q)
    p = fma32(c[:, 0], a, c[:, 1])
    p = fma32(p, a, c[:, 2])
    return fma32(p, a, c[:, 3])


def test_table_error_bound_and_symmetry():
    tab = load_table()
    rng = np.random.default_rng(11337)
    edges = np.array([0, 1, 2, 3, 4, 5, 7, 8, 255, 256, (1 << 24) - 1, 1 << 24, (1 << 24) + 1,
                      (1 << 31) - 65, (1 << 31) - 64, (1 << 31) - 1, 1 << 31, (1 << 31) + 1, (1 << 31) + 64,
                      (1 << 32) - (1 << 24), (1 << 32) - 8, (1 << 32) - 3, (1 << 32) - 2, (1 << 32) - 1],
                     dtype=np.uint64)
    # uniform, plus log-uniform in both tails
    tails = np.exp2(rng.uniform(0, 31, 200000)).astype(np.uint64)
    y = np.concatenate([edges, rng.integers(0, 1 << 32, 400000, dtype=np.uint64), tails,
                        (1 << 32) - 1 - tails]).astype(np.uint64) & 0xFFFFFFFF
    z = emulate(tab, y).astype(np.float64)
    ref = sp.ndtri((y.astype(np.float64) + 0.5) * 2.0**-32)
    err = np.abs(z - ref)
    # FP32 evaluation of the cubic in |q| (up to 2^31) sets the error: about 1e-7 relative in the
    # far tails, a few 1e-7 absolute in the body
    assert err.max() <= 7e-7, (err.max(), y[np.argmax(err)])
    assert err[np.abs(ref) < 0.5].max() <= 3e-7
    assert (err / np.abs(ref))[np.abs(ref) > 3].max() <= 2e-7
    # the two halves mirror each other: y and ~y give opposite normals up to the fit
    zm = emulate(tab, (~y) & 0xFFFFFFFF).astype(np.float64)
    assert np.abs(z + zm).max() <= 1.2e-6
    # monotone over a dense sweep through both tails and the middle
    for lo in (0, (1 << 31) - 5000, (1 << 32) - 5000):
        yy = np.arange(lo, lo + 5000, dtype=np.uint64)
        zz = emulate(tab, yy)
        assert np.all(np.diff(zz.astype(np.float64)) >= -1e-7)
