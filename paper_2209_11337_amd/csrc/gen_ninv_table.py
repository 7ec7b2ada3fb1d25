"""Write ninv_table.inc: two tables of cubics for the FP32 inverse normal.

The kernels convert the raw 32-bit Sobol coordinate y to FP32 as a signed
integer with one instruction: q = float(int32(y)), i.e. q = y for y < 2^31
and q = -(2^32 - y) otherwise, exact below 2^24 in magnitude and rounded to
24 bits above.  With a = |q|, u = (y + 1/2) 2^-32 is

    lower half (q >= 0):  u = (a + 1/2) 2^-32,      z = Phi^{-1}(u) <= 0,
    upper half (q <  0):  u = 1 - (a - 1/2) 2^-32,  z = -Phi^{-1}((a - 1/2) 2^-32) > 0,

so each half has its own function of a, and one table per half.  a is 0 or
lies in one of the binary octaves [2^e, 2^(e+1)), e = 0..30, or is exactly
2^31.  Each octave is cut into 2^c equal cells (c = 3: the cubic's error is
then at the level of FP32 rounding, and a small table keeps the random LDS
reads cheap).  The FP32 bits of q select the cell and the half at once:
bits 16..31 of q, masked with 0x8FF0, are 16 x (low 5 bits of the biased
exponent, top 3 mantissa bits) plus 0x8000 for a negative q -- one SDWA
instruction.  So the octaves sit in each table rotated by their exponent
modulo 32, and the upper-half table sits 32 KiB after the lower one.

On every cell the target is a cubic in a itself (the kernels take |q| as a
free source modifier): least squares over the values a can take in the cell
(the reachable integers there below 2^24, every FP32 value above), weight
1/max(|z|, 0.05), coefficients fixed one at a time from the highest degree,
each rounded to FP32 before the rest are refitted; a cell with k <= 4
reachable values gets the interpolating polynomial of degree k - 1.
Coefficients are stored highest degree first.

Shared and lone cells: in the lower table q = 0 has the bits of exponent
slot 0, cell 0, as does q = 2 (octave 1) -- that cell is the line through
both points; a = 2^31 (in both tables) is alone in its slot (30), where z
is 0 to within 4e-8.  In the upper table a >= 1, so octave 0 holds a = 1
only.

Max error of the FP32 evaluation (printed when run): about 5e-7 absolute in
the far tails (|z| ~ 4..6, about 1e-7 relative) and about 2e-7 absolute
next to z = 0.

Run from the repository root:  python paper_2209_11337_amd/csrc/gen_ninv_table.py
"""
import os

import numpy as np
import scipy.special as sp

CELL_BITS = 3   # 2^CELL_BITS cells per octave: bits 20..22 of q, fixed by the 0x8FF0 mask
DEG = 3
HERE = os.path.dirname(os.path.abspath(__file__))


def fma32(a, b, c):
    # FP32 fused multiply-add: the product of two FP32 values is exact in FP64
    return (a.astype(np.float64) * b.astype(np.float64) + c.astype(np.float64)).astype(np.float32)


def horner32(ck, q):
    p = np.full(q.shape, ck[0], np.float32)
    for c in ck[1:]:
        p = fma32(p, q, np.full(q.shape, c, np.float32))
    return p


def g_lo(a):
    return sp.ndtri((a + 0.5) * 2.0**-32)


def g_hi(a):
    return -sp.ndtri((a - 0.5) * 2.0**-32)


def fit_cell(g, a, h, e, amin):
    lo = np.float32(a).view(np.uint32)
    hi = np.float32(a + h).view(np.uint32)
    q = np.unique(np.linspace(lo, hi - 1, 1025).astype(np.uint32)).view(np.float32)
    if e < 24:
        q = np.unique(np.ceil(q).astype(np.float32))
        q = q[(q < a + h) & (q >= amin)]
    if len(q) == 0:
        return np.zeros(DEG + 1, dtype=np.float32), 0.0, 0.0
    qd = q.astype(np.float64)
    z = g(qd)
    deg = min(DEG, len(q) - 1)
    w = 1.0 / np.maximum(np.abs(z), 0.05)
    V = np.vander(qd, DEG + 1)
    sc = np.array([a ** (DEG - k) for k in range(DEG + 1)])
    fixed = [0.0] * (DEG - deg)
    for k in range(DEG - deg, DEG + 1):
        r = z - sum(fixed[j] * qd ** (DEG - j) for j in range(k))
        M = V[:, k:] / sc[k:]
        c = np.linalg.lstsq(M * w[:, None], r * w, rcond=None)[0] / sc[k:]
        fixed.append(float(np.float32(c[0])))
    ck = np.array(fixed, dtype=np.float32)
    err = np.abs(horner32(ck, q) - z)
    return ck, float(err.max()), float(np.max(err / np.maximum(np.abs(z), 0.05)))


def fit_table(g, amin):
    cells = 1 << CELL_BITS
    table = np.zeros((32 * cells, DEG + 1), dtype=np.float32)
    worst_abs = worst_rel = 0.0
    for e in range(0, 31):
        slot = (e + 127) & 31
        for i in range(cells):
            a = 2.0 ** e * (1 + i / cells)
            ck, ea, er = fit_cell(g, a, 2.0 ** e / cells, e, amin)
            table[slot * cells + i] = ck
            worst_abs, worst_rel = max(worst_abs, ea), max(worst_rel, er)
    # a = 2^31 alone in its slot: z within 4e-8 of 0
    top = (31 + 127) & 31
    assert top not in {(e + 127) & 31 for e in range(0, 31)}
    table[top * cells: (top + 1) * cells] = 0.0
    return table, worst_abs, worst_rel


def main():
    cells = 1 << CELL_BITS
    lo, lo_abs, lo_rel = fit_table(g_lo, 0.0)
    # lower half: q = 0 shares slot 0 / cell 0 with q = 2 (octave 1): the line through both
    assert (1 + 127) & 31 == 0
    z0, z2 = float(g_lo(0.0)), float(g_lo(2.0))
    lo[0] = np.array([0.0, 0.0, (z2 - z0) / 2.0, z0], dtype=np.float32)
    ends = horner32(lo[0], np.array([0.0, 2.0], dtype=np.float32))
    e_ends = max(abs(float(ends[0]) - z0), abs(float(ends[1]) - z2))
    hi, hi_abs, hi_rel = fit_table(g_hi, 1.0)
    e_top = max(abs(float(g_lo(2.0**31 - 64))), abs(float(g_hi(2.0**31 - 63))))
    print("cells %d + %d, max error: lower %.3g absolute %.3g relative, upper %.3g absolute %.3g relative "
          "(floor 0.05); q in {0, 2}: %.3g, |q| = 2^31: %.3g"
          % (len(lo), len(hi), lo_abs, lo_rel, hi_abs, hi_rel, e_ends, e_top))
    lines = ["// Generated by gen_ninv_table.py: z = Phi^{-1}((y + 1/2) 2^-32) as cubics in a = |q|,",
             "// q = float(int32(y)) for the raw 32-bit Sobol coordinate y; one table per half",
             "// (q >= 0: rows 0..255, q < 0: rows 256..511), one row per (octave, 1/8 of the octave)",
             "// cell; row within a table = bits 20..27 of q (octaves rotated by their biased",
             "// exponent mod 32); coefficients highest first.",
             "#define QCPW_NINV_TAB_CELLS %d   // cells per half" % len(lo),
             "#define QCPW_NINV_CELL_BITS %d   // mantissa bits of q that pick the cell" % CELL_BITS,
             "static const float QCPW_NINV_TAB[2 * QCPW_NINV_TAB_CELLS][4] = {"]
    for ck in np.concatenate([lo, hi]):
        lines.append("  {" + ", ".join("%.9ef" % x for x in ck) + "},")
    lines.append("};")
    with open(os.path.join(HERE, "ninv_table.inc"), "w") as f:
        f.write("\n".join(lines) + "\n")


if __name__ == "__main__":
    main()
