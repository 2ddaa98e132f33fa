"""The FP64 phase polynomials of the regular fill kernel, checked on the CPU
against 50-digit sine and cosine: the coefficients are read from the kernel
source, the argument reduction and the Horner chains are replayed in FP64
with exactly rounded fused multiply-adds, and the results must stay within
1.5 ulp of 1 (3.3e-16) over several revolutions (the phase factor e^{-jkR} of the
Green's function, Sec. II-B)."""
import os
import random
import re
from fractions import Fraction

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "paper_2111_11058_amd", "csrc", "fill.hip")


def _coefficients():
    src = open(SRC).read()
    body = src[src.index("void sincos_rev("):]
    body = body[:body.index("\n}\n")]

    def chain(v):
        first = re.search(r"double %s = ([-0-9.e]+);" % v, body).group(1)
        rest = re.findall(r"%s = fma\(%s, u, ([-0-9.e]+)\);" % (v, v), body)
        return [float(first)] + [float(x) for x in rest]

    cs, cc = chain("ps"), chain("pc")
    assert "fma(pc, u, 1.0)" in body
    return cs, cc + [1.0]


def _fma(a, b, c):
    return float(Fraction(a) * Fraction(b) + Fraction(c))


def _sincos_rev(x, cs, cc):
    q = float(round(2.0 * x))  # rint: ties never occur on the samples below
    f = _fma(-0.5, q, x)
    u = f * f
    ps = cs[0]
    for c in cs[1:]:
        ps = _fma(ps, u, c)
    sn = f * ps
    pc = cc[0]
    for c in cc[1:]:
        pc = _fma(pc, u, c)
    flip = -1.0 if int(q) & 1 else 1.0
    return flip * sn, flip * pc


def test_phase_polynomials_within_an_ulp():
    mp = pytest.importorskip("mpmath")
    mp.mp.dps = 40
    cs, cc = _coefficients()
    assert len(cs) == 9 and len(cc) == 9
    rng = random.Random(7)
    xs = [rng.uniform(-3.0, 3.0) for _ in range(3000)]
    xs += [k / 8.0 + s * 1e-12 for k in range(-16, 17) for s in (-1, 1)]  # near the quarter turns
    xs += [0.0, 1e-300, 0.2499999999999, 0.2500000000001]
    es = ec = 0.0
    for x in xs:
        s, c = _sincos_rev(x, cs, cc)
        t = 2 * mp.pi * mp.mpf(x)
        es = max(es, abs(s - float(mp.sin(t))))
        ec = max(ec, abs(c - float(mp.cos(t))))
    assert es <= 3.3e-16 and ec <= 3.3e-16, (es, ec)
