"""The FP64 reciprocal and reciprocal square root of the kernels refine the
hardware estimate r by one third-order step: with e = 1 - x r,
1/x ~ r + r (e + e^2); with e = 1 - x r^2, 1/sqrt(x) ~ r + r e (1/2 + 3e/8).
Here the same operation sequence runs with an exact fused multiply-add
(rational arithmetic, one rounding per operation, as on the device) on
estimates whose relative error reaches 2^-22, four times the largest error
measured for the gfx950 estimates (2^-24), and must land within one ulp of
the exact value (the reciprocal within half an ulp: correctly rounded).
The source is checked to hold these sequences."""
import math
import os
import random
import re
from fractions import Fraction as F

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _fma(a, b, c):
    return float(F(a) * F(b) + F(c))


def _mul(a, b):
    return float(F(a) * F(b))


def _rcp(x, r):
    e = _fma(-x, r, 1.0)
    return _fma(r, _fma(e, e, e), r)


def _rsq(x, r):
    e = _fma(-_mul(x, r), r, 1.0)
    return _fma(r, _mul(_fma(0.375, e, 0.5), e), r)


def _ulps(got, exact):
    return float(abs(F(got) - exact) / F(math.ulp(float(exact))))


def test_device_sequences():
    src = open(os.path.join(ROOT, "paper_1607_08710_amd", "csrc", "lf_device.h")).read()
    body = lambda name: re.search(r"double %s\(double x\) \{(.*?)\n\}" % name, src, re.S).group(1)
    assert re.sub(r"\s+", " ", body("rcp")).strip() == (
        "const double r = __builtin_amdgcn_rcp(x); const double e = fma(-x, r, 1.0); "
        "return fma(r, fma(e, e, e), r);")
    assert re.sub(r"\s+", " ", body("rsq")).strip() == (
        "const double r = __builtin_amdgcn_rsq(x); const double e = fma(-x * r, r, 1.0); "
        "// 1 - x r^2 return fma(r, fma(0.375, e, 0.5) * e, r);")


def test_refinement_error_bound():
    rng = random.Random(2024)
    worst_rcp = worst_rsq = 0.0
    for _ in range(3000):
        x = math.ldexp(rng.uniform(1.0, 2.0), rng.randint(-300, 300))
        exact = 1 / F(x)
        r0 = float(exact * (1 + F(rng.uniform(-1.0, 1.0)) / 2**22))
        worst_rcp = max(worst_rcp, _ulps(_rcp(x, r0), exact))
        xs = math.ldexp(rng.uniform(1.0, 4.0), 2 * rng.randint(-150, 150))
        y = 1 / F(math.sqrt(xs))
        for _ in range(4):  # Newton in exact arithmetic: 1/sqrt(xs) to far beyond double precision
            y = y * (3 - F(xs) * y * y) / 2
        r0 = float(y * (1 + F(rng.uniform(-1.0, 1.0)) / 2**22))
        worst_rsq = max(worst_rsq, _ulps(_rsq(xs, r0), y))
    assert worst_rcp <= 0.5 + 1e-9, worst_rcp
    assert worst_rsq < 1.0, worst_rsq
