"""The FP64 exponential of csrc/equilibrium.h: its polynomial coefficients
are those of the Remez fit in exp_minimax.py, and with those coefficients
rounded to double the polynomial stays within 3.2e-16 relative of e^r on
|r| <= ln(2)/2 (3.05e-16 measured; 2.1e-16 before rounding) (a mistyped coefficient would break either check)."""
import os
import re

import pytest

mp = pytest.importorskip("mpmath")

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _device_coefficients():
    src = open(os.path.join(ROOT, "paper_1910_13515_amd", "csrc", "equilibrium.h")).read()
    body = src[src.index("__device__ __forceinline__ double dexp<double>(double x)"):]
    body = body[:body.index("return __builtin_ldexp")]
    # the reduction constants come first; the polynomial is the p = ... chain
    chain = body[body.index("double p ="):]
    lits = re.findall(r"(0x[0-9a-f]\.[0-9a-f]+p[+-]\d+|1\.0)(?=\)?;)", chain)
    vals = [float.fromhex(v) if v.startswith("0x") else float(v) for v in lits]
    return vals[::-1]  # c_0 .. c_10


def test_coefficients_match_the_remez_fit():
    from paper_1910_13515_amd import exp_minimax
    coef, level, worst = exp_minimax.remez()
    assert float(level) < 2.2e-16
    dev = _device_coefficients()
    assert len(dev) == len(coef) == 11
    for c_dev, c_fit in zip(dev, coef):
        assert c_dev == float(c_fit)


def test_rounded_polynomial_error():
    mp.mp.dps = 40
    c = [mp.mpf(v) for v in _device_coefficients()]
    a = mp.log(2) / 2
    worst = mp.mpf(0)
    for k in range(801):
        r = -a + 2 * a * k / 800
        p = mp.polyval(c[::-1], r)
        worst = max(worst, abs(p / mp.exp(r) - 1))
    assert worst < 3.2e-16
