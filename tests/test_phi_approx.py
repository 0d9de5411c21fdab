"""The device approximation of the check-rule transform (csrc/phi.hpp), checked on the host.

The kernels evaluate g(x) = phi(x ln2) / ln2 with phi(x) = -ln tanh(x/2) (Sec. II-A,
eq. equ_s2e5) from two degree-3 polynomials and one hardware log2 / exp2.  This test reads
the coefficients out of the header, evaluates the same float32 operation sequence in numpy
(FMA emulated in float64 and rounded once) and compares with the closed form in float64.
"""
import re
from pathlib import Path

import numpy as np

HEADER = Path(__file__).resolve().parents[1] / "paper_2305_05286_amd" / "csrc" / "phi.hpp"
f32 = np.float32
LN2 = np.log(2.0)


def _coefficients():
    src = HEADER.read_text()
    body = src[src.index("float phi2(float x)"):]
    body = body[:body.index("\n}\n")]
    nums = [float(m) for m in re.findall(r"(-?\d+\.\d+(?:e-?\d+)?)f", body)]
    # p = c3; p = fma(p, uu, c2) ... c0 ; then u = d3; u = fma(u, s, d2) ... d0
    small, large = nums[:4], nums[4:8]
    return [f32(c) for c in small], [f32(c) for c in large]


def _fma(a, b, c):
    return f32(np.float64(a) * np.float64(b) + np.float64(c))


def _horner(cs, y):
    p = cs[0]
    for c in cs[1:]:
        p = _fma(p, y, c)
    return p


def phi2_emulated(x):
    small_c, large_c = _coefficients()
    x = f32(x)
    if x < f32(1.4426950408889634):
        return f32(-np.log2(f32(x * _horner(small_c, f32(x * x)))))
    t = f32(np.exp2(f32(-x)))
    return f32(t * _horner(large_c, f32(t * t)))


def phi2_exact(x):
    x = np.float64(x) * LN2
    return np.log1p(2.0 / np.expm1(x)) / LN2


def test_coefficients_parsed():
    small_c, large_c = _coefficients()
    assert len(small_c) == 4 and len(large_c) == 4
    # leading terms of the two expansions: tanh(ln2 sqrt(u)/2)/sqrt(u) -> ln2/2, and
    # (2/ln2) atanh(sqrt s)/sqrt s -> 2/ln2
    assert abs(small_c[-1] - LN2 / 2) < 1e-6
    assert abs(large_c[-1] - 2 / LN2) < 1e-6


def test_relative_error_bound():
    xs = np.concatenate([np.geomspace(5e-9, 60.0, 4000), np.linspace(1.40, 1.48, 400)])
    xs = xs.astype(np.float32)  # compare at the float32 input the kernel sees
    err = max(abs(float(phi2_emulated(x)) - phi2_exact(x)) / phi2_exact(x) for x in xs)
    assert err < 1e-6, err


def test_self_inverse():
    # g(g(x)) = x because phi is an involution (the property that lets one function
    # serve B2V and C2B in log2 units)
    for x in np.geomspace(1e-3, 25.0, 300):
        y = phi2_emulated(phi2_emulated(x))
        assert abs(float(y) - x) <= 2e-5 * max(x, 1.0), (x, y)


def test_split_is_continuous():
    lo = phi2_emulated(np.nextafter(f32(1.4426950408889634), f32(0)))
    hi = phi2_emulated(f32(1.4426950408889634))
    # each side is within the 1e-6 bound of the closed form, so they differ by under 2e-6
    assert abs(float(lo) - float(hi)) / float(hi) < 2e-6
