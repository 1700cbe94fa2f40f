"""The flat-sky pair kernel's reciprocal (exponent-negation seed and two
third-order Newton steps, `recip_newton` in csrc/flat.hip), emulated in FP32
on the CPU: every operation of the kernel is one correctly rounded FP32
operation (an FMA's product of two FP32 values is exact in FP64, so FP64
then one rounding to FP32 emulates it, up to a double rounding whose effect
is far below the bound).  Pinned against the exact 1/x in FP64: the error
bound follows from the seed's range x*y0 in [1, 1.125] and the cubing of the
relative error by each step (1.25e-1, 2.0e-3, 7.5e-9 before rounding), so
the result is within 0.6 ulp of 1/x, over the operand range the kernel
uses (products of two floored squared distances, [1e-36, 1e18))."""
import os
import re

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _seed_constant():
    src = open(os.path.join(ROOT, "paper_1204_5041_amd", "csrc", "flat.hip")).read()
    m = re.search(r"float recip_newton\(float x\) \{\s*float y = __uint_as_float\((0x[0-9A-Fa-f]+)u", src)
    assert m, "recip_newton's seed not found"
    return np.uint32(int(m.group(1), 16))


def _fma32(a, b, c):
    return (a.astype(np.float64) * b.astype(np.float64) + c.astype(np.float64)).astype(np.float32)


def _recip(x, k):
    y = (k - x.view(np.uint32)).view(np.float32)
    one = np.ones_like(x)
    for _ in range(2):
        e = _fma32(-x, y, one)
        y = _fma32(y, _fma32(e, e, e), y)
    return y, (k - x.view(np.uint32)).view(np.float32)


def test_seed_is_the_bits_of_two_to_127():
    # 2^127 = (127 + 127) << 23: subtracting x's bits negates its exponent.
    assert _seed_constant() == np.float32(2.0 ** 127).view(np.uint32)


def test_newton_reciprocal_within_0p6_ulp():
    rng = np.random.default_rng(17)
    m = rng.uniform(1.0, 2.0, 1_000_000)
    x = (m * 2.0 ** rng.integers(-119, 60, m.size)).astype(np.float32)
    p2 = (2.0 ** np.arange(-119, 60)).astype(np.float32)
    x = np.concatenate([x, p2, np.nextafter(p2, np.float32(np.inf)),
                        np.nextafter(p2, np.float32(0))])
    x = x[(x >= 1e-36) & (x < 1e18)]
    y, y0 = _recip(x, _seed_constant())
    ref = 1.0 / x.astype(np.float64)
    # the seed's range, which the error bound rests on
    s = x.astype(np.float64) * y0.astype(np.float64)
    assert s.min() >= 1.0 and s.max() <= 1.125
    ulp = np.spacing(ref.astype(np.float32)).astype(np.float64)
    err = np.abs(y.astype(np.float64) - ref) / ulp
    assert err.max() <= 0.6, err.max()
    # exact at powers of two
    yp, _ = _recip(p2, _seed_constant())
    assert np.array_equal(yp, (1.0 / p2.astype(np.float64)).astype(np.float32))
