"""The flat-sky pair kernel's reciprocal (exponent-negation seed, one
third-order and one second-order Newton step, `recip_newton` in
csrc/flat.hip), emulated in FP32 on the CPU: every operation of the kernel is one correctly rounded FP32
operation (an FMA's product of two FP32 values is exact in FP64, so FP64
then one rounding to FP32 emulates it, up to a double rounding whose effect
is far below the bound).  Pinned against the exact 1/x in FP64: the seed's
relative error is at most 5.05e-2 (the constant is the bits of 2^127 less
the shift that minimises it), the third-order step cubes it (1.3e-4) and the
second-order step squares it (1.7e-8 before rounding), so the result is
within 0.8 ulp of 1/x over [2^-125, 2^125].  The kernel's operands are
products of two floored squared distances: at least 1e-36 > 2^-125 by the
floor, and below 2^122 because csmap_render_flat rejects patches whose
pixel-segment offsets could exceed 2^30 pixels (tan(rho)/pix + max(nx, ny)
<= 2^30, so each squared distance is below 2 (2^30)^2)."""
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
    y0 = (k - x.view(np.uint32)).view(np.float32)
    one = np.ones_like(x)
    e = _fma32(-x, y0, one)
    y = _fma32(y0, _fma32(e, e, e), y0)
    e = _fma32(-x, y, one)
    return _fma32(y, e, y), y0


def _seed_error(k):
    mant = np.linspace(1.0, 2.0, 1 << 20, endpoint=False).astype(np.float32)
    y0 = (np.uint32(k) - mant.view(np.uint32)).view(np.float32)
    return np.abs(1.0 - mant.astype(np.float64) * y0.astype(np.float64)).max()


def test_seed_minimises_the_seed_error():
    # 2^127 = (127 + 127) << 23: subtracting x's bits negates its exponent
    # (seed error 12.5%); the constant is that one shifted to the minimum.
    k = int(_seed_constant())
    base = int(np.float32(2.0 ** 127).view(np.uint32))
    assert 0 < base - k < 1 << 20
    assert abs(_seed_error(base) - 0.125) < 1e-6
    e = _seed_error(k)
    assert e <= 0.0506
    assert e <= _seed_error(k - 256) and e <= _seed_error(k + 256)


def test_newton_reciprocal_within_0p8_ulp():
    rng = np.random.default_rng(17)
    m = rng.uniform(1.0, 2.0, 1_000_000)
    x = (m * 2.0 ** rng.integers(-125, 125, m.size)).astype(np.float32)
    p2 = (2.0 ** np.arange(-125, 126)).astype(np.float32)
    x = np.concatenate([x, p2, np.nextafter(p2, np.float32(np.inf)),
                        np.nextafter(p2, np.float32(0))])
    x = x[(x >= 2.0 ** -125) & (x <= 2.0 ** 125)]
    y, y0 = _recip(x, _seed_constant())
    ref = 1.0 / x.astype(np.float64)
    # the seed's error, which the bound rests on
    s = x.astype(np.float64) * y0.astype(np.float64)
    assert np.abs(1.0 - s).max() <= 0.0506
    ulp = np.spacing(ref.astype(np.float32)).astype(np.float64)
    err = np.abs(y.astype(np.float64) - ref) / ulp
    assert err.max() <= 0.8, err.max()


def test_operand_bound_of_the_flat_kernel():
    """The entry point's patch bound keeps the kernel's operands in range,
    and past 2^126 the seed wraps (why the bound is needed)."""
    off = 2.0 ** 30                       # largest pixel-segment offset admitted
    q_max = 2.0 * off * off               # squared distance, both axes at the bound
    assert q_max * q_max <= 2.0 ** 122 < 2.0 ** 125
    assert 1e-18 * 1e-18 >= 2.0 ** -125   # the floor of each squared distance
    big = np.array([1.7e38, 3e38], dtype=np.float32)
    y, _ = _recip(big, _seed_constant())
    assert not np.all(np.isfinite(y) & (np.abs(y * big.astype(np.float64) - 1.0) < 1e-6))
