"""Bounds the Legendre kernel (k_legendre in csrc/alm.hip) relies on: the
overflow margin of its scaled recursion and the bound with which it drops
whole blocks of negligible terms.

Overflow margin.  The kernel runs mu_l = (a_l z) mu_{l-1} + mu_{l-2}, a_l = A_l c_{l-1} / c_l,
c_m = c_{m+1} = 1, c_l = -A_l B_l c_{l-2}, with A_l and B_l the coefficients
of the normalised associated Legendre recursion (lambda_l = c_l mu_l).  A
ring whose lambda_mm lies below 2^-600 carries its values as v * 2^(600 e)
and divides them by 2^600 once max(|mu_l|, |mu_{l-1}|) exceeds 2^600; the
kernel tests this only every 32 degrees.  That is safe while 32 steps can
grow the pair by less than 2^424 (the room between 2^600 and the double
range).  With |z| <= 1, one step grows max(|mu_l|, |mu_{l-1}|) by at most
|a_l| + 1, so the product of |a_l| + 1 over any 32 consecutive degrees
bounds the growth.  Computed here from the coefficient formulas, in log2,
for lmax 4096 (every m) and lmax 32768, the largest the API accepts (every
m of the top 512, where the first steps' |a_l| ~ sqrt(2m) is largest, and
every 61st below)."""
import numpy as np
import pytest


def _window_growth_log2(m: int, lmax: int, window: int) -> float:
    l = np.arange(m, lmax + 1, dtype=np.float64)
    n = len(l)
    A = np.zeros(n)
    log_ab = np.zeros(n)
    if n > 1:
        A[1] = np.sqrt(2.0 * m + 3.0)
    if n > 2:
        ll = l[2:]
        A[2:] = np.sqrt((4 * ll * ll - 1) / (ll * ll - m * m))
        B = np.sqrt(((ll - 1) ** 2 - m * m) / (4 * (ll - 1) ** 2 - 1))
        log_ab[2:] = np.log2(A[2:] * B)
    # log2 |c_l|: the even and odd degrees form two product chains.
    log_c = np.zeros(n)
    log_c[0::2] = np.cumsum(log_ab[0::2])
    log_c[1::2] = np.cumsum(log_ab[1::2])
    step = np.zeros(n)
    step[1:] = np.log2(A[1:] * np.exp2(log_c[:-1] - log_c[1:]) + 1.0)
    cs = np.concatenate([[0.0], np.cumsum(step)])
    if n < window:
        return float(cs[-1])
    return float(np.max(cs[window:] - cs[:-window]))


def _worst(lmax: int, ms) -> float:
    return max(_window_growth_log2(m, lmax, 32) for m in ms)


def test_growth_bound_lmax4096_every_m():
    g = _worst(4096, range(0, 4097))
    assert 140.0 < g < 424.0 - 200.0, g


@pytest.mark.parametrize("lmax", [8192, 32768])
def test_growth_bound_large_lmax(lmax):
    ms = sorted(set(range(max(0, lmax - 511), lmax + 1)) | set(range(0, lmax + 1, 61)))
    g = _worst(lmax, ms)
    assert g < 424.0 - 200.0, g


def test_growth_bound_is_attained_by_the_first_steps():
    # The bound is largest where A_{m+1} = sqrt(2m + 3) is: at the top m.
    # Restricting to m <= lmax/2 must give a smaller bound, which makes the
    # sampled large-lmax cases above cover the maximum.
    lo = _worst(4096, range(0, 2049))
    hi = _worst(4096, range(4000, 4097))
    assert lo < hi



def test_gegenbauer_bound_on_oracle_lambda():
    """|lambda_lm(cos theta)| <= sqrt((2l+1)/4pi) sin^m sqrt((l+m)!/(l-m)!) /
    (2^m m!), the bound with which the Legendre kernel drops whole blocks,
    holds on the oracle's lambda_lm (log2, 1e-9 slack) over a grid of m and
    theta, at every degree up to lmax = 1024."""
    import math
    import oracle
    L = 1024
    for m in (0, 1, 5, 50, 300, 700, 1000):
        for th in (1e-3, 0.05, 0.3, 0.7, 1.2, 1.5707963267948966):
            s, z = math.sin(th), math.cos(th)
            lam = oracle.lambda_lm(L, m, z, s)
            l = np.arange(m, L + 1, dtype=np.float64)
            lg = (0.5 * np.log2((2 * l + 1) / (4 * math.pi)) + m * math.log2(s) +
                  (0.5 * (np.array([math.lgamma(x + m + 1) - math.lgamma(x - m + 1) for x in l]))
                   - math.lgamma(m + 1)) / math.log(2) - m)
            nz = lam != 0
            assert np.all(np.log2(np.abs(lam[nz])) <= lg[nz] + 1e-9), (m, th)

