"""The index arithmetic of the ring transforms' LDS FFT (csrc/alm.hip:
`fft_pass`, `fft_dif`, `fft_dit_inv`, `dif_pos`, `fft_slot`, `fft_twiddle`,
`tw_slot`), emulated on the CPU in complex128 and pinned against numpy's
FFT.  The map2alm parity tests check the kernels themselves; this checks the
layout decisions they rest on, at every transform size the kernels take:

- the radix-8 decimation-in-frequency passes (one radix-4 or radix-2 pass
  last when log2 P is not a multiple of 3) leave frequency k at
  `dif_pos(k)`, the base-8 digits of k reversed;
- the inverse passes, in reverse order, undo them up to the factor P;
- the point slots j ^ ((j >> 3) & 15) and the twiddle-table slots
  r ^ ((r >> 4) & 15) ^ (r >> 8) are permutations of their ranges, so that
  storing through them changes no result;
- every twiddle e^{-2 pi i k/4096} is exact from the quarter-period table,
  (-i)^q e^{-2 pi i r/4096} for k = 1024 q + r;
- the swizzled point slots put the lanes of every radix-8 pass in distinct
  banks of 16-byte slots, for groups of 8 and of 16 lanes."""
import numpy as np
import pytest

NMAX = 4096          # kFftMaxP
QTR = NMAX // 4      # kTwQ


def slot(j, swz):
    return j ^ ((j >> 3) & 15) if swz else j


def tw_slot(r):
    return r ^ ((r >> 4) & 15) ^ (r >> 8)


def _table():
    # The quarter table as the kernels hold it in LDS: entry r at tw_slot(r).
    t = np.zeros(QTR, dtype=np.complex128)
    r = np.arange(QTR)
    t[tw_slot(r)] = np.exp(-2j * np.pi * r / NMAX)
    return t


TAB = _table()


def twiddle(k):
    q, r = k >> 10, k & (QTR - 1)
    u = TAB[tw_slot(r)]
    x, y = (u.imag, u.real) if q & 1 else (u.real, u.imag)
    if q & 2:
        x = -x
    if (q ^ (q >> 1)) & 1:
        y = -y
    return complex(x, y)


def dft_small(v, inv):
    R = len(v)
    e = np.arange(R)
    return np.exp((1j if inv else -1j) * 2 * np.pi * np.outer(e, e) / R) @ v


def fft_pass(x, P, S, R, inv, swz):
    h, tw = S // R, NMAX // S
    for b in range(P // R):
        pos = b & (h - 1)
        base = (b - pos) * R + pos
        idx = [slot(base + q * h, swz) for q in range(R)]
        v = x[idx]
        if not inv:
            v = dft_small(v, False)
        w = np.array([twiddle((pos * q * tw) & (NMAX - 1)) for q in range(R)])
        v = v * (np.conj(w) if inv else w)
        if inv:
            v = dft_small(v, True)
        x[idx] = v


def fft_dif(x, P, swz):
    S = P
    while S >= 8:
        fft_pass(x, P, S, 8, False, swz)
        S >>= 3
    if S == 4:
        fft_pass(x, P, 4, 4, False, swz)
    if S == 2:
        fft_pass(x, P, 2, 2, False, swz)


def fft_dit_inv(x, P, swz):
    e = P.bit_length() - 1
    S = 1 << (e % 3)
    if S == 4:
        fft_pass(x, P, 4, 4, True, swz)
    if S == 2:
        fft_pass(x, P, 2, 2, True, swz)
    while S < P:
        S <<= 3
        fft_pass(x, P, S, 8, True, swz)


def dif_pos(k, e):
    p = 0
    while e >= 3:
        p |= (k & 7) << (e - 3)
        e -= 3
        k >>= 3
    return p | k


def test_slots_are_permutations():
    for e in range(1, 13):
        P = 1 << e
        j = np.arange(P)
        assert np.array_equal(np.sort(slot(j, True)), j), P
    r = np.arange(QTR)
    assert np.array_equal(np.sort(tw_slot(r)), r)


def test_quarter_table_twiddles_exact():
    k = np.arange(NMAX)
    got = np.array([twiddle(int(x)) for x in k])
    ref = np.exp(-2j * np.pi * k / NMAX)
    # The reference is numpy's exp at the rounded angle 2 pi k/4096, whose
    # argument error reaches about 5e-16 near k = 4096; the table entry a
    # quarter period away is rotated exactly.
    assert np.max(np.abs(got - ref)) < 1e-15


@pytest.mark.parametrize("e", list(range(1, 13)))
@pytest.mark.parametrize("swz", [False, True])
def test_forward_digit_reversed_and_inverse(e, swz):
    P = 1 << e
    rng = np.random.default_rng(100 + e)
    z = rng.standard_normal(P) + 1j * rng.standard_normal(P)
    x = np.zeros(P, dtype=np.complex128)
    x[slot(np.arange(P), swz)] = z
    fft_dif(x, P, swz)
    got = np.array([x[slot(dif_pos(k, e), swz)] for k in range(P)])
    Z = np.fft.fft(z)
    assert np.max(np.abs(got - Z)) <= 1e-14 * np.max(np.abs(Z))
    fft_dit_inv(x, P, swz)
    back = x[slot(np.arange(P), swz)] / P
    assert np.max(np.abs(back - z)) <= 1e-14 * np.max(np.abs(z))


@pytest.mark.parametrize("group", [8, 16])
def test_swizzled_radix8_passes_have_no_bank_conflicts(group):
    # 16-byte slots, one bank group per slot modulo `group`: within every
    # aligned group of lanes, the points a radix-8 pass reads or writes
    # (base + q h for a fixed q) fall into distinct slots modulo the group.
    for e in range(3, 13):
        P = 1 << e
        S = P
        while S >= 8:
            h = S // 8
            b = np.arange(P // 8)
            pos = b & (h - 1)
            base = (b - pos) * 8 + pos
            for q in range(8):
                s = slot(base + q * h, True) % group
                for g0 in range(0, P // 8, group):
                    chunk = s[g0:g0 + group]
                    assert len(set(chunk.tolist())) == len(chunk), (P, S, q, g0)
            S >>= 3
