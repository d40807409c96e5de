"""The integer carry step of the reduction kernel's 32-bit finish, checked on
the CPU with exact arithmetic.

For a digit base B (odd; p^e <= 169 for p >= 7) and a carry sum t with
|t| < 2^31, the kernel computes r = fma(t, 1/B, 1.5 2^52) in fp64, takes the
low 32-bit word of r as the carry q, and the digit as the low byte of
(q mod 2^24) (2^24 - B) + t.  The claims are: q = round(t / B) (no ties, B
odd), and the byte read as int8 is the balanced digit t - q B, |t - q B| <=
(B - 1) / 2.  A fused multiply-add rounds once, so r is the double nearest to
t * fl(1/B) + 1.5 2^52; Python's int / int division is correctly rounded,
which gives that double exactly from a Fraction.
"""
import random
import struct
from fractions import Fraction

import pytest

K = 3 << 51  # 1.5 2^52


def fma_exact(a, b, c):
    x = Fraction(a) * Fraction(b) + Fraction(c)
    return x.numerator / x.denominator  # correctly rounded to the nearest double


def low_word_signed(x):
    w = struct.unpack("<Q", struct.pack("<d", x))[0] & 0xFFFFFFFF
    return w - (1 << 32) if w >= 1 << 31 else w


def carry_step(t, B):
    q = low_word_signed(fma_exact(t, 1.0 / B, float(K)))
    du = (((q & 0xFFFFFF) * ((1 << 24) - B)) + (t & 0xFFFFFFFF)) & 0xFFFFFFFF
    d = du & 0xFF
    return q, d - 256 if d >= 128 else d


def digit_bases():
    bases = set()
    for p in (7, 11, 13, 17, 19, 23, 29, 31, 37, 41, 43, 47):
        e = 1
        while p ** (e + 1) <= 169:
            e += 1
        bases.add(p ** e)
    return sorted(bases)


def cases(B, rng):
    T = (1 << 31) - 1
    ts = [0, 1, -1, T, -T, B, -B, (B - 1) // 2, -(B - 1) // 2, (B + 1) // 2, -(B + 1) // 2]
    n_max = T // B
    for n in (n_max, -n_max, n_max - 1, -(n_max - 1)):
        for off in (-(B + 1) // 2, -(B - 1) // 2, 0, (B - 1) // 2, (B + 1) // 2):
            ts.append(n * B + off)
    for _ in range(300):
        n = rng.randint(-n_max, n_max)
        ts.append(n * B + rng.choice(((B - 1) // 2, -(B - 1) // 2, (B + 1) // 2)))
        ts.append(rng.randint(-T, T))
    return [t for t in ts if -T <= t <= T]


@pytest.mark.parametrize("B", digit_bases())
def test_integer_carry_is_exact(B):
    rng = random.Random(B)
    half = (B - 1) // 2
    for t in cases(B, rng):
        q, d = carry_step(t, B)
        want_q = (2 * t + B) // (2 * B)  # round(t / B); t / B is never a half-integer
        assert q == want_q, (B, t)
        assert d == t - want_q * B and -half <= d <= half, (B, t)


def test_balanced_digits_recombine():
    """Carrying a run of position sums z_0..z_(D-1) gives balanced digits
    whose value sum d_k B^k equals sum z_k B^k modulo B^D."""
    rng = random.Random(7)
    for B in digit_bases():
        D = 8
        for _ in range(50):
            z = [rng.randint(-(1 << 28), 1 << 28) for _ in range(D)]
            c, digits = 0, []
            for zk in z:
                c, d = carry_step(zk + c, B)
                digits.append(d)
            Q = B ** D
            assert sum(d * B ** k for k, d in enumerate(digits)) % Q == sum(zk * B ** k for k, zk in enumerate(z)) % Q
