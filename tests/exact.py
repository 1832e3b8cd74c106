"""Exact rational arithmetic used to pin the oracle (test helper).

Python's ``fractions.Fraction`` holds every binary floating-point value exactly,
and the sums and products below are exact.  ``round_to`` rounds an exact
rational to a binary format with a p-bit significand, to nearest with ties to
even, which is the IEEE default rounding.  Exponent range limits (overflow,
subnormals) are not modelled; the values used in the tests stay far from them.
"""
from __future__ import annotations

from fractions import Fraction

P_BITS = {"f64": 53, "f32": 24, "bf16": 8}


def round_to(q: Fraction, p: int) -> Fraction:
    q = Fraction(q)
    if q == 0:
        return Fraction(0)
    sign = -1 if q < 0 else 1
    a = abs(q)
    # find e with 2^(e) <= a < 2^(e+1)
    e = a.numerator.bit_length() - a.denominator.bit_length()
    if Fraction(2) ** e > a:
        e -= 1
    while Fraction(2) ** (e + 1) <= a:
        e += 1
    scale = Fraction(2) ** (p - 1 - e)  # a*scale in [2^(p-1), 2^p)
    t = a * scale
    fl = t.numerator // t.denominator
    rem = t - fl
    if rem > Fraction(1, 2) or (rem == Fraction(1, 2) and fl % 2 == 1):
        fl += 1
    return sign * Fraction(fl) / scale


def rn(q: Fraction, prec: str) -> Fraction:
    return round_to(q, P_BITS[prec])


def exact_dot(x, y) -> Fraction:
    s = Fraction(0)
    for a, b in zip(x, y):
        s += Fraction(float(a)) * Fraction(float(b))
    return s


def exact_dot_int(x, y) -> Fraction:
    """Exact inner product of float64 arrays via Python integers: each double is
    m * 2^e with integer m; all products are brought to the smallest exponent
    and summed as integers.  Much faster than Fraction for long vectors."""
    terms = []
    emin = None
    for a, b in zip(x, y):
        ma, ea = _split(float(a))
        mb, eb = _split(float(b))
        m, e = ma * mb, ea + eb
        terms.append((m, e))
        if m != 0 and (emin is None or e < emin):
            emin = e
    if emin is None:
        return Fraction(0)
    total = 0
    for m, e in terms:
        if m:
            total += m << (e - emin)
    return Fraction(total) * Fraction(2) ** emin if emin >= 0 else Fraction(total, 2 ** (-emin))


def _split(v: float):
    n, d = v.as_integer_ratio()  # d is a power of two
    return n, -(d.bit_length() - 1)


def dot2_bound(n: int, exact: Fraction, abs_sum: Fraction) -> float:
    """Error bound of Dot2 (Ogita, Rump, Oishi 2005):
    |res - x^T y| <= u |x^T y| + gamma_n^2 |x|^T |y|, u = 2^-53."""
    u = 2.0 ** -53
    g = n * u / (1 - n * u)
    return u * abs(float(exact)) + g * g * float(abs_sum)
