"""Host emulation of the per-event FP64 sequences of the device library
(reciprocal and reciprocal square root from a hardware seed plus one
Newton-Raphson step; the reciprocal with a further second-order term for the
logarithm; the logarithm by argument reduction and the atanh series), with
every fused multiply-add evaluated exactly and rounded once (rational
arithmetic), and with seeds perturbed to twice the worst relative error
measured for the gfx950 approximations (2^-24.1): the one-step results stay
within their second-order bounds (relative e^2 for the reciprocal, 1.5 e^2 for
the reciprocal square root, e the seed's error, plus the roundings), the
second-order reciprocal and the logarithm within about one unit in the last
place of the exact values; the grouped reciprocal (one reciprocal of a product
of up to four denominators) within the seed's term plus its roundings."""
import math
import random
from decimal import Decimal, getcontext
from fractions import Fraction

getcontext().prec = 60

SEED_ERR = 2.0 ** -23


def fma(a, b, c):
    return float(Fraction(a) * Fraction(b) + Fraction(c))


def seeded(exact, rng):
    """A seed with relative error uniform in [-SEED_ERR, SEED_ERR] (its ends included now and then)."""
    d = rng.choice([-SEED_ERR, SEED_ERR, rng.uniform(-SEED_ERR, SEED_ERR)])
    return float(exact * (1 + Fraction(d)))


def rcp_fast(x, rng):
    r = seeded(1 / Fraction(x), rng)
    e = fma(-x, r, 1.0)
    return fma(r, e, r)


def rcp_acc(x, rng):
    r = seeded(1 / Fraction(x), rng)
    e = fma(-x, r, 1.0)
    return fma(r, fma(e, e, e), r)


def rsqrt_fast(x, rng):
    exact = Fraction(1 / Decimal(x).sqrt())
    y = seeded(exact, rng)
    e = fma(-x * y, y, 1.0)
    return fma(y * 0.5, e, y)


def rel_err(v, exact):
    return float(abs(Fraction(v) - Fraction(exact)) / abs(Fraction(exact)))


def ulps(v, exact):
    """|v - exact| in units in the last place of exact."""
    ex = float(exact)
    return float(abs(Fraction(v) - Fraction(exact))) / math.ulp(ex)


def samples(rng, n):
    for _ in range(n):
        yield math.ldexp(1.0 + rng.random(), rng.randint(-60, 60))


def test_reciprocal_second_order_bound():
    """One Newton step: r (1 + e) = (1 - e^2) / x for a seed r = (1 - e) / x,
    so the relative error is e^2 plus the final rounding; seeds at the
    extremes of their error range reach it."""
    rng = random.Random(11)
    worst = max(rel_err(rcp_fast(x, rng), 1 / Fraction(x)) for x in samples(rng, 3000))
    assert worst <= SEED_ERR ** 2 + 2.0 ** -52, worst
    assert worst >= 0.5 * SEED_ERR ** 2, worst


def test_reciprocal_square_root_second_order_bound():
    """One Newton step on y = (1 - d) / sqrt(x): the result is
    (1 - 1.5 d^2 + 0.5 d^3) / sqrt(x), plus the roundings of x y and of the
    final FMA."""
    rng = random.Random(12)
    worst = 0.0
    for x in samples(rng, 2000):
        exact = Fraction(1 / Decimal(x).sqrt())
        worst = max(worst, rel_err(rsqrt_fast(x, rng), exact))
    assert worst <= 1.5 * SEED_ERR ** 2 + 2.0 ** -52 + 2.0 ** -53, worst
    assert worst >= 0.5 * SEED_ERR ** 2, worst


def test_second_order_reciprocal_within_one_ulp():
    """With the e^2 term the error is third order and the result is within one
    unit in the last place."""
    rng = random.Random(13)
    worst = max(ulps(rcp_acc(x, rng), 1 / Fraction(x)) for x in samples(rng, 3000))
    assert worst <= 1.0, worst


LN2_HI = float.fromhex("0x1.62e42ff000000p-1")
LN2_LO = float.fromhex("-0x1.718432a1b0e26p-35")


def log_fast(x, rng):
    m, e = math.frexp(x)  # m in [0.5, 1)
    if m < 0.70710678118654752440:
        m, e = 2.0 * m, e - 1
    f = (m - 1.0) * rcp_acc(m + 1.0, rng)
    f2 = f * f
    p = 1.0 / 23.0
    for c in (21, 19, 17, 15, 13, 11, 9, 7, 5, 3):
        p = fma(p, f2, 1.0 / c)
    f2x = 2.0 * f
    lm = fma(f2x * f2, p, f2x)
    de = float(e)
    return fma(de, LN2_HI, fma(de, LN2_LO, lm))


def test_log_split_constant():
    """ln 2 = head + tail to far below double precision, with a 32-bit head
    (so e * head is exact for |e| < 2^21)."""
    ln2 = Decimal(2).ln()
    assert abs(Decimal(LN2_HI) + Decimal(LN2_LO) - ln2) < Decimal(2) ** -85
    assert Fraction(LN2_HI).denominator.bit_length() - 1 <= 32


def test_log_series_truncation():
    """Eleven terms of 2 atanh(f) for |f| <= (sqrt 2 - 1)/(sqrt 2 + 1): the
    first omitted term, 2 f^23 / 23, is below 3e-17 of ln m."""
    fmax = (Decimal(2).sqrt() - 1) / (Decimal(2).sqrt() + 1)
    first_omitted = 2 * fmax ** 23 / 23
    lnm = Decimal(2).sqrt().ln()  # |ln m| at the end of the range
    assert first_omitted / lnm < Decimal("3e-17")


def test_log_accuracy():
    rng = random.Random(14)
    xs = list(samples(rng, 1500)) + [1.0, 2.0, 0.5, 0.7071067811865476, 0.7071067811865475,
                                     1.4142135623730951, 1e-300, 1e300, 1.0 + 2 ** -52, 1.0 - 2 ** -53]
    worst = 0.0
    for x in xs:
        exact = Decimal(x).ln()
        v = log_fast(x, rng)
        if exact == 0:
            assert v == 0.0
            continue
        # absolute error near x = 1 (where ln x -> 0) is measured against the ulp of 1e-16
        err = abs(Decimal(v) - exact)
        scale = max(abs(exact), Decimal("1e-16"))
        worst = max(worst, float(err / scale))
    assert worst < 2.5e-16, worst


class LogProd:
    """The device running product: m in [0.5, 1) times 2^e, split after every
    factor (frexp, as the hardware mantissa/exponent instructions for finite
    non-zero values), one logarithm at the end."""

    def __init__(self):
        self.m, self.e = 1.0, 0

    def mul(self, x):
        p = self.m * x  # one IEEE rounding, like the device multiply
        mant, ex = math.frexp(p)
        self.m, self.e = mant, self.e + ex

    def log(self, rng):
        de = float(self.e)
        return fma(de, LN2_HI, fma(de, LN2_LO, log_fast(self.m, rng)))


def test_logprod_sum_accuracy():
    """The sum of logarithms of n factors through the running product is within
    n 2^-53 + 3e-16 (absolute, scaled by max(1, |sum|)) of the exact sum, for
    factors spread over the double range and for long runs of factors near
    the density values of the fits (where the product alone would underflow)."""
    rng = random.Random(18)
    cases = []
    for n in (1, 2, 8, 64, 1000):
        cases.append([math.ldexp(1.0 + rng.random(), rng.randint(-300, 300)) for _ in range(n)])
        cases.append([rng.uniform(1e-4, 10.0) for _ in range(n)])
    cases.append([1e-300] * 50)  # the plain product would underflow after two factors
    cases.append([1e300] * 50)
    for xs in cases:
        lp = LogProd()
        for x in xs:
            lp.mul(x)
        v = lp.log(rng)
        exact = sum(Decimal(x).ln() for x in xs)
        bound = (len(xs) * Decimal(2) ** -53 + Decimal("3e-16")) * max(Decimal(1), abs(exact))
        assert abs(Decimal(v) - exact) <= bound, (len(xs), v, exact)


def test_logprod_special_factors():
    """A zero factor gives -inf, a negative one NaN, as the summed logarithms would."""
    rng = random.Random(19)
    lp = LogProd()
    for x in (2.0, 0.0, 3.0):
        lp.mul(x)
    assert lp.m == 0.0  # the device's log of 0 is -inf (checked in the log emulation's domain)
    lp = LogProd()
    for x in (2.0, -1.0):
        lp.mul(x)
    assert lp.m < 0.0  # log of a negative mantissa: NaN on the device


def rcp_group(D, rng):
    """The grouped reciprocal of csrc/fastmath.hpp: prefix products, one
    seeded reciprocal with its Newton step, then the reciprocals peeled from
    the top down (each product a correctly rounded double multiply)."""
    n = len(D)
    p = [D[0]]
    for j in range(1, n):
        p.append(p[j - 1] * D[j])
    r = rcp_fast(p[n - 1], rng)
    out = [0.0] * n
    for j in range(n - 1, 0, -1):
        out[j] = r * p[j - 1]
        r = r * D[j]
    out[0] = r
    return out


def test_grouped_reciprocals_within_bound():
    """1/D_j from one reciprocal of the product of n <= 4 denominators (spread
    over nine decades, as Breit-Wigner denominators are): the error stays
    below the seed's second-order term plus 3 n roundings."""
    rng = random.Random(17)
    for n in (1, 2, 3, 4):
        worst = 0.0
        for _ in range(400):
            D = [10.0 ** rng.uniform(-6.0, 3.0) for _ in range(n)]
            got = rcp_group(D, rng)
            worst = max(worst, max(rel_err(g, 1 / Fraction(d)) for g, d in zip(got, D)))
        assert worst <= SEED_ERR ** 2 + 3 * n * 2.0 ** -53, (n, worst)
