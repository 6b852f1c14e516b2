"""Field arithmetic for the oracle (test infrastructure only).

Three fields share one interface so that the recursion in ``oracle.bg`` is
written once:

* ``Fp(p)``      -- the prime field Z_p, elements are Python ints in [0, p).
                    The paper fixes p < 2^31 with default p = 2^31 - 19
                    (Sec. 3, finite-field representation); the oracle accepts
                    any odd prime.  Inverse by Fermat, x^(p-2) mod p; the
                    paper uses the extended Euclidean algorithm (Sec. 3), and
                    the inverse is unique, so both give the same residue.
* ``Complex128`` -- Python ``complex`` (IEEE binary64 real and imaginary parts),
                    the double-precision complex path of the paper (Sec. 3).
* ``Rationals``  -- ``fractions.Fraction``, exact; used to arbitrate FP64
                    rounding and to tie the two other fields together.
* ``GaussianRationals`` -- pairs of Fractions (a + b i), exact; the exact
                    value of an FP64 complex input (every binary64 number is a
                    dyadic rational), used to arbitrate complex rounding.

Minkowski products use the mostly-minus metric diag(+1, -1, ..., -1) of
Sec. 2.3 (the completeness relation is written with the "mostly negative
metric"), bilinear (no complex conjugation).

Parity: pinned.  F_p ops against Python's own integer arithmetic and
``pow(x, -1, p)``; Q ops against ``fractions``; see tests/test_oracle_fields.py.
"""
from __future__ import annotations

from fractions import Fraction


def is_prime(p: int) -> bool:
    """Deterministic trial division (oracle side; fine for p < 2^31)."""
    if p < 2:
        return False
    if p % 2 == 0:
        return p == 2
    f = 3
    while f * f <= p:
        if p % f == 0:
            return False
        f += 2
    return True


class Fp:
    """Z_p with canonical representatives in [0, p)."""

    name = "fp"
    exact = True

    def __init__(self, p: int):
        if not is_prime(p) or p == 2:
            raise ValueError(f"{p} is not an odd prime")
        self.p = p

    def __repr__(self):
        return f"Fp({self.p})"

    def elem(self, x) -> int:
        if isinstance(x, Fraction):
            return (x.numerator * pow(x.denominator, self.p - 2, self.p)) % self.p
        return int(x) % self.p

    zero = 0
    one = 1

    def add(self, a, b):
        return (a + b) % self.p

    def sub(self, a, b):
        return (a - b) % self.p

    def mul(self, a, b):
        return (a * b) % self.p

    def neg(self, a):
        return (-a) % self.p

    def inv(self, a):
        if a % self.p == 0:
            raise ZeroDivisionError("inverse of 0 in F_p")
        return pow(a, self.p - 2, self.p)

    def is_zero(self, a) -> bool:
        return a % self.p == 0


class Complex128:
    """IEEE binary64 complex numbers (Python ``complex``)."""

    name = "c128"
    exact = False
    zero = 0j
    one = 1 + 0j

    def elem(self, x) -> complex:
        return complex(x)

    def add(self, a, b):
        return a + b

    def sub(self, a, b):
        return a - b

    def mul(self, a, b):
        return a * b

    def neg(self, a):
        return -a

    def inv(self, a):
        if a == 0:
            raise ZeroDivisionError("inverse of 0 in C")
        return 1 / a

    def is_zero(self, a) -> bool:
        return a == 0


class Rationals:
    """Exact rationals; complex values are not needed on this field."""

    name = "q"
    exact = True
    zero = Fraction(0)
    one = Fraction(1)

    def elem(self, x) -> Fraction:
        return Fraction(x)

    def add(self, a, b):
        return a + b

    def sub(self, a, b):
        return a - b

    def mul(self, a, b):
        return a * b

    def neg(self, a):
        return -a

    def inv(self, a):
        if a == 0:
            raise ZeroDivisionError("inverse of 0 in Q")
        return 1 / a

    def is_zero(self, a) -> bool:
        return a == 0


def mdot(F, x, y):
    """Bilinear Minkowski product x.y = x^0 y^0 - sum_{mu>=1} x^mu y^mu."""
    s = F.mul(x[0], y[0])
    for mu in range(1, len(x)):
        s = F.sub(s, F.mul(x[mu], y[mu]))
    return s


def adot(F, x, y):
    """Bilinear product in the alternating metric diag(1, -1, 1, -1, ...)
    (the option of paper Sec. 3.1 that matches Caravel's convention):
    x.y = sum_mu (-1)^mu x^mu y^mu."""
    s = F.zero
    for mu in range(len(x)):
        t = F.mul(x[mu], y[mu])
        s = F.add(s, t) if mu % 2 == 0 else F.sub(s, t)
    return s


METRICS = {"mostly-minus": mdot, "alternating": adot}


def metric_dot(metric):
    """The bilinear product of a metric name ("mostly-minus" or "alternating")."""
    try:
        return METRICS[metric]
    except KeyError:
        raise ValueError(f"unknown metric {metric!r}") from None


def vadd(F, x, y):
    return [F.add(a, b) for a, b in zip(x, y)]


def vsub(F, x, y):
    return [F.sub(a, b) for a, b in zip(x, y)]


def vscale(F, c, x):
    return [F.mul(c, a) for a in x]


class GaussianRationals:
    """Exact complex rationals a + b i as (Fraction, Fraction) pairs."""

    name = "qi"
    exact = True
    zero = (Fraction(0), Fraction(0))
    one = (Fraction(1), Fraction(0))

    def elem(self, x):
        if isinstance(x, tuple):
            return (Fraction(x[0]), Fraction(x[1]))
        z = complex(x)
        return (Fraction(z.real), Fraction(z.imag))

    def add(self, a, b):
        return (a[0] + b[0], a[1] + b[1])

    def sub(self, a, b):
        return (a[0] - b[0], a[1] - b[1])

    def mul(self, a, b):
        return (a[0] * b[0] - a[1] * b[1], a[0] * b[1] + a[1] * b[0])

    def neg(self, a):
        return (-a[0], -a[1])

    def inv(self, a):
        n = a[0] * a[0] + a[1] * a[1]
        if n == 0:
            raise ZeroDivisionError("inverse of 0 in Q(i)")
        return (a[0] / n, -a[1] / n)

    def is_zero(self, a) -> bool:
        return a[0] == 0 and a[1] == 0

    @staticmethod
    def to_complex(a) -> complex:
        return complex(float(a[0]), float(a[1]))


class RunningError:
    """Complex binary64 values carried with a first-order rounding-error bound.

    Elements are (v, e): v the binary64 result of the operation exactly as
    ``Complex128`` computes it, e a bound, in units of the unit roundoff
    u = 2^-53, on |v - exact| accumulated to first order (running error
    analysis, Wilkinson 1963):
        e(a +- b) = e(a) + e(b) + |a +- b|
        e(a * b)  = |a| e(b) + |b| e(a) + 4 |a b|     (complex product, one rounding per part)
        e(1 / a)  = e(a) / |a|^2 + 4 |1 / a|
    Used only to size the tolerance floor of complex parity checks: two
    evaluations of the same amplitude in different orders differ by at most
    about u (e_1 + e_2).
    """

    name = "c128_err"
    exact = False
    zero = (0j, 0.0)
    one = (1 + 0j, 0.0)

    def elem(self, x):
        return (complex(x), 0.0)

    def add(self, a, b):
        v = a[0] + b[0]
        return (v, a[1] + b[1] + abs(v))

    def sub(self, a, b):
        v = a[0] - b[0]
        return (v, a[1] + b[1] + abs(v))

    def mul(self, a, b):
        v = a[0] * b[0]
        return (v, abs(a[0]) * b[1] + abs(b[0]) * a[1] + 4 * abs(v))

    def neg(self, a):
        return (-a[0], a[1])

    def inv(self, a):
        if a[0] == 0:
            raise ZeroDivisionError("inverse of 0 in C")
        v = 1 / a[0]
        return (v, a[1] / abs(a[0]) ** 2 + 4 * abs(v))

    def is_zero(self, a) -> bool:
        return a[0] == 0
