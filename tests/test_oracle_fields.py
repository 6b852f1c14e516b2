"""Pins for oracle.fields: the field operations against textbook definitions."""
import random
from fractions import Fraction

import pytest

from oracle import fields

P_DEFAULT = 2147483629  # 2^31 - 19, the paper's default prime (Sec. 3)
PRIMES = [P_DEFAULT, 2147483647, 1000000007, 10007, 97]


def test_primality_of_known_values():
    for p in PRIMES:
        assert fields.is_prime(p)
    for c in [1, 4, 9, 2147483627, 2147483649, 10007 * 97]:
        assert not fields.is_prime(c)
    assert P_DEFAULT == 2**31 - 19


@pytest.mark.parametrize("p", PRIMES)
def test_fp_ops_match_python_ints(p):
    F = fields.Fp(p)
    rng = random.Random(p)
    edge = [0, 1, 2, p - 2, p - 1]
    vals = edge + [rng.randrange(p) for _ in range(200)]
    for a in vals[:40]:
        for b in vals:
            assert F.add(a, b) == (a + b) % p
            assert F.sub(a, b) == (a - b) % p
            assert F.mul(a, b) == (a * b) % p
    for a in vals:
        if a:
            inv = F.inv(a)
            assert inv == pow(a, -1, p)           # Python's own modular inverse
            assert (a * inv) % p == 1
    with pytest.raises(ZeroDivisionError):
        F.inv(0)


def test_fp_rejects_non_primes():
    with pytest.raises(ValueError):
        fields.Fp(2147483631)   # 2^31 - 17 = 3 * 715827877
    with pytest.raises(ValueError):
        fields.Fp(2)


def test_fraction_to_fp_reduction():
    F = fields.Fp(P_DEFAULT)
    x = Fraction(-7, 13)
    assert (F.elem(x) * 13) % P_DEFAULT == (-7) % P_DEFAULT


def test_minkowski_product_signature():
    for F in (fields.Fp(97), fields.Complex128(), fields.Rationals()):
        e = [[F.elem(int(m == mu)) for m in range(5)] for mu in range(5)]
        assert fields.mdot(F, e[0], e[0]) == F.one
        for mu in range(1, 5):
            assert fields.mdot(F, e[mu], e[mu]) == F.neg(F.one)
            assert fields.mdot(F, e[0], e[mu]) == F.zero


def test_mdot_is_bilinear_not_sesquilinear():
    C = fields.Complex128()
    x = [1j, 2.0, 0.0, 1.0]
    # x.x = (i)^2 - 4 - 0 - 1 = -6 (no conjugation)
    assert fields.mdot(C, x, x) == -6


def test_gaussian_rationals_match_complex_arithmetic():
    G = fields.GaussianRationals()
    rng = random.Random(5)
    for _ in range(200):
        a = complex(rng.randint(-50, 50), rng.randint(-50, 50))
        b = complex(rng.randint(-50, 50), rng.randint(-50, 50))
        ga, gb = G.elem(a), G.elem(b)
        assert G.to_complex(G.mul(ga, gb)) == a * b          # small integers: exact in FP64
        assert G.to_complex(G.add(ga, gb)) == a + b
        if b != 0:
            q = G.mul(ga, G.inv(gb))
            assert G.mul(q, gb) == ga                          # exact inverse
    x = G.elem(0.1 + 0.3j)                                     # exact dyadic value of the binary64 input
    assert x[0] == Fraction(0.1) and x[1] == Fraction(0.3)


def test_running_error_bound_covers_actual_error():
    """The first-order rounding bound of oracle.fields.RunningError must cover
    the true error of the binary64 recursion (exact value from Gaussian
    rationals), on generic and vanishing helicity amplitudes."""
    import numpy as np
    from oracle import bg as obg
    from paper_2502_07060_amd import inputs as I
    R, G, C = fields.RunningError(), fields.GaussianRationals(), fields.Complex128()
    k, e, hel = I.random_helicity_c128(17, 5, 12)
    kc, ec = I.generic_c128(18, 6, 4, 6)
    for kk, ee in list(zip(k, e)) + list(zip(kc, ec)):
        kl, el = [list(v) for v in kk], [list(v) for v in ee]
        _, m = obg.amplitude(C, kl, el)
        _, mr = obg.amplitude(R, [[R.elem(x) for x in v] for v in kl], [[R.elem(x) for x in v] for v in el])
        _, mx = obg.amplitude(G, [[G.elem(x) for x in v] for v in kl], [[G.elem(x) for x in v] for v in el])
        assert mr[0] == m
        assert abs(m - G.to_complex(mx)) <= 2.0 ** -53 * mr[1]
