"""Pins of oracle/rational.py (F_p samples back to rational numbers):

* residues of fractions against Python's own modular inverse (pow(d, -1, p));
* Chinese remaindering against brute-force search for small moduli and the
  defining congruences for large ones;
* rational reconstruction: every coprime fraction within the bound comes
  back exactly from its residues (the uniqueness theorem), brute force over
  every residue of small moduli (the result is the only fraction in the
  bound, or there is none), validity of whatever is returned;
* amplitudes at rational kinematic points: the rational amplitude computed
  over Q equals the reconstruction of the F_p amplitudes of the same point
  modulo enough primes, and too few primes are detected.
"""
import random
from fractions import Fraction
from math import gcd

import pytest

from oracle import bg, fields
from oracle import rational as R
from test_oracle_pins import rational_point


def primes_below(top, count):
    """The `count` largest primes below `top`, by trial division."""
    out, c = [], top - 1
    while len(out) < count:
        if c % 2 and all(c % f for f in range(3, int(c ** 0.5) + 1, 2)):
            out.append(c)
        c -= 1
    return out


BIG = primes_below(2 ** 31, 16)


def test_primes_helper():
    assert BIG[0] == 2147483647 and 2147483629 in BIG


def test_residue_against_python_inverse():
    rng = random.Random(1)
    for p in (3, 7, 101, 2147483629, BIG[3]):
        for _ in range(50):
            n, d = rng.randint(-10 ** 20, 10 ** 20), rng.randint(-10 ** 9, 10 ** 9) or 1
            st, r = R.residue(n, d, p)
            if d % p == 0:
                assert st == 1
            else:
                assert st == 0 and r == n * pow(d, -1, p) % p
    assert R.residue(5, 14, 7) == (1, None)


def test_crt_brute_force_small():
    primes = [3, 5, 7, 11]
    M = 3 * 5 * 7 * 11
    for x in range(M):
        assert R.crt([x % p for p in primes], primes) == (x, M)


def test_crt_large():
    rng = random.Random(2)
    for k in (1, 2, 5, 16):
        ps = BIG[:k]
        M = 1
        for p in ps:
            M *= p
        for _ in range(20):
            x = rng.randrange(M)
            assert R.crt([x % p for p in ps], ps) == (x, M)


@pytest.mark.parametrize("k", [1, 2, 3, 5, 8, 13, 16])
def test_fractions_within_the_bound_come_back(k):
    ps = BIG[:k]
    M = 1
    for p in ps:
        M *= p
    B = R.bound(M)
    assert 2 * B * B < M <= 2 * (B + 1) ** 2 + 1
    rng = random.Random(k)
    cases = [(0, 1), (1, 1), (-1, 1), (B, 1), (-B, 1), (1, B), (-1, B)]
    for _ in range(200):
        bits = rng.randint(1, B.bit_length())
        a = rng.randint(-(2 ** bits), 2 ** bits)
        b = rng.randint(1, 2 ** rng.randint(1, B.bit_length()))
        if abs(a) <= B and b <= B:
            g = gcd(a, b)
            cases.append((a // g, b // g))
    for a, b in cases:
        res = [a % p * pow(b, -1, p) % p for p in ps]
        assert R.reconstruct(res, ps) == (0, a, b), (a, b)


@pytest.mark.parametrize("primes", [(7, 11), (3, 5, 7), (13,), (5, 7, 11), (2147483629,)])
def test_brute_force_every_residue(primes):
    M = 1
    for p in primes:
        M *= p
    B = R.bound(M)
    xs = range(M) if M < 5000 else random.Random(3).sample(range(M), 3000)
    cands = [(a, b) for b in range(1, B + 1) for a in range(-B, B + 1) if gcd(a, b) == 1] if B < 40 else None
    for x in xs:
        st, a, b = R.reconstruct([x % p for p in primes], list(primes))
        if st == 0:
            assert abs(a) <= B and 0 < b <= B and gcd(a, b) == 1 and (a - b * x) % M == 0
        if cands is not None:
            sols = [(a2, b2) for a2, b2 in cands if (a2 - b2 * x) % M == 0]
            assert len(sols) <= 1
            assert (st, a, b) == ((0,) + sols[0] if sols else (1, None, None)), x


def test_bad_residue_status():
    assert R.reconstruct([5, 2147483629], [7, 2147483629])[0] == 2
    assert R.reconstruct([0xFFFFFFFF], [2147483629])[0] == 2
    assert R.reconstruct([-1, 3], [7, 11])[0] == 2


@pytest.mark.parametrize("n,d", [(4, 4), (5, 4), (5, 6), (6, 4)])
def test_amplitudes_over_Q_from_F_p(n, d):
    """With the fewest primes whose bound covers the rational amplitude the
    reconstruction returns it (uniqueness theorem); with one prime fewer the
    amplitude lies outside the bound, so whatever comes back is not it."""
    Q = fields.Rationals()
    rng = random.Random(50 + 10 * n + d)
    done = 0
    while done < 2:
        ks, eps = rational_point(rng, n, d)
        st, mq = bg.amplitude(Q, ks, eps)
        if st != 0 or mq == 0:
            continue
        res, ps = [], []
        for p in BIG:
            F = fields.Fp(p)
            conv = [[R.residue(x.numerator, x.denominator, p) for x in v] for v in ks + eps]
            if any(c[0] for v in conv for c in v):
                continue
            kk = [[c[1] for c in v] for v in conv[:n]]
            ee = [[c[1] for c in v] for v in conv[n:]]
            s2, m = bg.amplitude(F, kk, ee)
            if s2 != 0:
                continue
            assert m == mq.numerator % p * pow(mq.denominator, -1, p) % p   # the F_p image of mq
            res.append(m)
            ps.append(p)
        height = max(abs(mq.numerator), mq.denominator)
        k, M = 0, 1
        while R.bound(M) < height:
            M *= ps[k]
            k += 1
        assert k <= len(ps), "not enough primes below 2^31 for this height"
        st, a, b = R.reconstruct(res[:k], ps[:k])
        assert st == 0 and Fraction(a, b) == mq, (n, d, mq)
        st1, a1, b1 = R.reconstruct(res[:k - 1], ps[:k - 1])
        assert st1 == 1 or Fraction(a1, b1) != mq
        done += 1
