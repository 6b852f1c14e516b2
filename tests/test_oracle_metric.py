"""Pins of the oracle's alternating-metric option (paper Sec. 3.1: the metric
diag(1, -1, 1, -1, ...) that matches Caravel's convention).

* The product itself against hand-evaluated vectors on which the two metrics
  disagree.
* The memoised recursion against brute-force Feynman diagrams built from the
  same metric tensor (full vertex tensors, explicit index lowering), for any
  inputs with the paper's vertex and for physical inputs with the symmetric
  one.
* Gauge invariance (eps_i -> k_i gives zero) on massless, momentum-conserving
  kinematics generated directly in the alternating metric.
* The congruence of the two metrics: multiplying the components 2, 4, 6, ...
  of every vector by a square root of -1 turns products in the alternating
  metric into products in the mostly-minus one, so the amplitude computed in
  the alternating metric equals the mostly-minus amplitude of the
  transformed vectors (exactly, over F_p and over Q(i)).
"""
import random
from fractions import Fraction

import pytest

from oracle import bg as obg
from oracle import feynman, fields
from paper_2502_07060_amd import inputs as I

P = I.DEFAULT_PRIME
FP = fields.Fp(P)
IP = I.fp_sqrt_minus_one(P)
ALT = "alternating"


def rand_vecs(rng, n, d, p=P):
    return [[rng.randrange(p) for _ in range(d)] for _ in range(n)]


def null_alt(rng, d, p=P):
    """A random vector with x.x = 0 in the alternating metric over F_p:
    components 2..d-1 uniform, then (k0 - k1)(k0 + k1) = -R with
    R = sum_{mu >= 2} (-1)^mu (k^mu)^2 solved on the light cone of axes 0, 1."""
    rest = [rng.randrange(p) for _ in range(d - 2)]
    R = sum((x * x if mu % 2 == 0 else -x * x) for mu, x in enumerate(rest, start=2)) % p
    kp = rng.randrange(1, p)
    km = (-R) * pow(kp, p - 2, p) % p
    h = (p + 1) // 2
    return [(kp + km) * h % p, (kp - km) * h % p] + rest


def physical_alt(rng, n, d, p=P):
    """n >= 4 massless momenta (alternating metric) summing to zero, and
    transverse polarisations eps_l = v_l - (v_l.k_l)/(q.k_l) q."""
    if n < 4:
        raise ValueError("three massless momenta summing to zero have no transverse states here")
    F = fields.Fp(p)
    dot = fields.adot
    while True:
        ks = [null_alt(rng, d, p) for _ in range(n - 2)]
        Q = [(-sum(k[m] for k in ks)) % p for m in range(d)]
        r = null_alt(rng, d, p)
        qr = dot(F, Q, r)
        if qr == 0:
            continue
        t = dot(F, Q, Q) * pow(2 * qr, p - 2, p) % p
        ks += [[t * x % p for x in r], [(a - t * x) % p for a, x in zip(Q, r)]]
        q = null_alt(rng, d, p)
        eps = []
        ok = True
        for k in ks:
            qk = dot(F, q, k)
            if qk == 0:
                ok = False
                break
            v = [rng.randrange(p) for _ in range(d)]
            c = dot(F, v, k) * pow(qk, p - 2, p) % p
            eps.append([(a - c * b) % p for a, b in zip(v, q)])
        if ok:
            return ks, eps


def transform(F, vecs, i_unit):
    """Components 2, 4, ... multiplied by i_unit."""
    return [[F.mul(i_unit, x) if mu >= 2 and mu % 2 == 0 else x for mu, x in enumerate(v)] for v in vecs]


def test_alternating_product_values():
    Q = fields.Rationals()
    one = [Fraction(1)] * 4
    assert fields.adot(Q, one, one) == 0 and fields.mdot(Q, one, one) == -2
    e4 = [Fraction(x) for x in (1, 0, 0, 0, 1)]
    assert fields.adot(Q, e4, e4) == 2 and fields.mdot(Q, e4, e4) == 0
    a = [Fraction(x) for x in (2, 3, 5, 7, 11, 13)]
    b = [Fraction(x) for x in (1, -1, 2, -2, 3, -3)]
    # products 2, -3, 10, -14, 33, -39: signs + - + - + - give 101, the
    # mostly-minus metric 2 - (-3 + 10 - 14 + 33 - 39) = 15
    assert fields.adot(Q, a, b) == 101 and fields.mdot(Q, a, b) == 15
    with pytest.raises(ValueError):
        fields.metric_dot("euclidean")


@pytest.mark.parametrize("n", [4, 5, 6])
@pytest.mark.parametrize("d", [4, 5, 6])
def test_recursion_vs_diagrams_any_inputs(n, d):
    rng = random.Random(31 * n + d)
    k, e = rand_vecs(rng, n, d), rand_vecs(rng, n, d)
    st, m = obg.amplitude(FP, k, e, metric=ALT)
    assert st == 0
    a, _ = feynman.amplitude_diagrams(FP, IP, k, e, form="paper", metric=ALT)
    assert a == FP.mul(IP, m)
    # the mostly-minus value differs: the metric really enters
    assert obg.amplitude(FP, k, e)[1] != m


@pytest.mark.parametrize("n,d", [(4, 4), (5, 6), (6, 5)])
def test_physical_inputs_symmetric_vertex_and_ward(n, d):
    rng = random.Random(100 + 10 * n + d)
    k, e = physical_alt(rng, n, d)
    st, m = obg.amplitude(FP, k, e, metric=ALT)
    assert st == 0 and m != 0
    a, _ = feynman.amplitude_diagrams(FP, IP, k, e, form="symmetric", metric=ALT)
    assert a == FP.mul(IP, m)
    for leg in range(n):
        e2 = [list(v) for v in e]
        e2[leg] = list(k[leg])
        st2, w = obg.amplitude(FP, k, e2, metric=ALT)
        assert st2 == 0 and w == 0, leg


@pytest.mark.parametrize("n", [4, 6, 8])
@pytest.mark.parametrize("d", [4, 7, 10])
def test_congruence_fp(n, d):
    rng = random.Random(7 * n + d)
    k, e = rand_vecs(rng, n, d), rand_vecs(rng, n, d)
    st, m = obg.amplitude(FP, k, e, metric=ALT)
    st2, m2 = obg.amplitude(FP, transform(FP, k, IP), transform(FP, e, IP))
    assert st == st2 == 0 and m == m2


def test_congruence_gaussian_rationals():
    G = fields.GaussianRationals()
    iu = G.elem((Fraction(0), Fraction(1)))
    rng = random.Random(5)
    n, d = 5, 6
    k = [[G.elem((Fraction(rng.randint(-9, 9)), Fraction(0))) for _ in range(d)] for _ in range(n)]
    e = [[G.elem((Fraction(rng.randint(-9, 9)), Fraction(rng.randint(-9, 9)))) for _ in range(d)] for _ in range(n)]
    st, m = obg.amplitude(G, k, e, metric=ALT)
    st2, m2 = obg.amplitude(G, transform(G, k, iu), transform(G, e, iu))
    assert st == st2 == 0 and m == m2
