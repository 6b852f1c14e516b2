"""Pins of oracle/states.py (the d-dimensional polarisation states of paper
Sec. 2.3): every state transverse to k, e_i . e_j~ = -delta_ij (the
orthonormality conditions), and the completeness relation
    sum_i e_i^mu e_i~^nu = -g^{mu nu} + (k^mu eta^nu + eta^mu k^nu) / (k.eta)
with eta = k_4d - k_2d (d >= 5) or the reference chi (d = 4), exactly over
F_p and over the Gaussian rationals; and, for d = 4, the Parke-Taylor
normalisation of the amplitude built from these states."""
import random
from fractions import Fraction

import pytest

from oracle import bg as obg
from oracle import fields
from oracle import states as S
from oracle.fields import mdot

P = 2147483629
I_P = 1518275076  # a square root of -1 mod P (paper-facts fixture)


def null_fp(rng, d, p=P):
    """A random massless d-vector over F_p (light-cone along the last axis)."""
    kp = rng.randrange(1, p)
    kt = [rng.randrange(p) for _ in range(d - 2)]
    km = sum(t * t for t in kt) * pow(kp, p - 2, p) % p
    h = (p + 1) // 2
    return [(kp + km) * h % p] + kt + [(kp - km) * h % p]


def null_q(rng, d, B=5):
    """A random massless d-vector with rational components (non-zero
    transverse components, so that no mu_y^2 vanishes)."""
    kp = Fraction(rng.randint(1, B))
    kt = [Fraction(rng.choice([-1, 1]) * rng.randint(1, B)) for _ in range(d - 2)]
    km = sum(t * t for t in kt) / kp
    return [(kp + km) / 2] + kt + [(kp - km) / 2]


def metric(F, d, mu, nu):
    if mu != nu:
        return F.zero
    return F.one if mu == 0 else F.neg(F.one)


def check_states(F, k, chi, i_unit, exact=True, tol=0.0):
    d = len(k)
    st, eps, epst = S.states(F, k, chi, i_unit)
    assert st == 0
    assert len(eps) == len(epst) == d - 2
    close = (lambda a, b: a == b) if exact else (lambda a, b: abs(a - b) <= tol)
    for e in eps + epst:
        assert close(mdot(F, k, e), F.zero)
    for i, e in enumerate(eps):
        for j, et in enumerate(epst):
            assert close(mdot(F, e, et), F.neg(F.one) if i == j else F.zero), (i, j)
    if d >= 5:
        eta = list(k[:4]) + [F.neg(x) for x in k[4:]]
    else:
        eta = list(chi[:4])
    ke = mdot(F, k, eta)
    for e in eps:
        assert close(mdot(F, eta, e), F.zero)
    inv_ke = F.inv(ke)
    for mu in range(d):
        for nu in range(d):
            lhs = F.zero
            for e, et in zip(eps, epst):
                lhs = F.add(lhs, F.mul(e[mu], et[nu]))
            rhs = F.sub(F.mul(F.add(F.mul(k[mu], eta[nu]), F.mul(eta[mu], k[nu])), inv_ke),
                        metric(F, d, mu, nu))
            assert close(lhs, rhs), (mu, nu)
    return eps, epst


@pytest.mark.parametrize("d", list(range(4, 11)))
def test_states_fp_exact(d):
    F = fields.Fp(P)
    rng = random.Random(100 + d)
    for _ in range(6):
        check_states(F, null_fp(rng, d), null_fp(rng, 4), I_P)


@pytest.mark.parametrize("d", [4, 5, 6, 7, 8])
def test_states_gaussian_rationals_exact(d):
    G = fields.GaussianRationals()
    rng = random.Random(200 + d)
    for _ in range(3):
        k = [G.elem((x, 0)) for x in null_q(rng, d)]
        chi = [G.elem((x, 0)) for x in null_q(rng, 4)]
        check_states(G, k, chi, (Fraction(0), Fraction(1)))


@pytest.mark.parametrize("d", [4, 6, 10])
def test_states_complex(d):
    C = fields.Complex128()
    rng = random.Random(300 + d)
    for _ in range(4):
        k = [complex(float(x)) for x in null_q(rng, d)]
        chi = [complex(float(x)) for x in null_q(rng, 4)]
        check_states(C, k, chi, 1j, exact=False, tol=1e-9)


def test_state_properties_printed_in_the_paper():
    """(e1, e2) = -1, (e3, e3) = (e4, e4) in the square-root-free form equal
    -mu^2, and the other products vanish (Sec. 2.3, d = 6)."""
    F = fields.Fp(P)
    rng = random.Random(7)
    k, chi = null_fp(rng, 6), null_fp(rng, 4)
    st, e, _ = S.states(F, k, chi, I_P)
    assert st == 0
    mu2 = (k[4] * k[4] + k[5] * k[5]) % P
    assert mdot(F, e[0], e[1]) == P - 1
    assert mdot(F, e[2], e[2]) == (-mu2) % P and mdot(F, e[3], e[3]) == (-mu2) % P
    for a, b in [(0, 0), (1, 1), (2, 3), (0, 2), (0, 3), (1, 2), (1, 3)]:
        assert mdot(F, e[a], e[b]) == 0
    # lower-dimensional states embed with zeros beyond their last component
    assert e[3][:4] == [0, 0, 0, 0]


@pytest.mark.parametrize("n", [4, 5, 6])
def test_d4_states_reproduce_parke_taylor(n):
    """With d = 4 (mu^2 = 0, so kb = k) e1 is the minus and e2 the plus
    helicity state: an MHV amplitude over F_p equals (-1)^n 2^(n-3) times the
    Parke-Taylor formula built from the same spinors."""
    F = fields.Fp(P)
    rng = random.Random(400 + n)
    # n-2 random null legs and a closing pair (momentum conservation)
    ks = [null_fp(rng, 4) for _ in range(n - 2)]
    Q = [(-sum(k[m] for k in ks)) % P for m in range(4)]
    while True:
        r = null_fp(rng, 4)
        qr = mdot(F, Q, r)
        if qr:
            break
    t = mdot(F, Q, Q) * pow(2 * qr, P - 2, P) % P
    ks += [[t * x % P for x in r], [(a - t * x) % P for a, x in zip(Q, r)]]
    chi = null_fp(rng, 4)
    a, b = 0, 2
    eps, lams = [], []
    for l, k in enumerate(ks):
        st, e, _ = S.states(F, k, chi, I_P)
        assert st == 0
        eps.append(e[0] if l in (a, b) else e[1])
        lams.append(S.spinors(F, k, I_P)[0])
    st, m = obg.amplitude(F, ks, eps)
    assert st == 0
    den = 1
    for l in range(n):
        den = den * S.bracket(F, lams[l], lams[(l + 1) % n]) % P
    pt = pow(S.bracket(F, lams[a], lams[b]), 4, P) * pow(den, P - 2, P) % P
    assert m == ((-1) ** n * 2 ** (n - 3) * pt) % P


def test_singular_reference():
    """chi along k (chi.k4 = 0) has no states: status 1."""
    F = fields.Fp(P)
    rng = random.Random(9)
    k = null_fp(rng, 4)
    assert S.states(F, k, list(k), I_P)[0] == 1


@pytest.mark.parametrize("d", [4, 5, 6, 8, 10])
def test_state_sum_closed_form(d):
    """The completeness relation turns the state sum into
    -K_L.K_R + ((K_L.k)(eta.K_R) + (K_L.eta)(k.K_R)) / (k.eta) for any K_L, K_R."""
    F = fields.Fp(P)
    rng = random.Random(500 + d)
    for _ in range(5):
        k, chi = null_fp(rng, d), null_fp(rng, 4)
        st, eps, epst = S.states(F, k, chi, I_P)
        assert st == 0
        KL = [rng.randrange(P) for _ in range(d)]
        KR = [rng.randrange(P) for _ in range(d)]
        eta = list(k[:4]) + [F.neg(x) for x in k[4:]] if d >= 5 else list(chi[:4])
        ke = mdot(F, k, eta)
        want = F.add(F.neg(mdot(F, KL, KR)),
                     F.mul(F.add(F.mul(mdot(F, KL, k), mdot(F, eta, KR)), F.mul(mdot(F, KL, eta), mdot(F, k, KR))),
                           F.inv(ke)))
        assert S.state_sum(F, KL, KR, eps, epst) == want


@pytest.mark.parametrize("nl,nr,d", [(4, 4, 4), (4, 5, 6), (5, 4, 7)])
def test_state_sum_equals_sum_of_amplitude_products(nl, nr, d):
    """With K_L, K_R the root currents of two trees whose last leg is the cut
    leg (l and -l), the state sum equals sum_s M_L(.., e_s) M_R(.., e~_s)
    evaluated with the amplitude oracle (the multilinearity in eps_n)."""
    F = fields.Fp(P)
    rng = random.Random(600 + nl + 10 * nr + d)
    l = null_fp(rng, d)                    # the other momenta are arbitrary: the identity is algebraic
    kl_ = [[rng.randrange(P) for _ in range(d)] for _ in range(nl - 1)] + [l]
    kr_ = [[rng.randrange(P) for _ in range(d)] for _ in range(nr - 1)] + [[(-x) % P for x in l]]
    el = [[rng.randrange(P) for _ in range(d)] for _ in range(nl)]
    er = [[rng.randrange(P) for _ in range(d)] for _ in range(nr)]
    st, eps, epst = S.states(F, l, null_fp(rng, 4), I_P)
    assert st == 0
    s1, _, KL = obg.currents(F, kl_, el)
    s2, _, KR = obg.currents(F, kr_, er)
    assert s1 == s2 == 0
    total = F.zero
    for e, et in zip(eps, epst):
        a1 = obg.amplitude(F, kl_, el[:-1] + [e])[1]
        a2 = obg.amplitude(F, kr_, er[:-1] + [et])[1]
        total = F.add(total, F.mul(a1, a2))
    assert S.state_sum(F, KL, KR, eps, epst) == total
