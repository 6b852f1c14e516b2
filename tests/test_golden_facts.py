"""Checks against the small set of values the paper prints (tests/golden/paper_facts.txt)."""
import os

import numpy as np

from oracle import bg, fields
from paper_2502_07060_amd import inputs as I

HERE = os.path.dirname(os.path.abspath(__file__))


def load_facts():
    facts = {}
    with open(os.path.join(HERE, "golden", "paper_facts.txt")) as f:
        for line in f:
            line = line.split("#", 1)[0].strip()
            if line:
                key, val = (s.strip() for s in line.split("=", 1))
                facts[key] = [int(x) for x in val.split()]
    return facts


def test_default_prime():
    f = load_facts()
    p = f["default_prime"][0]
    assert p == I.DEFAULT_PRIME == 2**31 - 19
    assert p < 2 ** f["prime_bound_bits"][0]
    assert fields.is_prime(p)
    if f["i_in_field"][0]:
        ip = I.fp_sqrt_minus_one(p)
        assert ip * ip % p == p - 1


def test_4d_state_gram_block():
    """The 4d block (eps_1, eps_2) of the printed Gram matrix, over C and F_p."""
    f = load_facts()
    gram = np.array([f[f"gram_row_{r}"] for r in range(1, 5)])
    rng = np.random.default_rng(0)
    k = I.collider_point(rng, 4, 1000.0, 8, 4).astype(complex)
    lam, lamt = I.spinors(k)
    chi = I.random_null_c(rng, 8)
    lc, tc = I.spinors(chi)
    e1 = I.pol_minus(lam, lamt, lc[:, None], tc[:, None])
    e2 = I.pol_plus(lam, lamt, lc[:, None], tc[:, None])
    assert np.allclose(I.c_mdot(e1, e2), gram[0, 1])
    p = f["default_prime"][0]
    kf = I.fp_point(rng, p, 4, 4, 8)
    hm = -np.ones((8, 4), int)
    em, *_ = I.fp_helicity_pols(np.random.default_rng(5), p, kf, hm)
    ep, *_ = I.fp_helicity_pols(np.random.default_rng(5), p, kf, -hm)
    assert np.all(I.fp_mdot(em, ep, p) == gram[0, 1] % p)
    assert np.all(I.fp_mdot(em, em, p) == gram[0, 0])
    assert np.all(I.fp_mdot(ep, ep, p) == gram[1, 1])


def test_pt_at_ci_multiplicity():
    f = load_facts()
    n = f["pt_ci_multiplicity"][0]
    k, eps, hel = I.mhv_c128(7, n, 4)
    lam, _ = I.spinors(k)
    for q in range(4):
        st, m = bg.amplitude(fields.Complex128(), [list(v) for v in k[q]], [list(v) for v in eps[q]])
        den = np.prod([I.angle(lam[q, l], lam[q, (l + 1) % n]) for l in range(n)])
        pt = I.angle(lam[q, 0], lam[q, 1]) ** 4 / den
        assert abs(m / pt - (-1) ** n * 2 ** (n - 3)) < 1e-10
