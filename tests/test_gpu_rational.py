"""F_p samples back to rationals on the GPU (next row f2): residues of int64
fractions, and Chinese remaindering plus rational reconstruction, each
against oracle/rational.py value by value (exact: statuses, numerators and
denominators), from 1 to 32 primes; then the whole chain at rational
kinematic points -- residues of the inputs for each prime, the F_p
amplitudes, reconstruction -- against the amplitude computed over Q."""
import random
from fractions import Fraction
from math import gcd

import numpy as np
import pytest

from oracle import bg as obg
from oracle import fields
from oracle import rational as R
from paper_2502_07060_amd import bg
from paper_2502_07060_amd import inputs as I

from test_gpu_parity import torch_dev  # noqa: F401
from test_oracle_pins import rational_point
from test_oracle_rational import primes_below

pytestmark = pytest.mark.gpu
BIG = primes_below(2 ** 31, 32)


def gpu_residues(torch_dev, p, num, den):
    torch, dev = torch_dev
    tn = torch.from_numpy(np.asarray(num, np.int64)).to(dev)
    td = torch.from_numpy(np.asarray(den, np.int64)).to(dev)
    out, st = bg.bg_fp_from_rational(p, tn, td)
    torch.cuda.synchronize()
    return out.cpu().numpy().view(np.uint32).astype(np.int64), st.cpu().numpy()


@pytest.mark.parametrize("count", [1, 15, 16, 17, 1000, 4099])
def test_fp_from_rational(torch_dev, count):
    rng = np.random.default_rng(count)
    num = rng.integers(-(2 ** 63), 2 ** 63 - 1, size=count, dtype=np.int64, endpoint=True)
    den = rng.integers(-(2 ** 62), 2 ** 62, size=count, dtype=np.int64)
    num[:3] = [0, -(2 ** 63), 2 ** 63 - 1][:min(3, count)]
    for p in (BIG[1], BIG[7], 3, 101):
        d2 = den.copy()
        if count > 5:
            d2[5] = -7 * p           # a denominator divisible by p
            d2[count // 2] = 0       # and a zero one
        out, st = gpu_residues(torch_dev, p, num, d2)
        for i in range(count):
            s, r = R.residue(int(num[i]), int(d2[i]), p)
            assert st[i] == s, (p, i)
            assert out[i] == (r if s == 0 else 0xFFFFFFFF), (p, i, num[i], d2[i])


def gpu_reconstruct(torch_dev, primes, residues):
    torch, dev = torch_dev
    res = torch.from_numpy(np.asarray(residues, np.uint32).view(np.int32)).to(dev)
    num, den, st = bg.bg_rational_reconstruct(primes, res)
    torch.cuda.synchronize()
    return (bg.limbs_to_ints(num.cpu().numpy(), True), bg.limbs_to_ints(den.cpu().numpy(), False),
            st.cpu().numpy())


def check_against_oracle(torch_dev, primes, residues):
    a_g, b_g, st_g = gpu_reconstruct(torch_dev, primes, residues)
    for q in range(residues.shape[1]):
        st, a, b = R.reconstruct([int(x) for x in residues[:, q]], primes)
        assert st_g[q] == st, (len(primes), q, st, st_g[q])
        if st == 0:
            assert (a_g[q], b_g[q]) == (a, b), (len(primes), q)
        else:
            assert a_g[q] == 0 and b_g[q] == 0
    return st_g


@pytest.mark.parametrize("k", [1, 2, 3, 5, 8, 9, 13, 16, 17, 24, 32])
def test_reconstruct_against_oracle(torch_dev, k):
    primes = BIG[:k] if k % 2 else BIG[32 - k:]      # both ends of the prime list
    M = 1
    for p in primes:
        M *= p
    B = R.bound(M)
    rng = random.Random(k)
    fr = [(0, 1), (1, 1), (-1, 1), (B, 1), (-B, 1), (1, B), (-1, B), (B, B - 1) if gcd(B, B - 1) == 1 else (1, 2)]
    for _ in range(120):
        a = rng.randint(-B, B)
        b = rng.randint(1, max(1, B >> rng.randint(0, B.bit_length() - 1)))
        g = gcd(a, b)
        fr.append((a // g, b // g))
    cols = [[a % p * pow(b, -1, p) % p for p in primes] for a, b in fr]
    cols += [[rng.randrange(p) for p in primes] for _ in range(60)]            # arbitrary residues
    cols += [[(p + 3 if i == 0 else 1) for i, p in enumerate(primes)]]        # a residue >= p
    cols += [[0xFFFFFFFF] + [0] * (k - 1)]                                     # the F_p sentinel
    residues = np.array(cols, dtype=np.int64).T.copy()
    st = check_against_oracle(torch_dev, primes, residues)
    assert (st[:len(fr)] == 0).all() and st[-1] == 2 and st[-2] == 2


def test_reconstruct_ragged_ld(torch_dev):
    """ld > npts: only the first npts columns are read and written."""
    torch, dev = torch_dev
    primes = BIG[:4]
    vals = np.array([[Fraction(-7, 3).numerator % p * pow(3, -1, p) % p for _ in range(5)] for p in primes])
    res = torch.from_numpy(vals.astype(np.uint32).view(np.int32)).to(dev)
    num, den, st = bg.bg_rational_reconstruct(primes, res, npts=3)
    torch.cuda.synchronize()
    assert st.shape[0] == 3 and (st.cpu().numpy() == 0).all()
    assert bg.limbs_to_ints(num.cpu().numpy(), True) == [-7] * 3
    assert bg.limbs_to_ints(den.cpu().numpy(), False) == [3] * 3


@pytest.mark.parametrize("n,d", [(4, 4), (5, 4), (5, 6), (6, 4)])
def test_rational_amplitudes_end_to_end(torch_dev, n, d):
    """Rational kinematics -> residues per prime (bg_fp_from_rational) ->
    bg_amplitudes_fp per prime -> bg_rational_reconstruct, against the
    amplitude over Q."""
    torch, dev = torch_dev
    Q = fields.Rationals()
    rng = random.Random(700 + 10 * n + d)
    pts, mqs = [], []
    while len(pts) < 6:
        ks, eps = rational_point(rng, n, d)
        st, mq = obg.amplitude(Q, ks, eps)
        if st == 0 and mq != 0:
            pts.append((ks, eps))
            mqs.append(mq)
    m = len(pts)
    height = max(max(abs(x.numerator), x.denominator) for x in mqs)
    k, M = 0, 1
    while R.bound(M) < height:
        M *= BIG[k]
        k += 1
    primes = BIG[:k]
    # [n][d][m] numerators and denominators of k and eps
    kn = np.array([[[pts[q][0][l][mu].numerator for q in range(m)] for mu in range(d)] for l in range(n)], np.int64)
    kd = np.array([[[pts[q][0][l][mu].denominator for q in range(m)] for mu in range(d)] for l in range(n)], np.int64)
    en = np.array([[[pts[q][1][l][mu].numerator for q in range(m)] for mu in range(d)] for l in range(n)], np.int64)
    ed = np.array([[[pts[q][1][l][mu].denominator for q in range(m)] for mu in range(d)] for l in range(n)], np.int64)
    T = lambda a: torch.from_numpy(a).to(dev)
    rows = []
    for p in primes:
        km, kst = bg.bg_fp_from_rational(p, T(kn), T(kd))
        em, est = bg.bg_fp_from_rational(p, T(en), T(ed))
        assert int(kst.sum()) == 0 and int(est.sum()) == 0
        out, st = bg.bg_amplitudes_fp(km, em, p)
        torch.cuda.synchronize()
        assert (st.cpu().numpy() == 0).all()
        rows.append(out)
    residues = torch.stack(rows).contiguous()
    num, den, st = bg.bg_rational_reconstruct(primes, residues)
    torch.cuda.synchronize()
    a = bg.limbs_to_ints(num.cpu().numpy(), True)
    b = bg.limbs_to_ints(den.cpu().numpy(), False)
    assert (st.cpu().numpy() == 0).all()
    assert [Fraction(x, y) for x, y in zip(a, b)] == mqs
    # one prime fewer: the amplitude of greatest height lies outside the bound
    num2, den2, st2 = bg.bg_rational_reconstruct(primes[:-1], residues[:-1].contiguous())
    torch.cuda.synchronize()
    worst = max(range(m), key=lambda q: max(abs(mqs[q].numerator), mqs[q].denominator))
    a2 = bg.limbs_to_ints(num2.cpu().numpy(), True)[worst]
    b2 = bg.limbs_to_ints(den2.cpu().numpy(), False)[worst]
    assert st2.cpu().numpy()[worst] == 1 or Fraction(a2, max(b2, 1)) != mqs[worst]
