"""Sub-range sums from two-part prefix sums, in IEEE doubles on the host.

The complex lane-group kernel (csrc/bg_wide.h, WideRecursion::load) keeps the
prefix sums Q_l = k_0 + ... + k_{l-1} of the primed momenta as unevaluated
sums hi_l + lo_l: hi takes an error-free two-sum with each leg (Knuth's
TwoSum) and lo collects the rounding errors.  A sub-range momentum is then
P_{i..j} = (hi_{j+1} - hi_i) + (lo_{j+1} - lo_i).  The claim is that this is
as accurate as a direct left-to-right sum of the legs, with an error relative
to |P| itself, where a difference of plain prefix sums has an error relative
to the prefix sums, which can be far larger than P (paper Sec. 3: the
double-precision path; momentum conservation makes partial sums of the legs
large while their sub-range sums are small).

This file restates the recipe with Python floats (IEEE binary64, the same
operations in the same order) and checks it against exact rational sums.
"""
from __future__ import annotations

import random
from fractions import Fraction

EPS = 2.0**-53


def two_part_prefix(ks):
    hi, lo = [0.0], [0.0]
    h = l = 0.0
    for k in ks:
        s = h + k
        b = s - h
        l += (h - (s - b)) + (k - b)
        h = s
        hi.append(h)
        lo.append(l)
    return hi, lo


def plain_prefix(ks):
    q, acc = [0.0], 0.0
    for k in ks:
        acc += k
        q.append(acc)
    return q


def exact_sum(ks, i, j):
    return sum((Fraction(k) for k in ks[i:j + 1]), Fraction(0))


def legs(rng, n, scale, small):
    """n legs whose partial sums reach `scale` while neighbouring legs nearly
    cancel, so that short sub-ranges sum to about `small`."""
    out = []
    for _ in range(n // 2):
        big = rng.uniform(0.5, 1.0) * scale * rng.choice((-1.0, 1.0))
        out += [big, -big + rng.uniform(-1.0, 1.0) * small]
    if n % 2:
        out.append(rng.uniform(-1.0, 1.0) * small)
    # a running offset makes the prefix sums themselves large
    out[0] += 7.0 * scale
    out[-1] -= 7.0 * scale
    return out


def test_two_part_differences_are_relative_to_the_sub_range():
    rng = random.Random(5)
    worst_dd = worst_plain = 0.0
    for trial in range(300):
        n = rng.randint(3, 13)
        ks = legs(rng, n, scale=10.0 ** rng.randint(2, 4), small=10.0 ** rng.randint(-3, 1))
        hi, lo = two_part_prefix(ks)
        q = plain_prefix(ks)
        qmax = max(abs(x) for x in hi)
        for i in range(n):
            for j in range(i, n):
                exact = exact_sum(ks, i, j)
                dd = (hi[j + 1] - hi[i]) + (lo[j + 1] - lo[i])
                err = abs(Fraction(dd) - exact)
                bound = 3 * EPS * abs(exact) + 4 * n * EPS * EPS * qmax
                assert err <= bound, (trial, i, j, float(err), float(bound))
                if exact != 0:
                    worst_dd = max(worst_dd, float(err / abs(exact)))
                    perr = abs(Fraction(q[j + 1] - q[i]) - exact)
                    worst_plain = max(worst_plain, float(perr / abs(exact)))
    # the plain difference really does lose the digits this recipe keeps
    assert worst_plain > 1e3 * worst_dd


def test_two_part_prefix_is_exact_up_to_the_low_part_rounding():
    rng = random.Random(11)
    for _ in range(200):
        ks = [rng.uniform(-1.0, 1.0) * 10.0 ** rng.randint(-8, 8) for _ in range(rng.randint(1, 13))]
        hi, lo = two_part_prefix(ks)
        for l in range(len(ks) + 1):
            exact = sum((Fraction(k) for k in ks[:l]), Fraction(0))
            err = abs(Fraction(hi[l]) + Fraction(lo[l]) - exact)
            # only lo's own additions round, each by at most eps |lo|
            assert err <= l * EPS * (abs(lo[l]) + EPS * max(map(abs, hi)))
