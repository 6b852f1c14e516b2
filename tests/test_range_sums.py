"""Host model of how the lane-group kernel's item slots combine their partial
sums (csrc/bg_wide.h, WideRecursion::range_sum and, for Z_p ranges below the
root, WideRecursion::rs_finish).

A range's items sit in a block of `per` slots (a power of two); after the cuts
every slot holds a partial sum of each of the DL components of K'(S) that its
lane covers.  The butterfly leaves every slot with all totals.  The
reduce-scatter halves, at each step, the components a slot holds (of each pair
it keeps the one its bit selects and adds the partner's partial of it), then
adds whole values for the steps left once the count is odd; each slot finishes
the components it ends with, and P_S . J_S is summed over the slots that hold
different components.  These tests replay that bookkeeping with exact
integers for every (DL, per) the kernels can meet and check that each
component's total reaches exactly the slots that finish it and that the P.J
sum counts every component once.
"""
import random

import pytest


def butterfly(parts):
    """parts[u][c]: slot u's partial of component c -> every slot's totals."""
    per, out = len(parts), [list(p) for p in parts]
    st = 1
    while st < per:
        out = [[out[u][c] + out[u ^ st][c] for c in range(len(out[u]))] for u in range(per)]
        st *= 2
    return out


def reduce_scatter(parts):
    """The rs_finish schedule: per slot, (component indices, totals, steps
    taken by halving)."""
    per, DL = len(parts), len(parts[0])
    lg = per.bit_length() - 1
    # state per slot: list of (component index, value); the first base/stride
    # bookkeeping of the kernel (cb + q cs) is checked against it below
    held = [[(c, parts[u][c]) for c in range(DL)] for u in range(per)]
    cb, cs = [0] * per, [1] * per
    k, st = 0, 1
    while k < lg and len(held[0]) % 2 == 0:
        new = []
        for u in range(per):
            b = (u & st) != 0
            mine, partner = held[u], held[u ^ st]
            row = []
            for p in range(len(mine) // 2):
                keep = mine[2 * p + 1] if b else mine[2 * p]
                # the partner sends the element of the pair this slot keeps
                sent = partner[2 * p + 1] if b else partner[2 * p]
                assert keep[0] == sent[0]
                row.append((keep[0], keep[1] + sent[1]))
            new.append(row)
            if b:
                cb[u] += cs[u]
            cs[u] *= 2
        held = new
        k += 1
        st *= 2
    # steps left: whole values
    while st < per:
        held = [[(c, v + held[u ^ st][q][1]) for q, (c, v) in enumerate(held[u])] for u in range(per)]
        st *= 2
    for u in range(per):
        assert [c for c, _ in held[u]] == [cb[u] + q * cs[u] for q in range(len(held[u]))]
    return held, k


# components per lane of the Z_p lane-group kernels (DMAX / LC) and the slot
# blocks a range can take (per <= G <= 64)
@pytest.mark.parametrize("DL", [2, 3, 4, 5, 6, 8, 10])
@pytest.mark.parametrize("per", [1, 2, 4, 8, 16, 32])
def test_reduce_scatter_matches_the_butterfly(DL, per):
    rng = random.Random(1000 * DL + per)
    parts = [[rng.randrange(-2**40, 2**40) for _ in range(DL)] for _ in range(per)]
    totals = butterfly(parts)[0]
    assert all(row == totals for row in butterfly(parts))
    held, k = reduce_scatter(parts)
    owners = {c: [] for c in range(DL)}
    for u in range(per):
        for c, v in held[u]:
            assert v == totals[c], (u, c)          # the slot holds the complete sum
            owners[c].append(u)
    # every component is finished, by 2^(lg - k) slots that differ only in the
    # bits above the halving steps, and those write the same value
    lg = per.bit_length() - 1
    low = (1 << k) - 1
    for c, us in owners.items():
        assert len(us) == 1 << (lg - k), (c, us)
        assert len({u & low for u in us}) == 1
    # P_S . J_S: the slots' partials summed over the halving distances only
    pj = [sum(totals[c] * (c + 1) for c, _ in held[u]) for u in range(per)]
    st = 1
    for _ in range(k):
        pj = [pj[u] + pj[u ^ st] for u in range(per)]
        st *= 2
    assert all(x == sum(t * (c + 1) for c, t in enumerate(totals)) for x in pj)


def test_summing_pj_over_every_step_would_overcount():
    """The mistake the P.J sum must avoid: when the halving stops early
    (an odd component count), adding the partials over all steps counts each
    component several times."""
    DL, per = 6, 8
    parts = [[1] * DL for _ in range(per)]
    held, k = reduce_scatter(parts)
    assert k == 1
    pj = [sum(v for _, v in held[u]) for u in range(per)]
    st = 1
    while st < per:
        pj = [pj[u] + pj[u ^ st] for u in range(per)]
        st *= 2
    assert pj[0] == 4 * DL * per  # 2^(lg - k) = 4 times the true sum
