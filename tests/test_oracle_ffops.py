"""Pins of oracle/ffops.py (the paper's standalone F_p operations, Sec. 3):
contractions against numpy's integer matrix products of operands small
enough that int64 is exact, reduced afterwards; bilinearity and
associativity modulo p at full size; division against Python's own modular
inverse and x / y * y = x."""
import random

import numpy as np
import pytest

from oracle import ffops

P = 2147483629


@pytest.mark.parametrize("I,J,K", [(1, 1, 1), (4, 4, 1), (6, 6, 6), (3, 10, 7), (16, 2, 5)])
def test_contract_matches_numpy_small_operands(I, J, K):
    rng = np.random.default_rng(I * 100 + J * 10 + K)
    n = 5
    x = rng.integers(0, 1000, size=(n, I, J))
    y = rng.integers(0, 1000, size=(n, J, K))
    z = ffops.contract(x.tolist(), y.tolist(), P)
    assert np.array_equal(np.array(z), np.matmul(x, y) % P)
    y1 = rng.integers(0, 1000, size=(J, K))
    z1 = ffops.contract(x.tolist(), y1.tolist(), P, batched_y=False)
    assert np.array_equal(np.array(z1), np.matmul(x, y1) % P)


def test_contract_algebra_full_size():
    rng = random.Random(4)
    n, I, J, K, L = 3, 3, 4, 5, 2
    R = lambda a, b: [[rng.randrange(P) for _ in range(b)] for _ in range(a)]
    x = [R(I, J) for _ in range(n)]
    y = [R(J, K) for _ in range(n)]
    y2 = [R(J, K) for _ in range(n)]
    w = [R(K, L) for _ in range(n)]
    ysum = [[[(a + b) % P for a, b in zip(r1, r2)] for r1, r2 in zip(m1, m2)] for m1, m2 in zip(y, y2)]
    lhs = ffops.contract(x, ysum, P)
    a, b = ffops.contract(x, y, P), ffops.contract(x, y2, P)
    assert lhs == [[[(u + v) % P for u, v in zip(r1, r2)] for r1, r2 in zip(m1, m2)] for m1, m2 in zip(a, b)]
    assert ffops.contract(ffops.contract(x, y, P), w, P) == ffops.contract(x, ffops.contract(y, w, P), P)


def test_divide():
    rng = random.Random(5)
    x = [rng.randrange(P) for _ in range(100)] + [5, 0]
    y = [rng.randrange(1, P) for _ in range(100)] + [0, 7]
    st, v = ffops.divide(x, y, P)
    for a, b, s, q in zip(x, y, st, v):
        if b == 0:
            assert s == 1 and q is None
        else:
            assert s == 0 and q == a * pow(b, -1, P) % P and q * b % P == a
