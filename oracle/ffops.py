"""Standalone finite-field tensor operations (test infrastructure only; see
oracle/__init__.py).

The paper's F_p library (Sec. 3) provides, besides the recursion, batched
tensor contractions over any number of indices and a division:

* double-batched:  z[n, i, k] = sum_j x[n, i, j] y[n, j, k]
* single-batched:  z[n, i, k] = sum_j x[n, i, j] y[j, k]
* division:        z[n] = x[n] / y[n]  (or one y for every n)

with the free indices i, k and the summed indices j each standing for any
group of tensor indices (flattened).  Written out with Python integers
(exact sums, one reduction mod p at the end) and Fermat inverses.  Status of
a division: 0, or 1 when y = 0 (no inverse).

Parity: pinned by tests/test_oracle_ffops.py -- numpy integer products of
small operands reduced afterwards, Python's own modular inverse, and the
algebra (bilinearity, associativity, x / y * y = x).
"""
from __future__ import annotations


def contract(x, y, p: int, batched_y: bool = True):
    """x: [n][I][J] ints; y: [n][J][K] (batched) or [J][K]; -> [n][I][K] mod p."""
    out = []
    for e, xe in enumerate(x):
        ye = y[e] if batched_y else y
        I, J = len(xe), len(xe[0]) if xe else 0
        K = len(ye[0]) if ye else 0
        out.append([[sum(xe[i][j] * ye[j][k] for j in range(J)) % p for k in range(K)] for i in range(I)])
    return out


def divide(x, y, p: int):
    """Elementwise x / y mod p: ([status], [value or None])."""
    st, val = [], []
    for a, b in zip(x, y):
        if b % p == 0:
            st.append(1)
            val.append(None)
        else:
            st.append(0)
            val.append(a * pow(b, p - 2, p) % p)
    return st, val
