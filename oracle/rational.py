"""Multi-prime evaluation, Chinese remaindering and rational reconstruction
(test infrastructure only; see oracle/__init__.py).

The paper computes over F_p so that exact rational results can be recovered
from finite-field samples (Sec. 1 and Sec. 3: F_p values at rational
kinematic points are turned into rational numbers, e.g. to compare with
Caravel "up to a power of 2").  The steps, in Python integers:

* residue of a rational:  n/d mod p = n * d^(p-2) mod p, undefined (status 1)
  when p divides d;
* Chinese remaindering: the unique 0 <= x < M = p_1 ... p_k with x = r_i
  (mod p_i), written out as x = sum_i r_i (M/p_i) ((M/p_i)^-1 mod p_i) mod M;
* rational reconstruction (Wang; the form of von zur Gathen and Gerhard,
  Modern Computer Algebra, Sec. 5.10): with B = floor(sqrt((M - 1) / 2)), so
  that 2 B^2 < M, run the extended Euclidean algorithm on r_0 = M, r_1 = x
  with t_0 = 0, t_1 = 1 (every remainder r_j = s_j M + t_j x); stop at the
  first j with r_j <= B.  If |t_j| <= B and gcd(r_j, t_j) = 1, the result is
  a / b = sign(t_j) r_j / |t_j|, else there is none.  When a fraction a / b
  with |a| <= B, 0 < b <= B, gcd(a, b) = 1 and a = b x (mod M) exists, it is
  unique and this returns it.

Status codes: 0 reconstructed; 1 no fraction within the bound (more primes
are needed); 2 an input residue is not in [0, p_i) (e.g. the sentinel of a
singular point).

Parity: pinned by tests/test_oracle_rational.py -- fractions reduced mod
primes come back exactly, brute force over every residue for small moduli,
Python's own modular inverse for the residues, and amplitudes over Q against
the reconstruction of the F_p amplitudes.
"""
from __future__ import annotations

from math import gcd, isqrt

STATUS_OK = 0
STATUS_NO_FRACTION = 1
STATUS_BAD_RESIDUE = 2


def residue(num: int, den: int, p: int):
    """(status, num / den mod p): status 1 when p divides den."""
    if den % p == 0:
        return 1, None
    return 0, num % p * pow(den % p, p - 2, p) % p


def crt(residues, primes):
    """(x, M): 0 <= x < M with x = r_i mod p_i for distinct primes p_i."""
    M = 1
    for p in primes:
        M *= p
    x = 0
    for r, p in zip(residues, primes):
        Mi = M // p
        x += r * Mi * pow(Mi % p, p - 2, p)
    return x % M, M


def bound(M: int) -> int:
    """B = floor(sqrt((M - 1) / 2)): the numerator and denominator bound."""
    return isqrt((M - 1) // 2)


def rational_reconstruct(x: int, M: int):
    """(status, a, b) for 0 <= x < M, following the definition above."""
    B = bound(M)
    r0, r1 = M, x
    t0, t1 = 0, 1
    while r1 > B:
        q = r0 // r1
        r0, r1 = r1, r0 - q * r1
        t0, t1 = t1, t0 - q * t1
    if t1 == 0 or abs(t1) > B or gcd(r1, t1) != 1:
        return STATUS_NO_FRACTION, None, None
    return STATUS_OK, (r1 if t1 > 0 else -r1), abs(t1)


def reconstruct(residues, primes):
    """(status, a, b) from one residue per prime."""
    for r, p in zip(residues, primes):
        if not isinstance(r, int) or r < 0 or r >= p:
            return STATUS_BAD_RESIDUE, None, None
    x, M = crt(residues, primes)
    return rational_reconstruct(x, M)
