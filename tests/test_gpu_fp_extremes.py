"""Z_p parity at the extremes of the lazily reduced int64 accumulators (paper
Sec. 3: 64-bit products reduced modulo p < 2^31; Sec. 3.1: the finite-field
kernels validated on their own).

Uniformly random residues give sums of products with random signs, far from
the largest magnitudes an overflow would need.  Here the inputs are built so
that the kernels' first products reach the extremes: the kernel reads a
canonical residue x as the balanced value x (x <= h) or x - p (x > h), with
h = (p - 1) / 2, so x = h and x = h + 1 give +h and -h.

* aligned legs: polarisations alternate between (-h, +h, +h, ...) and
  (+h, +h, +h, ...), so every product of a primed dot product of adjacent
  legs has the same sign and the largest size;
* extreme prefix sums: per component, momenta h, 1, p - 1, 1, p - 1, ...
  (with a per-component shift) make the prefix sums Q_l alternate between
  +h and -h, so the unreduced differences P_S = Q_{j+1} - Q_i reach 2h;
* draws from {0, 1, 2, h - 1, h, h + 1, h + 2, p - 2, p - 1} per component.

Every compiled kernel variant of each (n, d) is compared with the oracle bit
for bit, statuses included, at six primes: 2^31 - 1 (largest h),
2^31 - 19 (the default), the two primes whose fold constant 2^32 mod p is the
widest the small-fold-constant schedule accepts (+-2^22), and the two primes
below 2^31 whose fold constant is closest to +h and to -h (general schedule).
"""
import numpy as np
import pytest

from paper_2502_07060_amd import bg

import bgtest
from test_fp_bounds import _c32_extreme_prime, _sc_extreme_prime
from test_gpu_parity import assert_fp_equal, gpu_fp, torch_dev  # noqa: F401

pytestmark = pytest.mark.gpu

# 2^31 - 1 and 2^31 - 19 and the two primes with the widest fold constants the
# small-fold-constant schedule accepts run that schedule; the two primes with
# fold constants near +-h run the general one
PRIMES = [2**31 - 1, 2147483629, _sc_extreme_prime(+1), _sc_extreme_prime(-1),
          _c32_extreme_prime(+1), _c32_extreme_prime(-1)]


def extreme_inputs(seed, n, d, npts, p):
    rng = np.random.default_rng(seed)
    h = (p - 1) // 2
    S = np.array([0, 1, 2, h - 1, h, h + 1, h + 2, p - 2, p - 1], np.int64)
    k = np.empty((npts, n, d), np.int64)
    e = np.empty((npts, n, d), np.int64)
    for q in range(npts):
        kind = q % 4
        if kind == 0:
            # aligned legs and extreme prefix sums
            pat = np.array([h, 1] + [p - 1, 1] * n, np.int64)
            for mu in range(d):
                sh = (mu + q // 4) % 2
                k[q, :, mu] = pat[sh:sh + n]
            e[q] = h
            e[q, 1::2, 0] = h + 1
            # make a few components random so that not every P_S^2 vanishes
            mask = rng.random((n, d)) < 0.3
            k[q][mask] = rng.choice(S, size=mask.sum())
        elif kind == 1:
            k[q] = rng.choice(S, size=(n, d))
            e[q] = rng.choice(S, size=(n, d))
        elif kind == 2:
            # aligned legs with extreme but random-sign momenta
            k[q] = np.where(rng.random((n, d)) < 0.75, rng.choice(np.array([h, h + 1], np.int64), size=(n, d)),
                            rng.integers(0, p, size=(n, d)))
            e[q] = h
            e[q, 0::2, 0] = h + 1
        else:
            # extreme signs mixed with uniform residues
            k[q] = np.where(rng.random((n, d)) < 0.5, rng.choice(S, size=(n, d)),
                            rng.integers(0, p, size=(n, d)))
            e[q] = np.where(rng.random((n, d)) < 0.7, rng.choice(np.array([h, h + 1], np.int64), size=(n, d)),
                            rng.integers(0, p, size=(n, d)))
    return k, e


def _npts(n):
    return {4: 320, 8: 300, 11: 64, 14: 20}[n]


@pytest.mark.parametrize("p", PRIMES)
@pytest.mark.parametrize("n", [4, 8, 11, 14])
@pytest.mark.parametrize("d", [4, 6, 10])
def test_every_fp_variant_at_the_extremes(torch_dev, p, n, d):
    k, e = extreme_inputs(p % 1000 + 31 * n + d, n, d, _npts(n), p)
    st_o, v_o = bgtest.oracle_fp(k, e, p)
    # the inputs must exercise the arithmetic, not only the singular path
    assert (st_o == 0).mean() >= 0.5, f"only {(st_o == 0).mean():.2f} of the points are regular"
    variants = bg.bg_variants(bg.BG_FIELD_FP, n, d)
    assert variants
    try:
        for v in variants:
            bg.bg_select_variant(bg.BG_FIELD_FP, n, d, v["index"])
            st_g, v_g = gpu_fp(torch_dev, k, e, p)
            assert_fp_equal(st_g, v_g, st_o, v_o, f"extremes p={p} n={n} d={d} variant {v}")
    finally:
        bg.bg_select_variant(bg.BG_FIELD_FP, n, d, -1)
