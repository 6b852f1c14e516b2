"""Generator pins: on-shell, momentum conservation, transversality and the
polarisation identities of the paper (Sec. 2.3: (k, eps_i) = 0,
(eps_1, eps_2) = -1, (eps_1, eps_1) = (eps_2, eps_2) = 0)."""
import numpy as np
import pytest

from paper_2502_07060_amd import inputs as I

P = I.DEFAULT_PRIME


@pytest.mark.parametrize("d", [4, 6, 10])
def test_rambo_on_shell_and_conserved(d):
    rng = np.random.default_rng(0)
    k = I.collider_point(rng, 8, 1000.0, 200, d)
    k2 = k[..., 0] ** 2 - np.sum(k[..., 1:] ** 2, axis=-1)
    assert np.max(np.abs(k2)) < 1e-9 * 1000.0 ** 2
    assert np.max(np.abs(k.sum(axis=1))) < 1e-9 * 1000.0
    assert np.allclose(k[:, 2:, 0].sum(axis=1), 1000.0)
    assert np.all(k[:, 2:, 0] > 0)


def test_spinors_factorise_momenta():
    rng = np.random.default_rng(1)
    k = I.collider_point(rng, 6, 1000.0, 50, 4).astype(complex)
    lam, lamt = I.spinors(k)
    v = I.vec_of(lam, lamt)
    assert np.allclose(v, k, atol=1e-9)
    a = I.angle(lam[:, :, None, :], lam[:, None, :, :])
    s = I.square(lamt[:, :, None, :], lamt[:, None, :, :])
    two_kk = 2 * I.c_mdot(k[:, :, None, :], k[:, None, :, :])
    assert np.allclose(a * s, two_kk, rtol=1e-10, atol=1e-6)


def test_helicity_polarisation_identities():
    rng = np.random.default_rng(2)
    npts, n = 40, 7
    k = I.collider_point(rng, n, 1000.0, npts, 4).astype(complex)
    lam, lamt = I.spinors(k)
    chi = I.random_null_c(rng, npts)
    lc, tc = I.spinors(chi)
    lc, tc = lc[:, None, :], tc[:, None, :]
    em = I.pol_minus(lam, lamt, lc, tc)
    ep = I.pol_plus(lam, lamt, lc, tc)
    md = I.c_mdot
    assert np.allclose(md(em, ep), -1)
    # the square-root-free chart gives |eps_-| ~ 1/|k| and |eps_+| ~ |k|, so
    # the vanishing products are checked relative to the natural scale
    nrm = lambda v: np.sqrt(np.sum(np.abs(v) ** 2, axis=-1))
    assert np.max(np.abs(md(em, em)) / nrm(em) ** 2) < 1e-13
    assert np.max(np.abs(md(ep, ep)) / nrm(ep) ** 2) < 1e-13
    assert np.max(np.abs(md(em, k)) / (nrm(em) * nrm(k))) < 1e-13
    assert np.max(np.abs(md(ep, k)) / (nrm(ep) * nrm(k))) < 1e-13
    chi_b = chi[:, None, :]
    assert np.max(np.abs(md(em, chi_b)) / (nrm(em) * nrm(chi_b))) < 1e-13
    assert np.max(np.abs(md(ep, chi_b)) / (nrm(ep) * nrm(chi_b))) < 1e-13


@pytest.mark.parametrize("d", [4, 6, 8, 10])
def test_fp_points_exact(d):
    rng = np.random.default_rng(3)
    k = I.fp_point(rng, P, 8, d, 300)
    assert k.min() >= 0 and k.max() < P
    assert np.all(I.fp_mdot(k, k, P) == 0)
    assert np.all(k.sum(axis=1) % P == 0)
    eps = I.fp_transverse_pols(rng, P, k)
    assert np.all(I.fp_mdot(eps, k, P) == 0)


def test_fp_helicity_identities_exact():
    rng = np.random.default_rng(4)
    ip = I.fp_sqrt_minus_one(P)
    assert (ip * ip) % P == P - 1
    k = I.fp_point(rng, P, 6, 4, 50)
    hel = np.ones((50, 6), np.int64)
    hel[:, :3] = -1
    eps, lam, lamt, _ = I.fp_helicity_pols(rng, P, k, hel)
    assert np.all(I.fp_mdot(eps, k, P) == 0)
    assert np.all(I.fp_mdot(eps, eps, P) == 0)
    v = I.fp_vec_of(lam, lamt, P, ip)
    assert np.array_equal(v % P, k % P)
    # (eps_-, eps_+) = -1 on the same leg and reference: build both for leg 0
    hel_m = -np.ones((50, 6), np.int64)
    hel_p = np.ones((50, 6), np.int64)
    rng_a, rng_b = np.random.default_rng(9), np.random.default_rng(9)
    em, *_ = I.fp_helicity_pols(rng_a, P, k, hel_m)
    epl, *_ = I.fp_helicity_pols(rng_b, P, k, hel_p)
    assert np.all(I.fp_mdot(em, epl, P) == P - 1)


def test_soa_roundtrip():
    rng = np.random.default_rng(5)
    a = rng.standard_normal((10, 5, 4)) + 1j * rng.standard_normal((10, 5, 4))
    s = I.to_soa(a, ld=16)
    assert s.shape == (5, 4, 16) and s.dtype == np.complex128
    assert np.array_equal(I.from_soa(s, 10), a)
    u = rng.integers(0, P, size=(7, 3, 6)).astype(np.uint32)
    su = I.to_soa(u)
    assert su.dtype == np.uint32 and su[2, 4, 5] == u[5, 2, 4]


def test_workloads_are_seeded():
    a = I.config_workload("fp8_d6", npts=64)
    b = I.config_workload("fp8_d6", npts=64)
    assert np.array_equal(a["k"], b["k"]) and np.array_equal(a["eps"], b["eps"])
    c = I.config_workload("c5_small", npts=32)
    assert c["k"].shape == (32, 5, 4) and np.all(c["hel"][:, :2] == -1)


def test_rational_points_are_physical():
    """rational_points: massless momenta summing to zero and transverse
    polarisations, exactly (fractions rebuilt from the int64 arrays)."""
    from fractions import Fraction
    n, d = 6, 5
    kn, kd, en, ed = I.rational_points(3, n, d, 4)
    dot = lambda x, y: x[0] * y[0] - sum(a * b for a, b in zip(x[1:], y[1:]))
    for q in range(4):
        k = [[Fraction(int(kn[q, l, m]), int(kd[q, l, m])) for m in range(d)] for l in range(n)]
        e = [[Fraction(int(en[q, l, m]), int(ed[q, l, m])) for m in range(d)] for l in range(n)]
        assert all(dot(v, v) == 0 for v in k)
        assert all(sum(v[m] for v in k) == 0 for m in range(d))
        assert all(dot(a, b) == 0 for a, b in zip(k, e))
        assert (kd[q] > 0).all() and (ed[q] > 0).all()
