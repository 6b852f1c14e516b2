"""Seeded synthetic inputs: momenta and polarisation vectors (host, numpy).

This module feeds both the GPU path and the test oracle.  It holds none of the
Berends-Giele recursion's arithmetic: only phase-space generation, spinor
helicity polarisation vectors, finite-field kinematics and layout helpers.

Conventions
-----------
* Metric diag(+1, -1, ..., -1) (paper Sec. 2.3).  Momenta are all-outgoing,
  sum_l k_l = 0; incoming beams are negated.
* Arrays are (npts, n, d) here; ``to_soa`` produces the C-ABI layout
  [n][d][npts] with the point index fastest (complex interleaved re/im).
* Spinors: for a null vector k the 2x2 matrix
      K = [[k0 + k3, k1 - i k2], [k1 + i k2, k0 - k3]],  det K = k^2 = 0,
  factors as K = lam lamt^T.  We pick the square-root-free chart
      lam = (1, (k1 + i k2)/k+),  lamt = (k+, k1 - i k2)        if |k+| >= |k-|
      lam = ((k1 - i k2)/k-, 1),  lamt = (k1 + i k2, k-)        otherwise
  (k+- = k0 +- k3); any factorisation is a valid little-group frame, and the
  same spinors feed the polarisations and the Parke-Taylor check.
  <ab> = lam_a^1 lam_b^2 - lam_a^2 lam_b^1,  [ab] = lamt_a^1 lamt_b^2 - lamt_a^2 lamt_b^1,
  so 2 a.b = <ab>[ab].  The vector of a rank-one matrix M = u w^T is
      vec(M) = ((M11+M22)/2, (M12+M21)/2, i(M12-M21)/2, (M11-M22)/2),
  and <a|gamma^mu|b] = 2 vec(lam_a lamt_b^T).
* Polarisations with the paper's square-root-free normalisation (Sec. 2.3,
  the d = 6 states and their d > 6 re-normalised form):
      eps_1 = <k|gamma^mu|chi] / (2 [k chi])   ("minus", carries lam_k)
      eps_2 = [k|gamma^mu|chi> / <k chi>       ("plus",  carries lamt_k)
  with a null reference chi; (eps_1, eps_2) = -1 and (eps_i, eps_i) = 0.
* Finite-field points (d dimensions, prime p): light-cone coordinates
  k+ = k^0 + k^{d-1}, k- = k^0 - k^{d-1}, transverse k^1..k^{d-2}; null
  vectors have k- = |k_T|^2 / k+.  The last two legs close momentum
  conservation: Q = -sum_{l<=n-2} k_l, r null, t = Q^2/(2 Q.r),
  k_{n-1} = t r, k_n = Q - t r.  Polarisations eps = v - (v.k)/(q.k) q
  with v random and q a random null vector (transverse by construction).
"""
from __future__ import annotations

import numpy as np

DEFAULT_PRIME = 2147483629  # 2^31 - 19, the paper's default (Sec. 3)


# ----------------------------------------------------------------------------
# modular helpers (numpy int64; every operand is a canonical residue < 2^31 so
# a single product fits in int64 before reduction)
# ----------------------------------------------------------------------------

def _mm(a, b, p):
    return (np.asarray(a, np.int64) * np.asarray(b, np.int64)) % p


def _pow(a, e, p):
    a = np.asarray(a, np.int64) % p
    r = np.ones_like(a)
    while e:
        if e & 1:
            r = _mm(r, a, p)
        a = _mm(a, a, p)
        e >>= 1
    return r


def _inv(a, p):
    return _pow(a, p - 2, p)


def fp_mdot(x, y, p):
    """Minkowski product over F_p along the last axis (mostly minus)."""
    s = _mm(x[..., 0], y[..., 0], p)
    for mu in range(1, x.shape[-1]):
        s = (s - _mm(x[..., mu], y[..., mu], p)) % p
    return s


def fp_sqrt_minus_one(p: int) -> int:
    """A square root of -1 mod p (p = 1 mod 4): g^((p-1)/4) for a non-residue g."""
    if p % 4 != 1:
        raise ValueError("i is in F_p only for p = 1 mod 4")
    g = 2
    while pow(g, (p - 1) // 2, p) != p - 1:
        g += 1
    return pow(g, (p - 1) // 4, p)


def c_mdot(x, y):
    """Bilinear Minkowski product over C along the last axis."""
    return x[..., 0] * y[..., 0] - np.sum(x[..., 1:] * y[..., 1:], axis=-1)


# ----------------------------------------------------------------------------
# real phase space
# ----------------------------------------------------------------------------

def rambo(rng, n_out: int, sqrt_s: float, npts: int, d: int = 4):
    """Massless flat phase space (Kleiss, Stirling, Ellis, RAMBO, 1986).

    Returns (npts, n_out, d) outgoing momenta summing to (sqrt_s, 0, ..., 0).
    In d dimensions the isotropic directions are uniform on S^{d-2} and the
    energies are Gamma(d-2, 1) distributed (the d = 4 case is -ln(r1 r2)).
    """
    q0 = rng.gamma(shape=d - 2, scale=1.0, size=(npts, n_out))
    dirs = rng.standard_normal(size=(npts, n_out, d - 1))
    dirs /= np.linalg.norm(dirs, axis=-1, keepdims=True)
    q = np.empty((npts, n_out, d))
    q[..., 0] = q0
    q[..., 1:] = q0[..., None] * dirs
    Q = q.sum(axis=1)                                   # (npts, d)
    M = np.sqrt(Q[:, 0] ** 2 - np.sum(Q[:, 1:] ** 2, axis=-1))
    b = -Q[:, 1:] / M[:, None]
    x = sqrt_s / M
    gamma = Q[:, 0] / M
    a = 1.0 / (1.0 + gamma)
    bq = np.einsum("pi,pli->pl", b, q[..., 1:])
    out = np.empty_like(q)
    out[..., 0] = x[:, None] * (gamma[:, None] * q[..., 0] + bq)
    out[..., 1:] = x[:, None, None] * (q[..., 1:] + b[:, None, :] * q[..., :1]
                                       + a[:, None, None] * bq[..., None] * b[:, None, :])
    return out


def collider_point(rng, n: int, sqrt_s: float, npts: int, d: int = 4):
    """All-outgoing momenta of a 2 -> n-2 massless process.

    Beams p1, p2 = (sqrt_s/2)(1, 0, ..., 0, +-1) along the last axis enter
    negated: k1 = -p1, k2 = -p2, k3..kn from ``rambo``.
    """
    k = np.zeros((npts, n, d))
    e = sqrt_s / 2
    k[:, 0, 0], k[:, 0, d - 1] = -e, -e
    k[:, 1, 0], k[:, 1, d - 1] = -e, e
    k[:, 2:, :] = rambo(rng, n - 2, sqrt_s, npts, d)
    return k


# ----------------------------------------------------------------------------
# spinor helicity (complex, d = 4)
# ----------------------------------------------------------------------------

def spinors(k):
    """(lam, lamt), each (..., 2) complex, with lam lamt^T = K(k) (see header)."""
    k = np.asarray(k, dtype=complex)
    kp = k[..., 0] + k[..., 3]
    km = k[..., 0] - k[..., 3]
    kt = k[..., 1] + 1j * k[..., 2]
    ktb = k[..., 1] - 1j * k[..., 2]
    use_p = np.abs(kp) >= np.abs(km)
    safe_kp = np.where(use_p, kp, 1.0)
    safe_km = np.where(use_p, 1.0, km)
    lam = np.empty(k.shape[:-1] + (2,), complex)
    lamt = np.empty_like(lam)
    lam[..., 0] = np.where(use_p, 1.0, ktb / safe_km)
    lam[..., 1] = np.where(use_p, kt / safe_kp, 1.0)
    lamt[..., 0] = np.where(use_p, kp, kt)
    lamt[..., 1] = np.where(use_p, ktb, km)
    return lam, lamt


def angle(la, lb):
    return la[..., 0] * lb[..., 1] - la[..., 1] * lb[..., 0]


def square(ta, tb):
    return ta[..., 0] * tb[..., 1] - ta[..., 1] * tb[..., 0]


def vec_of(u, w):
    """vec(u w^T) for 2-spinors u, w (complex)."""
    m11 = u[..., 0] * w[..., 0]
    m12 = u[..., 0] * w[..., 1]
    m21 = u[..., 1] * w[..., 0]
    m22 = u[..., 1] * w[..., 1]
    return np.stack([(m11 + m22) / 2, (m12 + m21) / 2, 1j * (m12 - m21) / 2,
                     (m11 - m22) / 2], axis=-1)


def pol_minus(lam_k, lamt_k, lam_c, lamt_c):
    """eps_1 = <k|gamma|chi]/(2[k chi]) = vec(lam_k lamt_chi^T)/[k chi]."""
    return vec_of(lam_k, lamt_c) / square(lamt_k, lamt_c)[..., None]


def pol_plus(lam_k, lamt_k, lam_c, lamt_c):
    """eps_2 = [k|gamma|chi>/<k chi> = 2 vec(lam_chi lamt_k^T)/<k chi>."""
    return 2 * vec_of(lam_c, lamt_k) / angle(lam_k, lam_c)[..., None]


def random_null_c(rng, npts, d=4):
    """Random real null vectors with unit-scale energy (isotropic direction)."""
    dirs = rng.standard_normal(size=(npts, d - 1))
    dirs /= np.linalg.norm(dirs, axis=-1, keepdims=True)
    e = rng.uniform(0.5, 1.5, size=npts)
    return np.concatenate([e[:, None], e[:, None] * dirs], axis=-1)


def helicity_pols(rng, k, hel, min_bracket=1e-3):
    """Spinor-helicity polarisations for d = 4 complex momenta.

    hel: (npts, n) array of -1 / +1.  One random null reference chi per point,
    shared by all legs, redrawn where some |<chi k>| or |[chi k]| is below
    ``min_bracket`` times the scale of the brackets.
    Returns (eps (npts, n, 4) complex, lam, lamt, chi).
    """
    npts, n, _ = k.shape
    lam, lamt = spinors(k)
    chi = random_null_c(rng, npts)
    for _ in range(100):
        lc, tc = spinors(chi)
        a = np.abs(angle(lam, lc[:, None, :]))
        s = np.abs(square(lamt, tc[:, None, :]))
        scale = np.sqrt(np.abs(k[..., 0]) * np.abs(chi[:, None, 0]))
        bad = np.any((a * s) < (min_bracket * scale) ** 2 * 4, axis=1)
        if not bad.any():
            break
        chi[bad] = random_null_c(rng, int(bad.sum()))
    lc, tc = spinors(chi)
    em = pol_minus(lam, lamt, lc[:, None, :], tc[:, None, :])
    ep = pol_plus(lam, lamt, lc[:, None, :], tc[:, None, :])
    eps = np.where((np.asarray(hel) < 0)[..., None], em, ep)
    return eps, lam, lamt, chi


def transverse_pols_c(rng, k):
    """eps = v - (v.k)/(q.k) q over C, v complex Gaussian, q random real null."""
    npts, n, d = k.shape
    q = random_null_c(rng, npts, d)
    for _ in range(100):
        qk = c_mdot(q[:, None, :], k)
        bad = np.any(np.abs(qk) < 1e-6 * np.abs(k[..., 0]), axis=1)
        if not bad.any():
            break
        q[bad] = random_null_c(rng, int(bad.sum()), d)
    v = rng.standard_normal((npts, n, d)) + 1j * rng.standard_normal((npts, n, d))
    qk = c_mdot(q[:, None, :], k)
    vk = c_mdot(v, k)
    return v - (vk / qk)[..., None] * q[:, None, :]


# ----------------------------------------------------------------------------
# finite-field kinematics
# ----------------------------------------------------------------------------

def fp_null(rng, p, shape, d):
    """Uniform null vectors over F_p in light-cone coordinates (k+ != 0)."""
    kp = rng.integers(1, p, size=shape, dtype=np.int64)
    kt = rng.integers(0, p, size=shape + (d - 2,), dtype=np.int64)
    t2 = np.zeros(shape, np.int64)
    for i in range(d - 2):
        t2 = (t2 + _mm(kt[..., i], kt[..., i], p)) % p
    km = _mm(t2, _inv(kp, p), p)
    half = (p + 1) // 2
    v = np.empty(shape + (d,), np.int64)
    v[..., 0] = _mm((kp + km) % p, half, p)
    v[..., d - 1] = _mm((kp - km) % p, half, p)
    v[..., 1:d - 1] = kt
    return v


def fp_point(rng, p, n, d, npts):
    """F_p momenta for n legs: n-2 random null legs plus the closing pair.

    Points whose closing pair needs a division by zero (Q.r = 0) are redrawn.
    Returns int64 (npts, n, d) canonical residues.
    """
    k = np.empty((npts, n, d), np.int64)
    todo = np.arange(npts)
    while todo.size:
        m = todo.size
        kk = fp_null(rng, p, (m, n - 2), d)
        Q = (-kk.sum(axis=1)) % p
        r = fp_null(rng, p, (m,), d)
        Qr = fp_mdot(Q, r, p)
        ok = Qr != 0
        Q2 = fp_mdot(Q, Q, p)
        t = _mm(Q2, _inv(_mm(2, np.where(ok, Qr, 1), p), p), p)
        k1 = _mm(t[:, None], r, p)
        k2 = (Q - k1) % p
        sel = todo[ok]
        k[sel, : n - 2] = kk[ok]
        k[sel, n - 2] = k1[ok]
        k[sel, n - 1] = k2[ok]
        todo = todo[~ok]
    return k


def fp_transverse_pols(rng, p, k):
    """eps = v - (v.k)/(q.k) q over F_p, one random null q per point.

    Points where some q.k_l = 0 get a fresh q.
    """
    npts, n, d = k.shape
    q = fp_null(rng, p, (npts,), d)
    for _ in range(100):
        qk = fp_mdot(q[:, None, :], k, p)
        bad = np.any(qk == 0, axis=1)
        if not bad.any():
            break
        q[bad] = fp_null(rng, p, (int(bad.sum()),), d)
    v = rng.integers(0, p, size=(npts, n, d), dtype=np.int64)
    qk = fp_mdot(q[:, None, :], k, p)
    vk = fp_mdot(v, k, p)
    c = _mm(vk, _inv(qk, p), p)
    return (v - _mm(c[..., None], q[:, None, :], p)) % p


def fp_spinors(k, p, ip):
    """Square-root-free spinors over F_p (d = 4 components), ip^2 = -1 mod p."""
    kp = (k[..., 0] + k[..., 3]) % p
    km = (k[..., 0] - k[..., 3]) % p
    kt = (k[..., 1] + _mm(ip, k[..., 2], p)) % p
    ktb = (k[..., 1] - _mm(ip, k[..., 2], p)) % p
    use_p = kp != 0
    lam = np.empty(k.shape[:-1] + (2,), np.int64)
    lamt = np.empty_like(lam)
    lam[..., 0] = np.where(use_p, 1, _mm(ktb, _inv(np.where(use_p, 1, km), p), p))
    lam[..., 1] = np.where(use_p, _mm(kt, _inv(np.where(use_p, kp, 1), p), p), 1)
    lamt[..., 0] = np.where(use_p, kp, kt)
    lamt[..., 1] = np.where(use_p, ktb, km)
    return lam, lamt


def fp_angle(la, lb, p):
    return (_mm(la[..., 0], lb[..., 1], p) - _mm(la[..., 1], lb[..., 0], p)) % p


def fp_square(ta, tb, p):
    return (_mm(ta[..., 0], tb[..., 1], p) - _mm(ta[..., 1], tb[..., 0], p)) % p


def fp_vec_of(u, w, p, ip):
    half = (p + 1) // 2
    m11 = _mm(u[..., 0], w[..., 0], p)
    m12 = _mm(u[..., 0], w[..., 1], p)
    m21 = _mm(u[..., 1], w[..., 0], p)
    m22 = _mm(u[..., 1], w[..., 1], p)
    return np.stack([_mm(m11 + m22, half, p), _mm(m12 + m21, half, p),
                     _mm(_mm(ip, (m12 - m21) % p, p), half, p),
                     _mm((m11 - m22) % p, half, p)], axis=-1)


def fp_helicity_pols(rng, p, k, hel):
    """Spinor-helicity polarisations over F_p for d = 4 (needs p = 1 mod 4).

    Returns (eps, lam, lamt, ip).
    """
    ip = fp_sqrt_minus_one(p)
    npts, n, _ = k.shape
    lam, lamt = fp_spinors(k, p, ip)
    chi = fp_null(rng, p, (npts,), 4)
    for _ in range(100):
        lc, tc = fp_spinors(chi, p, ip)
        a = fp_angle(lam, lc[:, None, :], p)
        s = fp_square(lamt, tc[:, None, :], p)
        bad = np.any((a == 0) | (s == 0), axis=1)
        if not bad.any():
            break
        chi[bad] = fp_null(rng, p, (int(bad.sum()),), 4)
    lc, tc = fp_spinors(chi, p, ip)
    lc, tc = lc[:, None, :], tc[:, None, :]
    em = _mm(fp_vec_of(lam, tc, p, ip), _inv(fp_square(lamt, tc, p), p)[..., None], p)
    ep = _mm(_mm(2, fp_vec_of(lc, lamt, p, ip), p),
             _inv(fp_angle(lam, lc, p), p)[..., None], p)
    eps = np.where((np.asarray(hel) < 0)[..., None], em, ep)
    return eps, lam, lamt, ip


# ----------------------------------------------------------------------------
# workloads
# ----------------------------------------------------------------------------

def mhv_c128(seed: int, n: int, npts: int, sqrt_s: float = 1000.0, minus=(0, 1)):
    """Complex d = 4 points, fixed helicities (legs in ``minus`` negative)."""
    rng = np.random.default_rng(seed)
    k = collider_point(rng, n, sqrt_s, npts, 4)
    hel = np.ones((npts, n), np.int64)
    for l in minus:
        hel[:, l] = -1
    eps, lam, lamt, chi = helicity_pols(rng, k, hel)
    return k.astype(complex), eps, hel


def random_helicity_c128(seed: int, n: int, npts: int, sqrt_s: float = 1000.0):
    """Complex d = 4 points with iid uniform helicities per leg per point."""
    rng = np.random.default_rng(seed)
    k = collider_point(rng, n, sqrt_s, npts, 4)
    hel = rng.choice(np.array([-1, 1]), size=(npts, n))
    eps, lam, lamt, chi = helicity_pols(rng, k, hel)
    return k.astype(complex), eps, hel


def generic_c128(seed: int, n: int, d: int, npts: int, sqrt_s: float = 1000.0):
    """Complex points in d dimensions: RAMBO momenta, transverse random eps."""
    rng = np.random.default_rng(seed)
    k = collider_point(rng, n, sqrt_s, npts, d)
    eps = transverse_pols_c(rng, k)
    return k.astype(complex), eps


def generic_fp(seed: int, n: int, d: int, npts: int, p: int = DEFAULT_PRIME):
    """F_p points in d dimensions: light-cone momenta with closing pair,
    transverse eps.  Returns uint32 arrays (npts, n, d)."""
    rng = np.random.default_rng(seed)
    k = fp_point(rng, p, n, d, npts)
    eps = fp_transverse_pols(rng, p, k)
    return k.astype(np.uint32), eps.astype(np.uint32)


def rational_points(seed: int, n: int, d: int, npts: int, kmax: int = 9, wmax: int = 5):
    """Physical kinematic points with rational components (exact, Python
    Fractions): n - 2 light-cone null momenta with integer k+ in [1, kmax]
    and transverse components in [-kmax, kmax], a closing null pair
    t r, Q - t r (Q = -sum of the others, r null, t = Q.Q / (2 Q.r)), one null
    reference q per point and polarisations eps = w - (w.k)/(q.k) q with
    integer w in [-wmax, wmax]; points with a vanishing sub-range P_S^2 are
    redrawn.  Returns int64 numerator and denominator
    arrays (knum, kden, enum, eden), each [npts][n][d]."""
    from fractions import Fraction
    import random
    rng = random.Random(seed)

    def dot(x, y):
        return x[0] * y[0] - sum(a * b for a, b in zip(x[1:], y[1:]))

    def null():
        kp = Fraction(rng.randint(1, kmax))
        kt = [Fraction(rng.randint(-kmax, kmax)) for _ in range(d - 2)]
        km = sum(x * x for x in kt) / kp
        return [(kp + km) / 2] + kt + [(kp - km) / 2]

    out = np.zeros((4, npts, n, d), np.int64)
    q = 0
    while q < npts:
        ks = [null() for _ in range(n - 2)]
        Qv = [-sum(v[mu] for v in ks) for mu in range(d)]
        r = null()
        qr = dot(Qv, r)
        if qr == 0:
            continue
        t = dot(Qv, Qv) / (2 * qr)
        ks += [[t * x for x in r], [a - t * b for a, b in zip(Qv, r)]]
        ref = null()
        if any(dot(ref, v) == 0 for v in ks):
            continue
        # no vanishing propagator: P_S^2 != 0 for the contiguous S of legs 1..n-1, 2 <= |S| <= n-2
        sing = False
        for i in range(n - 1):
            P = list(ks[i])
            for j in range(i + 1, n - 1):
                P = [a + b for a, b in zip(P, ks[j])]
                if j - i + 1 <= n - 2 and dot(P, P) == 0:
                    sing = True
        if sing:
            continue
        eps = []
        for v in ks:
            w = [Fraction(rng.randint(-wmax, wmax)) for _ in range(d)]
            c = dot(w, v) / dot(ref, v)
            eps.append([a - c * b for a, b in zip(w, ref)])
        vals = [ks, eps]
        if any(abs(x.numerator) >= 2 ** 62 or x.denominator >= 2 ** 62 for vs in vals for v in vs for x in v):
            continue
        for s, vs in enumerate(vals):
            for l in range(n):
                for mu in range(d):
                    out[2 * s, q, l, mu] = vs[l][mu].numerator
                    out[2 * s + 1, q, l, mu] = vs[l][mu].denominator
        q += 1
    return out[0], out[1], out[2], out[3]


def config_workload(name: str, npts: int | None = None):
    """The named synthetic workloads:

    c5_small   n=5, d=4, complex128, helicities (--+++), 10^4 points, seed 1
    c8_d4      n=8, d=4, complex128, uniform random helicities, 2^20 points, seed 2
    fp8_d6     n=8, d=6, F_p (p = 2^31-19), 2^20 points, seed 3
    Returns a dict with field, n, d, p, k, eps (and hel for complex).
    """
    if name == "c5_small":
        m = 10_000 if npts is None else npts
        k, eps, hel = mhv_c128(1, 5, m)
        return dict(field="c128", n=5, d=4, p=0, k=k, eps=eps, hel=hel)
    if name == "c8_d4":
        m = 1 << 20 if npts is None else npts
        k, eps, hel = random_helicity_c128(2, 8, m)
        return dict(field="c128", n=8, d=4, p=0, k=k, eps=eps, hel=hel)
    if name == "fp8_d6":
        m = 1 << 20 if npts is None else npts
        k, eps = generic_fp(3, 8, 6, m)
        return dict(field="fp", n=8, d=6, p=DEFAULT_PRIME, k=k, eps=eps)
    raise KeyError(name)


def batched_groups(total: int = 4_000_000, seed: int = 4, ns=range(4, 15), ds=(4, 6, 8, 10),
                   fields=("c128", "fp"), zipf_s: float = 1.2):
    """Group shapes and sizes of the mixed batched workload.

    Groups are (field, n, d) over the given ranges; their sizes are a
    multinomial draw of `total` points with weights proportional to
    r^-zipf_s over the ranks r = 1..G, ranks assigned to groups by a seeded
    permutation.  Returns a list of dicts (field, n, d, npts, seed).
    """
    rng = np.random.default_rng(seed)
    shapes = [(f, n, d) for f in fields for n in ns for d in ds]
    w = np.arange(1, len(shapes) + 1, dtype=float) ** (-zipf_s)
    w /= w.sum()
    sizes = rng.multinomial(total, w)
    order = rng.permutation(len(shapes))
    out = []
    for rank, g in enumerate(order):
        f, n, d = shapes[g]
        out.append(dict(field=f, n=n, d=d, npts=int(sizes[rank]), seed=int(seed * 1000 + g)))
    return out


def group_inputs(g, p: int = DEFAULT_PRIME):
    """Inputs for one group of ``batched_groups``: F_p groups use the F_p
    light-cone generator, complex d = 4 groups spinor-helicity points with
    random helicities, complex d > 4 groups RAMBO momenta in d dimensions with
    transverse random polarisations."""
    m = max(g["npts"], 1)
    if g["field"] == "fp":
        k, e = generic_fp(g["seed"], g["n"], g["d"], m, p)
    elif g["d"] == 4:
        k, e, _ = random_helicity_c128(g["seed"], g["n"], m)
    else:
        k, e = generic_c128(g["seed"], g["n"], g["d"], m)
    return k[:g["npts"]], e[:g["npts"]]


# ----------------------------------------------------------------------------
# layout
# ----------------------------------------------------------------------------

def to_soa(a, ld: int | None = None):
    """(npts, n, d) -> (n, d, ld) contiguous, point index fastest.

    Complex input becomes complex128, integer input uint32.  Columns past
    npts (ld > npts) are zero.
    """
    a = np.asarray(a)
    npts, n, d = a.shape
    ld = npts if ld is None else ld
    dt = np.complex128 if np.iscomplexobj(a) else np.uint32
    out = np.zeros((n, d, ld), dt)
    out[:, :, :npts] = np.transpose(a, (1, 2, 0))
    return out


def from_soa(a, npts: int):
    """(n, d, ld) -> (npts, n, d)."""
    return np.ascontiguousarray(np.transpose(np.asarray(a)[:, :, :npts], (2, 0, 1)))
