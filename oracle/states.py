"""Polarisation states of a massless d-dimensional gluon (paper Sec. 2.3).

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).  Plain field arithmetic
over any field of ``oracle.fields`` that contains a square root of -1 (F_p
with p = 1 mod 4, complex binary64, Gaussian rationals), written from the
definitions of Sec. 2.3 in the square-root-free normalisation:

Given a massless d-vector k (d >= 4, metric diag(+1, -1, ..., -1), component
indices 0..d-1) and a massless reference chi with components beyond index 3
equal to zero:

    k4  = (k^0, k^1, k^2, k^3, 0, ...),   mu^2 = k4.k4 (= sum_{i>=4} (k^i)^2),
    kb  = k4 - mu^2 / (2 chi.k4) chi      (massless, four-dimensional),
    e1  = <kb|gamma|chi] / (2 [kb chi]),  e2 = [kb|gamma|chi> / <kb chi>,
    e1~ = e2,  e2~ = e1,
and for d >= 5
    e3  = kb - mu^2 / (2 chi.k4) chi,     e3~ = e3 / mu^2,
for d >= 6
    e4  = (0, 0, 0, 0, k^5, -k^4, 0, ...),          e4~ = e4 / mu_6^2,
and for 5 <= x <= d - 2 the extra states, in the reading of the garbled
printed formula recorded with the design notes (indices counted as the
components above):
    ex^i = k^i k^{x+1}  (4 <= i <= x),  ex^{x+1} = -mu_{x+1}^2,  zero above,
    ex~  = ex / (mu_{x+1}^2 mu_{x+2}^2),
with mu_y^2 = sum_{i=4}^{y-1} (k^i)^2.  Then every state is transverse to k,
e_i . e_j~ = -delta_ij, and sum_i e_i^mu e_i~^nu = -g^{mu nu} + (k^mu eta^nu
+ eta^mu k^nu) / (k.eta) with eta = k4 - (0, 0, 0, 0, k^4, ...) (the
completeness relation of Sec. 2.3); for d = 4 the same holds with eta = chi.

Spinors of a massless four-vector v (the paper defers its conventions to
Gnendiger et al.; any factorisation is a valid little-group frame, and the
same one is used on every side): with v+ = v^0 + v^3, v- = v^0 - v^3,
vt = v^1 + i v^2, vtb = v^1 - i v^2, the matrix [[v+, vtb], [vt, v-]] has
determinant v.v = 0 and equals lam lamt^T for

    lam = (1, vt / v+),   lamt = (v+, vtb)     if the "plus chart" is used,
    lam = (vtb / v-, 1),  lamt = (vt, v-)      otherwise;

the plus chart is used when v+ != 0 (exact fields) or |v+|^2 >= |v-|^2
(complex binary64, squares of real and imaginary parts summed).  <ab> = a_1 b_2 - a_2 b_1 on lam, [ab] likewise on
lamt, and the four-vector of a rank-one matrix u w^T is
((M11 + M22)/2, (M12 + M21)/2, i (M12 - M21)/2, (M11 - M22)/2), so that
<a|gamma|b] = 2 vec(lam_a lamt_b^T).

State sum of a cut leg (Sec. 2.1, the leading pole of the cut equation):
with K_L, K_R the root currents of two trees whose last leg is the cut leg,
    S = sum_s (e_s . K_L)(e~_s . K_R).

Status: 0 ok; 1 singular (chi.k4 = 0, a zero bracket, an all-zero spinor
chart, or a zero mu^2 product needed by d >= 5).

Parity: pinned by tests/test_oracle_states.py (transversality,
orthonormality and the completeness relation exactly over F_p and Q(i), the
d = 4 states against Parke-Taylor through the amplitude oracle; the state
sum against the closed form the completeness relation gives, and against the
sum of products of amplitudes with the states as polarisations).
"""
from __future__ import annotations

from .fields import mdot


def _chart_plus(F, vp, vm):
    if F.name in ("fp", "q", "qi"):
        return not F.is_zero(vp)
    return vp.real * vp.real + vp.imag * vp.imag >= vm.real * vm.real + vm.imag * vm.imag


def spinors(F, v, i_unit):
    """(lam, lamt) of a massless four-vector v (first four components)."""
    vp = F.add(v[0], v[3])
    vm = F.sub(v[0], v[3])
    iv2 = F.mul(i_unit, v[2])
    vt = F.add(v[1], iv2)
    vtb = F.sub(v[1], iv2)
    if _chart_plus(F, vp, vm):
        if F.is_zero(vp):
            raise ZeroDivisionError("zero spinor chart")
        return (F.one, F.mul(vt, F.inv(vp))), (vp, vtb)
    if F.is_zero(vm):
        raise ZeroDivisionError("zero spinor chart")
    return (F.mul(vtb, F.inv(vm)), F.one), (vt, vm)


def bracket(F, a, b):
    return F.sub(F.mul(a[0], b[1]), F.mul(a[1], b[0]))


def vec_of(F, u, w, i_unit):
    """Four-vector of the rank-one matrix u w^T."""
    half = F.inv(F.add(F.one, F.one))
    m11, m12 = F.mul(u[0], w[0]), F.mul(u[0], w[1])
    m21, m22 = F.mul(u[1], w[0]), F.mul(u[1], w[1])
    return [F.mul(F.add(m11, m22), half), F.mul(F.add(m12, m21), half),
            F.mul(F.mul(i_unit, F.sub(m12, m21)), half), F.mul(F.sub(m11, m22), half)]


def states(F, k, chi, i_unit):
    """(status, [e_1..e_{d-2}], [e_1~..e_{d-2}~]) for the d-vector k."""
    d = len(k)
    z = F.zero
    try:
        k4 = list(k[:4]) + [z] * (d - 4)
        chi_d = list(chi[:4]) + [z] * (d - 4)
        mu2 = mdot(F, k4, k4)
        ck = mdot(F, chi_d, k4)
        if F.is_zero(ck):
            return 1, None, None
        c = F.mul(mu2, F.inv(F.add(ck, ck)))            # mu^2 / (2 chi.k4)
        kb = [F.sub(a, F.mul(c, b)) for a, b in zip(k4, chi_d)]
        lk, tk = spinors(F, kb, i_unit)
        lc, tc = spinors(F, chi_d, i_unit)
        sq = bracket(F, tk, tc)
        an = bracket(F, lk, lc)
        if F.is_zero(sq) or F.is_zero(an):
            return 1, None, None
        two = F.add(F.one, F.one)
        e1 = [F.mul(x, F.inv(sq)) for x in vec_of(F, lk, tc, i_unit)] + [z] * (d - 4)
        e2 = [F.mul(F.mul(two, x), F.inv(an)) for x in vec_of(F, lc, tk, i_unit)] + [z] * (d - 4)
        eps, epst = [e1, e2], [e2, e1]
        if d >= 5:
            if F.is_zero(mu2):
                return 1, None, None
            e3 = [F.sub(a, F.mul(c, b)) for a, b in zip(kb, chi_d)]
            eps.append(e3)
            epst.append([F.mul(x, F.inv(mu2)) for x in e3])

        def mu2y(y):  # sum_{i=4}^{y-1} (k^i)^2
            s = z
            for i in range(4, y):
                s = F.add(s, F.mul(k[i], k[i]))
            return s

        if d >= 6:
            e4 = [z] * d
            e4[4], e4[5] = k[5], F.neg(k[4])
            m6 = mu2y(6)
            if F.is_zero(m6):
                return 1, None, None
            eps.append(e4)
            epst.append([F.mul(x, F.inv(m6)) for x in e4])
        for x in range(5, d - 1):
            ex = [z] * d
            for i in range(4, x + 1):
                ex[i] = F.mul(k[i], k[x + 1])
            ex[x + 1] = F.neg(mu2y(x + 1))
            nrm = F.mul(mu2y(x + 1), mu2y(x + 2))
            if F.is_zero(nrm):
                return 1, None, None
            eps.append(ex)
            epst.append([F.mul(v, F.inv(nrm)) for v in ex])
        return 0, eps, epst
    except ZeroDivisionError:
        return 1, None, None


def state_sum(F, KL, KR, eps, epst):
    """sum_s (e_s . K_L)(e~_s . K_R), mostly-minus products."""
    s = F.zero
    for e, et in zip(eps, epst):
        s = F.add(s, F.mul(mdot(F, e, KL), mdot(F, et, KR)))
    return s
