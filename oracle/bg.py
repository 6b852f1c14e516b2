"""Berends-Giele recursion, oracle version (test infrastructure only).

What is computed (paper Sec. 2.2, the current recursion, the vertices V3 and
V4, and the sub-range momenta P_{i,j}):

* Legs 1..n carry momenta k_l and polarisation vectors eps_l (d components
  each, mostly-minus metric).  Let N = n - 1; currents live on contiguous
  sub-ranges S = [i..j] of the legs 1..N, and P_S = sum_{l in S} k_l.
* Base case: J([l]) = eps_l  (reading 1: the one-leg current is the leg's
  polarisation vector; the paper does not print the base case).
* For 2 <= |S| <= N - 1 the paper's recursion reads
      J^mu(S) = (-i / P_S^2) [ sum_{A|B = S} V3^{mu nu rho}(P_A, P_B) J_nu(A) J_rho(B)
                              + sum_{A|B|C = S} V4^{mu nu rho sigma} J_nu(A) J_rho(B) J_sigma(C) ]
  with V3(P,Q) = i (g^{nu rho}(P-Q)^mu + 2 g^{rho mu} Q^nu - 2 g^{mu nu} P^rho)
  and  V4 = i (2 g^{mu rho} g^{nu sigma} - g^{mu nu} g^{rho sigma} - g^{mu sigma} g^{nu rho}).
  Contracting the metric tensors gives, per split,
      V3 . J_A J_B   = i [ (J_A.J_B)(P_A - P_B) + 2 (P_B.J_A) J_B - 2 (P_A.J_B) J_A ]
      V4 . J_A J_B J_C = i [ 2 (J_A.J_C) J_B - (J_A.J_B) J_C - (J_B.J_C) J_A ]
  so every vertex carries one factor i and the propagator one factor -i;
  (-i)(i) = 1 and the current is J(S) = K(S) / P_S^2 with K(S) the sum of the
  bracketed, i-free terms.  This needs no square root of -1, so the same code
  runs over any field.
* The amplitude (paper: build the n-point matrix element from the (n-1)-point
  current by removing the off-shell propagator and contracting with eps_n):
  removing -i/P^2 from J([1..N]) leaves i K([1..N]); contracting with eps_n
  gives A = i * (eps_n . K([1..N])).  The oracle returns M = eps_n . K([1..N])
  (reading 2: the i-stripped amplitude, field independent); A = i M.
  Momentum conservation enters only through the caller's k_l; k_n itself is
  never read (reading 3).
* Singular point (reading 9): if some P_S^2 == 0 for 2 <= |S| <= N-1 the
  amplitude is undefined; status 1 and the sentinel are returned.
* Non-canonical residue (F_p only, reading 11): if any component that the
  recursion reads (k_1..k_{n-1}, eps_1..eps_n) is not an integer in [0, p),
  status 2 and the sentinel are returned.  Status 2 takes precedence.

* Metric: mostly-minus diag(1, -1, ..., -1) (paper Sec. 2.2) by default;
  ``metric="alternating"`` uses diag(1, -1, 1, -1, ...) in every product
  (the propagators' P_S^2, the vertices' contractions and the root), the
  option paper Sec. 3.1 adds to match Caravel.

Parity: pinned by tests/test_oracle_pins.py -- brute-force Feynman diagrams
with full vertex tensors (``oracle.feynman``), Parke-Taylor for MHV and
anti-MHV, the vanishing helicity configurations, the Ward identity, current
conservation, cyclicity, reflection, U(1) decoupling, multilinearity, scaling
and cross-field agreement.
"""
from __future__ import annotations

from .fields import Fp, mdot, metric_dot

STATUS_OK = 0
STATUS_SINGULAR = 1
STATUS_BAD_RESIDUE = 2

FP_SENTINEL = 0xFFFFFFFF
C_SENTINEL = complex(float("nan"), float("nan"))


def sentinel(F):
    return FP_SENTINEL if isinstance(F, Fp) else C_SENTINEL


def subrange_momenta(F, k, N):
    """P[(i, j)] = k_i + k_{i+1} + ... + k_j, summed left to right (0-based i <= j < N)."""
    d = len(k[0])
    P = {}
    for i in range(N):
        acc = list(k[i])
        P[(i, i)] = acc
        for j in range(i + 1, N):
            acc = [F.add(acc[mu], k[j][mu]) for mu in range(d)]
            P[(i, j)] = acc
    return P


def _kernel_vector(F, J, P, i, j, d, mdot=mdot):
    """K(S) for S = [i..j]: the i-free bracket of the recursion, summed over
    all V3 splits [i..s]|[s+1..j] and all V4 splits [i..s]|[s+1..t]|[t+1..j]
    (``mdot`` is the metric's bilinear product)."""
    K = [F.zero] * d
    # three-gluon vertex, A = [i..s], B = [s+1..j]
    for s in range(i, j):
        JA, JB = J[(i, s)], J[(s + 1, j)]
        PA, PB = P[(i, s)], P[(s + 1, j)]
        ab = mdot(F, JA, JB)
        pb_ja = mdot(F, PB, JA)
        pa_jb = mdot(F, PA, JB)
        two_pb_ja = F.add(pb_ja, pb_ja)
        two_pa_jb = F.add(pa_jb, pa_jb)
        for mu in range(d):
            t = F.mul(ab, F.sub(PA[mu], PB[mu]))
            t = F.add(t, F.mul(two_pb_ja, JB[mu]))
            t = F.sub(t, F.mul(two_pa_jb, JA[mu]))
            K[mu] = F.add(K[mu], t)
    # four-gluon vertex, A = [i..s], B = [s+1..t], C = [t+1..j]
    for s in range(i, j - 1):
        for t in range(s + 1, j):
            JA, JB, JC = J[(i, s)], J[(s + 1, t)], J[(t + 1, j)]
            ac = mdot(F, JA, JC)
            ab = mdot(F, JA, JB)
            bc = mdot(F, JB, JC)
            two_ac = F.add(ac, ac)
            for mu in range(d):
                u = F.mul(two_ac, JB[mu])
                u = F.sub(u, F.mul(ab, JC[mu]))
                u = F.sub(u, F.mul(bc, JA[mu]))
                K[mu] = F.add(K[mu], u)
    return K


def _check_canonical(F, k, eps, n):
    if not isinstance(F, Fp):
        return True
    p = F.p
    for l in range(n):
        vecs = (eps[l],) if l == n - 1 else (k[l], eps[l])
        for v in vecs:
            for x in v:
                if not isinstance(x, int) or x < 0 or x >= p:
                    return False
    return True


def currents(F, k, eps, metric="mostly-minus"):
    """All currents J(S), 1 <= |S| <= N-1, plus K([1..N]).

    Returns (status, J, Kroot) with J keyed by 0-based (i, j).  On a non-zero
    status J and Kroot are None.
    """
    n = len(k)
    if n < 3 or len(eps) != n:
        raise ValueError("need n >= 3 legs with one polarisation per leg")
    d = len(k[0])
    N = n - 1
    dot = metric_dot(metric)
    if not _check_canonical(F, k, eps, n):
        return STATUS_BAD_RESIDUE, None, None
    P = subrange_momenta(F, k, N)
    J = {(l, l): list(eps[l]) for l in range(N)}
    for m in range(2, N):
        for i in range(0, N - m + 1):
            j = i + m - 1
            K = _kernel_vector(F, J, P, i, j, d, dot)
            den = dot(F, P[(i, j)], P[(i, j)])
            if F.is_zero(den):
                return STATUS_SINGULAR, None, None
            inv = F.inv(den)
            J[(i, j)] = [F.mul(x, inv) for x in K]
    Kroot = _kernel_vector(F, J, P, 0, N - 1, d, dot)
    return STATUS_OK, J, Kroot


def amplitude(F, k, eps, metric="mostly-minus"):
    """(status, M) for one phase-space point; M = eps_n . K([1..n-1])."""
    status, _, Kroot = currents(F, k, eps, metric)
    if status != STATUS_OK:
        return status, sentinel(F)
    return STATUS_OK, metric_dot(metric)(F, eps[-1], Kroot)


def amplitudes(F, k_pts, eps_pts, metric="mostly-minus"):
    """Loop of ``amplitude`` over points; returns (status list, value list)."""
    st, out = [], []
    for k, e in zip(k_pts, eps_pts):
        s, m = amplitude(F, k, e, metric)
        st.append(s)
        out.append(m)
    return st, out
