"""Brute-force colour-ordered Feynman diagrams (test infrastructure only).

An independent pin for ``oracle.bg``: every planar tree diagram with cubic and
quartic vertices on the ordered legs 1..n-1 (leg n at the root) is listed
explicitly and evaluated on its own, with the vertices built as full d^3 and
d^4 tensors, the metric applied explicitly to lower indices, and every factor
of i kept.  Nothing is memoised and no contracted closed form is used, so a
dropped term, a wrong sign, a wrong split enumeration or a transposed operand
in ``oracle.bg`` shows up as a mismatch.

Two three-gluon vertices are available:

* ``"paper"``     -- V3^{mu nu rho}(P, Q) exactly as printed in the paper
  (Sec. 2.2), P the momentum of the left (nu) current, Q of the right (rho)
  current.  Agrees with the recursion for *any* inputs.
* ``"symmetric"`` -- the cyclically symmetric colour-ordered rule
  -i [ g^{nu rho}(q_nu - q_rho)^mu + g^{rho mu}(q_rho - q_mu)^nu
       + g^{mu nu}(q_mu - q_nu)^rho ]
  with q the momenta leaving the vertex along each leg (parent, left, right).
  It differs from the paper's V3 by terms proportional to P_A.J_A and
  P_B.J_B, which vanish for conserved currents, i.e. on physical inputs
  (on-shell momenta, transverse polarisations, momentum conservation).  It
  checks that the paper's simplified vertex is the right physics.

The four-gluon vertex is the printed V4 (already the full colour-ordered
tensor).  Propagators are -i/P^2 (paper Sec. 2.2), the root amplitude is
A = eps_n . T with the off-shell propagator removed.  With the recursion's
M = eps_n . K([1..N]) (``oracle.bg``) the expected relation is A = i M.

The metric is mostly-minus by default; ``metric="alternating"`` builds the
tensors and the propagators from diag(1, -1, 1, -1, ...) instead.

The caller passes the imaginary unit ``I`` of the field: ``1j`` over C, a
square root of -1 mod p over F_p (exists for p = 1 mod 4).

Parity: this module *is* a pin.  Diagram counts 3, 10, 38 for n = 4, 5, 6 are
checked in tests (the planar cubic+quartic tree counts).
"""
from __future__ import annotations

from .fields import metric_dot


def trees(i, j):
    """All planar trees on the ordered leaves i..j (inclusive)."""
    if i == j:
        return [("leaf", i)]
    out = []
    for s in range(i, j):
        for ta in trees(i, s):
            for tb in trees(s + 1, j):
                out.append(("v3", ta, tb))
    for s in range(i, j - 1):
        for t in range(s + 1, j):
            for ta in trees(i, s):
                for tb in trees(s + 1, t):
                    for tc in trees(t + 1, j):
                        out.append(("v4", ta, tb, tc))
    return out


def _metric(F, d, metric="mostly-minus"):
    """g^{mu nu} = g_{mu nu}: diag(1, -1, ..., -1), or diag(1, -1, 1, -1, ...)."""
    g = [[F.zero] * d for _ in range(d)]
    for mu in range(d):
        plus = mu == 0 if metric == "mostly-minus" else mu % 2 == 0
        g[mu][mu] = F.one if plus else F.neg(F.one)
    return g


def _lower(F, g, v):
    d = len(v)
    return [sum_f(F, (F.mul(g[mu][nu], v[nu]) for nu in range(d))) for mu in range(d)]


def sum_f(F, it):
    s = F.zero
    for x in it:
        s = F.add(s, x)
    return s


def _v3_tensor(F, I, g, form, PA, PB):
    """V3^{mu nu rho} as a nested list, legs (parent mu, left nu, right rho)."""
    d = len(PA)
    if form == "paper":
        P, Q = PA, PB
        coup = I
        vec_mu = [F.sub(P[m], Q[m]) for m in range(d)]   # (P - Q)^mu with g^{nu rho}
        vec_nu = [F.add(Q[m], Q[m]) for m in range(d)]   # 2 Q^nu with g^{rho mu}
        vec_rho = [F.neg(F.add(P[m], P[m])) for m in range(d)]  # -2 P^rho with g^{mu nu}
    elif form == "symmetric":
        q_par = [F.add(PA[m], PB[m]) for m in range(d)]
        q_a = [F.neg(x) for x in PA]
        q_b = [F.neg(x) for x in PB]
        coup = F.neg(I)
        vec_mu = [F.sub(q_a[m], q_b[m]) for m in range(d)]
        vec_nu = [F.sub(q_b[m], q_par[m]) for m in range(d)]
        vec_rho = [F.sub(q_par[m], q_a[m]) for m in range(d)]
    else:
        raise ValueError(form)
    V = [[[F.zero] * d for _ in range(d)] for _ in range(d)]
    for mu in range(d):
        for nu in range(d):
            for rho in range(d):
                t = F.mul(g[nu][rho], vec_mu[mu])
                t = F.add(t, F.mul(g[rho][mu], vec_nu[nu]))
                t = F.add(t, F.mul(g[mu][nu], vec_rho[rho]))
                V[mu][nu][rho] = F.mul(coup, t)
    return V


def _v4_tensor(F, I, g, d):
    V = [[[[F.zero] * d for _ in range(d)] for _ in range(d)] for _ in range(d)]
    for mu in range(d):
        for nu in range(d):
            for rho in range(d):
                for sg in range(d):
                    t = F.mul(F.add(F.one, F.one), F.mul(g[mu][rho], g[nu][sg]))
                    t = F.sub(t, F.mul(g[mu][nu], g[rho][sg]))
                    t = F.sub(t, F.mul(g[mu][sg], g[nu][rho]))
                    V[mu][nu][rho][sg] = F.mul(I, t)
    return V


def _eval(F, I, g, V4, form, tree, k, eps, is_root, dot):
    """Returns (T or J vector with upper index, momentum flowing in)."""
    d = len(k[0])
    if tree[0] == "leaf":
        l = tree[1]
        return list(eps[l]), list(k[l])
    kids = [_eval(F, I, g, V4, form, t, k, eps, False, dot) for t in tree[1:]]
    Ps = [c[1] for c in kids]
    low = [_lower(F, g, c[0]) for c in kids]
    P = Ps[0]
    for q in Ps[1:]:
        P = [F.add(a, b) for a, b in zip(P, q)]
    T = [F.zero] * d
    if tree[0] == "v3":
        V = _v3_tensor(F, I, g, form, Ps[0], Ps[1])
        for mu in range(d):
            T[mu] = sum_f(F, (F.mul(V[mu][nu][rho], F.mul(low[0][nu], low[1][rho]))
                              for nu in range(d) for rho in range(d)))
    else:
        for mu in range(d):
            T[mu] = sum_f(F, (F.mul(V4[mu][nu][rho][sg],
                                    F.mul(low[0][nu], F.mul(low[1][rho], low[2][sg])))
                              for nu in range(d) for rho in range(d) for sg in range(d)))
    if is_root:
        return T, P
    prop = F.mul(F.neg(I), F.inv(dot(F, P, P)))
    return [F.mul(prop, x) for x in T], P


def amplitude_diagrams(F, I, k, eps, form="paper", metric="mostly-minus"):
    """A = sum over diagrams of eps_n . T(root); returns (A, number of diagrams)."""
    n = len(k)
    N = n - 1
    d = len(k[0])
    dot = metric_dot(metric)
    g = _metric(F, d, metric)
    V4 = _v4_tensor(F, I, g, d)
    total = F.zero
    diags = trees(0, N - 1)
    for tr in diags:
        T, _ = _eval(F, I, g, V4, form, tr, k, eps, True, dot)
        total = F.add(total, dot(F, eps[n - 1], T))
    return total, len(diags)
