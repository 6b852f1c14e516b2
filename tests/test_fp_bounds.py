"""Worst-case int64 bounds of the Z_p kernels' lazy reduction, in exact
Python integers (paper Sec. 3: 64-bit integer arithmetic reduced modulo a
prime p < 2^31 must never overflow).

The kernels keep sums of products of 31-bit residues in int64 accumulators
and reduce them only where the next product could overflow.  Where they fold
or reduce is fixed at compile time.  This file restates, independently of the
device code:

* the three primitives of ``csrc/field_fp.h`` (fold, one 32-bit REDC step,
  two-step REDC) with 64-bit wrap-around emulated bit by bit, checked for
  congruence and for their documented output bounds at the extremes of their
  inputs, for primes that push each bound (p near 2^31, where |v| <= h is
  largest, and primes whose fold constant 2^32 mod p is near +-h);
* the accumulation schedule of every Z_p kernel family (the field policy's
  dot products, the register kernel, the lane-group kernel, the
  one-point-per-lane kernel, the standalone contraction), replayed with the
  largest magnitude each operand can have.  The fold decisions mirror the
  kernels' own (unit counters and fixed positions); the safety check does
  not use those units: every partial sum is bounded exactly and must stay
  inside int64, and every REDC input inside that step's limit.

A kernel whose fold schedule changes must change its replay here.
"""
from __future__ import annotations

import random

import pytest

I64 = 2**63 - 1          # largest int64 magnitude allowed (|x| <= 2^63 - 1)
I32 = 2**31 - 1


def balanced(x, p):
    x %= p
    return x - p if x > (p - 1) // 2 else x


def is_prime(n):
    if n < 2:
        return False
    for q in (2, 3, 5, 7, 11, 13, 17, 19, 23, 29, 31, 37):
        if n % q == 0:
            return n == q
    d, s = n - 1, 0
    while d % 2 == 0:
        d //= 2
        s += 1
    for a in (2, 3, 5, 7, 11, 13, 17):
        x = pow(a, d, n)
        if x in (1, n - 1):
            continue
        for _ in range(s - 1):
            x = x * x % n
            if x == n - 1:
                break
        else:
            return False
    return True


def _prime_near(x, step):
    while not is_prime(x):
        x += step
    return x


def _c32_extreme_prime(sign):
    """The prime p < 2^31 with the balanced 2^32 mod p closest to sign * h.
    For p in (2^32/3, 2^31), 2^32 mod p = 2^32 - 2p, which is near +h when
    p is near 2^32 / 2.5 and near -h (i.e. p/2 + ... mod p) when p is near
    2^32 / 2.5 from the other side of the balanced cut."""
    x = int(2**32 / 2.5)
    best = None
    for p in range(x - 4000, x + 4000):
        if p % 2 == 0 or not is_prime(p):
            continue
        c = balanced(2**32, p)
        h = (p - 1) // 2
        score = abs(c - sign * h)
        if best is None or score < best[0]:
            best = (score, p)
    return best[1]


def _sc_extreme_prime(sign):
    """The prime whose balanced fold constant 2^32 mod p is the largest
    (sign +1) or the most negative (sign -1) value the small-fold-constant
    schedule accepts, |2^32 mod p| <= 2^22.  For p = 2^31 - c (c <= 2^21) the
    constant is 2c; just above 2^32 / 3 it is -(3p - 2^32)."""
    if sign > 0:
        p = 2**31 - 2**21
        while not is_prime(p):
            p += 1
        return p
    p = -(-2**32 // 3) + 2**22 // 3
    while not is_prime(p):
        p -= 1
    return p


def small_fold(p):
    return abs(balanced(2**32, p)) <= 2**22


PRIMES = sorted({
    2**31 - 1,                     # Mersenne: the largest h
    2147483629,                    # 2^31 - 19, the default prime
    _prime_near(2**31 - 10**6, -1),
    _c32_extreme_prime(+1),        # fold constant near +h
    _c32_extreme_prime(-1),        # fold constant near -h
    _prime_near(3 * 2**29 + 1, 2),
    65537, 13, 5, 3,
})


# ---------------------------------------------------------------------------
# the primitives, with int64 / uint32 wrap-around written out
# ---------------------------------------------------------------------------
def s64(x):
    x &= 2**64 - 1
    return x - 2**64 if x >= 2**63 else x


def s32(x):
    x &= 2**32 - 1
    return x - 2**32 if x >= 2**31 else x


class Consts:
    def __init__(self, p):
        self.p = p
        self.h = (p - 1) // 2
        self.pinv = pow(p, -1, 2**32)
        self.negp = -p
        self.c32 = balanced(2**32, p)
        self.c64 = balanced(2**64, p)


def fold(T, k):
    """T = hi 2^32 + lo -> lo + hi c32, formed as (T + hi c32) mod 2^64 with
    hi then subtracted from the high word (as the device code does)."""
    hi = s32(T >> 32)
    r = (T + hi * k.c32) & (2**64 - 1)
    lo_w, hi_w = r & (2**32 - 1), r >> 32
    hi_w = (hi_w - hi) & (2**32 - 1)
    return s64((hi_w << 32) | lo_w)


def redc1(T, k):
    t1 = s32((T & (2**32 - 1)) * k.pinv)
    x = s64(t1 * k.negp + T)
    return s32(x >> 32)


def redc2(T, k):
    t1 = s32((T & (2**32 - 1)) * k.pinv)
    T1 = s32(s64(t1 * k.negp + T) >> 32)
    t2 = s32((T1 & (2**32 - 1)) * k.pinv)
    return s32(s64(t2 * k.negp + T1) >> 32)


def _extreme_int64():
    vals = [0, 1, -1, 2**31, -2**31, 2**32 - 1, 2**32, -2**32, 2**62, -2**62,
            2**63 - 1, -2**63, 2**63 - 2**32, -2**63 + 2**32 - 1]
    return vals


@pytest.mark.parametrize("p", PRIMES)
def test_fold_congruent_and_bounded(p):
    k = Consts(p)
    rng = random.Random(p)
    vals = _extreme_int64() + [rng.randrange(-2**63, 2**63) for _ in range(2000)]
    for T in vals:
        f = fold(T, k)
        hi, lo = T >> 32, T & (2**32 - 1)
        assert f == lo + hi * k.c32                      # no wrap in the result
        assert (f - T) % p == 0
        # documented bound: below 2^31 h + 2^32 for any int64 input
        assert abs(f) < 2**31 * k.h + 2**32
        assert abs(f) < 2**61 + 2**32
    # the second fold of an already folded value: below 2^59 + 2^33
    for T in (2**61 + 2**32 - 1, -(2**61 + 2**32 - 1), 2**61, -2**61):
        f2 = fold(fold(T, k), k) if abs(T) > 2**61 else fold(T, k)
        assert abs(fold(T, k)) < 2**59 + 2**33
        assert (f2 - T) % p == 0


@pytest.mark.parametrize("p", PRIMES)
def test_redc_steps_at_their_input_limits(p):
    k = Consts(p)
    h = k.h
    rng = random.Random(p + 1)
    lim1 = 2**61 + 2**32 - 1       # one 32-bit REDC step
    lim2 = 2**62 - 1               # two-step REDC
    for lim, fn in ((lim1, redc1), (lim2, redc2)):
        vals = [lim, -lim, lim - 1, -(lim - 1), 0, 1, -1]
        vals += [rng.randrange(-lim, lim + 1) for _ in range(3000)]
        # every low word pattern at the limit (t1 takes its extreme values)
        for low in (0, 1, 2**31 - 1, 2**31, 2**32 - 1):
            vals += [(lim & ~(2**32 - 1)) | low, -((lim & ~(2**32 - 1)) | low)]
        for T in vals:
            if abs(T) > lim:
                continue
            r = fn(T, k)
            if fn is redc1:
                assert (r * 2**32 - T) % p == 0
                assert abs(r) < 2**30 + 2**29 + 1      # 1.5 2^30 + 1
            else:
                assert (r * 2**64 - T) % p == 0
                assert abs(r) <= h                     # balanced, no final select
    # REDC2 of products of balanced values (fp_mul) and of a lazily reduced
    # scalar times a balanced value (finish_mul32)
    for a in (h, -h, h - 1, 1, 0):
        for b in (h, -h, 2**30 + 2**29, -(2**30 + 2**29)):
            if abs(b) > h and abs(a) > h:
                continue
            r = redc2(a * b, k)
            assert abs(r) <= h and (r * 2**64 - a * b) % p == 0


# ---------------------------------------------------------------------------
# exact worst-case magnitudes of the primitives' outputs
# ---------------------------------------------------------------------------
class Bounds:
    """Largest magnitudes at prime p; every method checks the limit of the
    step it models before returning the output bound."""

    def __init__(self, p):
        self.k = Consts(p)
        self.p = p
        self.h = self.k.h

    def chk(self, b, what=""):
        assert b <= I64, f"int64 overflow in {what}: {b} > 2^63 - 1"
        return b

    def fold(self, b):
        self.chk(b, "fold input")
        hi = (b >> 32) + 1                  # |hi| for |T| <= b
        return min(2**32 - 1 + hi * abs(self.k.c32), 2**32 - 1 + 2**31 * abs(self.k.c32))

    def redc1(self, b):
        assert b + 2**31 * self.p <= I64, "redc1: T - t1 p overflows"
        assert b < 2**61 + 2**32, "redc1 input above its documented limit"
        return (b + 2**31 * self.p) >> 32

    def redc2(self, b):
        assert b + 2**31 * self.p <= I64, "redc2: T - t1 p overflows"
        assert b < 2**62, "redc2 input above its documented limit"
        T1 = (b + 2**31 * self.p) >> 32
        assert T1 <= I32, "redc2: intermediate is not an int32"
        T2 = (T1 + 2**31 * self.p) >> 32
        assert T2 <= self.h, "redc2 output not balanced"
        return T2


class FieldModel:
    """The dot-product helpers of the Z_p field policy (DL components per
    lane, L lanes per point): where they fold mirrors the unit counter of the
    device code (half-units of 2^59, at most 15); the bound is exact."""

    MAXU = 15

    def __init__(self, B: Bounds, DL, L):
        self.B, self.DL, self.L = B, DL, L
        self.h = B.h

    def acc_dot(self, t, u, bx, by, UX):
        for _ in range(self.DL):
            if u + UX > self.MAXU:
                t, u = self.B.fold(t), 4
            t = self.B.chk(t + bx * by, "acc_dot")
            u += UX
        return t, u

    def finish_dot(self, t, u, lazy):
        L = self.L
        if L > 1:
            if L * u > self.MAXU:
                t, u = self.B.fold(t), 4
                if L * u > self.MAXU:
                    t, u = self.B.fold(t), 2
            t = self.B.chk(L * t, "group sum")
            u *= L
        if lazy:
            if u > 4:
                t = self.B.fold(t)
            return self.B.redc1(t)
        if u > 7:
            t = self.B.fold(t)
        return self.B.redc2(t)

    def ndot(self, bx, by, UX=2, lazy=False):
        t, u = self.acc_dot(0, 0, bx, by, UX)
        return self.finish_dot(t, u, lazy)

    def ndot_sub(self, bx, by, bz, UX=2, UZ=2, lazy=False):
        t, u = self.acc_dot(0, 0, bx, by, UX)
        if u + UZ > self.MAXU:
            t, u = self.B.fold(t), 4
        lift = abs(self.B.k.c32) if UZ == 3 else abs(self.B.k.c64)
        t = self.B.chk(t + bz * lift, "ndot_sub lift")
        return self.finish_dot(t, u + UZ, lazy)

    def ndot_sub2(self, bx, by, bz, bw, UX=2, UZ=2, UW=2, lazy=False):
        """ndot_sub with a second term w, lifted by R (UW = 2) or 2^32 (UW = 3)."""
        t, u = self.acc_dot(0, 0, bx, by, UX)
        if u + UZ > self.MAXU:
            t, u = self.B.fold(t), 4
        lift = abs(self.B.k.c32) if UZ == 3 else abs(self.B.k.c64)
        t = self.B.chk(t + bz * lift, "ndot_sub2 lift z")
        u += UZ
        if u + UW > self.MAXU:
            t, u = self.B.fold(t), 4
        lift = abs(self.B.k.c32) if UW == 3 else abs(self.B.k.c64)
        t = self.B.chk(t + bw * lift, "ndot_sub2 lift w")
        return self.finish_dot(t, u + UW, lazy)


class Vec:
    """An accumulator vector K (every component has the same bound)."""

    def __init__(self, B: Bounds):
        self.B, self.b = B, 0

    def axpy(self, bc, bv):
        self.b = self.B.chk(self.b + bc * bv, "axpy")

    def fold(self):
        self.b = self.B.fold(self.b)


# ---------------------------------------------------------------------------
# register kernel (csrc/bg_kernel.h, Recursion::run, Z_p path)
# ---------------------------------------------------------------------------
def replay_register_kernel(p, N, DL, L):
    B = Bounds(p)
    F = FieldModel(B, DL, L)
    h = B.h
    lazyP = 2 * h             # Q_{j+1} - Q_i, unreduced
    # legs: nc(l) = -(k_l . eps_l), lazily reduced
    nc_leg = F.ndot(h, h, UX=2, lazy=True)
    # propagators: y = -(P.P) from reduced primed P, non-lazy
    F.ndot(h, h, UX=2, lazy=False)
    # batched inversion: products of balanced values, REDC2
    B.redc2(h * h)
    B.redc2(h * 2)            # the factor -2
    nc_cur = nc_leg
    worst = {}
    for j in range(1, N):
        for i in range(j - 1, -1, -1):
            root = i == 0 and j == N - 1
            K = Vec(B)
            nDacc = 0
            for t in range(i, j):
                nDm = F.ndot(h, h, UX=2, lazy=True)                       # ndot_u<lazy>
                ncA = max(nc_leg, nc_cur)
                nc2 = F.ndot_sub(lazyP, h, ncA, UX=4, UZ=3, lazy=True)
                nc3 = F.ndot_sub(lazyP, h, ncA, UX=4, UZ=3, lazy=True)
                K.axpy(nDm, h)        # -nDm * Q_{t+1}
                K.axpy(nc2, h)        # -nc2 * J_B
                K.axpy(nc3, h)        # nc3 * J_A
                K.fold()
                if t > i and (t - i) % 3 == 0:
                    nDacc = B.fold(nDacc)
                nDacc = B.chk(nDacc + nDm * h, "nDacc")   # times the constant 1/2
            nDhS = B.redc2(B.fold(nDacc))
            K.axpy(nDhS, 2 * h)       # times Q_i + Q_{j+1}, unreduced
            K.fold()
            qn = 0
            for s1 in range(i, j - 1):
                for t in range(s1 + 1, j):
                    ne = F.ndot(h, h, UX=2, lazy=True)
                    K.axpy(ne, h)
                    if qn % 3 == 2:
                        K.fold()
                    qn += 1
            K.fold()
            for t in range(i + 1, j):
                K.axpy(h, h)          # nDh (balanced) times J
                if (t - i) % 5 == 4:
                    K.fold()
            K.fold()
            for s1 in range(i, j - 1):
                K.axpy(h, h)
                if (s1 - i) % 5 == 4:
                    K.fold()
            if not root:
                s = B.redc1(B.fold(K.b))              # finish_mul32
                B.redc2(B.chk(s * h, "finish_mul32"))
                nc_cur = max(nc_cur, F.ndot(lazyP, h, UX=4, lazy=True))
            else:
                B.redc2(B.fold(K.b))                  # finish
                F.ndot(h, h, UX=2, lazy=False)        # eps_n . K
            worst[(i, j)] = K.b
    # output fix-up: products of balanced values
    B.redc2(h * h)
    return worst


# ---------------------------------------------------------------------------
# register kernel, small-fold-constant schedule (|2^32 mod p| <= 2^22): units
# of 2^54, an int64 holds 511, a fold leaves 1; the current accumulators are
# folded only when the next product would pass the budget
# ---------------------------------------------------------------------------
class FieldModelSC:
    """The dot-product helpers of FpField<DL, L, true>: fold decisions mirror
    the device code's unit counter; the bound is exact."""

    MAXU = 511
    FOLDU = 1
    LAZYIN = 2
    REDC2IN = 256

    def __init__(self, B: Bounds, DL, L):
        self.B, self.DL, self.L = B, DL, L
        assert small_fold(B.p)

    @staticmethod
    def ux_units(UX):
        return 129 if UX == 4 else 66

    def acc_dot(self, t, u, bx, by, UX):
        for _ in range(self.DL):
            if u + self.ux_units(UX) > self.MAXU:
                t, u = self.B.fold(t), self.FOLDU
            t = self.B.chk(t + bx * by, "acc_dot")
            u += self.ux_units(UX)
        return t, u

    def finish_dot(self, t, u, lazy):
        L = self.L
        if L > 1:
            if L * u > self.MAXU:
                t, u = self.B.fold(t), self.FOLDU
            t = self.B.chk(L * t, "group sum")
            u *= L
        if lazy:
            if u > self.LAZYIN:
                t = self.B.fold(t)
            return self.B.redc1(t)
        if u >= self.REDC2IN:
            t = self.B.fold(t)
        return self.B.redc2(t)

    def ndot(self, bx, by, UX=2, lazy=False):
        t, u = self.acc_dot(0, 0, bx, by, UX)
        return self.finish_dot(t, u, lazy)

    def ndot_sub(self, bx, by, bz, UX=2, UZ=2, lazy=False):
        t, u = self.acc_dot(0, 0, bx, by, UX)
        uz = 1 if UZ == 3 else 64
        if u + uz > self.MAXU:
            t, u = self.B.fold(t), self.FOLDU
        lift = abs(self.B.k.c32) if UZ == 3 else abs(self.B.k.c64)
        t = self.B.chk(t + bz * lift, "ndot_sub lift")
        return self.finish_dot(t, u + uz, lazy)

    def ndot_sub2(self, bx, by, bz, bw, UX=2, UZ=2, lazy=False):
        """ndot_sub with a second, balanced term w lifted by 2^32 mod p."""
        t, u = self.acc_dot(0, 0, bx, by, UX)
        uz = 1 if UZ == 3 else 64
        if u + uz > self.MAXU:
            t, u = self.B.fold(t), self.FOLDU
        lift = abs(self.B.k.c32) if UZ == 3 else abs(self.B.k.c64)
        t = self.B.chk(t + bz * lift, "ndot_sub2 lift z")
        u += uz
        if u + 1 > self.MAXU:
            t, u = self.B.fold(t), self.FOLDU
        t = self.B.chk(t + bw * abs(self.B.k.c32), "ndot_sub2 lift w")
        return self.finish_dot(t, u + 1, lazy)


class TrackedVec(Vec):
    """A current accumulator under the small-fold schedule (kaxpy)."""

    def __init__(self, B: Bounds):
        super().__init__(B)
        self.u = 0

    def kaxpy(self, UP, bc, bv):
        if self.u + UP > FieldModelSC.MAXU:
            self.fold()
            self.u = FieldModelSC.FOLDU
        self.u += UP
        self.axpy(bc, bv)


def replay_register_kernel_sc(p, N, DL, L):
    B = Bounds(p)
    F = FieldModelSC(B, DL, L)
    h = B.h
    nb = h + 2**23             # the bound the unit counts assume for currents and lazy scalars
    lazyP = 2 * h              # Q_{j+1} - Q_i, unreduced
    # legs: nc(l) = -(k_l . eps_l), lazily reduced
    nc = F.ndot(h, h, UX=2, lazy=True)
    assert nc <= nb
    # propagators: P lazily normalised (one product with 2^32 mod p, one
    # 32-bit REDC step), y = -(P.P) reduced by REDC2
    Pn = B.redc1(B.chk(lazyP * abs(B.k.c32), "lazy_norm"))
    assert Pn <= nb
    ybound = F.ndot(Pn, Pn, UX=5, lazy=False)
    # batched inversion in the Montgomery domain of 2^32: mulp = fold and one
    # 32-bit REDC step of a product; factors are y (balanced), the running
    # products, the powers and the plain residue -2
    def mulp(a, b):
        return B.redc1(B.fold(B.chk(a * b, "mulp")))
    v = max(ybound, abs(B.k.c32))
    for _ in range(4):          # the running values' bound reaches its fixed point
        v = max(v, mulp(v, max(v, ybound)), mulp(v, 2))
    inv = v
    assert inv <= nb
    for j in range(1, N):
        for i in range(j - 1, -1, -1):
            root = i == 0 and j == N - 1
            K = TrackedVec(B)
            nDacc, uD = 0, 0
            for t in range(i, j):
                nDm = F.ndot(nb, nb, UX=2, lazy=True)
                # -Dh(A) (t > i) and -Dh(B) (t + 1 < j), balanced, ride in the
                # scalars of the J_B and J_A axpys
                if t > i:
                    nc2 = F.ndot_sub2(lazyP, nb, nc, h, UX=4, UZ=3, lazy=True)
                else:
                    nc2 = F.ndot_sub(lazyP, nb, nc, UX=4, UZ=3, lazy=True)
                if t + 1 < j:
                    nc3 = F.ndot_sub2(lazyP, nb, nc, h, UX=4, UZ=3, lazy=True)
                else:
                    nc3 = F.ndot_sub(lazyP, nb, nc, UX=4, UZ=3, lazy=True)
                assert max(nDm, nc2, nc3) <= nb
                K.kaxpy(66, nDm, h)       # times Q_{t+1} (balanced)
                K.kaxpy(66, nc2, nb)      # times J_B
                K.kaxpy(66, nc3, nb)      # times J_A
                if uD + 66 > FieldModelSC.MAXU:
                    nDacc, uD = B.fold(nDacc), FieldModelSC.FOLDU
                uD += 66
                nDacc = B.chk(nDacc + nDm * h, "nDacc")   # times the constant 1/2
            nDhS = B.redc2(B.fold(nDacc))
            K.kaxpy(128, nDhS, 2 * h)     # times Q_i + Q_{j+1}, unreduced
            for s1 in range(i, j - 1):
                for t in range(s1 + 1, j):
                    ne = F.ndot(nb, nb, UX=2, lazy=True)
                    K.kaxpy(66, ne, nb)
            if not root:
                s = B.redc1(B.fold(K.b))                  # finish_mul32, small fold
                J = B.redc1(B.fold(B.chk(s * inv, "finish product")))
                assert J <= nb
                nc = max(nc, F.ndot(lazyP, nb, UX=4, lazy=True))
                assert nc <= nb
            else:
                B.redc2(B.fold(K.b))                      # finish
                F.ndot(h, h, UX=2, lazy=False)            # eps_n . K
    B.redc2(h * h)


# every register-kernel instantiation of the build list
def _register_variants():
    from paper_2502_07060_amd import build as b
    return sorted({(N, DL, L) for f, N, DL, L, _lt, _w in b.REGISTER_VARIANTS if f == "fp"})


@pytest.mark.parametrize("p", [2**31 - 1, 2147483629, _c32_extreme_prime(+1), _c32_extreme_prime(-1)])
def test_register_kernel_schedule(p):
    variants = _register_variants()
    assert variants, "no Z_p register kernels in the build list"
    for N, DL, L in variants:
        replay_register_kernel(p, N, DL, L)


@pytest.mark.parametrize("p", [2**31 - 1, 2147483629, _sc_extreme_prime(+1), _sc_extreme_prime(-1), 65537, 13])
def test_register_kernel_small_fold_schedule(p):
    assert small_fold(p)
    for N, DL, L in _register_variants():
        replay_register_kernel_sc(p, N, DL, L)


def test_small_fold_replay_catches_a_wider_fold_constant():
    """The small-fold schedule relies on |2^32 mod p| <= 2^22: at a prime whose
    constant is near h the same fold decisions overflow."""
    p = _c32_extreme_prime(+1)
    B = Bounds(p)
    with pytest.raises(AssertionError):
        F = FieldModelSC.__new__(FieldModelSC)
        F.B, F.DL, F.L = B, 6, 1
        h = B.h
        K = TrackedVec(B)
        for _ in range(16):
            K.kaxpy(66, h + 2**23, h + 2**23)
        B.redc1(B.fold(K.b))
        nDm = F.ndot(h, h, UX=2, lazy=True)
        assert nDm <= h + 2**23


def test_register_kernel_replay_catches_a_missing_fold():
    """The replay is able to fail: with the fold after each three-gluon split
    taken out, sums grow past int64 at the longest ranges."""
    B = Bounds(2**31 - 1)
    F = FieldModel(B, 3, 2)
    h = B.h
    K = Vec(B)
    with pytest.raises(AssertionError):
        for _ in range(8):
            nDm = F.ndot(h, h, UX=2, lazy=True)
            nc2 = F.ndot_sub(2 * h, h, nDm, UX=4, UZ=3, lazy=True)
            K.axpy(nDm, h)
            K.axpy(nc2, h)
            K.axpy(nc2, h)


# ---------------------------------------------------------------------------
# lane-group kernel (csrc/bg_wide.h, Z_p path) and one-point-per-lane kernel
# (csrc/bg_generic.h): L = 1 or 2 lanes per item, balanced scalars
# ---------------------------------------------------------------------------
def replay_lane_group_kernel(p, N, DL, LC):
    B = Bounds(p)
    F = FieldModel(B, DL, LC)
    h = B.h
    lazyP = 2 * h
    nc = F.ndot(h, h, UX=2)                       # legs: balanced
    nc = max(nc, F.ndot(lazyP, h, UX=4))          # ranges: ndot<4>, balanced
    F.ndot(h, h)                                  # propagators
    for m in range(2, N + 1):
        pairs = m // 2                            # items per range: a pair of cuts each
        per = 1
        while per < pairs:                        # item slots per range (a power of two)
            per *= 2
        # every item: two three-gluon cuts (the middle item of an odd number
        # of cuts has one; two is the larger bound), then m - 2 splits
        Kp = Vec(B)
        nDs = 0
        for _cut in range(2):
            nDm = F.ndot(h, h)
            # -Dh of the parts (balanced) ride in the scalars, lifted by R
            nc2 = F.ndot_sub2(lazyP, h, nc, h, UX=4)
            nc3 = F.ndot_sub2(lazyP, h, nc, h, UX=4)
            Kp.axpy(nDm, h)
            Kp.axpy(nc2, h)
            Kp.axpy(nc3, h)
            nDs = B.fold(B.chk(nDs + nDm * h, "nDs"))  # folded after every cut
        Kp.fold()                                 # once after the item's cuts
        cnt = 0
        for _q in range(max(0, m - 2)):           # four-gluon splits of the item
            ne = F.ndot(h, h)
            Kp.axpy(ne, h)
            cnt += 1
            if cnt == 5:
                Kp.fold()
                cnt = 0
        Kp.fold()
        # the range's slots add their sums, refolding after every step
        # (add_acc): a butterfly for the root and for nDs, a reduce-scatter
        # with the same per-step sums otherwise; every slot may hold a
        # worst-case sum
        acc, nd = Kp.b, nDs
        s = 1
        while s < per:
            acc = B.fold(B.chk(acc + acc, "butterfly"))
            nd = B.fold(B.chk(nd + nd, "butterfly nDs"))
            s *= 2
        # P_S . J_S of the spread finish: a slot's components (DL at most),
        # folded, added over the slots with a refold per step, then the
        # item's lanes and REDC2
        t, _u = F.acc_dot(0, 0, lazyP, h, UX=4)
        t = B.fold(t)
        s = 1
        while s < per:
            t = B.fold(B.chk(t + t, "P.J over slots"))
            s *= 2
        assert F.finish_dot(t, 4, lazy=False) <= h
        B.redc2(B.fold(nd))
        K = Vec(B)
        K.b = acc
        K.axpy(h, 2 * h)                          # -Dh(S)(Q_i + Q_{j+1})
        K.fold()
        s1 = B.redc1(B.fold(K.b))
        B.redc2(B.chk(s1 * h, "finish_mul32"))
        B.redc2(B.fold(K.b))


def replay_one_point_kernel(p, N, DMAX):
    B = Bounds(p)
    F = FieldModel(B, DMAX, 1)
    h = B.h
    nc = F.ndot(h, h)
    for j in range(1, N):
        for i in range(j - 1, -1, -1):
            K = Vec(B)
            for _t in range(i, j):
                nDm = F.ndot(h, h)
                nc2 = F.ndot_sub(h, h, nc)        # reduced primed P
                nc3 = F.ndot_sub(h, h, nc)
                K.axpy(nDm, h)
                K.axpy(nc2, h)
                K.axpy(nc3, h)
                K.fold()
            K.axpy(h, h)                          # nDh Q_i
            K.axpy(h, h)                          # nDh Q_{j+1}
            K.fold()
            for loop in range(3):
                cnt = 0
                nsplit = {0: (j - i) * (j - i - 1) // 2, 1: j - i - 1, 2: j - i - 1}[loop]
                for _q in range(nsplit):
                    if loop == 0:
                        F.ndot(h, h)
                    K.axpy(h, h)
                    cnt += 1
                    if cnt == 5:
                        K.fold()
                        cnt = 0
                K.fold()
            B.redc2(B.chk(B.redc2(B.fold(K.b)) * h, "mul"))
            nc = max(nc, F.ndot(h, h))


@pytest.mark.parametrize("p", [2**31 - 1, 2147483629, _c32_extreme_prime(+1), _c32_extreme_prime(-1)])
def test_runtime_n_kernel_schedules(p):
    from paper_2502_07060_amd import build as b
    for f, dm, G, _pad, LC in b.WIDE_VARIANTS:
        if f != "fp":
            continue
        for N in range(2, 14):
            replay_lane_group_kernel(p, N, dm // LC, LC)
    for f, dm in b.GENERIC_VARIANTS:
        if f == "fp":
            for N in range(2, 14):
                replay_one_point_kernel(p, N, dm)


# ---------------------------------------------------------------------------
# standalone contraction (csrc/bg_ffops.hip): a fold after every four
# products of balanced values, one REDC2 per output
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("p", [2**31 - 1, _c32_extreme_prime(+1)])
def test_contraction_schedule(p):
    B = Bounds(p)
    h = B.h
    t = 0
    for q in range(4096):
        t = B.chk(t + h * h, "contract")
        if q % 4 == 3:
            t = B.fold(t)
    B.redc2(B.fold(t))


@pytest.mark.parametrize("p", [2**31 - 1, _c32_extreme_prime(+1)])
def test_state_sum_and_residue_schedules(p):
    """csrc/bg_states.hip: two dot products of balanced values with a fold
    after every four products, then a fold per state of the running sum;
    csrc/bg_rational.hip: a uint32 limb times a balanced weight added to a
    folded sum, refolded after every limb."""
    B = Bounds(p)
    h = B.h
    for d in range(1, 11):
        acc = 0
        for _s in range(d - 2 if d > 2 else 1):
            t = 0
            for mu in range(d):
                t = B.chk(t + h * h, "state dot")
                if mu % 4 == 3:
                    t = B.fold(t)
            dl = B.redc2(B.fold(t))
            acc = B.fold(B.chk(acc + dl * dl, "state sum"))
        B.redc2(acc)
    T = 0
    for _k in range(32):
        T = B.fold(B.chk(T + (2**32 - 1) * h, "limb"))
    B.redc2(T)


def test_primes_cover_the_extremes():
    """The prime list reaches each bound: h within 2^-20 of 2^30, and fold
    constants within 1 % of +h and of -h."""
    assert any((p - 1) // 2 > 2**30 - 2**10 for p in PRIMES)
    for sign in (+1, -1):
        p = _c32_extreme_prime(sign)
        h = (p - 1) // 2
        assert abs(balanced(2**32, p) - sign * h) < 0.01 * h
