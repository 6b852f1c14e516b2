"""Shared helpers for the parity tests: batch oracle evaluation and the
complex-path tolerance rule.

Tolerance (complex128).  The bar is relative 1e-11:
    |gpu - oracle| <= 1e-11 |oracle|.
Where FP64 itself cannot deliver that (amplitudes that vanish exactly, such
as tree-level all-plus / one-minus in d = 4, or ill-conditioned points), the
floor is the oracle's own first-order rounding-error bound u * e(M)
(oracle.fields.RunningError, u = 2^-53): a point also passes when
    |gpu - oracle| <= 1e-11 |oracle| + 2 u e(M),
i.e. the GPU value lies within the worst-case rounding of the oracle's own
evaluation order.  A point that still fails is arbitrated by the exact value
of the same binary64 inputs (Gaussian rationals): it passes only if the GPU
value is no further from the exact amplitude than
max(1e-11 |exact|, 4 x the oracle's own error).
"""
from __future__ import annotations

import atexit
import multiprocessing as mp
import os

import numpy as np

from oracle import bg as obg
from oracle import fields

_POOL = None


def _workers():
    return max(1, min(16, os.cpu_count() or 1))


def pool():
    global _POOL
    if _POOL is None:
        _POOL = mp.get_context("fork").Pool(_workers())
        atexit.register(_close_pool)
    return _POOL


def _close_pool():
    global _POOL
    if _POOL is not None:
        _POOL.terminate()
        _POOL.join()
        _POOL = None


MM = "mostly-minus"


def _fp_one(args):
    p, k, e, metric = args
    F = fields.Fp(p)
    return obg.amplitude(F, [[int(x) for x in v] for v in k], [[int(x) for x in v] for v in e], metric)


def _c_one(args):
    k, e, metric = args
    F = fields.Complex128()
    return obg.amplitude(F, [[complex(x) for x in v] for v in k], [[complex(x) for x in v] for v in e], metric)


def _exact_one(args):
    k, e, metric = args
    G = fields.GaussianRationals()
    st, m = obg.amplitude(G, [[G.elem(complex(x)) for x in v] for v in k],
                          [[G.elem(complex(x)) for x in v] for v in e], metric)
    return st, (G.to_complex(m) if st == 0 else complex("nan"))


def oracle_fp(k, e, p, metric=MM):
    """k, e: (npts, n, d) integer arrays -> (status array, value array int64)."""
    jobs = [(p, k[i], e[i], metric) for i in range(len(k))]
    res = pool().map(_fp_one, jobs, chunksize=max(1, len(jobs) // (4 * _workers())))
    st = np.array([r[0] for r in res], np.uint8)
    val = np.array([r[1] for r in res], np.int64)
    return st, val


def oracle_c(k, e, metric=MM):
    jobs = [(k[i], e[i], metric) for i in range(len(k))]
    res = pool().map(_c_one, jobs, chunksize=max(1, len(jobs) // (4 * _workers())))
    st = np.array([r[0] for r in res], np.uint8)
    val = np.array([r[1] for r in res], np.complex128)
    return st, val


def _err_one(args):
    k, e, metric = args
    R = fields.RunningError()
    st, m = obg.amplitude(R, [[R.elem(x) for x in v] for v in k], [[R.elem(x) for x in v] for v in e], metric)
    return m[1] if st == 0 else float("inf")


def error_bound_c(k, e, metric=MM):
    """u * e(M): the oracle's running rounding-error bound per point."""
    jobs = [(k[i], e[i], metric) for i in range(len(k))]
    res = pool().map(_err_one, jobs, chunksize=max(1, len(jobs) // (4 * _workers())))
    return np.array(res) * 2.0 ** -53


def exact_c(k, e, metric=MM):
    jobs = [(k[i], e[i], metric) for i in range(len(k))]
    res = pool().map(_exact_one, jobs, chunksize=1)
    return np.array([r[1] for r in res], np.complex128)


def natural_size(k, e):
    n = k.shape[1]
    scale = np.max(np.abs(k[..., 0]), axis=1)
    return np.prod(np.linalg.norm(e, axis=-1), axis=1) * scale ** (4 - n)


def check_c(gpu, ref, k, e, rel=1e-11, label="", metric=MM, vanishing=None, conditioned_only=False):
    """Apply the tolerance rule; returns the number of points that needed the
    rounding-error floor and the number that needed exact arbitration, and
    prints both (they show in the test log with -s or on failure).

    vanishing: optional mask of points whose amplitude is exactly zero (the
    relative bar cannot hold there, so they always need the floor);
    conditioned_only: a non-vanishing point may pass through the floor only if
    it is ill-conditioned, i.e. the oracle's own worst-case rounding bound
    2 u e(M) reaches a tenth of the relative bar.  Running-error bounds
    overstate the actual error by orders of magnitude, so on a well-conditioned
    point (bound below a tenth of the bar) an error beyond the bar would be a
    fault of the kernel, not rounding."""
    err = np.abs(gpu - ref)
    bad = np.nonzero(~(err <= rel * np.abs(ref)))[0]
    nvan = 0 if vanishing is None else int(np.count_nonzero(vanishing))
    nb_reg = bad.size if vanishing is None else int(np.count_nonzero(~vanishing[bad]))
    nreg = len(gpu) - nvan
    print(f"[tolerance] {label}: {len(gpu)} points, {bad.size} outside the relative bar "
          f"({nb_reg} of {nreg} non-vanishing)", flush=True)
    if conditioned_only and nb_reg:
        reg = bad if vanishing is None else bad[~vanishing[bad]]
        ubr = error_bound_c(k[reg], e[reg], metric)
        well = reg[2 * ubr < 0.1 * rel * np.abs(ref[reg])]
        assert well.size == 0, (
            f"{label}: {well.size} well-conditioned points outside the relative bar, first {well[:5]}, "
            f"err/|ref| {err[well[:5]] / np.abs(ref[well[:5]])}")
    if bad.size == 0:
        return 0, 0
    ub = error_bound_c(k[bad], e[bad], metric)
    still = bad[~(err[bad] <= rel * np.abs(ref[bad]) + 2 * ub)]
    if still.size == 0:
        return bad.size, 0
    print(f"[tolerance] {label}: {still.size} points arbitrated by exact evaluation", flush=True)
    assert still.size <= max(3, len(gpu) // 1000), (
        f"{label}: {still.size} of {len(gpu)} points outside tolerance, first {still[:5]}, "
        f"err {err[still[:5]]}, |ref| {np.abs(ref[still[:5]])}")
    ex = exact_c(k[still], e[still], metric)
    for t, idx in enumerate(still):
        e_gpu = abs(gpu[idx] - ex[t])
        e_orc = abs(ref[idx] - ex[t])
        assert e_gpu <= max(rel * abs(ex[t]), 4 * e_orc), (
            f"{label}: point {idx}: gpu {gpu[idx]} oracle {ref[idx]} exact {ex[t]}")
    return bad.size, still.size
