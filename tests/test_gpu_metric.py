"""Alternating metric diag(1, -1, 1, -1, ...) (paper Sec. 3.1) on the GPU:
bg_amplitudes_*_metric against the oracle computed directly in that metric,
for every kernel variant of a spread of (n, d) (register, lane-group and
one-point-per-lane kernels all load through the same metric map), on
arbitrary inputs and on massless momentum-conserving kinematics generated in
the alternating metric; bit-exact over Z_p, the complex tolerance rule over
C.  The mostly-minus tag through the same entry points reproduces the plain
calls exactly."""
import random

import numpy as np
import pytest

from paper_2502_07060_amd import bg
from paper_2502_07060_amd import inputs as I

import bgtest
from test_gpu_parity import assert_fp_equal, gpu_c, gpu_fp, torch_dev  # noqa: F401
from test_oracle_metric import physical_alt

pytestmark = pytest.mark.gpu
P = I.DEFAULT_PRIME
ALT = bg.BG_METRIC_ALTERNATING


def fp_inputs(n, d, m, seed):
    rng = np.random.default_rng(seed)
    k = rng.integers(0, P, size=(m, n, d))
    e = rng.integers(0, P, size=(m, n, d))
    if n >= 4:  # three massless legs summing to zero are collinear: no physical point
        r = random.Random(seed)
        phys = [physical_alt(r, n, d) for _ in range(4)]
        k = np.concatenate([k, np.array([x[0] for x in phys], np.int64)])
        e = np.concatenate([e, np.array([x[1] for x in phys], np.int64)])
    return k, e


@pytest.mark.parametrize("n,d", [(3, 4), (4, 5), (5, 6), (6, 4), (8, 6), (8, 10), (9, 6), (10, 8), (11, 6), (12, 8), (14, 4)])
def test_fp_every_variant(torch_dev, n, d):
    k, e = fp_inputs(n, d, 60 if n <= 8 else 12, 50 + 10 * n + d)
    st_o, v_o = bgtest.oracle_fp(k, e, P, metric="alternating")
    assert (st_o == 0).all()
    try:
        for v in bg.bg_variants(bg.BG_FIELD_FP, n, d):
            # the alternating metric's own pin: that variant's alternating body runs
            bg.bg_select_variant(bg.BG_FIELD_FP, n, d, v["index"], metric=ALT)
            st_g, v_g = gpu_fp(torch_dev, k, e, P, metric=ALT)
            assert_fp_equal(st_g, v_g, st_o, v_o, f"alt fp n={n} d={d} variant {v}")
    finally:
        bg.bg_select_variant(bg.BG_FIELD_FP, n, d, -1, metric=ALT)
    # unpinned: the mostly-minus choice (two lanes instead of one)
    st_g, v_g = gpu_fp(torch_dev, k, e, P, metric=ALT)
    assert_fp_equal(st_g, v_g, st_o, v_o, f"alt fp n={n} d={d} default")


@pytest.mark.parametrize("n,d", [(4, 4), (5, 6), (8, 4), (8, 7), (9, 4), (10, 6), (11, 4), (14, 10)])
def test_c128_every_variant(torch_dev, n, d):
    m = 60 if n <= 8 else 10
    rng = np.random.default_rng(900 + 10 * n + d)
    shape = (m, n, d)
    k = 100 * (rng.standard_normal(shape) + 1j * rng.standard_normal(shape))
    e = rng.standard_normal(shape) + 1j * rng.standard_normal(shape)
    st_o, v_o = bgtest.oracle_c(k, e, metric="alternating")
    try:
        for v in bg.bg_variants(bg.BG_FIELD_C128, n, d):
            bg.bg_select_variant(bg.BG_FIELD_C128, n, d, v["index"], metric=ALT)
            st_g, v_g = gpu_c(torch_dev, k, e, metric=ALT)
            assert np.array_equal(st_g, st_o)
            bgtest.check_c(v_g, v_o, k, e, label=f"alt c128 n={n} d={d} variant {v}", metric="alternating")
    finally:
        bg.bg_select_variant(bg.BG_FIELD_C128, n, d, -1, metric=ALT)


def test_mostly_minus_tag_matches_plain_calls(torch_dev):
    n, d = 7, 6
    k, e = fp_inputs(n, d, 100, 3)
    st1, v1 = gpu_fp(torch_dev, k, e, P)
    st2, v2 = gpu_fp(torch_dev, k, e, P, metric=bg.BG_METRIC_MOSTLY_MINUS)
    assert np.array_equal(st1, st2) and np.array_equal(v1, v2)
    kc, ec = I.generic_c128(4, n, d, 50)
    s1, c1 = gpu_c(torch_dev, kc, ec)
    s2, c2 = gpu_c(torch_dev, kc, ec, metric=bg.BG_METRIC_MOSTLY_MINUS)
    assert np.array_equal(s1, s2) and np.array_equal(c1.view(np.uint64), c2.view(np.uint64))
    # and the alternating metric really differs on these inputs
    s3, v3 = gpu_fp(torch_dev, k, e, P, metric=ALT)
    assert (v3 != v1).mean() > 0.9


def test_alternating_statuses(torch_dev):
    """Bad residues and singular propagators are reported as in the plain call."""
    n, d = 6, 6
    k, e = fp_inputs(n, d, 20, 9)
    k[3, 1, 2] = P + 5                       # a residue >= p
    k[5, 0] = 0                              # k_1 = k_2 = 0: P_{12} = 0, so P_{12}^2 = 0
    k[5, 1] = 0
    st_o, v_o = bgtest.oracle_fp(k, e, P, metric="alternating")
    assert st_o[3] == 2 and st_o[5] == 1
    st_g, v_g = gpu_fp(torch_dev, k, e, P, metric=ALT)
    assert_fp_equal(st_g, v_g, st_o, v_o, "alt statuses")


def test_alternating_autotune_pins_its_own_variant(torch_dev):
    """bg_autotune_metric in the alternating metric pins a variant for that
    metric only: the mostly-minus selection is untouched, and both metrics
    still match the oracle."""
    n, d = 8, 10
    field = bg.BG_FIELD_FP
    k, e = fp_inputs(n, d, 40, 77)
    before = [v["index"] for v in bg.bg_variants(field, n, d) if v["selected"]]
    try:
        chosen, timed = bg.bg_autotune(field, n, d, P, npts=1 << 14, reps=2, metric=ALT)
        assert chosen in [v["index"] for v, _ in timed] and all(ms > 0 for _, ms in timed)
        assert [v["index"] for v in bg.bg_variants(field, n, d) if v["selected"]] == before
        st_o, v_o = bgtest.oracle_fp(k, e, P, metric="alternating")
        st_g, v_g = gpu_fp(torch_dev, k, e, P, metric=ALT)
        assert_fp_equal(st_g, v_g, st_o, v_o, "alt after tuning")
        st_m, v_m = bgtest.oracle_fp(k, e, P)
        st_h, v_h = gpu_fp(torch_dev, k, e, P)
        assert_fp_equal(st_h, v_h, st_m, v_m, "mostly-minus after alt tuning")
    finally:
        bg.bg_select_variant(field, n, d, -1, metric=ALT)
