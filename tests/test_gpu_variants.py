"""Every compiled kernel variant (lanes per point, components per lane,
tables in registers or LDS, runtime-n kernel) against the oracle, for every
multiplicity with a register-resident instantiation: any of them may be
selected by a tuner, so each must be right on its own."""
import numpy as np
import pytest

from paper_2502_07060_amd import bg
from paper_2502_07060_amd import inputs as I

import bgtest
from test_gpu_parity import assert_fp_equal, gpu_c, gpu_fp, torch_dev  # noqa: F401

pytestmark = pytest.mark.gpu
P = I.DEFAULT_PRIME


@pytest.mark.parametrize("n", [3, 4, 5, 6, 7, 8])
@pytest.mark.parametrize("d", [4, 6, 8, 10])
def test_every_fp_variant(torch_dev, n, d):
    m = 150 if n <= 6 else 100
    k, e = I.generic_fp(700 + 10 * n + d, n, d, m)
    rng = np.random.default_rng(n + 100 * d)
    k = np.concatenate([k.astype(np.int64), rng.integers(0, P, size=(m + 7, n, d))])
    e = np.concatenate([e.astype(np.int64), rng.integers(0, P, size=(m + 7, n, d))])
    st_o, v_o = bgtest.oracle_fp(k, e, P)
    try:
        for v in bg.bg_variants(bg.BG_FIELD_FP, n, d):
            bg.bg_select_variant(bg.BG_FIELD_FP, n, d, v["index"])
            st_g, v_g = gpu_fp(torch_dev, k, e, P)
            assert_fp_equal(st_g, v_g, st_o, v_o, f"fp n={n} d={d} variant {v}")
    finally:
        bg.bg_select_variant(bg.BG_FIELD_FP, n, d, -1)


@pytest.mark.parametrize("n", [4, 5, 6, 7, 8])
@pytest.mark.parametrize("d", [4, 6, 8, 10])
def test_every_c128_variant(torch_dev, n, d):
    m = 150 if n <= 6 else 100
    k, e = I.generic_c128(800 + 10 * n + d, n, d, m)
    rng = np.random.default_rng(n + 1000 * d)
    shape = (m + 7, n, d)
    k = np.concatenate([k, 100 * (rng.standard_normal(shape) + 1j * rng.standard_normal(shape))])
    e = np.concatenate([e, rng.standard_normal(shape) + 1j * rng.standard_normal(shape)])
    st_o, v_o = bgtest.oracle_c(k, e)
    try:
        for v in bg.bg_variants(bg.BG_FIELD_C128, n, d):
            bg.bg_select_variant(bg.BG_FIELD_C128, n, d, v["index"])
            st_g, v_g = gpu_c(torch_dev, k, e)
            assert np.array_equal(st_g, st_o)
            bgtest.check_c(v_g, v_o, k, e, label=f"c128 n={n} d={d} variant {v}")
    finally:
        bg.bg_select_variant(bg.BG_FIELD_C128, n, d, -1)


@pytest.mark.parametrize("n", [9, 10, 11, 12, 14])
@pytest.mark.parametrize("d", [4, 6, 10])
def test_every_runtime_n_variant_large_n(torch_dev, n, d):
    """Every variant at n ≥ 9, both fields: the runtime-n kernels (one point
    per lane, or a group of lanes per point) and the register-resident
    kernels compiled for F_p at n = 9..11 and complex at n = 9..12."""
    m = 24 if n <= 11 else 10
    k, e = I.generic_fp(900 + 10 * n + d, n, d, m)
    rng = np.random.default_rng(n + 100 * d + 7)
    k = np.concatenate([k.astype(np.int64), rng.integers(0, P, size=(5, n, d))])
    e = np.concatenate([e.astype(np.int64), rng.integers(0, P, size=(5, n, d))])
    st_o, v_o = bgtest.oracle_fp(k, e, P)
    kc, ec = I.generic_c128(950 + 10 * n + d, n, d, m)
    stc_o, vc_o = bgtest.oracle_c(kc, ec)
    try:
        for v in bg.bg_variants(bg.BG_FIELD_FP, n, d):
            bg.bg_select_variant(bg.BG_FIELD_FP, n, d, v["index"])
            st_g, v_g = gpu_fp(torch_dev, k, e, P)
            assert_fp_equal(st_g, v_g, st_o, v_o, f"fp n={n} d={d} variant {v}")
        for v in bg.bg_variants(bg.BG_FIELD_C128, n, d):
            bg.bg_select_variant(bg.BG_FIELD_C128, n, d, v["index"])
            st_g, v_g = gpu_c(torch_dev, kc, ec)
            assert np.array_equal(st_g, stc_o)
            bgtest.check_c(v_g, vc_o, kc, ec, label=f"c128 n={n} d={d} variant {v}")
    finally:
        bg.bg_select_variant(bg.BG_FIELD_FP, n, d, -1)
        bg.bg_select_variant(bg.BG_FIELD_C128, n, d, -1)
