"""GPU parity: the HIP path through the C ABI against the oracle.

F_p results must match bit for bit (values and status); complex128 results
follow the tolerance rule in tests/bgtest.py (relative 1e-11 with a
natural-size floor, exact-rational arbitration).  Inputs are seeded and
synthetic (paper_2502_07060_amd.inputs), physical (on-shell, conserving,
transverse) and deliberately non-physical, so that no kernel shortcut that
relies on transversality or conservation can pass.
"""
import numpy as np
import pytest

from paper_2502_07060_amd import bg
from paper_2502_07060_amd import inputs as I

import bgtest

pytestmark = pytest.mark.gpu
P = I.DEFAULT_PRIME


@pytest.fixture(scope="module")
def torch_dev():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    bg.lib()
    return torch, torch.device("cuda:0")


def gpu_fp(torch_dev, k, e, p, ld=None, pad_value=None, metric=None):
    torch, dev = torch_dev
    npts = len(k)
    ks, es = I.to_soa(k.astype(np.uint32), ld), I.to_soa(e.astype(np.uint32), ld)
    if pad_value is not None and ks.shape[2] > npts:
        ks[:, :, npts:] = pad_value
        es[:, :, npts:] = pad_value
    tk = torch.from_numpy(ks.view(np.int32)).to(dev)
    te = torch.from_numpy(es.view(np.int32)).to(dev)
    out, st = bg.bg_amplitudes_fp(tk, te, p, npts=npts, metric=metric)
    torch.cuda.synchronize()
    return st.cpu().numpy(), out.cpu().numpy().view(np.uint32).astype(np.int64)


def gpu_c(torch_dev, k, e, ld=None, metric=None):
    torch, dev = torch_dev
    tk = torch.from_numpy(I.to_soa(k.astype(np.complex128), ld)).to(dev)
    te = torch.from_numpy(I.to_soa(e.astype(np.complex128), ld)).to(dev)
    out, st = bg.bg_amplitudes_c128(tk, te, npts=len(k), metric=metric)
    torch.cuda.synchronize()
    return st.cpu().numpy(), out.cpu().numpy()


def assert_fp_equal(st_g, v_g, st_o, v_o, label):
    assert np.array_equal(st_g, st_o), f"{label}: status mismatch at {np.nonzero(st_g != st_o)[0][:8]}"
    ok = st_o == 0
    v_o = np.where(ok, v_o, bg.FP_SENTINEL)
    bad = np.nonzero(v_g != v_o)[0]
    assert bad.size == 0, f"{label}: {bad.size} mismatches, first {bad[:8]}: {v_g[bad[:4]]} vs {v_o[bad[:4]]}"


def npts_for(n):
    # several 256-point tiles plus a ragged tail for the register kernels,
    # a few LDS tiles for the runtime-n kernel
    return 600 if n <= 8 else (70 if n <= 11 else 24)


# ----------------------------------------------------------------------------
# every multiplicity and dimension
# ----------------------------------------------------------------------------

@pytest.mark.parametrize("n", list(range(3, 15)))
@pytest.mark.parametrize("d", [3, 4, 5, 6, 8, 10])
def test_fp_shapes_bit_exact(torch_dev, n, d):
    m = npts_for(n)
    k, e = I.generic_fp(1000 * n + d, n, d, m // 2)
    rng = np.random.default_rng(n * 31 + d)
    kr = rng.integers(0, P, size=(m - m // 2, n, d))   # non-physical inputs
    er = rng.integers(0, P, size=(m - m // 2, n, d))
    k = np.concatenate([k.astype(np.int64), kr])
    e = np.concatenate([e.astype(np.int64), er])
    st_g, v_g = gpu_fp(torch_dev, k, e, P)
    st_o, v_o = bgtest.oracle_fp(k, e, P)
    assert_fp_equal(st_g, v_g, st_o, v_o, f"fp n={n} d={d}")


@pytest.mark.parametrize("n", list(range(3, 15)))
@pytest.mark.parametrize("d", [3, 4, 6, 8, 10])
def test_c128_shapes(torch_dev, n, d):
    m = npts_for(n)
    # a real massless 2 -> 1 process does not exist, so n = 3 uses random inputs only
    mphys = m // 2 if n > 3 else 0
    k, e = I.generic_c128(2000 * n + d, n, d, mphys)
    rng = np.random.default_rng(n * 37 + d)
    shape = (m - mphys, n, d)
    kr = rng.standard_normal(shape) + 1j * rng.standard_normal(shape)
    er = rng.standard_normal(shape) + 1j * rng.standard_normal(shape)
    k = np.concatenate([k, kr * 100])
    e = np.concatenate([e, er])
    st_g, v_g = gpu_c(torch_dev, k, e)
    st_o, v_o = bgtest.oracle_c(k, e)
    assert np.array_equal(st_g, st_o)
    bgtest.check_c(v_g, v_o, k, e, label=f"c128 n={n} d={d}")


@pytest.mark.parametrize("n", [4, 5, 6, 7, 8])
def test_c128_helicity_points(torch_dev, n):
    """Spinor-helicity inputs with random helicities, vanishing ones included."""
    k, e, hel = I.random_helicity_c128(300 + n, n, 600)
    st_g, v_g = gpu_c(torch_dev, k, e)
    st_o, v_o = bgtest.oracle_c(k, e)
    assert np.array_equal(st_g, st_o)
    nminus = (hel < 0).sum(axis=1)
    van = (nminus <= 1) | (nminus >= n - 1)      # tree-level zeros in d = 4
    bgtest.check_c(v_g, v_o, k, e, label=f"helicity n={n}", vanishing=van, conditioned_only=True)


# ----------------------------------------------------------------------------
# the benchmark workloads: small case in full, the 2^20-point cases sampled,
# plus properties over every point
# ----------------------------------------------------------------------------

def pt_mhv(k, a=0, b=1):
    lam, _ = I.spinors(k)
    n = k.shape[1]
    den = np.ones(len(k), complex)
    for l in range(n):
        den = den * I.angle(lam[:, l], lam[:, (l + 1) % n])
    return I.angle(lam[:, a], lam[:, b]) ** 4 / den


def test_c5_small_full(torch_dev):
    w = I.config_workload("c5_small")
    k, e = w["k"], w["eps"]
    st_g, v_g = gpu_c(torch_dev, k, e)
    st_o, v_o = bgtest.oracle_c(k, e)
    assert np.all(st_g == 0) and np.array_equal(st_g, st_o)
    bgtest.check_c(v_g, v_o, k, e, label="c5_small", conditioned_only=True)
    ratio = v_g / pt_mhv(k)
    assert np.max(np.abs(ratio - (-1) ** 5 * 4)) < 1e-9      # M / PT = (-1)^n 2^(n-3)


def sample_idx(npts, count, seed):
    rng = np.random.default_rng(seed)
    idx = rng.choice(npts, size=count, replace=False)
    return np.unique(np.concatenate([idx, np.arange(64), np.arange(npts - 64, npts)]))


def test_fp8_d6_full_size(torch_dev):
    w = I.config_workload("fp8_d6")
    k, e = w["k"].astype(np.int64), w["eps"].astype(np.int64)
    st_g, v_g = gpu_fp(torch_dev, k, e, P)
    idx = sample_idx(len(k), 768, 11)
    st_o, v_o = bgtest.oracle_fp(k[idx], e[idx], P)
    assert_fp_equal(st_g[idx], v_g[idx], st_o, v_o, "fp8_d6 sampled")
    # Ward identity on every point: eps_1 -> k_1 gives exactly 0
    e2 = e.copy()
    e2[:, 0, :] = k[:, 0, :]
    st_w, v_w = gpu_fp(torch_dev, k, e2, P)
    ok = st_w == 0
    assert ok.mean() > 0.999
    assert np.all(v_w[ok] == 0)
    # cyclicity on every point
    st_c, v_c = gpu_fp(torch_dev, np.roll(k, 1, axis=1), np.roll(e, 1, axis=1), P)
    both = (st_c == 0) & (st_g == 0)
    assert both.mean() > 0.999 and np.array_equal(v_c[both], v_g[both])


def test_c8_d4_full_size(torch_dev):
    w = I.config_workload("c8_d4")
    k, e, hel = w["k"], w["eps"], w["hel"]
    st_g, v_g = gpu_c(torch_dev, k, e)
    assert np.all(st_g == 0)
    idx = sample_idx(len(k), 768, 12)
    st_o, v_o = bgtest.oracle_c(k[idx], e[idx])
    nminus = (hel < 0).sum(axis=1)
    van = (nminus <= 1) | (nminus >= 7)
    bgtest.check_c(v_g[idx], v_o, k[idx], e[idx], label="c8_d4 sampled", vanishing=van[idx],
                   conditioned_only=True)
    # Parke-Taylor on every MHV point with legs 1, 2 negative
    sel = (nminus == 2) & (hel[:, 0] < 0) & (hel[:, 1] < 0)
    r = v_g[sel] / pt_mhv(k[sel])
    assert sel.sum() > 1000
    assert np.max(np.abs(r - 32)) < 1e-8 * 32
    # vanishing configurations (0, 1, n-1 or n negative helicities): zero
    # within the oracle's rounding-error bound, on a sample of 512 of them
    van = np.nonzero((nminus <= 1) | (nminus >= 7))[0]
    assert van.size > 50000
    pick = np.random.default_rng(13).choice(van, size=512, replace=False)
    ub = bgtest.error_bound_c(k[pick], e[pick])
    assert np.all(np.abs(v_g[pick]) <= 2 * ub)


# ----------------------------------------------------------------------------
# edge cases
# ----------------------------------------------------------------------------

def test_one_point_and_ragged_and_padding(torch_dev):
    for n, d in [(8, 6), (5, 4), (11, 6)]:
        for m in (1, 257, 515):
            k, e = I.generic_fp(5 + m, n, d, m)
            st_g, v_g = gpu_fp(torch_dev, k.astype(np.int64), e.astype(np.int64), P, ld=m + 37,
                               pad_value=0xFFFFFFFF)
            st_o, v_o = bgtest.oracle_fp(k, e, P)
            assert_fp_equal(st_g, v_g, st_o, v_o, f"n={n} m={m}")
    for n in (5, 8):
        k, e = I.generic_c128(9, n, 4, 130)
        st_g, v_g = gpu_c(torch_dev, k, e, ld=133)
        st_o, v_o = bgtest.oracle_c(k, e)
        bgtest.check_c(v_g, v_o, k, e, label="ld")


@pytest.mark.parametrize("p", [3, 5, 13, 97, 10007, 1000000007, 2147483647, 2147483629])
@pytest.mark.parametrize("n,d", [(5, 4), (8, 6), (10, 4)])
def test_primes_and_singular_points(torch_dev, p, n, d):
    rng = np.random.default_rng(p % 1000 + n)
    m = 300 if n <= 8 else 40
    k = rng.integers(0, p, size=(m, n, d))
    e = rng.integers(0, p, size=(m, n, d))
    st_g, v_g = gpu_fp(torch_dev, k, e, p)
    st_o, v_o = bgtest.oracle_fp(k, e, p)
    assert_fp_equal(st_g, v_g, st_o, v_o, f"p={p} n={n}")
    if p <= 13:
        assert (st_o == 1).any()


def test_bad_residues(torch_dev):
    for n, d in [(6, 4), (8, 6), (12, 4)]:
        k, e = I.generic_fp(77, n, d, 40)
        k, e = k.astype(np.int64), e.astype(np.int64)
        e[3, 2, 1] = P
        k[5, 0, 0] = P + 7
        k[7, n - 1, 0] = 0xFFFFFFFF        # k_n is never read: no error
        k[9, 1, 1] = (k[9, 0, 1] * 3) % P  # whatever it does, status must match the oracle
        st_g, v_g = gpu_fp(torch_dev, k, e, P)
        st_o, v_o = bgtest.oracle_fp(k, e, P)
        assert st_g[3] == 2 and st_g[5] == 2 and st_g[7] == 0
        assert_fp_equal(st_g, v_g, st_o, v_o, f"bad residues n={n}")


def test_complex_singular_point(torch_dev):
    k, e = I.generic_c128(3, 6, 4, 8)
    k[2, 0] = np.array([1, 0, 0, 1])
    k[2, 1] = np.array([3, 0, 0, 3])     # P_12^2 = 0 exactly
    st_g, v_g = gpu_c(torch_dev, k, e)
    st_o, v_o = bgtest.oracle_c(k, e)
    assert np.array_equal(st_g, st_o) and st_g[2] == 1 and np.isnan(v_g[2].real)


def test_non_default_stream(torch_dev):
    torch, dev = torch_dev
    k, e = I.generic_fp(8, 7, 6, 1000)
    s = torch.cuda.Stream()
    tk = torch.from_numpy(I.to_soa(k).view(np.int32)).to(dev)
    te = torch.from_numpy(I.to_soa(e).view(np.int32)).to(dev)
    torch.cuda.synchronize()
    with torch.cuda.stream(s):
        out, st = bg.bg_amplitudes_fp(tk, te, P)
    s.synchronize()
    st_o, v_o = bgtest.oracle_fp(k, e, P)
    assert_fp_equal(st.cpu().numpy(), out.cpu().numpy().view(np.uint32).astype(np.int64), st_o, v_o, "stream")
