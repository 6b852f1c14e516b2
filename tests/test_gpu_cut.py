"""Root currents and sums over the states of a cut leg on the GPU (rest of
next row f1): bg_currents_* against the oracle's K([1..n-1]) for every
kernel variant (register, lane-group and one-point-per-lane kernels all have
the root-current mode), consistency eps_n . K = M with the amplitude entry
point, statuses; bg_state_sum_* against the oracle's state sum; and the
whole cut -- states of the cut leg, the two trees' root currents, the state
sum -- against sum_s M_L(e_s) M_R(e~_s) from the amplitude oracle."""
import numpy as np
import pytest

from oracle import bg as obg
from oracle import fields
from oracle import states as S
from paper_2502_07060_amd import bg
from paper_2502_07060_amd import inputs as I

from test_gpu_parity import torch_dev  # noqa: F401
from test_gpu_states import fp_points, gpu_fp_states

pytestmark = pytest.mark.gpu
P = I.DEFAULT_PRIME
U = 2.0 ** -53


def soa(torch_dev, a, dtype=np.uint32):
    torch, dev = torch_dev
    arr = I.to_soa(a.astype(dtype))
    return torch.from_numpy(arr.view(np.int32) if dtype == np.uint32 else arr).to(dev)


def oracle_fp_currents(k, e, p=P):
    F = fields.Fp(p)
    out = []
    for q in range(len(k)):
        st, _, K = obg.currents(F, [[int(x) for x in v] for v in k[q]], [[int(x) for x in v] for v in e[q]])
        out.append((st, K))
    return out


@pytest.mark.parametrize("n,d", [(3, 4), (4, 6), (6, 5), (8, 6), (8, 10), (9, 6), (10, 6), (11, 8), (12, 4), (14, 8)])
def test_currents_fp_every_variant(torch_dev, n, d):
    torch, _ = torch_dev
    m = 40 if n <= 8 else 10
    k, e = I.generic_fp(300 + 10 * n + d, n, d, m)
    rng = np.random.default_rng(n + d)
    k = np.concatenate([k.astype(np.int64), rng.integers(0, P, size=(6, n, d))])
    e = np.concatenate([e.astype(np.int64), rng.integers(0, P, size=(6, n, d))])
    e[2, 0, 1] = P + 3                                   # a bad residue
    ref = oracle_fp_currents(k, e)
    tk, te = soa(torch_dev, k), soa(torch_dev, e)
    try:
        for v in bg.bg_variants(bg.BG_FIELD_FP, n, d):
            bg.bg_select_variant(bg.BG_FIELD_FP, n, d, v["index"])
            cur, st = bg.bg_currents_fp(tk, te, P)
            amp, st2 = bg.bg_amplitudes_fp(tk, te, P)
            torch.cuda.synchronize()
            cur = cur.cpu().numpy().view(np.uint32).astype(np.int64)
            st, amp = st.cpu().numpy(), amp.cpu().numpy().view(np.uint32).astype(np.int64)
            assert np.array_equal(st, st2.cpu().numpy())
            for q, (so, K) in enumerate(ref):
                assert st[q] == so, (v, q)
                if so:
                    assert (cur[:, q] == 0xFFFFFFFF).all()
                    continue
                assert [int(x) for x in cur[:, q]] == K, (n, d, v, q)
                en = e[q, n - 1]
                m_from_k = (int(en[0]) * K[0] - sum(int(en[mu]) * K[mu] for mu in range(1, d))) % P
                assert amp[q] == m_from_k
    finally:
        bg.bg_select_variant(bg.BG_FIELD_FP, n, d, -1)


@pytest.mark.parametrize("n,d", [(4, 4), (6, 6), (8, 4), (9, 4), (10, 6), (11, 4), (11, 7), (12, 4), (14, 10)])
def test_currents_c128_every_variant(torch_dev, n, d):
    torch, _ = torch_dev
    m = 30 if n <= 8 else 6
    k, e = I.generic_c128(400 + 10 * n + d, n, d, m)
    R = fields.RunningError()
    ref = []
    for q in range(m):
        st, _, K = obg.currents(R, [[R.elem(complex(x)) for x in v] for v in k[q]],
                                [[R.elem(complex(x)) for x in v] for v in e[q]])
        ref.append((st, K))
    tk, te = soa(torch_dev, k, np.complex128), soa(torch_dev, e, np.complex128)
    try:
        for v in bg.bg_variants(bg.BG_FIELD_C128, n, d):
            bg.bg_select_variant(bg.BG_FIELD_C128, n, d, v["index"])
            cur, st = bg.bg_currents_c128(tk, te)
            torch.cuda.synchronize()
            cur, st = cur.cpu().numpy(), st.cpu().numpy()
            for q, (so, K) in enumerate(ref):
                assert st[q] == so
                vals = np.array([x[0] for x in K])
                errs = np.array([x[1] for x in K])
                scale = np.abs(vals).max()
                # the oracle's own rounding-error bound per component (the GPU
                # sums in another order), plus 1e-11 of the current's size
                assert (np.abs(cur[:, q] - vals) <= 1e-11 * scale + 4 * U * errs).all(), (n, d, v, q)
    finally:
        bg.bg_select_variant(bg.BG_FIELD_C128, n, d, -1)


@pytest.mark.parametrize("d", [4, 6, 10])
def test_state_sum_fp_against_oracle(torch_dev, d):
    torch, dev = torch_dev
    m = 64
    l, chi = fp_points(70 + d, m, d)
    eps, epst, st = gpu_fp_states(torch_dev, l, chi)
    assert (st == 0).all()
    rng = np.random.default_rng(d)
    KL = rng.integers(0, P, size=(d, m))
    KR = rng.integers(0, P, size=(d, m))
    KL[0, 5] = 0xFFFFFFFF                                  # a sentinel input
    T = lambda a: torch.from_numpy(np.ascontiguousarray(a.astype(np.uint32)).view(np.int32)).to(dev)
    out, sst = bg.bg_state_sum(T(KL), T(KR), T(eps), T(epst), p=P)
    torch.cuda.synchronize()
    out, sst = out.cpu().numpy().view(np.uint32), sst.cpu().numpy()
    F = fields.Fp(P)
    for q in range(m):
        if q == 5:
            assert sst[q] == 2 and out[q] == 0xFFFFFFFF
            continue
        e = [[int(x) for x in eps[s, :, q]] for s in range(d - 2)]
        et = [[int(x) for x in epst[s, :, q]] for s in range(d - 2)]
        want = S.state_sum(F, [int(x) for x in KL[:, q]], [int(x) for x in KR[:, q]], e, et)
        assert sst[q] == 0 and out[q] == want, q


def test_state_sum_c128_against_oracle(torch_dev):
    torch, dev = torch_dev
    d, m = 6, 50
    rng = np.random.default_rng(3)
    c = lambda *s: rng.standard_normal(s) + 1j * rng.standard_normal(s)
    KL, KR, eps, epst = c(d, m), c(d, m), c(d - 2, d, m), c(d - 2, d, m)
    T = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)
    out, st = bg.bg_state_sum(T(KL), T(KR), T(eps), T(epst))
    torch.cuda.synchronize()
    out = out.cpu().numpy()
    C = fields.Complex128()
    for q in range(m):
        want = S.state_sum(C, list(KL[:, q]), list(KR[:, q]), [list(eps[s, :, q]) for s in range(d - 2)],
                           [list(epst[s, :, q]) for s in range(d - 2)])
        assert abs(out[q] - want) <= 1e-13 * (1 + abs(want)) * d * d


@pytest.mark.parametrize("nl,nr,d", [(4, 4, 4), (5, 4, 6), (4, 6, 5), (9, 4, 6)])
def test_cut_end_to_end_fp(torch_dev, nl, nr, d):
    """States of the cut leg l, root currents of L(.., l) and R(.., -l), state
    sum -- all on the GPU -- equal sum_s M_L(e_s) M_R(e~_s) (amplitude oracle
    with the states as the last leg's polarisation)."""
    torch, dev = torch_dev
    m = 24
    rng = np.random.default_rng(nl * 100 + nr * 10 + d)
    l, chi = fp_points(900 + d, m, d)
    kL = rng.integers(0, P, size=(m, nl, d))
    kR = rng.integers(0, P, size=(m, nr, d))
    kL[:, nl - 1] = l
    kR[:, nr - 1] = (-l) % P
    eL = rng.integers(0, P, size=(m, nl, d))
    eR = rng.integers(0, P, size=(m, nr, d))
    eps, epst, st = gpu_fp_states(torch_dev, l, chi)
    assert (st == 0).all()
    KL, s1 = bg.bg_currents_fp(soa(torch_dev, kL), soa(torch_dev, eL), P)
    KR, s2 = bg.bg_currents_fp(soa(torch_dev, kR), soa(torch_dev, eR), P)
    T = lambda a: torch.from_numpy(np.ascontiguousarray(a.astype(np.uint32)).view(np.int32)).to(dev)
    out, sst = bg.bg_state_sum(KL, KR, T(eps), T(epst), p=P)
    torch.cuda.synchronize()
    out, sst = out.cpu().numpy().view(np.uint32), sst.cpu().numpy()
    F = fields.Fp(P)
    for q in range(m):
        total = 0
        for s in range(d - 2):
            e = [int(x) for x in eps[s, :, q]]
            et = [int(x) for x in epst[s, :, q]]
            a1 = obg.amplitude(F, [[int(x) for x in v] for v in kL[q]],
                               [[int(x) for x in v] for v in eL[q, :nl - 1]] + [e])
            a2 = obg.amplitude(F, [[int(x) for x in v] for v in kR[q]],
                               [[int(x) for x in v] for v in eR[q, :nr - 1]] + [et])
            assert a1[0] == 0 and a2[0] == 0
            total = (total + a1[1] * a2[1]) % P
        assert sst[q] == 0 and out[q] == total, q
