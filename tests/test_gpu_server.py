"""Serving loop: every request's results equal the single-call entry points'
on the same inputs (bit for bit in both fields: same kernels, same per-point
arithmetic), whatever the request was batched with; admission keeps the
arena within its budget; the plain mode gives the same results; argument
errors are reported at submit.  A few points per shape are also checked
against the oracle."""
import numpy as np
import pytest

from paper_2502_07060_amd import bg
from paper_2502_07060_amd import inputs as I

import bgtest
from test_gpu_parity import assert_fp_equal, torch_dev  # noqa: F401

pytestmark = pytest.mark.gpu
P = I.DEFAULT_PRIME


class HostReq:
    """Inputs (pinned host, [n][d][ld]) and output buffers of one request."""

    def __init__(self, torch, field, n, d, m, seed, ld_extra=0):
        self.field, self.n, self.d, self.m = field, n, d, m
        g = dict(field=field, n=n, d=d, npts=m, seed=seed)
        if m:
            self.k, self.e = I.group_inputs(g)
        else:
            dt = np.uint32 if field == "fp" else np.complex128
            self.k = self.e = np.zeros((0, n, d), dt)
        ld = max(m + ld_extra, 1)
        if field == "fp":
            ks = I.to_soa(self.k.astype(np.uint32), ld).view(np.int32)
            es = I.to_soa(self.e.astype(np.uint32), ld).view(np.int32)
            self.out = torch.full((max(m, 1),), -1, dtype=torch.int32).pin_memory()
        else:
            ks = I.to_soa(self.k.astype(np.complex128), ld)
            es = I.to_soa(self.e.astype(np.complex128), ld)
            self.out = torch.full((max(m, 1),), complex(7, 7), dtype=torch.complex128).pin_memory()
        self.tk = torch.from_numpy(ks).pin_memory()
        self.te = torch.from_numpy(es).pin_memory()
        self.st = torch.full((max(m, 1),), 9, dtype=torch.uint8).pin_memory()

    def submit(self, srv):
        return srv.submit(self.tk, self.te, self.out, self.st, p=P, npts=self.m)

    def result(self):
        return self.out[:self.m].numpy().copy(), self.st[:self.m].numpy().copy()

    def direct(self, torch_dev):
        torch, dev = torch_dev
        tk, te = self.tk.to(dev), self.te.to(dev)
        if self.field == "fp":
            o, s = bg.bg_amplitudes_fp(tk, te, P, npts=self.m)
        else:
            o, s = bg.bg_amplitudes_c128(tk, te, npts=self.m)
        torch.cuda.synchronize()
        return o.cpu().numpy(), s.cpu().numpy()


def same_bits(a, b):
    return np.array_equal(np.asarray(a).view(np.uint8), np.asarray(b).view(np.uint8))


def random_requests(torch, count, seed, sizes=(1, 7, 64, 300, 1000), ns=range(4, 15), ds=(4, 6, 10)):
    rng = np.random.default_rng(seed)
    out = []
    for t in range(count):
        field = ("c128", "fp")[rng.integers(2)]
        n = int(rng.choice(list(ns)))
        d = int(rng.choice(ds))
        m = int(rng.choice(sizes))
        if n >= 12:
            m = min(m, 64)   # keeps the oracle samples and the generators quick
        out.append(HostReq(torch, field, n, d, m, seed * 1000 + t, ld_extra=int(rng.integers(0, 3)) * 5))
    return out


def run_all(srv, reqs):
    ids = [r.submit(srv) for r in reqs]
    return [srv.wait(i, timeout=120) for i in ids]


def test_mixed_requests_match_direct_calls_and_oracle(torch_dev):
    torch, _ = torch_dev
    reqs = random_requests(torch, 40, 1) + [HostReq(torch, "fp", 8, 6, 0, 5), HostReq(torch, "c128", 5, 4, 0, 6)]
    with bg.Server(1 << 30) as srv:
        times = run_all(srv, reqs)
        st = srv.stats()
    assert st["completed"] == st["submitted"] == len(reqs)
    assert st["arena_peak"] <= st["arena_bytes"] and st["arena_in_use"] == 0
    assert all(t["done_ns"] >= t["launch_ns"] >= t["submit_ns"] for t in times)
    for r in reqs:
        if r.m == 0:
            continue
        o, s = r.result()
        od, sd = r.direct(torch_dev)
        assert np.array_equal(s, sd) and same_bits(o, od), (r.field, r.n, r.d, r.m)
    rng = np.random.default_rng(2)
    for r in reqs[:12]:
        if r.m == 0:
            continue
        idx = rng.choice(r.m, size=min(3, r.m), replace=False)
        o, s = r.result()
        if r.field == "fp":
            so, vo = bgtest.oracle_fp(r.k[idx].astype(np.int64), r.e[idx].astype(np.int64), P)
            assert_fp_equal(s[idx], o[idx].view(np.uint32).astype(np.int64), so, vo, f"server {r.n},{r.d}")
        else:
            so, vo = bgtest.oracle_c(r.k[idx], r.e[idx])
            assert np.array_equal(s[idx], so)
            bgtest.check_c(o[idx], vo, r.k[idx], r.e[idx], label=f"server {r.n},{r.d}")


def test_alone_equals_in_mix(torch_dev):
    torch, _ = torch_dev
    probes = [HostReq(torch, "fp", 8, 6, 500, 11), HostReq(torch, "c128", 7, 4, 300, 12),
              HostReq(torch, "c128", 11, 10, 40, 13)]
    alone = []
    for x in probes:
        with bg.Server(1 << 28) as srv:
            run_all(srv, [x])
        alone.append(x.result())
        x.out.fill_(0)
        x.st.fill_(9)
    # the same requests among others of the same shapes (so they share launches) and of other shapes
    mix = random_requests(torch, 60, 3)
    same = [HostReq(torch, p.field, p.n, p.d, 200, 900 + t) for t, p in enumerate(probes * 5)]
    order = mix[:20] + same[:5] + [probes[0]] + same[5:10] + [probes[1]] + mix[20:40] + [probes[2]] + same[10:] + mix[40:]
    with bg.Server(1 << 30) as srv:
        times = run_all(srv, order)
    shared = sum(1 for t in times if t["batch_requests"] > 1)
    for x, (o, s) in zip(probes, alone):
        o2, s2 = x.result()
        assert np.array_equal(s, s2) and same_bits(o, o2), (x.field, x.n, x.d)
    print(f"requests that shared a launch: {shared} of {len(order)}")


def test_admission_under_a_small_arena(torch_dev):
    torch, _ = torch_dev
    reqs = random_requests(torch, 30, 4, sizes=(64, 300, 1000), ns=range(4, 10))
    biggest = max(r.m * (2 * r.n * r.d * (16 if r.field == "c128" else 4) + 17) for r in reqs)
    budget = 3 * biggest
    with bg.Server(budget) as srv:
        run_all(srv, reqs)
        st = srv.stats()
        huge = HostReq(torch, "c128", 14, 10, 4000, 7)
        with pytest.raises(bg.BGError) as ei:
            huge.submit(srv)
        assert ei.value.code == bg.BG_ENOMEM
    assert st["arena_peak"] <= st["arena_bytes"] and st["completed"] == len(reqs)
    for r in reqs:
        o, s = r.result()
        od, sd = r.direct(torch_dev)
        assert np.array_equal(s, sd) and same_bits(o, od)


def test_same_shape_requests_share_launches(torch_dev):
    torch, _ = torch_dev
    # a long request first keeps the device busy while the rest queue up
    head = HostReq(torch, "c128", 13, 10, 3000, 20)
    reqs = [head] + [HostReq(torch, "fp", 9, 6, 64, 21 + t) for t in range(40)]
    with bg.Server(1 << 30) as srv:
        run_all(srv, reqs)
        st = srv.stats()
    assert st["batches"] < st["completed"], st
    for r in reqs[1:6]:
        o, s = r.result()
        od, sd = r.direct(torch_dev)
        assert np.array_equal(s, sd) and same_bits(o, od)


def test_plain_mode_gives_the_same_results(torch_dev):
    torch, _ = torch_dev
    reqs = random_requests(torch, 15, 5)
    with bg.Server(1 << 29) as srv:
        run_all(srv, reqs)
    first = [r.result() for r in reqs]
    for r in reqs:
        r.out.zero_()
        r.st.fill_(9)
    with bg.Server(1 << 29, plain=True) as srv:
        times = run_all(srv, reqs)
        st = srv.stats()
    assert st["batches"] == len(reqs) and all(t["batch_requests"] == 1 for t in times)
    for r, (o, s) in zip(reqs, first):
        o2, s2 = r.result()
        assert np.array_equal(s, s2) and same_bits(o, o2)


def test_submit_errors(torch_dev):
    torch, _ = torch_dev
    with bg.Server(1 << 24) as srv:
        r = HostReq(torch, "fp", 6, 4, 10, 30)
        with pytest.raises(bg.BGError) as ei:
            srv.submit(r.tk, r.te, r.out, r.st, p=2147483631)
        assert ei.value.code == bg.BG_ENOTPRIME
        with pytest.raises(bg.BGError) as ei:
            srv.wait(123456789)
        assert ei.value.code == bg.BG_EINVAL
        assert srv.stats()["submitted"] == 0
