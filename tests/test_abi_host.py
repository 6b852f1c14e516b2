"""C-ABI checks that need no GPU: the library loads, exports every symbol that
include/bg.h declares, and rejects bad arguments on the host before any
launch (paper Sec. 3: p < 2^31 prime; n and d within the supported range)."""
import ctypes
import os
import re

import pytest

from paper_2502_07060_amd import bg

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_symbols():
    syms = set()
    for name in os.listdir(os.path.join(ROOT, "include")):
        if name.endswith(".h"):
            text = open(os.path.join(ROOT, "include", name)).read()
            text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
            syms |= set(re.findall(r"\b(bg_[a-z0-9_]+)\s*\(", text))
    return syms


def test_library_exports_every_declared_symbol():
    L = bg.lib()
    syms = declared_symbols()
    assert {"bg_amplitudes_c128", "bg_amplitudes_fp", "bg_strerror", "bg_version"} <= syms
    for s in syms:
        assert hasattr(L, s), s
    assert set(bg._SIGNATURES) >= syms


def test_version_and_strerror():
    assert bg.bg_version() >= 100
    for code in range(-7, 1):
        assert bg.strerror(code) != "unknown error code"
    assert bg.strerror(-99) == "unknown error code"


NULL = ctypes.c_void_p(0)
DUMMY = ctypes.c_void_p(0x1000)   # never dereferenced: every case below fails validation first


def call_fp(n=8, d=6, npts=10, ld=10, p=2147483629, m=DUMMY, e=DUMMY, o=DUMMY):
    return bg.lib().bg_amplitudes_fp(n, d, npts, ld, ctypes.c_uint32(p), m, e, o, NULL, NULL)


def call_c(n=8, d=4, npts=10, ld=10, m=DUMMY, e=DUMMY, o=DUMMY):
    return bg.lib().bg_amplitudes_c128(n, d, npts, ld, m, e, o, NULL, NULL)


@pytest.mark.parametrize("n", [-1, 0, 1, 2, 15, 100])
def test_bad_multiplicity(n):
    assert call_fp(n=n) == bg.BG_EDOMAIN
    assert call_c(n=n) == bg.BG_EDOMAIN


@pytest.mark.parametrize("d", [0, -3, 11, 64])
def test_bad_dimension(d):
    assert call_fp(d=d) == bg.BG_EDOMAIN
    assert call_c(d=d) == bg.BG_EDOMAIN


@pytest.mark.parametrize("p", [0, 1, 2, 4, 9, 2147483631, 2147483648, 4294967291, 2147483649])
def test_bad_prime(p):
    assert call_fp(p=p) == bg.BG_ENOTPRIME


def test_null_pointers_and_ld():
    assert call_fp(m=NULL) == bg.BG_EINVAL
    assert call_fp(e=NULL) == bg.BG_EINVAL
    assert call_fp(o=NULL) == bg.BG_EINVAL
    assert call_fp(ld=9) == bg.BG_EINVAL
    assert call_fp(npts=-1) == bg.BG_EINVAL
    assert call_c(m=NULL) == bg.BG_EINVAL
    assert call_c(ld=3) == bg.BG_EINVAL


def test_zero_points_is_a_noop():
    assert call_fp(npts=0, ld=0, m=NULL, e=NULL, o=NULL) == bg.BG_OK
    assert call_c(npts=0, ld=0, m=NULL, e=NULL, o=NULL) == bg.BG_OK


def test_primality_matches_oracle():
    from oracle.fields import is_prime
    import random
    rng = random.Random(1)
    cands = [rng.randrange(3, 2**31) | 1 for _ in range(300)] + [2147483629, 2147483647, 10007, 3, 5]
    for p in cands:
        rc = call_fp(p=p, npts=0, ld=0)
        assert (rc == bg.BG_OK) == is_prime(p), p


def test_every_built_register_kernel_is_listed():
    """Host-side: each register-resident instantiation in the build list shows
    up in bg_variants for its (field, n) at some d <= 10, with its lanes,
    components per lane and table placement, and no register kernel is listed
    that the build does not compile."""
    from paper_2502_07060_amd import build as B
    want = {}
    for field, N, DL, L, LT, W in B.REGISTER_VARIANTS:
        f = bg.BG_FIELD_FP if field == "fp" else bg.BG_FIELD_C128
        want.setdefault((f, N + 1), set()).add((L, DL, int(LT)))
    for f in (bg.BG_FIELD_C128, bg.BG_FIELD_FP):
        for n in range(3, 15):
            got = set()
            for d in range(1, 11):
                for v in bg.bg_variants(f, n, d):
                    if not v["generic"]:
                        got.add((v["lanes"], v["comps_per_lane"], v["lds_tables"]))
            assert got == want.get((f, n), set()), (f, n)


def test_variant_listing_and_selection():
    """Host-side: every (field, n, d) has at least one variant, one is marked
    selected, pinning and unpinning work, and bad indices are rejected."""
    for field in (bg.BG_FIELD_C128, bg.BG_FIELD_FP):
        for n in range(3, 15):
            for d in range(1, 11):
                vs = bg.bg_variants(field, n, d)
                assert vs, (field, n, d)
                assert sum(v["selected"] for v in vs) == 1
                for v in vs:
                    assert v["lanes"] * v["comps_per_lane"] >= d or v["generic"]
    vs = bg.bg_variants(bg.BG_FIELD_FP, 8, 6)
    last = vs[-1]["index"]
    bg.bg_select_variant(bg.BG_FIELD_FP, 8, 6, last)
    assert [v["selected"] for v in bg.bg_variants(bg.BG_FIELD_FP, 8, 6)][-1] == 1
    bg.bg_select_variant(bg.BG_FIELD_FP, 8, 6, -1)
    with pytest.raises(bg.BGError):
        bg.bg_select_variant(bg.BG_FIELD_FP, 8, 6, 10**6)
    assert bg.lib().bg_variants(7, 8, 6, None, 0) == bg.BG_EINVAL
    assert bg.lib().bg_variants(bg.BG_FIELD_FP, 20, 6, None, 0) == bg.BG_EDOMAIN


def test_server_argument_checks_without_gpu():
    """Server entry points reject bad handles and flags before touching the GPU."""
    L = bg.lib()
    h = ctypes.c_void_p()
    assert L.bg_server_create(0, 0, ctypes.byref(h)) == bg.BG_EINVAL
    assert L.bg_server_create(1 << 20, 2, ctypes.byref(h)) == bg.BG_EINVAL
    assert L.bg_server_create(1 << 20, 0, None) == bg.BG_EINVAL
    rid = ctypes.c_uint64()
    g = bg.bg_group(bg.BG_FIELD_FP, 8, 6, 2147483629, 10, 10, 0x1000, 0x1000, 0x1000, None)
    assert L.bg_server_submit(None, ctypes.byref(g), ctypes.byref(rid)) == bg.BG_EINVAL
    assert L.bg_server_poll(None, 1) == bg.BG_EINVAL
    assert L.bg_server_wait(None, 1, 0.0, None) == bg.BG_EINVAL
    assert L.bg_server_get_stats(None, None) == bg.BG_EINVAL
    assert L.bg_server_destroy(None) == bg.BG_OK
    t0 = bg.bg_server_now_ns()
    assert bg.bg_server_now_ns() >= t0


def test_states_argument_checks():
    """bg_states_*: dimension range, prime and p = 1 (mod 4), pointers."""
    L = bg.lib()
    D = ctypes.c_void_p(0x1000)
    st = lambda d=6, npts=10, ld=10, p=2147483629, m=D, c=D, e=D, t=D: L.bg_states_fp(
        d, npts, ld, ctypes.c_uint32(p), m, c, e, t, NULL, NULL)
    assert st(d=3) == bg.BG_EDOMAIN and st(d=11) == bg.BG_EDOMAIN
    assert st(p=2147483631) == bg.BG_ENOTPRIME
    assert st(p=2147483647) == bg.BG_EDOMAIN        # prime, but 3 mod 4: no sqrt(-1)
    assert st(m=NULL) == bg.BG_EINVAL and st(ld=5) == bg.BG_EINVAL
    assert st(npts=0, ld=0, m=NULL, c=NULL, e=NULL, t=NULL) == bg.BG_OK
    assert L.bg_states_c128(6, 10, 10, NULL, D, D, D, NULL, NULL) == bg.BG_EINVAL
    assert L.bg_states_c128(2, 10, 10, D, D, D, D, NULL, NULL) == bg.BG_EDOMAIN


def test_metric_argument_checks():
    """bg_amplitudes_*_metric: metric tag, p = 1 (mod 4) for the alternating
    metric over Z_p, and the checks of the plain entry points."""
    L = bg.lib()
    D = ctypes.c_void_p(0x1000)
    fp = lambda metric=1, n=5, d=6, npts=10, ld=10, p=2147483629, m=D: L.bg_amplitudes_fp_metric(
        metric, n, d, npts, ld, ctypes.c_uint32(p), m, D, D, NULL, NULL)
    assert fp(metric=2) == bg.BG_EINVAL and fp(metric=-1) == bg.BG_EINVAL
    assert fp(p=2147483647) == bg.BG_EDOMAIN            # prime, but 3 mod 4: no sqrt(-1)
    assert fp(p=2147483631) == bg.BG_ENOTPRIME
    assert fp(n=15) == bg.BG_EDOMAIN and fp(m=NULL) == bg.BG_EINVAL
    assert fp(npts=0, ld=0, m=NULL) == bg.BG_OK
    assert fp(metric=0, p=2147483647, npts=0, ld=0) == bg.BG_OK   # mostly-minus: any odd prime
    c = lambda metric=1, n=5, d=6, npts=10, ld=10, m=D: L.bg_amplitudes_c128_metric(
        metric, n, d, npts, ld, m, D, D, NULL, NULL)
    assert c(metric=7) == bg.BG_EINVAL and c(d=0) == bg.BG_EDOMAIN and c(ld=3) == bg.BG_EINVAL
    assert c(npts=0, ld=0, m=NULL) == bg.BG_OK


def test_rational_argument_checks():
    """bg_fp_from_rational / bg_rational_reconstruct: prime checks, prime
    count, duplicates, pointers; zero points is a no-op."""
    L = bg.lib()
    D = ctypes.c_void_p(0x1000)
    assert L.bg_fp_from_rational(ctypes.c_uint32(2147483631), 4, D, D, D, NULL, NULL) == bg.BG_ENOTPRIME
    assert L.bg_fp_from_rational(ctypes.c_uint32(2147483629), -1, D, D, D, NULL, NULL) == bg.BG_EINVAL
    assert L.bg_fp_from_rational(ctypes.c_uint32(2147483629), 4, NULL, D, D, NULL, NULL) == bg.BG_EINVAL
    assert L.bg_fp_from_rational(ctypes.c_uint32(2147483629), 0, NULL, NULL, NULL, NULL, NULL) == bg.BG_OK

    def rr(primes, npts=10, ld=10, res=D, num=D, den=D):
        arr = (ctypes.c_uint32 * max(len(primes), 1))(*primes)
        return L.bg_rational_reconstruct(len(primes), ctypes.cast(arr, ctypes.c_void_p), npts, ld, res, num, den,
                                         NULL, NULL)
    good = [2147483629, 2147483587]
    assert rr([]) == bg.BG_EINVAL
    assert rr([2147483629] * 33) == bg.BG_EINVAL
    assert rr([2147483629, 2147483629]) == bg.BG_EINVAL          # not distinct
    assert rr([2147483629, 2147483631]) == bg.BG_ENOTPRIME
    assert rr(good, ld=5) == bg.BG_EINVAL and rr(good, res=NULL) == bg.BG_EINVAL
    assert rr(good, npts=0, ld=0, res=NULL, num=NULL, den=NULL) == bg.BG_OK
    assert bg.bg_rr_limbs(1) == 1 and bg.bg_rr_limbs(8) == 5 and bg.bg_rr_limbs(32) == 17


def test_limbs_to_ints():
    import numpy as np
    a = np.array([[0xFFFFFFFF, 5, 0], [0xFFFFFFFF, 0, 1]], dtype=np.uint32)
    assert bg.limbs_to_ints(a, signed=True) == [-1, 5, 1 << 32]
    assert bg.limbs_to_ints(a, signed=False) == [(1 << 64) - 1, 5, 1 << 32]


def test_ffops_argument_checks():
    L = bg.lib()
    D = ctypes.c_void_p(0x1000)
    c = lambda p=2147483629, I=2, J=3, K=4, npts=10, ld=10, x=D, y=D, z=D: L.bg_fp_contract(
        ctypes.c_uint32(p), I, J, K, npts, ld, x, y, 1, z, NULL, NULL)
    assert c(p=2147483631) == bg.BG_ENOTPRIME
    assert c(I=0) == bg.BG_EDOMAIN and c(K=bg.BG_FP_MAX_DIM + 1) == bg.BG_EDOMAIN
    assert c(ld=3) == bg.BG_EINVAL and c(y=NULL) == bg.BG_EINVAL and c(npts=-1) == bg.BG_EINVAL
    assert c(npts=0, ld=0, x=NULL, y=NULL, z=NULL) == bg.BG_OK
    P = ctypes.c_uint32(2147483629)
    assert L.bg_fp_divide(P, 4, D, NULL, D, NULL, NULL) == bg.BG_EINVAL
    assert L.bg_fp_divide(P, 0, NULL, NULL, NULL, NULL, NULL) == bg.BG_OK
    assert L.bg_fp_divide_scalar(P, 4, D, ctypes.c_uint32(0), D, NULL, NULL) == bg.BG_EDOMAIN
    assert L.bg_fp_divide_scalar(P, 4, D, ctypes.c_uint32(2147483629), D, NULL, NULL) == bg.BG_EINVAL


def test_currents_and_state_sum_argument_checks():
    L = bg.lib()
    D = ctypes.c_void_p(0x1000)
    P = ctypes.c_uint32(2147483629)
    assert L.bg_currents_fp(15, 4, 10, 10, P, D, D, D, NULL, NULL) == bg.BG_EDOMAIN
    assert L.bg_currents_fp(5, 4, 10, 10, ctypes.c_uint32(2147483631), D, D, D, NULL, NULL) == bg.BG_ENOTPRIME
    assert L.bg_currents_fp(5, 4, 10, 10, P, D, D, NULL, NULL, NULL) == bg.BG_EINVAL
    assert L.bg_currents_c128(5, 4, 10, 5, D, D, D, NULL, NULL) == bg.BG_EINVAL
    assert L.bg_currents_c128(5, 4, 0, 0, NULL, NULL, NULL, NULL, NULL) == bg.BG_OK
    assert L.bg_state_sum_fp(3, 10, 10, P, D, D, D, D, D, NULL, NULL) == bg.BG_EDOMAIN
    assert L.bg_state_sum_fp(6, 10, 10, ctypes.c_uint32(2147483631), D, D, D, D, D, NULL, NULL) == bg.BG_ENOTPRIME
    assert L.bg_state_sum_c128(6, 10, 10, D, D, NULL, D, D, NULL, NULL) == bg.BG_EINVAL
    assert L.bg_state_sum_c128(6, 0, 0, NULL, NULL, NULL, NULL, NULL, NULL, NULL) == bg.BG_OK


def test_tune_save_and_load_roundtrip(tmp_path):
    """Pins written by bg_tune_save come back with bg_tune_load, including
    the lane-group variants that differ only in padding or in lanes per item."""
    picks = {}
    for field, n, d in ((bg.BG_FIELD_C128, 14, 6), (bg.BG_FIELD_C128, 13, 6), (bg.BG_FIELD_FP, 12, 8),
                        (bg.BG_FIELD_FP, 8, 6)):
        vs = bg.bg_variants(field, n, d)
        # prefer a padded or split lane-group variant when there is one
        pick = next((v for v in vs if v["generic"] and (v["padded"] or v["comps_per_lane"] < 6)), vs[-1])
        bg.bg_select_variant(field, n, d, pick["index"])
        picks[(field, n, d)] = pick["index"]
    # an alternating-metric pin of its own, on another variant
    ALT = bg.BG_METRIC_ALTERNATING
    alt_pick = bg.bg_variants(bg.BG_FIELD_FP, 8, 6)[0]["index"]
    bg.bg_select_variant(bg.BG_FIELD_FP, 8, 6, alt_pick, metric=ALT)
    path, again = str(tmp_path / "tune.txt"), str(tmp_path / "again.txt")
    try:
        bg.bg_tune_save(path)
        lines = [ln.split() for ln in open(path) if not ln.startswith("#")]
        assert sum(ln[-1] == str(ALT) for ln in lines) == 1
        assert sum(ln[-1] == str(bg.BG_METRIC_MOSTLY_MINUS) for ln in lines) >= len(picks)
        for (field, n, d) in picks:
            bg.bg_select_variant(field, n, d, -1)
        bg.bg_select_variant(bg.BG_FIELD_FP, 8, 6, -1, metric=ALT)
        assert bg.bg_tune_load(path) >= len(picks) + 1
        for (field, n, d), idx in picks.items():
            sel = [v["index"] for v in bg.bg_variants(field, n, d) if v["selected"]]
            assert sel == [idx], (field, n, d)
        bg.bg_tune_save(again)  # the alternating pin came back too
        assert open(again).read() == open(path).read()
    finally:
        for (field, n, d) in picks:
            bg.bg_select_variant(field, n, d, -1)
        bg.bg_select_variant(bg.BG_FIELD_FP, 8, 6, -1, metric=ALT)


def test_tune_load_reads_lines_without_metric(tmp_path):
    """A selection line without the metric column pins the mostly-minus metric."""
    v = bg.bg_variants(bg.BG_FIELD_FP, 8, 6)[-1]
    path = tmp_path / "old.txt"
    path.write_text("%d 8 6 %d %d %d %d %d %d\n" % (bg.BG_FIELD_FP, v["lanes"], v["comps_per_lane"],
                                                     v["lds_tables"], v["generic"], v["padded"], v["max_d"]))
    try:
        assert bg.bg_tune_load(str(path)) == 1
        assert [x["index"] for x in bg.bg_variants(bg.BG_FIELD_FP, 8, 6) if x["selected"]] == [v["index"]]
    finally:
        bg.bg_select_variant(bg.BG_FIELD_FP, 8, 6, -1)


def test_failed_autotune_keeps_the_previous_pin():
    """A tuning call that fails (here: synthetic inputs too large to allocate,
    or no GPU at all) leaves a pinned (field, n, d) on its pinned variant and
    an unpinned one on its default."""
    field, n, d = bg.BG_FIELD_FP, 8, 6
    vs = bg.bg_variants(field, n, d)
    default = [v["index"] for v in vs if v["selected"]]
    pick = next(v for v in vs if not v["selected"])
    try:
        bg.bg_select_variant(field, n, d, pick["index"])
        rc = bg.lib().bg_autotune(field, n, d, ctypes.c_uint32(2147483629), 1 << 40, 1, None, 0, None)
        assert rc < 0
        assert [v["index"] for v in bg.bg_variants(field, n, d) if v["selected"]] == [pick["index"]]
        bg.bg_select_variant(field, n, d, -1)
        rc = bg.lib().bg_autotune(field, n, d, ctypes.c_uint32(2147483629), 1 << 40, 1, None, 0, None)
        assert rc < 0
        assert [v["index"] for v in bg.bg_variants(field, n, d) if v["selected"]] == default
    finally:
        bg.bg_select_variant(field, n, d, -1)


def test_metric_selection_and_tuning_arguments():
    """Alternating-metric pins are separate from the mostly-minus ones (which
    bg_variants reports), and the per-metric entry points reject an unknown
    metric and, over Z_p, a prime with no square root of -1, before touching
    the GPU."""
    L = bg.lib()
    field, n, d = bg.BG_FIELD_FP, 8, 6
    vs = bg.bg_variants(field, n, d)
    default = [v["index"] for v in vs if v["selected"]]
    pick = next(v for v in vs if not v["selected"])
    try:
        bg.bg_select_variant(field, n, d, pick["index"], metric=bg.BG_METRIC_ALTERNATING)
        assert [v["index"] for v in bg.bg_variants(field, n, d) if v["selected"]] == default
        bg.bg_select_variant(field, n, d, -1, metric=bg.BG_METRIC_ALTERNATING)
    finally:
        bg.bg_select_variant(field, n, d, -1, metric=bg.BG_METRIC_ALTERNATING)
    assert L.bg_select_variant_metric(7, field, n, d, -1) == bg.BG_EINVAL
    assert L.bg_select_variant_metric(bg.BG_METRIC_ALTERNATING, field, n, d, 10**6) == bg.BG_EINVAL
    assert L.bg_select_variant_metric(bg.BG_METRIC_ALTERNATING, field, 20, d, -1) == bg.BG_EDOMAIN
    p = ctypes.c_uint32(2147483629)
    assert L.bg_autotune_metric(7, field, n, d, p, 1024, 1, None, 0, None) == bg.BG_EINVAL
    # 2^31 - 1 = 3 (mod 4): no square root of -1, so no alternating metric
    assert L.bg_autotune_metric(bg.BG_METRIC_ALTERNATING, field, n, d, ctypes.c_uint32(2**31 - 1), 1024, 1,
                                None, 0, None) == bg.BG_EDOMAIN


def _bad_batch():
    g = bg.bg_group(bg.BG_FIELD_FP, 8, 6, 2147483631, 10, 10, DUMMY.value, DUMMY.value, DUMMY.value, None)
    return (bg.bg_group * 1)(g)


def test_batch_entry_points_validate_on_the_host():
    """The batched calls check flags and every group before any device work
    (the allocation-free one included)."""
    L = bg.lib()
    arr = _bad_batch()
    p = ctypes.cast(arr, ctypes.c_void_p)
    assert L.bg_batch_run_ex(p, 1, 2, NULL) == bg.BG_EINVAL          # unknown flag
    assert L.bg_batch_run_ex(p, 1, bg.BG_BATCH_QUEUE, NULL) == bg.BG_ENOTPRIME
    assert L.bg_batch_run_noalloc(p, 1, NULL) == bg.BG_ENOTPRIME
    assert L.bg_batch_run_noalloc(p, -1, NULL) == bg.BG_EINVAL
    assert L.bg_batch_run_noalloc(NULL, 1, NULL) == bg.BG_EINVAL
    plan = ctypes.c_void_p()
    assert L.bg_batch_plan_create_ex(p, 1, 4, ctypes.byref(plan)) == bg.BG_EINVAL
    assert not plan.value
