"""Batched form: one call over mixed (field, n, d) groups gives, group by
group, exactly what the single-group entry points give (same kernels, so
bit-identical in both fields), and the oracle's values; recorded plans
(hipGraph) give the same on every replay; an invalid group rejects the
whole batch before anything runs.  The queue form (persistent lane-group
launches over a device work queue) is held to the same bar."""
import numpy as np
import pytest

from paper_2502_07060_amd import bg
from paper_2502_07060_amd import inputs as I

import bgtest
from test_gpu_parity import assert_fp_equal, torch_dev  # noqa: F401

pytestmark = pytest.mark.gpu
P = I.DEFAULT_PRIME

SHAPES = [("fp", 4, 4, 300), ("fp", 8, 6, 700), ("fp", 11, 8, 40), ("fp", 14, 10, 9),
          ("c128", 5, 4, 500), ("c128", 8, 4, 600), ("c128", 10, 6, 50), ("c128", 13, 10, 7),
          ("fp", 6, 5, 0), ("c128", 7, 8, 130)]


# lane-group (runtime-n) groups of several tiles each, two of them sharing a
# kernel variant (one persistent launch serves both), mixed with register ones
QSHAPES = [("fp", 12, 8, 150), ("fp", 13, 8, 61), ("c128", 12, 6, 90), ("c128", 14, 4, 37),
           ("fp", 8, 6, 700), ("c128", 8, 4, 300), ("fp", 14, 10, 9), ("c128", 5, 4, 0)]


def make_groups(torch_dev, shapes=SHAPES):
    torch, dev = torch_dev
    groups, data = [], []
    for t, (field, n, d, m) in enumerate(shapes):
        g = dict(field=field, n=n, d=d, npts=m, seed=900 + t)
        k, e = I.group_inputs(g) if m else (np.zeros((0, n, d), np.uint32 if field == "fp" else complex),) * 2
        if field == "fp":
            tk = torch.from_numpy(I.to_soa(k.astype(np.uint32), max(m, 1)).view(np.int32)).to(dev)
            te = torch.from_numpy(I.to_soa(e.astype(np.uint32), max(m, 1)).view(np.int32)).to(dev)
            out = torch.full((max(m, 1),), -1, dtype=torch.int32, device=dev)
        else:
            tk = torch.from_numpy(I.to_soa(k.astype(complex), max(m, 1))).to(dev)
            te = torch.from_numpy(I.to_soa(e.astype(complex), max(m, 1))).to(dev)
            out = torch.full((max(m, 1),), complex(7, 7), dtype=torch.complex128, device=dev)
        st = torch.full((max(m, 1),), 9, dtype=torch.uint8, device=dev)
        groups.append(bg.make_group(tk, te, out, st, p=P, npts=m))
        data.append(dict(field=field, n=n, d=d, m=m, k=k, e=e, tk=tk, te=te, out=out, st=st))
    return groups, data


def single_call(x):
    if x["field"] == "fp":
        o, s = bg.bg_amplitudes_fp(x["tk"], x["te"], P, npts=x["m"])
    else:
        o, s = bg.bg_amplitudes_c128(x["tk"], x["te"], npts=x["m"])
    return o, s


def check_against_single_and_oracle(torch_dev, data, with_oracle):
    torch, _ = torch_dev
    torch.cuda.synchronize()
    for x in data:
        if x["m"] == 0:
            continue
        o1, s1 = single_call(x)
        torch.cuda.synchronize()
        ob, sb = x["out"][:x["m"]].cpu().numpy(), x["st"][:x["m"]].cpu().numpy()
        assert np.array_equal(sb, s1.cpu().numpy())
        if x["field"] == "fp":
            assert np.array_equal(ob, o1.cpu().numpy())
        else:
            a, b = ob, o1.cpu().numpy()
            assert np.array_equal(a.view(np.uint64), b.view(np.uint64)), "complex batch differs from single call"
        if with_oracle:
            if x["field"] == "fp":
                st_o, v_o = bgtest.oracle_fp(x["k"].astype(np.int64), x["e"].astype(np.int64), P)
                assert_fp_equal(sb, ob.view(np.uint32).astype(np.int64), st_o, v_o, f"batch {x['n']},{x['d']}")
            else:
                st_o, v_o = bgtest.oracle_c(x["k"], x["e"])
                assert np.array_equal(sb, st_o)
                bgtest.check_c(ob, v_o, x["k"], x["e"], label=f"batch {x['n']},{x['d']}")


def test_batch_run_matches_single_calls_and_oracle(torch_dev):
    groups, data = make_groups(torch_dev)
    bg.bg_batch_run(groups)
    check_against_single_and_oracle(torch_dev, data, with_oracle=True)


def test_plan_replays(torch_dev):
    torch, _ = torch_dev
    groups, data = make_groups(torch_dev)
    plan = bg.BatchPlan(groups)
    try:
        for rep in range(3):
            for x in data:                  # eager work between replays: poison the outputs
                x["out"].fill_(-1 if x["field"] == "fp" else complex(7, 7))
                x["st"].fill_(9)
            torch.cuda.synchronize()
            plan.launch()
            check_against_single_and_oracle(torch_dev, data, with_oracle=(rep == 0))
    finally:
        plan.close()


def test_queue_form_matches_single_calls_and_oracle(torch_dev):
    groups, data = make_groups(torch_dev, QSHAPES)
    bg.bg_batch_run_ex(groups, bg.BG_BATCH_QUEUE)
    check_against_single_and_oracle(torch_dev, data, with_oracle=True)
    # and the small shapes (one lane-group group per variant, few points)
    groups, data = make_groups(torch_dev)
    bg.bg_batch_run_ex(groups, bg.BG_BATCH_QUEUE)
    check_against_single_and_oracle(torch_dev, data, with_oracle=False)


def test_queue_plan_replays(torch_dev):
    torch, _ = torch_dev
    groups, data = make_groups(torch_dev, QSHAPES)
    plan = bg.BatchPlan(groups, bg.BG_BATCH_QUEUE)
    try:
        for rep in range(3):
            for x in data:                  # eager work between replays: poison the outputs
                x["out"].fill_(-1 if x["field"] == "fp" else complex(7, 7))
                x["st"].fill_(9)
            torch.cuda.synchronize()
            plan.launch()
            check_against_single_and_oracle(torch_dev, data, with_oracle=False)
    finally:
        plan.close()


def test_queue_form_rejects_unknown_flags(torch_dev):
    groups, _ = make_groups(torch_dev)
    with pytest.raises(bg.BGError) as ei:
        bg.bg_batch_run_ex(groups, 2)
    assert ei.value.code == bg.BG_EINVAL


def test_invalid_group_rejects_whole_batch(torch_dev):
    torch, _ = torch_dev
    groups, data = make_groups(torch_dev)
    bad = list(groups)
    bad[3] = bg.bg_group(bg.BG_FIELD_FP, groups[3].n, groups[3].d, 2147483631, groups[3].npts, groups[3].ld,
                         groups[3].momenta, groups[3].pols, groups[3].out, groups[3].status)
    with pytest.raises(bg.BGError) as ei:
        bg.bg_batch_run(bad)
    assert ei.value.code == bg.BG_ENOTPRIME
    torch.cuda.synchronize()
    assert (data[0]["st"] == 9).all()          # nothing ran
    bg.bg_batch_run([])                        # empty batch is fine


@pytest.mark.parametrize("flags", [0, bg.BG_BATCH_QUEUE])
def test_full_batched_workload_sampled(torch_dev, flags):
    """The measured batched workload itself (88 groups, 4*10^6 points, the
    bench's launch configuration after autotuning), as a graph of per-group
    launches and in the queue form: two sampled points per group against the
    oracle, and no status other than OK."""
    import multiprocessing as mp
    from concurrent.futures import ProcessPoolExecutor

    import bench
    torch, dev = torch_dev
    groups = [g for g in I.batched_groups() if g["npts"] > 0]
    with ProcessPoolExecutor(max_workers=bench._gen_workers(), mp_context=mp.get_context("spawn")) as ex:
        soa = list(ex.map(bench._gen_group_soa, groups))
    descs, keep = [], []
    for g, (ks, es) in zip(groups, soa):
        field = bg.BG_FIELD_FP if g["field"] == "fp" else bg.BG_FIELD_C128
        bg.bg_autotune(field, g["n"], g["d"], P if g["field"] == "fp" else 0,
                       npts=min(max(g["npts"], 4096), 1 << 18), reps=1)
        if g["field"] == "fp":
            tk = torch.from_numpy(ks.view(np.int32)).to(dev)
            te = torch.from_numpy(es.view(np.int32)).to(dev)
            out = torch.empty(g["npts"], dtype=torch.int32, device=dev)
        else:
            tk = torch.from_numpy(ks).to(dev)
            te = torch.from_numpy(es).to(dev)
            out = torch.empty(g["npts"], dtype=torch.complex128, device=dev)
        st = torch.full((g["npts"],), 9, dtype=torch.uint8, device=dev)
        descs.append(bg.make_group(tk, te, out, st, p=P))
        keep.append((g, ks, es, out, st, tk, te))  # the descriptors hold raw pointers only
    plan = bg.BatchPlan(descs, flags)
    try:
        plan.launch()
        torch.cuda.synchronize()
    finally:
        plan.close()
    rng = np.random.default_rng(3)
    for g, ks, es, out, st, _, _ in keep:
        sts = st.cpu().numpy()
        assert (sts == 0).all(), (g["field"], g["n"], g["d"])
        idx = rng.choice(g["npts"], size=min(2, g["npts"]), replace=False)
        k = I.from_soa(ks[:, :, idx], len(idx))
        e = I.from_soa(es[:, :, idx], len(idx))
        o = out.cpu().numpy()[idx]
        if g["field"] == "fp":
            so, vo = bgtest.oracle_fp(k.astype(np.int64), e.astype(np.int64), P)
            assert_fp_equal(sts[idx], o.view(np.uint32).astype(np.int64), so, vo, f"fp n={g['n']} d={g['d']}")
        else:
            so, vo = bgtest.oracle_c(k, e)
            bgtest.check_c(o, vo, k, e, label=f"c128 n={g['n']} d={g['d']}")
    for f in (bg.BG_FIELD_FP, bg.BG_FIELD_C128):
        for g, *_ in keep:
            bg.bg_select_variant(f, g["n"], g["d"], -1)
