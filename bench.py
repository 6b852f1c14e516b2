#!/usr/bin/env python3
"""Throughput of the batched Berends-Giele recursion on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu-baseline]

A step is one pass of the hot path over one batch resident in HBM: one call
of bg_amplitudes_c128 on the n = 8, d = 4 complex128 workload (2^20
phase-space points: RAMBO momenta at sqrt(s) = 1000, uniform random
helicities, random null reference per point).  The same line carries the
n = 8, d = 6 F_p workload (p = 2^31 - 19, 2^20 points) measured the same way.

Prints one JSON line.  Kernel durations are taken with HIP events recorded on
the stream the kernels run on, around every launch.  The roofline figure
uses the algorithmic work per amplitude, W = d (6 C(n,3) + 4 C(n,4) + 2 R + 1)
field multiply-adds with R = (n-1)(n-2)/2 - 1 propagators; a complex
multiply-add is 8 FP64 flops, an F_p multiply-add at least one 32x32->64-bit
integer multiply-add issue.
"""
from __future__ import annotations

import argparse
import ctypes
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

FP64_PEAK_TFLOPS = 78.6          # MI355X vector FP64 (published)
LANE_SLOTS_PER_S = 256 * 4 * 16 * 2.4e9   # 256 CU x 4 SIMD x 16 lanes x 2.4 GHz = 39.3e12
# Z_p roofline: the 32x32->64-bit integer multiply-add issue rate.  It has no
# published figure; run_issue_rate measures it beside the FP64 FMA and the
# peak is the published FP64 FMA rate scaled by the measured ratio of the two
# (both measured at the same clock).  This constant is the nominal value (one
# per lane slot per cycle at 2.4 GHz), used only where nothing was measured.
INT_MAD_PEAK_TOPS = LANE_SLOTS_PER_S / 1e12


def kernel_source_digest() -> str:
    """Hash of what decides the recursion kernels' code and launch shape: the
    kernel headers, the launch layer (bg_api.hip) and the build script that
    instantiates them with its compiler flags."""
    import hashlib
    pkg = os.path.join(ROOT, "paper_2502_07060_amd")
    csrc = os.path.join(pkg, "csrc")
    files = [os.path.join(csrc, f) for f in sorted(os.listdir(csrc)) if f.endswith(".h")]
    files += [os.path.join(csrc, "bg_api.hip"), os.path.join(pkg, "build.py")]
    h = hashlib.sha256()
    for f in files:
        with open(f, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(kind: str):
    """HBM bytes per launch from the committed rocprofv3 counter runs, or None
    when the kernel sources changed since those counters were taken."""
    path = os.path.join(ROOT, "profiles", "traffic.txt")
    if not os.path.exists(path):
        return None
    vals = {}
    for line in open(path):
        line = line.split("#", 1)[0].strip()
        if "=" in line:
            k, v = (x.strip() for x in line.split("=", 1))
            vals[k] = v
    if vals.get("source_digest") != kernel_source_digest() or kind not in vals:
        return None
    return int(vals[kind])


def work_per_amplitude(n: int, d: int) -> int:
    R = (n - 1) * (n - 2) // 2 - 1
    return d * (6 * math.comb(n, 3) + 4 * math.comb(n, 4) + 2 * R + 1)


def time_launches(fn, steps: int, warmup: int):
    import torch
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(steps)]
    t_all0 = torch.cuda.Event(enable_timing=True)
    t_all1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    wall0 = time.perf_counter()
    t_all0.record()
    for a, b in ev:
        a.record()
        fn()
        b.record()
    t_all1.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - wall0
    total_ms = t_all0.elapsed_time(t_all1)
    per = [a.elapsed_time(b) for a, b in ev]
    return total_ms, sum(per) / len(per), wall


PROBE_NAMES = {0: "v_mad_i64_i32", 1: "v_mad_u64_u32", 2: "v_fma_f64", 3: "v_mul_lo_u32", 4: "v_mov_b32_dpp"}


def run_issue_rate(blocks: int = 8192, iters: int = 2048, reps: int = 5):
    """Issue rates of the recursion kernels' instruction classes on this
    device (bg_issue_rate: 8 independent chains per lane, 2^21 lanes), the
    derived Z_p peak, and the time of an almost empty launch."""
    from paper_2502_07060_amd import bg
    rates = {}
    for kind, name in PROBE_NAMES.items():
        r, ms = bg.bg_issue_rate(kind, blocks=blocks, iters=iters, reps=reps)
        rates[name] = {"lane_ops_per_s": r, "ms_per_launch": ms, "per_lane_slot_cycle_at_2.4GHz": r / LANE_SLOTS_PER_S}
    _, empty_ms = bg.bg_issue_rate(bg.BG_PROBE_MAD_I64_I32, blocks=1, iters=4, reps=50)
    ratio = rates["v_mad_i64_i32"]["lane_ops_per_s"] / rates["v_fma_f64"]["lane_ops_per_s"]
    return {
        "method": f"{blocks} blocks x 256 lanes, 8 independent dependency chains per lane, {iters} rounds, "
                  f"{reps} timed launches after one warm-up, HIP events on the launch stream",
        "rates": rates,
        "int_mad_over_fp64_fma": ratio,
        "int_mad_peak_tops": ratio * FP64_PEAK_TFLOPS / 2,
        "int_mad_peak_basis": "published FP64 FMA rate (78.6 TFLOP/s / 2 flops) x measured v_mad_i64_i32 / v_fma_f64",
        "implied_clock_ghz": rates["v_fma_f64"]["lane_ops_per_s"] / (256 * 4 * 16) / 1e9,
        "empty_launch_ms": empty_ms,
    }


def run_c5_small(steps: int, warmup: int, empty_launch_ms: float | None):
    """Config c1: n = 5, d = 4, complex128, 10^4 points: HBM / launch bound."""
    r = run_workload("c5_small", steps, warmup)
    n, d, npts = r["n"], r["d"], r["npts"]
    nbytes = npts * ((2 * n - 1) * d * 16 + 16 + 1)
    achieved = nbytes / (r["kernel_ms"] * 1e-3) / 1e9
    r["roofline"] = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_TBS * 1e3, "unit": "GB/s",
                     "frac": achieved / (HBM_PEAK_TBS * 1e3), "traffic": None,
                     "hbm_floor_ms": nbytes / (HBM_PEAK_TBS * 1e12) * 1e3}
    r["empty_launch_ms"] = empty_launch_ms
    r["workload"] = ("c5_small: n=5, d=4, complex128, 10^4 points, helicities (--+++), RAMBO sqrt(s)=1000, "
                     "one launch per step")
    return r


def cpu_baseline(kind: str, npts: int):
    """The oracle, as it stands, on a bounded sample of the same workload."""
    import multiprocessing as mp
    import numpy as np

    sys.path.insert(0, os.path.join(ROOT, "tests"))
    import bgtest
    from paper_2502_07060_amd import inputs as I

    w = I.config_workload(kind, npts=npts)
    k, e = w["k"], w["eps"]
    cores = bgtest._workers()
    bgtest.pool()  # start workers before timing
    t0 = time.perf_counter()
    if w["field"] == "fp":
        bgtest.oracle_fp(k.astype(np.int64), e.astype(np.int64), w["p"])
    else:
        bgtest.oracle_c(k, e)
    dt = time.perf_counter() - t0
    one = cpu_single_core(kind, 4096 if kind != "c5_small" else 10_000)
    return {"value": npts / dt, "unit": "amplitudes/s", "cores": cores, "kind": "oracle",
            "all_cores_per_core": npts / dt / cores, "single_core": one,
            "cpu_model": _cpu_model(), "host_cpus": os.cpu_count(),
            "sample": f"{npts} points of {kind} drawn with the same recipe and seed, pure-Python oracle, "
                      f"{cores} worker processes, {dt:.1f} s wall"}


def cpu_single_core(kind: str, npts: int):
    """The oracle in this process alone (one core) on the first npts points of
    the same recipe and seed."""
    import numpy as np

    sys.path.insert(0, os.path.join(ROOT, "tests"))
    import bgtest
    from paper_2502_07060_amd import inputs as I

    w = I.config_workload(kind, npts=npts)
    k, e = w["k"], w["eps"]
    t0 = time.perf_counter()
    if w["field"] == "fp":
        for q in range(npts):
            bgtest._fp_one((w["p"], k[q].astype(np.int64), e[q].astype(np.int64), bgtest.MM))
    else:
        for q in range(npts):
            bgtest._c_one((k[q], e[q], bgtest.MM))
    dt = time.perf_counter() - t0
    return {"value": npts / dt, "unit": "amplitudes/s", "cores": 1,
            "sample": f"first {npts} points of {kind} (same recipe and seed), one process, {dt:.1f} s"}


def _cpu_model() -> str:
    """The host CPU's model name, from /proc/cpuinfo (empty if unreadable)."""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return ""


def run_workload(kind: str, steps: int, warmup: int, int_peak_tops: float | None = None):
    import numpy as np
    import torch

    from paper_2502_07060_amd import bg
    from paper_2502_07060_amd import inputs as I

    w = I.config_workload(kind)
    dev = torch.device("cuda:0")
    n, d = w["n"], w["d"]
    npts = len(w["k"])
    # the library's autotuner picks the kernel variant for this (field, n, d)
    # on synthetic inputs of the same shape and size, before anything is timed
    # (same size, so every launch of the chosen kernel in a trace is alike)
    field = bg.BG_FIELD_FP if w["field"] == "fp" else bg.BG_FIELD_C128
    chosen, tuned = bg.bg_autotune(field, n, d, w["p"] if w["field"] == "fp" else 0, npts=npts, reps=5)
    if w["field"] == "fp":
        tk = torch.from_numpy(I.to_soa(w["k"]).view(np.int32)).to(dev)
        te = torch.from_numpy(I.to_soa(w["eps"]).view(np.int32)).to(dev)
        out = torch.empty(npts, dtype=torch.int32, device=dev)
        st = torch.empty(npts, dtype=torch.uint8, device=dev)
        fn = lambda: bg.bg_amplitudes_fp(tk, te, w["p"], out=out, status=st)
    else:
        tk = torch.from_numpy(I.to_soa(w["k"])).to(dev)
        te = torch.from_numpy(I.to_soa(w["eps"])).to(dev)
        out = torch.empty(npts, dtype=torch.complex128, device=dev)
        st = torch.empty(npts, dtype=torch.uint8, device=dev)
        fn = lambda: bg.bg_amplitudes_c128(tk, te, out=out, status=st)
    total_ms, launch_ms, wall = time_launches(fn, steps, warmup)
    bad = int((st != 0).sum().item())
    W = work_per_amplitude(n, d)
    if w["field"] == "fp":
        peak = int_peak_tops or INT_MAD_PEAK_TOPS
        achieved = W * npts / (launch_ms * 1e-3) / 1e12
        roof = {"bound": "alu", "achieved": achieved, "peak": peak, "unit": "TOP/s",
                "frac": achieved / peak, "traffic": measured_traffic(kind),
                "peak_basis": "measured (issue_rate)" if int_peak_tops else "nominal: one per lane slot per cycle"}
    else:
        achieved = 8 * W * npts / (launch_ms * 1e-3) / 1e12
        roof = {"bound": "alu", "achieved": achieved, "peak": FP64_PEAK_TFLOPS, "unit": "TFLOP/s",
                "frac": achieved / FP64_PEAK_TFLOPS, "traffic": measured_traffic(kind)}
    return {
        "value": npts * steps / (total_ms * 1e-3),
        "ms_per_step": total_ms / steps,
        "kernel_ms": launch_ms,
        "host_wall_ms_per_step": 1e3 * wall / steps,
        "npts": npts, "n": n, "d": d, "field": w["field"], "nonzero_status": bad,
        "work_per_amplitude": W, "roofline": roof,
        "variant": next({k: v[k] for k in ("lanes", "comps_per_lane", "lds_tables", "generic", "padded")}
                        for v, _ in tuned if v["index"] == chosen),
    }


def run_group(spec: str, steps: int, warmup: int):
    """One group of the batched workload alone, e.g. "c128:14:6" (the group's
    size and seed from the batched draw) or "fp:12:8:65536" (that many points,
    same generator): autotuned at its size, then timed like the n = 8
    workloads.  Used to profile the runtime-n kernels one group at a time."""
    import numpy as np
    import torch

    from paper_2502_07060_amd import bg
    from paper_2502_07060_amd import inputs as I

    parts = spec.split(":")
    field, n, d = parts[0], int(parts[1]), int(parts[2])
    g = next(dict(x) for x in I.batched_groups() if (x["field"], x["n"], x["d"]) == (field, n, d))
    if len(parts) > 3:
        g["npts"] = int(parts[3])
    p = I.DEFAULT_PRIME
    k, e = I.group_inputs(g, p)
    dev = torch.device("cuda:0")
    npts = g["npts"]
    fid = bg.BG_FIELD_FP if field == "fp" else bg.BG_FIELD_C128
    chosen, tuned = bg.bg_autotune(fid, n, d, p if field == "fp" else 0, npts=npts, reps=5)
    if field == "fp":
        tk = torch.from_numpy(I.to_soa(k.astype(np.uint32)).view(np.int32)).to(dev)
        te = torch.from_numpy(I.to_soa(e.astype(np.uint32)).view(np.int32)).to(dev)
        fn = lambda: bg.bg_amplitudes_fp(tk, te, p)
    else:
        tk = torch.from_numpy(I.to_soa(k.astype(np.complex128))).to(dev)
        te = torch.from_numpy(I.to_soa(e.astype(np.complex128))).to(dev)
        fn = lambda: bg.bg_amplitudes_c128(tk, te)
    total_ms, launch_ms, _ = time_launches(fn, steps, warmup)
    roof = group_roofline_ms(field, n, d, npts)
    return {"workload": f"batched group {field} n={n} d={d}, {npts} points (seed {g['seed']})",
            "npts": npts, "kernel_ms": launch_ms, "ms_per_step": total_ms / steps,
            "value": npts / (launch_ms * 1e-3), "unit": "amplitudes/s",
            "roofline_ms": roof, "frac": roof / launch_ms,
            "variant": next({kk: v[kk] for kk in ("lanes", "comps_per_lane", "lds_tables", "generic", "padded")}
                            for v, _ in tuned if v["index"] == chosen)}


def run_alternating(kind: str, steps: int, warmup: int, mostly_minus_ms: float):
    """The same workload through bg_amplitudes_*_metric in the alternating
    metric of Sec. 3.1 (the loaders map it onto the mostly-minus one), tuned
    in that metric (its own variant pin), against the mostly-minus kernel time
    measured before."""
    import numpy as np
    import torch

    from paper_2502_07060_amd import bg
    from paper_2502_07060_amd import inputs as I

    w = I.config_workload(kind)
    dev = torch.device("cuda:0")
    npts = len(w["k"])
    alt = bg.BG_METRIC_ALTERNATING
    field = bg.BG_FIELD_FP if w["field"] == "fp" else bg.BG_FIELD_C128
    chosen, tuned = bg.bg_autotune(field, w["n"], w["d"], w["p"] if w["field"] == "fp" else 0, npts=npts, reps=5,
                                   metric=alt)
    if w["field"] == "fp":
        tk = torch.from_numpy(I.to_soa(w["k"]).view(np.int32)).to(dev)
        te = torch.from_numpy(I.to_soa(w["eps"]).view(np.int32)).to(dev)
        out = torch.empty(npts, dtype=torch.int32, device=dev)
        st = torch.empty(npts, dtype=torch.uint8, device=dev)
        fn = lambda: bg.bg_amplitudes_fp(tk, te, w["p"], out=out, status=st, metric=alt)
    else:
        tk = torch.from_numpy(I.to_soa(w["k"])).to(dev)
        te = torch.from_numpy(I.to_soa(w["eps"])).to(dev)
        out = torch.empty(npts, dtype=torch.complex128, device=dev)
        st = torch.empty(npts, dtype=torch.uint8, device=dev)
        fn = lambda: bg.bg_amplitudes_c128(tk, te, out=out, status=st, metric=alt)
    _, launch_ms, _ = time_launches(fn, steps, warmup)
    v = next(v for v, _ in tuned if v["index"] == chosen)
    return {"kernel_ms": launch_ms, "mostly_minus_kernel_ms": mostly_minus_ms,
            "ratio": launch_ms / mostly_minus_ms, "value": npts / (launch_ms * 1e-3),
            "variant": {k: v[k] for k in ("lanes", "comps_per_lane", "lds_tables", "generic")}}


# ----------------------------------------------------------------------------
# rational amplitudes from F_p samples (residues, F_p amplitudes, reconstruction)
# ----------------------------------------------------------------------------

def _largest_primes_below(top: int, count: int):
    out, c = [], top - 1
    while len(out) < count:
        if c % 2 and all(c % f for f in range(3, int(c ** 0.5) + 1, 2)):
            out.append(c)
        c -= 1
    return out


def run_rational(steps: int, warmup: int, n: int = 5, d: int = 4, npts: int = 1 << 18, nprimes: int = 14,
                 pool: int = 512):
    """Rational amplitudes at rational kinematic points: for each prime the
    inputs' residues (bg_fp_from_rational) and the F_p amplitudes
    (bg_amplitudes_fp), then Chinese remaindering and rational reconstruction
    (bg_rational_reconstruct), all on the GPU with inputs resident."""
    import numpy as np
    import torch

    from paper_2502_07060_amd import bg
    from paper_2502_07060_amd import inputs as I

    dev = torch.device("cuda:0")
    primes = _largest_primes_below(2 ** 31, nprimes)
    kn, kd, en, ed = I.rational_points(11, n, d, pool)
    reps = npts // pool
    soa = lambda a: torch.from_numpy(np.ascontiguousarray(np.tile(np.transpose(a, (1, 2, 0)), (1, 1, reps)))).to(dev)
    tkn, tkd, ten, ted = soa(kn), soa(kd), soa(en), soa(ed)
    km = torch.empty((n, d, npts), dtype=torch.int32, device=dev)
    em = torch.empty_like(km)
    kst = torch.empty((n, d, npts), dtype=torch.uint8, device=dev)
    est = torch.empty_like(kst)
    res = torch.empty((nprimes, npts), dtype=torch.int32, device=dev)
    ast = torch.empty((nprimes, npts), dtype=torch.uint8, device=dev)
    bg.bg_autotune(bg.BG_FIELD_FP, n, d, primes[0], npts=npts, reps=3)

    def residues_and_amplitudes():
        for i, p in enumerate(primes):
            bg.bg_fp_from_rational(p, tkn, tkd, out=km, status=kst)
            bg.bg_fp_from_rational(p, ten, ted, out=em, status=est)
            bg.bg_amplitudes_fp(km, em, p, out=res[i], status=ast[i])

    box = {}

    def reconstruct():
        box["r"] = bg.bg_rational_reconstruct(primes, res)

    def whole():
        residues_and_amplitudes()
        reconstruct()

    total_ms, launch_ms, _ = time_launches(whole, steps, warmup)
    _, rr_ms, _ = time_launches(reconstruct, steps, warmup)
    _, fa_ms, _ = time_launches(residues_and_amplitudes, steps, warmup)
    num, den, st = box["r"]
    bad = int((st != 0).sum().item()) + int((ast != 0).sum().item())
    L = bg.bg_rr_limbs(nprimes)
    rr_bytes = npts * (4 * nprimes + 8 * L + 1)
    return {
        "workload": f"n={n}, d={d} rational kinematic points (light-cone integers in [-9, 9], exact closing pair, "
                    f"integer w in [-5, 5]; {pool} distinct points tiled to {npts}), {nprimes} primes below 2^31",
        "value": npts * steps / (total_ms * 1e-3), "unit": "rational amplitudes/s",
        "ms_per_step": total_ms / steps, "ms_residues_and_fp_amplitudes": fa_ms, "ms_reconstruct": rr_ms,
        "reconstruct": {"bound": "hbm", "achieved": rr_bytes / (rr_ms * 1e-3) / 1e9, "peak": HBM_PEAK_TBS * 1e3,
                        "unit": "GB/s", "frac": rr_bytes / (rr_ms * 1e-3) / (HBM_PEAK_TBS * 1e12),
                        "points_per_s": npts / (rr_ms * 1e-3)},
        "nonzero_status": bad, "npts": npts, "nprimes": nprimes,
    }


# ----------------------------------------------------------------------------
# one-leg cut: states of the cut leg, two root currents, the state sum
# ----------------------------------------------------------------------------

def run_cut(steps: int, warmup: int, n: int = 6, d: int = 6, npts: int = 1 << 20):
    """sum_s M_L(.., e_s) M_R(.., e~_s) over Z_p for two n-point trees joined
    by a cut leg l: bg_states_fp (l), bg_currents_fp (both trees),
    bg_state_sum_fp; random residues for the other legs (the identities are
    algebraic), inputs resident."""
    import numpy as np
    import torch

    from paper_2502_07060_amd import bg
    from paper_2502_07060_amd import inputs as I

    p = I.DEFAULT_PRIME
    dev = torch.device("cuda:0")
    rng = np.random.default_rng(21)
    l = I.fp_null(rng, p, (npts,), d).astype(np.uint32)
    chi = I.fp_null(rng, p, (npts,), 4).astype(np.uint32)
    up = lambda a: torch.from_numpy(np.ascontiguousarray(a).view(np.int32)).to(dev)
    tl, tchi = up(l.T), up(chi.T)
    g = torch.Generator(device=dev)
    g.manual_seed(22)
    rnd = lambda *shape: torch.randint(0, p, shape, generator=g, device=dev, dtype=torch.int64).to(torch.int32)
    kL, kR, eL, eR = rnd(n, d, npts), rnd(n, d, npts), rnd(n, d, npts), rnd(n, d, npts)
    kL[n - 1].copy_(tl)
    kR[n - 1].copy_(torch.remainder(p - tl.to(torch.int64).bitwise_and(0xFFFFFFFF), p).to(torch.int32))
    bg.bg_autotune(bg.BG_FIELD_FP, n, d, p, npts=npts, reps=3)
    box = {}

    def states():
        box["s"] = bg.bg_states_fp(tl, tchi, p)

    def currents():
        box["L"] = bg.bg_currents_fp(kL, eL, p)
        box["R"] = bg.bg_currents_fp(kR, eR, p)

    def ssum():
        e, et, _ = box["s"]
        box["S"] = bg.bg_state_sum(box["L"][0], box["R"][0], e, et, p=p)

    def whole():
        states()
        currents()
        ssum()

    total_ms, _, _ = time_launches(whole, steps, warmup)
    _, st_ms, _ = time_launches(states, steps, warmup)
    _, cu_ms, _ = time_launches(currents, steps, warmup)
    _, ss_ms, _ = time_launches(ssum, steps, warmup)
    bad = int((box["S"][1] != 0).sum().item()) + int((box["L"][1] != 0).sum().item())
    ss_bytes = npts * 4 * (2 * d + 2 * (d - 2) * d + 1) + npts
    return {
        "workload": f"two {n}-point trees joined by one cut leg, d={d}, Z_p p=2^31-19, {npts} points",
        "value": npts * steps / (total_ms * 1e-3), "unit": "state-summed cut products/s",
        "ms_per_step": total_ms / steps, "ms_states": st_ms, "ms_two_root_currents": cu_ms, "ms_state_sum": ss_ms,
        "state_sum_roofline": {"bound": "hbm", "achieved": ss_bytes / (ss_ms * 1e-3) / 1e9,
                               "peak": HBM_PEAK_TBS * 1e3, "unit": "GB/s",
                               "frac": ss_bytes / (ss_ms * 1e-3) / (HBM_PEAK_TBS * 1e12)},
        "nonzero_status": bad,
    }


# ----------------------------------------------------------------------------
# standalone Z_p operations (contraction and division)
# ----------------------------------------------------------------------------

def run_ffops(steps: int, warmup: int, npts: int = 1 << 20, dim: int = 6, ndiv: int = 1 << 24):
    """bg_fp_contract with I = J = K = dim, second operand per event, over npts
    events; bg_fp_divide over ndiv values.  HBM rooflines on the algorithmic
    bytes (each input read once, each output written once)."""
    import numpy as np
    import torch

    from paper_2502_07060_amd import bg
    from paper_2502_07060_amd import inputs as I

    p = I.DEFAULT_PRIME
    dev = torch.device("cuda:0")
    g = torch.Generator(device=dev)
    g.manual_seed(12)
    rnd = lambda *shape: torch.randint(0, p, shape, generator=g, device=dev, dtype=torch.int64).to(torch.int32)
    x, y = rnd(dim, dim, npts), rnd(dim, dim, npts)
    box = {}
    _, c_ms, _ = time_launches(lambda: box.__setitem__("c", bg.bg_fp_contract(p, x, y)), steps, warmup)
    dx, dy = rnd(ndiv), rnd(ndiv)
    _, d_ms, _ = time_launches(lambda: box.__setitem__("d", bg.bg_fp_divide(p, dx, dy)), steps, warmup)
    c_bytes = npts * (3 * dim * dim * 4 + 1)
    d_bytes = ndiv * (3 * 4 + 1)
    roof = lambda b, ms: {"bound": "hbm", "achieved": b / (ms * 1e-3) / 1e9, "peak": HBM_PEAK_TBS * 1e3,
                          "unit": "GB/s", "frac": b / (ms * 1e-3) / (HBM_PEAK_TBS * 1e12)}
    bad = int((box["c"][1] != 0).sum().item()) + int((box["d"][1] != 0).sum().item())
    return {
        "contract": {"workload": f"z = x y per event, {dim}x{dim} times {dim}x{dim}, {npts} events, Z_p p=2^31-19",
                     "kernel_ms": c_ms, "value": npts / (c_ms * 1e-3), "unit": "events/s",
                     "roofline": roof(c_bytes, c_ms)},
        "divide": {"workload": f"z = x / y elementwise, {ndiv} values", "kernel_ms": d_ms,
                   "value": ndiv / (d_ms * 1e-3), "unit": "values/s", "roofline": roof(d_bytes, d_ms)},
        "nonzero_status": bad,
    }


# ----------------------------------------------------------------------------
# polarisation states (d-dimensional states and duals of Sec. 2.3)
# ----------------------------------------------------------------------------

def run_states(steps: int, warmup: int, d: int = 6, npts: int = 1 << 20):
    """States and duals of 2^20 massless d-vectors, F_p and complex128."""
    import numpy as np
    import torch

    from paper_2502_07060_amd import bg
    from paper_2502_07060_amd import inputs as I

    dev = torch.device("cuda:0")
    rng = np.random.default_rng(12)
    p = I.DEFAULT_PRIME
    res = {}
    for field in ("fp", "c128"):
        if field == "fp":
            k = I.fp_null(rng, p, (npts,), d).astype(np.uint32)
            chi = I.fp_null(rng, p, (npts,), 4).astype(np.uint32)
            tk = torch.from_numpy(np.ascontiguousarray(k.T).view(np.int32)).to(dev)
            tc = torch.from_numpy(np.ascontiguousarray(chi.T).view(np.int32)).to(dev)
            fn = lambda: bg.bg_states_fp(tk, tc, p)
            s = 4
        else:
            k = I.random_null_c(rng, npts, d).astype(np.complex128)
            chi = I.random_null_c(rng, npts, 4).astype(np.complex128)
            tk = torch.from_numpy(np.ascontiguousarray(k.T)).to(dev)
            tc = torch.from_numpy(np.ascontiguousarray(chi.T)).to(dev)
            fn = lambda: bg.bg_states_c128(tk, tc)
            s = 16
        total_ms, launch_ms, _ = time_launches(fn, steps, warmup)
        nbytes = npts * ((d + 4) * s + 2 * (d - 2) * d * s + 1)
        achieved = nbytes / (launch_ms * 1e-3) / 1e9
        res[field] = {"value": npts / (launch_ms * 1e-3), "unit": "points/s", "kernel_ms": launch_ms,
                      "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_TBS * 1e3,
                                   "unit": "GB/s", "frac": achieved / (HBM_PEAK_TBS * 1e3), "traffic": None}}
    return {"workload": f"d = {d} polarisation states and duals of 2^20 massless vectors (reference chi per "
                        "point), F_p p = 2^31-19 and complex128", "d": d, "npts": npts, **res}


# ----------------------------------------------------------------------------
# batched form: 88 (field, n, d) groups in one call
# ----------------------------------------------------------------------------

HBM_PEAK_TBS = 8.0


def _gen_group_soa(g):
    """Worker: one group's inputs in the C-ABI layout (host)."""
    import numpy as np
    from paper_2502_07060_amd import inputs as I
    k, e = I.group_inputs(g)
    if g["field"] == "fp":
        return I.to_soa(k.astype(np.uint32)), I.to_soa(e.astype(np.uint32))
    return I.to_soa(k.astype(np.complex128)), I.to_soa(e.astype(np.complex128))


def _gen_workers():
    return max(1, min(16, os.cpu_count() or 1))


def group_roofline_ms(field: str, n: int, d: int, npts: int) -> float:
    """max(HBM time, ALU time) of one group at the peaks used above."""
    s = 16 if field == "c128" else 4
    nbytes = npts * ((2 * n - 1) * d * s + s + 1)
    W = work_per_amplitude(n, d) * npts
    t_alu = 8 * W / (FP64_PEAK_TFLOPS * 1e12) if field == "c128" else W / (INT_MAD_PEAK_TOPS * 1e12)
    return 1e3 * max(nbytes / (HBM_PEAK_TBS * 1e12), t_alu)


def run_batched(steps: int, warmup: int):
    import multiprocessing as mp
    from concurrent.futures import ProcessPoolExecutor, as_completed

    import numpy as np
    import torch

    from paper_2502_07060_amd import bg
    from paper_2502_07060_amd import inputs as I

    p = I.DEFAULT_PRIME
    groups = [g for g in I.batched_groups() if g["npts"] > 0]
    dev = torch.device("cuda:0")
    t_gen = time.perf_counter()
    tens = {}
    with ProcessPoolExecutor(max_workers=_gen_workers(), mp_context=mp.get_context("spawn")) as ex:
        order = sorted(range(len(groups)), key=lambda i: -groups[i]["npts"])
        futs = {ex.submit(_gen_group_soa, groups[i]): i for i in order}
        for fu in as_completed(futs):
            i = futs[fu]
            ks, es = fu.result()
            g = groups[i]
            if g["field"] == "fp":
                tk = torch.from_numpy(ks.view(np.int32)).to(dev)
                te = torch.from_numpy(es.view(np.int32)).to(dev)
                out = torch.empty(g["npts"], dtype=torch.int32, device=dev)
            else:
                tk = torch.from_numpy(ks).to(dev)
                te = torch.from_numpy(es).to(dev)
                out = torch.empty(g["npts"], dtype=torch.complex128, device=dev)
            st = torch.full((g["npts"],), 9, dtype=torch.uint8, device=dev)
            tens[i] = (tk, te, out, st)
    t_gen = time.perf_counter() - t_gen
    # the autotuner picks each (field, n, d) group's kernel variant
    t_tune = time.perf_counter()
    for g in groups:
        field = bg.BG_FIELD_FP if g["field"] == "fp" else bg.BG_FIELD_C128
        bg.bg_autotune(field, g["n"], g["d"], p if g["field"] == "fp" else 0,
                       npts=min(max(g["npts"], 4096), 1 << 18), reps=3)
    t_tune = time.perf_counter() - t_tune
    descs = [bg.make_group(*tens[i], p=p) for i in range(len(groups))]
    total = sum(g["npts"] for g in groups)

    run = lambda: bg.bg_batch_run(descs)
    total_ms, launch_ms, wall = time_launches(run, steps, warmup)
    bad = sum(int((tens[i][3] != 0).sum().item()) for i in range(len(groups)))
    for i in range(len(groups)):       # the plan must rewrite every status
        tens[i][3].fill_(9)
    plan = bg.BatchPlan(descs)
    try:
        p_total_ms, p_launch_ms, _ = time_launches(plan.launch, steps, warmup)
    finally:
        plan.close()
    bad += sum(int((tens[i][3] != 0).sum().item()) for i in range(len(groups)))
    # queue form: one persistent launch per lane-group kernel variant over a
    # device work queue, as a call and as a graph plan
    for i in range(len(groups)):
        tens[i][3].fill_(9)
    runq = lambda: bg.bg_batch_run_ex(descs, bg.BG_BATCH_QUEUE)
    _, q_launch_ms, _ = time_launches(runq, steps, warmup)
    bad += sum(int((tens[i][3] != 0).sum().item()) for i in range(len(groups)))
    for i in range(len(groups)):
        tens[i][3].fill_(9)
    qplan = bg.BatchPlan(descs, bg.BG_BATCH_QUEUE)
    try:
        _, qp_launch_ms, _ = time_launches(qplan.launch, steps, warmup)
    finally:
        qplan.close()
    bad += sum(int((tens[i][3] != 0).sum().item()) for i in range(len(groups)))
    roof_ms = sum(group_roofline_ms(g["field"], g["n"], g["d"], g["npts"]) for g in groups)
    best = min(launch_ms, p_launch_ms, q_launch_ms, qp_launch_ms)
    # each group alone (same kernels), to show where the time goes
    per_group = []
    for i, g in enumerate(groups):
        one = [descs[i]]
        _, ms, _ = time_launches(lambda: bg.bg_batch_run(one), 3, 1)
        field = bg.BG_FIELD_FP if g["field"] == "fp" else bg.BG_FIELD_C128
        sel = next(v for v in bg.bg_variants(field, g["n"], g["d"]) if v["selected"])
        per_group.append({"field": g["field"], "n": g["n"], "d": g["d"], "npts": g["npts"], "ms": ms,
                          "roofline_ms": group_roofline_ms(g["field"], g["n"], g["d"], g["npts"]),
                          "variant": {k: sel[k] for k in ("lanes", "comps_per_lane", "lds_tables", "generic", "padded")}})
    per_group.sort(key=lambda r: -r["ms"])
    return {
        "workload": "88 groups (n 4..14 x d {4,6,8,10} x {complex128, Z_p}), 4*10^6 points, "
                    "Zipf(1.2) group sizes, seed 4",
        "value": total / (best * 1e-3), "unit": "amplitudes/s", "npts": total, "groups": len(groups),
        "ms_batch_run": launch_ms, "ms_graph_plan": p_launch_ms,
        "ms_queue_run": q_launch_ms, "ms_queue_graph_plan": qp_launch_ms,
        "roofline": {"bound": "mixed (per group max of HBM and ALU time)", "roofline_ms": roof_ms,
                     "measured_ms": best, "frac": roof_ms / best},
        "nonzero_status": bad, "host_generation_s": t_gen, "autotune_s": t_tune,
        "sum_of_groups_alone_ms": sum(r["ms"] for r in per_group), "slowest_groups": per_group[:12],
    }


# ----------------------------------------------------------------------------
# serving form: Poisson request stream, served vs plain per-request launches
# ----------------------------------------------------------------------------

SERVE_NS = list(range(4, 15))
SERVE_DS = [4, 6, 10]
SERVE_POOL = 65536        # columns of each host input pool (largest request)
SERVE_DISTINCT = 2048     # distinct points per pool, tiled across its columns


def serve_trace(count: int, seed: int = 5):
    """Request shapes and sizes: field and n, d uniform; size floor(exp(U[0, ln 65536])) in [1, 65536]."""
    import numpy as np
    rng = np.random.default_rng(seed)
    fields = rng.integers(0, 2, size=count)
    ns = rng.choice(SERVE_NS, size=count)
    ds = rng.choice(SERVE_DS, size=count)
    sizes = np.clip(np.floor(np.exp(rng.uniform(0, math.log(SERVE_POOL), size=count))), 1, SERVE_POOL).astype(np.int64)
    offs = (rng.random(count) * (SERVE_POOL - sizes + 1)).astype(np.int64)
    gaps = rng.exponential(1.0, size=count)      # unit-rate Poisson gaps, scaled per rate
    return [dict(field=("c128", "fp")[f], n=int(n), d=int(d), npts=int(m), off=int(o))
            for f, n, d, m, o in zip(fields, ns, ds, sizes, offs)], np.cumsum(gaps) - gaps[0]


def _serve_pool_inputs(key):
    import numpy as np
    from paper_2502_07060_amd import inputs as I
    field, n, d = key
    g = dict(field=field, n=n, d=d, npts=SERVE_DISTINCT, seed=50_000 + 100 * n + d + (7 if field == "fp" else 0))
    k, e = I.group_inputs(g)
    if field == "fp":
        return I.to_soa(k.astype(np.uint32)).view(np.int32), I.to_soa(e.astype(np.uint32)).view(np.int32)
    return I.to_soa(k.astype(np.complex128)), I.to_soa(e.astype(np.complex128))


def copy_bandwidth(mib: int = 512, reps: int = 5):
    """Pinned host <-> device copy bandwidth (bytes/s), each direction alone
    and both at once, timed with events on one stream per direction."""
    import torch
    n = mib << 20
    h_src = torch.empty(n, dtype=torch.uint8, pin_memory=True)
    h_dst = torch.empty(n, dtype=torch.uint8, pin_memory=True)
    d_a = torch.empty(n, dtype=torch.uint8, device="cuda:0")
    d_b = torch.empty(n, dtype=torch.uint8, device="cuda:0")
    s1, s2 = torch.cuda.Stream(), torch.cuda.Stream()

    def timed(fns):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            for st, f in fns:
                with torch.cuda.stream(st):
                    f()
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) / reps

    h2d = lambda: d_a.copy_(h_src, non_blocking=True)
    d2h = lambda: h_dst.copy_(d_b, non_blocking=True)
    timed([(s1, h2d), (s2, d2h)])  # warm-up
    t_in = timed([(s1, h2d)])
    t_out = timed([(s2, d2h)])
    t_both = timed([(s1, h2d), (s2, d2h)])
    return {"h2d_bytes_per_s": n / t_in, "d2h_bytes_per_s": n / t_out, "bidirectional_bytes_per_s": 2 * n / t_both,
            "method": f"{mib} MiB pinned <-> device, {reps} copies per direction, wall clock around the copies"}


def run_served(count: int, fracs=(0.5, 0.7, 0.9), budget_gib: float = 8.0):
    import multiprocessing as mp
    from concurrent.futures import ProcessPoolExecutor

    import numpy as np
    import torch

    from paper_2502_07060_amd import bg
    from paper_2502_07060_amd import inputs as I

    p = I.DEFAULT_PRIME
    trace, unit_arrivals = serve_trace(count)
    keys = sorted({(r["field"], r["n"], r["d"]) for r in trace})
    t_gen = time.perf_counter()
    pools = {}
    with ProcessPoolExecutor(max_workers=_gen_workers(), mp_context=mp.get_context("spawn")) as ex:
        for key, (ks, es) in zip(keys, ex.map(_serve_pool_inputs, keys)):
            reps = SERVE_POOL // SERVE_DISTINCT
            dt = torch.int32 if key[0] == "fp" else torch.complex128
            n, d = key[1], key[2]
            pk = torch.empty((n, d, SERVE_POOL), dtype=dt, pin_memory=True)
            pe = torch.empty((n, d, SERVE_POOL), dtype=dt, pin_memory=True)
            pk.numpy().reshape(n, d, reps, SERVE_DISTINCT)[:] = ks[:, :, None, :]
            pe.numpy().reshape(n, d, reps, SERVE_DISTINCT)[:] = es[:, :, None, :]
            pools[key] = (pk, pe)
    # per-request output slices of two pinned pools
    tot_c = sum(r["npts"] for r in trace if r["field"] == "c128")
    tot_f = sum(r["npts"] for r in trace if r["field"] == "fp")
    out_c = torch.empty(max(tot_c, 1), dtype=torch.complex128, pin_memory=True)
    out_f = torch.empty(max(tot_f, 1), dtype=torch.int32, pin_memory=True)
    st_all = torch.empty(max(tot_c + tot_f, 1), dtype=torch.uint8, pin_memory=True)
    descs = []
    oc = of = 0
    for r in trace:
        pk, pe = pools[(r["field"], r["n"], r["d"])]
        es = 16 if r["field"] == "c128" else 4
        m = r["npts"]
        if r["field"] == "c128":
            optr = out_c.data_ptr() + oc * es
            sptr = st_all.data_ptr() + oc
            oc += m
        else:
            optr = out_f.data_ptr() + of * es
            sptr = st_all.data_ptr() + tot_c + of
            of += m
        field = bg.BG_FIELD_FP if r["field"] == "fp" else bg.BG_FIELD_C128
        descs.append(bg.bg_group(field, r["n"], r["d"], p if r["field"] == "fp" else 0, m, SERVE_POOL,
                                 pk.data_ptr() + r["off"] * es, pe.data_ptr() + r["off"] * es, optr, sptr))
    t_gen = time.perf_counter() - t_gen
    for field, n, d in keys:
        f = bg.BG_FIELD_FP if field == "fp" else bg.BG_FIELD_C128
        bg.bg_autotune(f, n, d, p if field == "fp" else 0, npts=1 << 16, reps=3)
    mean_size = sum(r["npts"] for r in trace) / len(trace)
    # host <-> device bytes of the whole trace: inputs in, results and statuses out
    es_of = lambda r: 16 if r["field"] == "c128" else 4
    bytes_in = sum(2 * r["n"] * r["d"] * es_of(r) * r["npts"] for r in trace)
    bytes_out = sum((es_of(r) + 1) * r["npts"] for r in trace)
    bw = copy_bandwidth()
    # copies in and out run on separate DMA engines: the copy-bound span is the
    # longer of the two directions (both directions at once measured too)
    copy_bound_s = max(bytes_in / bw["h2d_bytes_per_s"], bytes_out / bw["d2h_bytes_per_s"],
                       (bytes_in + bytes_out) / bw["bidirectional_bytes_per_s"])
    L = bg.lib()
    budget = int(budget_gib * (1 << 30))

    def replay(plain: bool, rate):
        """Submits the trace at arrival times unit_arrivals / rate (all at once
        if rate is None); returns throughput and latency percentiles."""
        srv = bg.Server(budget, plain=plain)
        try:
            ids = []
            rid = ctypes.c_uint64()
            t0 = bg.bg_server_now_ns()
            arr = [0.0] * len(descs) if rate is None else list(unit_arrivals / rate)
            base = time.perf_counter()
            for dsc, at in zip(descs, arr):
                while time.perf_counter() - base < at:
                    pass
                rc = L.bg_server_submit(srv._h, ctypes.byref(dsc), ctypes.byref(rid))
                if rc != bg.BG_OK:
                    raise bg.BGError(rc, "bg_server_submit")
                ids.append(rid.value)
            lat, done_max, shared = [], 0, 0
            tm = bg.bg_request_times()
            for i, at in zip(ids, arr):
                rc = L.bg_server_wait(srv._h, i, -1.0, ctypes.byref(tm))
                if rc != bg.BG_OK:
                    raise bg.BGError(rc, "bg_server_wait")
                lat.append((tm.done_ns - (t0 + at * 1e9)) * 1e-6)
                done_max = max(done_max, tm.done_ns)
                shared += tm.batch_requests > 1
            st = srv.stats()
        finally:
            srv.close()
        lat = np.array(lat)
        span = (done_max - t0) * 1e-9
        return {"throughput": sum(r["npts"] for r in trace) / span, "p50_ms": float(np.percentile(lat, 50)),
                "p99_ms": float(np.percentile(lat, 99)), "launches": st["batches"],
                "requests_sharing_a_launch": shared, "arena_peak_bytes": st["arena_peak"], "span_s": span,
                "host_device_bytes_per_s": (bytes_in + bytes_out) / span,
                "frac_of_copy_bound": copy_bound_s / span}

    replay(False, None)            # warm-up: first touches of pinned pages and kernels
    plain_sat = replay(True, None)
    served_sat = replay(False, None)
    rates = []
    for fr in fracs:
        lam = fr * plain_sat["throughput"] / mean_size
        rates.append({"frac_of_plain_throughput": fr, "requests_per_s": lam,
                      "served": replay(False, lam), "plain": replay(True, lam)})
    bad = int((st_all != 0).sum().item())
    return {
        "workload": f"{count} requests, Poisson arrivals, sizes floor(exp(U[0, ln 65536])), n 4..14, "
                    "d {4,6,10}, complex128 or Z_p, seed 5; inputs and outputs in pinned host memory, "
                    "latency from arrival to results on the host",
        "mean_request_points": mean_size, "arena_gib": budget_gib,
        "copy_bound": {**bw, "trace_bytes_in": bytes_in, "trace_bytes_out": bytes_out,
                       "copy_bound_span_s": copy_bound_s},
        "saturated": {"plain": plain_sat, "served": served_sat,
                      "served_over_plain": served_sat["throughput"] / plain_sat["throughput"]},
        "rates": rates, "nonzero_status": bad, "host_setup_s": t_gen,
    }


def calibrate_copy(mib: int):
    if mib <= 0:
        return
    import torch
    src = torch.ones(mib << 18, dtype=torch.float32, device="cuda:0")
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    dst.copy_(src)
    torch.cuda.synchronize()


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-sample", type=int, default=600_000,
                    help="points of c8_d4 for the oracle baseline (a quarter as many for fp8_d6)")
    ap.add_argument("--no-batched", action="store_true", help="skip the batched 88-group workload")
    ap.add_argument("--no-served", action="store_true", help="skip the serving workload")
    ap.add_argument("--serve-requests", type=int, default=10000)
    ap.add_argument("--workload", choices=["both", "c8_d4", "fp8_d6", "c5_small", "issue_rate", "batched", "served",
                                           "states", "rational", "ffops", "cut"],
                    default="both",
                    help="restrict to one workload (profiling runs)")
    ap.add_argument("--group", metavar="FIELD:N:D[:NPTS]",
                    help="time one group of the batched workload alone (profiling runs)")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="after timing, run one device-to-device copy of MIB MiB: a plain copy "
                         "kernel of known traffic that scales hardware byte counters")
    a = ap.parse_args(argv)
    if a.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on one GPU only: the recursion shards by point range with no "
              "communication, so the single-GPU figure is the per-rank figure", file=sys.stderr)
        sys.exit(2)
    import torch
    assert torch.cuda.is_available(), "bench.py needs a GPU"

    if a.group:
        r = run_group(a.group, a.steps, a.warmup)
        calibrate_copy(a.calibrate_copy)
        print(json.dumps(r), flush=True)
        return
    if a.workload == "batched":
        print(json.dumps(run_batched(a.steps, a.warmup)), flush=True)
        return
    if a.workload == "served":
        print(json.dumps(run_served(a.serve_requests)), flush=True)
        return
    if a.workload == "states":
        print(json.dumps(run_states(a.steps, a.warmup)), flush=True)
        return
    if a.workload == "rational":
        print(json.dumps(run_rational(a.steps, a.warmup)), flush=True)
        return
    if a.workload == "ffops":
        print(json.dumps(run_ffops(a.steps, a.warmup)), flush=True)
        return
    if a.workload == "cut":
        print(json.dumps(run_cut(a.steps, a.warmup)), flush=True)
        return
    if a.workload == "issue_rate":
        print(json.dumps(run_issue_rate()), flush=True)
        return
    if a.workload == "c5_small":
        ir = run_issue_rate(iters=256)
        print(json.dumps(run_c5_small(a.steps, a.warmup, ir["empty_launch_ms"])), flush=True)
        return
    if a.workload != "both":
        r = run_workload(a.workload, a.steps, a.warmup)
        calibrate_copy(a.calibrate_copy)
        print(json.dumps({"workload": a.workload, **r}), flush=True)
        return
    issue = run_issue_rate()
    main_run = run_workload("c8_d4", a.steps, a.warmup)
    fp_run = run_workload("fp8_d6", a.steps, a.warmup, int_peak_tops=issue["int_mad_peak_tops"])
    calibrate_copy(a.calibrate_copy)
    line = {
        "metric": "amplitudes/s at n=8 (C d=4, F_p d=6); served p50/p99 latency vs plain launch",
        "value": main_run["value"],
        "unit": "amplitudes/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": main_run["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "c128",
        "data": "synthetic",
        "config": {
            "workload": "c8_d4: n=8 gluons, d=4, complex128, 2^20 phase-space points "
                        "(RAMBO sqrt(s)=1000, uniform random helicities, random null reference)",
            "npts": main_run["npts"], "n": 8, "d": 4,
        },
        "roofline": main_run["roofline"],
        "kernel_ms": main_run["kernel_ms"],
        "variant": main_run["variant"],
        "fp8_d6": {
            "workload": "n=8 gluons, d=6, Z_p p=2^31-19 (uint32), 2^20 points, light-cone momenta "
                        "with closing pair, transverse random polarisations",
            "value": fp_run["value"], "unit": "amplitudes/s", "dtype": "int32 Montgomery (int64 accumulate)",
            "ms_per_step": fp_run["ms_per_step"], "kernel_ms": fp_run["kernel_ms"],
            "roofline": fp_run["roofline"], "nonzero_status": fp_run["nonzero_status"],
            "variant": fp_run["variant"],
        },
    }
    def progress(what):
        print(f"[bench] {what} done", file=sys.stderr, flush=True)

    progress("n = 8 workloads")
    line["issue_rate"] = issue
    line["c5_small"] = run_c5_small(a.steps, a.warmup, issue["empty_launch_ms"])
    progress("c5_small")
    line["alternating_metric"] = {
        "workload": "the two n = 8 workloads through bg_amplitudes_*_metric, metric diag(1,-1,1,-1,...)",
        "c8_d4": run_alternating("c8_d4", a.steps, a.warmup, main_run["kernel_ms"]),
        "fp8_d6": run_alternating("fp8_d6", a.steps, a.warmup, fp_run["kernel_ms"]),
    }
    progress("alternating metric")
    line["states"] = run_states(a.steps, a.warmup)
    progress("states")
    line["rational"] = run_rational(a.steps, a.warmup)
    progress("rational")
    line["ffops"] = run_ffops(a.steps, a.warmup)
    progress("ffops")
    line["cut"] = run_cut(a.steps, a.warmup)
    progress("cut")
    if not a.no_batched:
        line["batched"] = run_batched(a.steps, a.warmup)
        progress("batched")
    if not a.no_served:
        line["served"] = run_served(a.serve_requests)
        progress("served")
    if not a.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline("c8_d4", a.cpu_sample)
        line["fp8_d6"]["cpu_baseline"] = cpu_baseline("fp8_d6", a.cpu_sample // 4)
        line["c5_small"]["cpu_baseline"] = {"single_core": cpu_single_core("c5_small", 10_000)}
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
