"""Build libbg_mi355x.so for gfx950 with hipcc.

Every kernel variant listed below becomes an explicit template instantiation
in a generated translation unit under ``_build/gen``; the units compile in
parallel and link, with the host C-ABI layer, into
``paper_2502_07060_amd/libbg_mi355x.so``.

    python -m paper_2502_07060_amd.build            # full rebuild
    python -m paper_2502_07060_amd.build --incremental
"""
from __future__ import annotations

import argparse
import hashlib
import os
import re
import shutil
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
INCLUDE = os.path.join(ROOT, "include")
BUILD = os.path.join(ROOT, "_build")
LIB = os.path.join(PKG, "libbg_mi355x.so")

ARCH = "gfx950"
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
CXXFLAGS = [
    f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC",
    # packed FP32 instructions are kept out of every kernel
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-I", INCLUDE, "-I", CSRC,
]

# Register-resident kernels: (field, N = n - 1, DL = components per lane,
# L = lanes per point, LT = per-point tables in LDS, W = waves per SIMD the
# register allocation must allow)
REGISTER_VARIANTS = []
for N in range(2, 8):
    # F_p: one, two or four lanes per point, per-point tables in LDS
    for DL, L in ((4, 1), (6, 1), (2, 2), (3, 2), (4, 2), (5, 2), (2, 4), (3, 4)):
        REGISTER_VARIANTS.append(("fp", N, DL, L, True, 1))
    # complex: two or four lanes per point; one lane while the table is small
    for DL, L, LT in ((2, 2, True), (3, 2, True), (4, 2, True), (5, 2, True),
                      (1, 4, False), (2, 4, True), (3, 4, True)):
        REGISTER_VARIANTS.append(("c128", N, DL, L, LT, 1))
    if N <= 4:
        REGISTER_VARIANTS.append(("c128", N, 4, 1, True, 1))
# n = 9 to 12 (35 to 65 currents per point): F_p on two lanes per point up
# to n = 11; complex with one component per lane on four lanes (d <= 4, up to
# n = 12) or two on two, and up to n = 11 two on four or three on two.  Some of these spill to scratch
# and still beat the runtime-n kernels.
for N in (8, 9, 10):
    for DL in (3, 4, 5):
        REGISTER_VARIANTS.append(("fp", N, DL, 2, True, 1))
for N in (8, 9, 10):
    REGISTER_VARIANTS += [("c128", N, 1, 4, True, 1), ("c128", N, 2, 2, True, 1)]
for N in (8, 9):
    REGISTER_VARIANTS += [("c128", N, 2, 4, True, 1), ("c128", N, 3, 2, True, 1)]
REGISTER_VARIANTS += [("c128", 10, 2, 4, True, 1), ("c128", 11, 1, 4, True, 1)]
# Runtime-n kernels with LDS tables: (field, DMAX), one point per lane
GENERIC_VARIANTS = [(f, dm) for f in ("fp", "c128") for dm in (4, 6, 8, 10)]
# Runtime-n kernels with G lanes sharing each point's tables: (field, DMAX, G,
# padded rows).  Padded rows (an odd number of 16-byte units) are compiled
# where the plain row stride puts many rows on the same LDS banks and the
# padding costs little LDS: complex DMAX 4, 8, 10 and F_p DMAX 8.
_PADDED = {("c128", 4), ("c128", 8), ("c128", 10), ("fp", 8)}
# (field, DMAX, G, padded, LC): LC lanes per work item; complex items also run
# on two lanes (half the components each), so that more lanes share the same
# LDS footprint per point
WIDE_VARIANTS = [(f, dm, G, pad, 1) for f in ("fp", "c128") for dm in (4, 6, 8, 10) for G in (16, 32, 64)
                 for pad in ((False, True) if (f, dm) in _PADDED else (False,))]
WIDE_VARIANTS += [("c128", dm, G, pad, 2) for dm in (4, 6, 8, 10) for G in (16, 32)
                  for pad in ((False, True) if ("c128", dm) in _PADDED else (False,))]
WIDE_VARIANTS += [("c128", 6, G, True, 2) for G in (16, 32)]
WIDE_VARIANTS += [("c128", dm, 16, pad, 4) for dm in (4, 8) for pad in (False, True)]
WIDE_VARIANTS += [("fp", dm, G, pad, 2) for dm in (8, 10) for G in (16, 32)
                  for pad in ((False, True) if ("fp", dm) in _PADDED else (False,))]

FIELD = {"fp": ("FIELD_FP", "FpField"), "c128": ("FIELD_C128", "C128Field")}


def lds_bytes_per_wave(field, N, DL, L, LT):
    """LDS of one 64-lane wavefront of a register kernel with per-point tables
    in LDS (mirrors Recursion::Lds in csrc/bg_kernel.h)."""
    if not LT:
        return 0
    ncur = N * (N + 1) // 2 - 1
    nprop = max(0, N * (N - 1) // 2 - 1)
    size = 4 if field == "fp" else 16
    scal = (2 * nprop + ncur) if field == "fp" else nprop
    vec = (N + 1) * DL if field == "fp" else N * DL
    return scal * (64 // L) * size + vec * 64 * size


# one wave per SIMD on all four SIMDs of a CU must fit the 160 KiB of LDS
REGISTER_VARIANTS = [v for v in REGISTER_VARIANTS if 4 * lds_bytes_per_wave(*v[:5]) <= 160 * 1024]


def generated_units():
    units = {}
    for field, N, DL, L, LT, W in REGISTER_VARIANTS:
        tag, cls = FIELD[field]
        # one unit per (field, n, lanes) keeps the units similar in size; from
        # n = 9 on each kernel takes minutes to compile, so each gets its own
        # unit and they compile in parallel
        name = f"inst_{field}_n{N + 1}_l{L}" + (f"_dl{DL}" if N >= 8 else "")
        lt = 'true' if LT else 'false'
        units.setdefault(name, []).append(
            f"BG_REGISTER_RECURSION_FP({N}, {DL}, {L}, {lt}, {W})" if field == "fp" else
            f"BG_REGISTER_RECURSION({tag}, {cls}, {N}, {DL}, {L}, {lt}, {W})")
    for field, dm in GENERIC_VARIANTS:
        tag, cls = FIELD[field]
        units.setdefault(f"inst_{field}_generic", []).append(
            f"BG_REGISTER_GENERIC({tag}, {cls}, {dm})")
    for field, dm, G, pad, lc in WIDE_VARIANTS:
        tag, cls = FIELD[field]
        units.setdefault(f"inst_{field}_wide_g{G}{'_pad' if pad else ''}{'_s' + str(lc) if lc > 1 else ''}", []).append(
            f"BG_REGISTER_WIDE({tag}, {cls}, {dm}, {G}, {'true' if pad else 'false'}, {lc})")
    out = {}
    for name, lines in units.items():
        out[name] = ("// generated by paper_2502_07060_amd/build.py\n"
                     "#include \"bg_wide.h\"\n#include \"bg_registry.h\"\n"
                     + "\n".join(lines) + "\n")
    return out


def unit_flags(src):
    """Extra flags per translation unit.  The n ≥ 8 register-resident
    recursion kernels hold so much of the register file that a few more
    registers cost no occupancy, so they are scheduled for instruction-level
    parallelism rather than occupancy (measured on gfx950: complex n = 8 about
    1.5 % and F_p n = 8 about 2.5 % faster than the default strategy).  At
    smaller n the same strategy costs F_p kernels a wave per SIMD, so they
    keep the default."""
    name = os.path.basename(src)
    if name.startswith("inst_") and any(f"_n{n}_" in name for n in (8, 9, 10, 11, 12)):
        return ["-mllvm", "-amdgpu-sched-strategy=max-ilp"]
    return []


def _digest(paths, extra=""):
    h = hashlib.sha256(extra.encode())
    for p in sorted(paths):
        with open(p, "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def build(incremental: bool = False, jobs: int | None = None, verbose: bool = False) -> str:
    gen = os.path.join(BUILD, "gen")
    objd = os.path.join(BUILD, "obj")
    if not incremental and os.path.isdir(BUILD):
        shutil.rmtree(BUILD)
    os.makedirs(gen, exist_ok=True)
    os.makedirs(objd, exist_ok=True)
    headers = [os.path.join(CSRC, f) for f in os.listdir(CSRC) if f.endswith(".h")]
    headers.append(os.path.join(INCLUDE, "bg.h"))
    hdr_digest = _digest(headers, " ".join(CXXFLAGS))

    sources = []
    for name, text in generated_units().items():
        path = os.path.join(gen, name + ".hip")
        old = open(path).read() if os.path.exists(path) else None
        if old != text:
            with open(path, "w") as f:
                f.write(text)
        sources.append(path)
    sources += [os.path.join(CSRC, f) for f in sorted(os.listdir(CSRC)) if f.endswith(".hip")]

    def compile_one(src):
        obj = os.path.join(objd, os.path.basename(src).replace(".hip", ".o"))
        stamp = obj + ".sha"
        key = _digest([src], hdr_digest + " ".join(unit_flags(src)))
        if incremental and os.path.exists(obj) and os.path.exists(stamp) and open(stamp).read() == key:
            return obj
        cmd = [HIPCC, *CXXFLAGS, *unit_flags(src), "-c", src, "-o", obj]
        r = subprocess.run(cmd, capture_output=True, text=True)
        if r.returncode != 0:
            raise RuntimeError(f"hipcc failed for {src}:\n{r.stderr[-6000:]}")
        if verbose and r.stderr.strip():
            print(r.stderr[-2000:], file=sys.stderr)
        with open(stamp, "w") as f:
            f.write(key)
        return obj

    jobs = jobs or min(8, os.cpu_count() or 4)
    # the biggest units (largest n) first, so the long poles start early
    def size_rank(src):
        m = re.search(r"inst_\w+?_n(\d+)_", os.path.basename(src))
        return -int(m.group(1)) if m else 0
    sources.sort(key=size_rank)
    with ThreadPoolExecutor(max_workers=jobs) as ex:
        objs = list(ex.map(compile_one, sources))
    tmp = LIB + ".tmp"
    cmd = [HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp, *objs]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stderr[-6000:]}")
    os.replace(tmp, LIB)
    return LIB


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--incremental", action="store_true")
    ap.add_argument("-j", "--jobs", type=int, default=None)
    ap.add_argument("-v", "--verbose", action="store_true")
    a = ap.parse_args(argv)
    print(build(a.incremental, a.jobs, a.verbose))


if __name__ == "__main__":
    main()
