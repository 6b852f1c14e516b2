"""The allocation-free batched entry point (bg_batch_run_noalloc, for callers
that cannot allocate device memory) against the allocating queue form
(bg_batch_run_ex with BG_BATCH_QUEUE): identical outputs and statuses, bit
for bit, on two calls in a row, the second with fewer groups and fewer
points (the library's fixed queue array keeps the first call's contents)."""
import numpy as np
import pytest

from paper_2502_07060_amd import bg

from test_gpu_batch import QSHAPES, make_groups
from test_gpu_parity import torch_dev  # noqa: F401

pytestmark = pytest.mark.gpu


def _snapshot(torch_dev, data):
    torch, _ = torch_dev
    torch.cuda.synchronize()
    return [(x["out"][:x["m"]].cpu().numpy().view(np.uint8).copy(), x["st"][:x["m"]].cpu().numpy().copy())
            for x in data]


def _poison(data):
    for x in data:
        x["out"].fill_(-1 if x["field"] == "fp" else complex(7, 7))
        x["st"].fill_(9)


def _compare(torch_dev, shapes):
    groups, data = make_groups(torch_dev, shapes)
    bg.bg_batch_run_ex(groups, bg.BG_BATCH_QUEUE)
    ref = _snapshot(torch_dev, data)
    _poison(data)
    bg.bg_batch_run_noalloc(groups)
    got = _snapshot(torch_dev, data)
    for x, (ro, rs), (go, gs) in zip(data, ref, got):
        assert np.array_equal(rs, gs), (x["field"], x["n"], x["d"])
        assert np.array_equal(ro, go), (x["field"], x["n"], x["d"])
        assert x["m"] == 0 or (rs != 9).all()


def test_noalloc_matches_queue_form_twice(torch_dev):
    _compare(torch_dev, QSHAPES)
    # second call: fewer groups, fewer points each
    smaller = [(f, n, d, m // 3) for f, n, d, m in QSHAPES[:5]]
    _compare(torch_dev, smaller)
