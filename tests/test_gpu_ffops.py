"""Standalone Z_p operations on the GPU (next row f4) against
oracle/ffops.py, value by value: contractions with the second operand per
event or shared, shapes from a scalar product to tall, wide and long ones
(every J mod 4 for the fold schedule, K across the blocks of eight columns),
ragged ld, non-canonical inputs; elementwise and scalar division with zero
and non-canonical divisors."""
import numpy as np
import pytest

from oracle import ffops
from paper_2502_07060_amd import bg
from paper_2502_07060_amd import inputs as I

from test_gpu_parity import torch_dev  # noqa: F401

pytestmark = pytest.mark.gpu
P = I.DEFAULT_PRIME


def dev_u32(torch_dev, a):
    torch, dev = torch_dev
    return torch.from_numpy(np.ascontiguousarray(np.asarray(a, np.int64).astype(np.uint32)).view(np.int32)).to(dev)


@pytest.mark.parametrize("Id,J,K", [(1, 1, 1), (1, 6, 1), (6, 6, 6), (5, 8, 8), (9, 3, 8), (4, 7, 9), (3, 17, 16), (10, 10, 10),
                                    (2, 100, 3), (1, 5, 33)])
@pytest.mark.parametrize("batched", [True, False])
def test_contract(torch_dev, Id, J, K, batched):
    torch, _ = torch_dev
    p = P if (Id + J + K) % 2 else 2147483587
    rng = np.random.default_rng(Id * 1000 + J * 10 + K + batched)
    n, ld = 37, 40
    x = rng.integers(0, p, size=(Id, J, ld))
    y = rng.integers(0, p, size=(J, K, ld) if batched else (J, K))
    x[0, 0, 3] = p + 1             # a non-canonical residue in event 3
    if batched:
        y[J - 1, K - 1, 7] = 0xFFFFFFFF
    z, st = bg.bg_fp_contract(p, dev_u32(torch_dev, x), dev_u32(torch_dev, y), y_batched=batched, npts=n)
    torch.cuda.synchronize()
    z = z.cpu().numpy().view(np.uint32)[:, :, :n].astype(np.int64)
    st = st.cpu().numpy()
    xe = [x[:, :, q].tolist() for q in range(n)]
    ye = [y[:, :, q].tolist() for q in range(n)] if batched else y.tolist()
    zo = ffops.contract(xe, ye, p, batched_y=batched)
    for q in range(n):
        bad = q == 3 or (batched and q == 7)
        assert st[q] == (2 if bad else 0), q
        if bad:
            assert (z[:, :, q] == 0xFFFFFFFF).all()
        else:
            assert np.array_equal(z[:, :, q], np.array(zo[q])), q


@pytest.mark.parametrize("count", [1, 15, 16, 17, 1000])
def test_divide(torch_dev, count):
    torch, _ = torch_dev
    rng = np.random.default_rng(count)
    x = rng.integers(0, P, size=count)
    y = rng.integers(1, P, size=count)
    if count > 4:
        y[2] = 0
        x[4] = P + 9
    z, st = bg.bg_fp_divide(P, dev_u32(torch_dev, x), dev_u32(torch_dev, y))
    torch.cuda.synchronize()
    z, st = z.cpu().numpy().view(np.uint32), st.cpu().numpy()
    so, vo = ffops.divide([int(a) for a in x], [int(b) for b in y], P)
    for i in range(count):
        if x[i] >= P:
            assert st[i] == 2 and z[i] == 0xFFFFFFFF
        elif so[i]:
            assert st[i] == 1 and z[i] == 0xFFFFFFFF
        else:
            assert st[i] == 0 and z[i] == vo[i]
    ys = 123456789
    z2, st2 = bg.bg_fp_divide(P, dev_u32(torch_dev, x), ys)
    torch.cuda.synchronize()
    z2, st2 = z2.cpu().numpy().view(np.uint32), st2.cpu().numpy()
    so2, vo2 = ffops.divide([int(a) for a in x], [ys] * count, P)
    for i in range(count):
        if x[i] >= P:
            assert st2[i] == 2
        else:
            assert st2[i] == 0 and z2[i] == vo2[i]
