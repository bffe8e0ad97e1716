"""Host checks of the spatial-order statement used by the GPU order tests:
the Hilbert index is a bijection of the grid whose consecutive cells are
edge neighbours (the defining property of the curve), and the Morton key
interleaves bits as stated."""
import numpy as np
import pytest

from tests import order_ref


@pytest.mark.parametrize("b", [1, 2, 3, 4, 5, 6])
def test_hilbert_bijective_and_continuous(b):
    side = 1 << b
    qx, qy = np.meshgrid(np.arange(side), np.arange(side), indexing="ij")
    h = order_ref.hilbert(qx.ravel(), qy.ravel(), b)
    assert sorted(h.tolist()) == list(range(side * side))
    inv = np.empty((side * side, 2), dtype=np.int64)
    inv[h.astype(np.int64)] = np.stack([qx.ravel(), qy.ravel()], 1)
    steps = np.abs(np.diff(inv, axis=0)).sum(1)
    assert np.all(steps == 1)
    # the curve starts at the origin and ends on the x axis's far corner
    assert tuple(inv[0]) == (0, 0)
    assert tuple(inv[-1]) == (side - 1, 0)


def test_hilbert_16_bit_range():
    q = np.array([0, 65535, 12345, 65535], dtype=np.uint64)
    r = np.array([0, 0, 54321, 65535], dtype=np.uint64)
    h = order_ref.hilbert(q, r, 16)
    assert h.max() < 2 ** 32
    assert h[0] == 0 and h[1] == 2 ** 32 - 1


def test_morton_interleave():
    x = np.array([[0.0, 0.0, 0.0], [1.0, 0.0, 0.0], [0.0, 1.0, 0.0], [0.0, 0.0, 1.0],
                  [1.0, 1.0, 1.0]])
    k = order_ref.keys(x)
    top = (1 << 10) - 1
    want = [0, 0, 0, 0, 0]
    for i, row in enumerate(x):
        v = 0
        for bit in range(10):
            for d in range(3):
                q = top if row[d] == 1.0 else 0
                v |= ((q >> bit) & 1) << (bit * 3 + d)
        want[i] = v
    assert k.tolist() == want
    assert k[1] < k[2] < k[3] < k[4]


def test_quantise_edges_and_order_is_stable():
    x = np.array([[2.0], [np.nan], [2.0], [-1.0], [5.0]])
    q = order_ref.keys(x)
    assert q[3] == 0 and q[1] == 0 and q[4] == 2 ** 32 - 1
    assert order_ref.spatial_order(x).tolist() == [1, 3, 0, 2, 4]
    flat = np.ones((4, 2))
    assert order_ref.spatial_order(flat).tolist() == [0, 1, 2, 3]
