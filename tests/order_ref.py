"""Plain numpy statement of the spatial order the library computes (a test
helper: keys and a stable sort, written independently of the HIP code).

Coordinates are quantised over the bounding box of X to b bits,
q = floor((v - lo) / (hi - lo) * (2^b - 1)), with b = 32 for D = 1, 16 for
D = 2 and floor(32 / D) otherwise; NaN and a flat box give 0.  The key is the
Hilbert index of (q_0, q_1) for D = 2 and the bit interleaving of the q_d
(bit k of coordinate d at position k*D + d) for other D.  The order sorts
the keys stably (ties keep index order).
"""
import numpy as np


def order_bits(d):
    return 32 if d == 1 else (16 if d == 2 else 32 // d)


def quantise(v, lo, hi, b):
    top = float((1 << b) - 1)
    if not hi > lo:
        return np.zeros(v.shape, dtype=np.uint64)
    t = (v - lo) / (hi - lo)
    t = np.where(t >= 0.0, t, 0.0)          # also maps NaN to 0
    t = np.minimum(t, 1.0)
    return np.floor(t * top).astype(np.uint64)


def hilbert(qx, qy, b):
    """Hilbert index of cells (qx, qy) of a 2^b x 2^b grid (arrays)."""
    qx = np.asarray(qx, dtype=np.uint64).copy()
    qy = np.asarray(qy, dtype=np.uint64).copy()
    full = np.uint64((1 << b) - 1)
    h = np.zeros(qx.shape, dtype=np.uint64)
    for k in range(b - 1, -1, -1):
        s = np.uint64(1 << k)
        rx = ((qx & s) != 0).astype(np.uint64)
        ry = ((qy & s) != 0).astype(np.uint64)
        h += s * s * ((np.uint64(3) * rx) ^ ry)
        flip = (ry == 0) & (rx == 1)
        qx[flip] ^= full
        qy[flip] ^= full
        swap = ry == 0
        tx = qx[swap].copy()
        qx[swap] = qy[swap]
        qy[swap] = tx
    return h


def keys(x):
    x = np.asarray(x, dtype=np.float64)
    n, d = x.shape
    b = order_bits(d)
    with np.errstate(invalid="ignore", all="ignore"):
        lo = np.array([np.nanmin(x[:, k]) if np.any(~np.isnan(x[:, k])) else np.inf
                       for k in range(d)])
        hi = np.array([np.nanmax(x[:, k]) if np.any(~np.isnan(x[:, k])) else -np.inf
                       for k in range(d)])
        q = [quantise(x[:, k], lo[k], hi[k], b) for k in range(d)]
    if d == 1:
        return q[0]
    if d == 2:
        return hilbert(q[0], q[1], b)
    key = np.zeros(n, dtype=np.uint64)
    for k in range(b):
        for dd in range(d):
            key |= ((q[dd] >> np.uint64(k)) & np.uint64(1)) << np.uint64(k * d + dd)
    return key


def spatial_order(x):
    return np.argsort(keys(x), kind="stable").astype(np.int64)
