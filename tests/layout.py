"""The state layout of P (the data contract of the library and the oracle),
restated for the tests by enumeration: each block's region holds first its
interior cells (x fastest), then the ghost slots of its (size + 2g) box (g layers
per side along every axis in use) in box order with the interior skipped, the
region rounded up to 32 slots; the remaining slots are padding."""
import numpy as np


def ghost_box(params, size):
    g, nd = int(params["nghost"]), int(params["ndim"])
    return (int(size[0]) + 2 * g, int(size[1]) + 2 * g, int(size[2]) + (2 * g if nd > 2 else 0))


def region_size(params, size):
    return -(-int(np.prod(ghost_box(params, size))) // 32) * 32


def box_locals(params, size):
    """Local coordinates of every slot of a block's region, in storage order, and
    the mask of its padding slots."""
    g, nd = int(params["nghost"]), int(params["ndim"])
    gz = g if nd > 2 else 0
    s = [int(v) for v in size]
    k, j, i = np.meshgrid(np.arange(s[2]), np.arange(s[1]), np.arange(s[0]), indexing="ij")
    inner = [i.ravel(), j.ravel(), k.ravel()]
    k, j, i = np.meshgrid(np.arange(-gz, s[2] + gz), np.arange(-g, s[1] + g), np.arange(-g, s[0] + g),
                          indexing="ij")
    i, j, k = i.ravel(), j.ravel(), k.ravel()
    out = ~((i >= 0) & (i < s[0]) & (j >= 0) & (j < s[1]) & (k >= 0) & (k < s[2]))
    n = region_size(params, size)
    npad = n - inner[0].size - int(out.sum())
    big = np.full(npad, 10 ** 6)
    x = np.concatenate([inner[0], i[out], big])
    y = np.concatenate([inner[1], j[out], big])
    z = np.concatenate([inner[2], k[out], big])
    pad = np.zeros(n, bool)
    pad[n - npad:] = True
    return x, y, z, pad


def _lut(key):
    params = dict(nghost=key[0], ndim=key[1])
    x, y, z, pad = box_locals(params, key[2:])
    return {(int(a), int(b), int(c)): q for q, (a, b, c) in enumerate(zip(x, y, z)) if not pad[q]}


_LUTS = {}


def pad_index(params, off_b, size, i, j, k):
    """Index in P of block-local position (i, j, k) (interior cell or ghost slot)."""
    key = (int(params["nghost"]), int(params["ndim"])) + tuple(int(v) for v in size)
    if key not in _LUTS:
        _LUTS[key] = _lut(key)
    lut = _LUTS[key]
    i, j, k = np.broadcast_arrays(np.asarray(i), np.asarray(j), np.asarray(k))
    out = np.array([lut[(int(a), int(b), int(c))] for a, b, c in zip(i.ravel(), j.ravel(), k.ravel())])
    out = int(off_b) + out.reshape(i.shape)
    return int(out) if out.ndim == 0 else out
