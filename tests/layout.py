"""The state layout of P (the data contract of the library and the oracle),
restated for the tests. Each block's region holds the cells and ghost slots of
its (size + 2g) box (g layers per side along every axis in use).
Independent patches (amr = 0): the interior cells first (x fastest), then the
ghost slots in box order with the interior skipped, the region rounded up to 32
slots. Block trees: the padded box, x fastest; along x the interior starts at
slot xo = roundup(g, A) of a row of roundup(xo + size + g, A) slots, A = 16 for
a double state and 1 for a float state. Unnamed slots are padding."""
import numpy as np


def interior_first(params):
    return not int(params.get("amr", 0))


def x_layout(params):
    xa = 1 if interior_first(params) or int(params.get("precision", 0)) == 1 else 16
    g = int(params["nghost"])
    return xa, -(-g // xa) * xa


def ghost_box(params, size):
    g, nd = int(params["nghost"]), int(params["ndim"])
    return (int(size[0]) + 2 * g, int(size[1]) + 2 * g, int(size[2]) + (2 * g if nd > 2 else 0))


def region_size(params, size):
    if interior_first(params):
        return -(-int(np.prod(ghost_box(params, size))) // 32) * 32
    return int(np.prod(box(params, size)))


def box(params, size):
    """Padded boxes: the box's extents in slots."""
    g, nd = int(params["nghost"]), int(params["ndim"])
    xa, xo = x_layout(params)
    return (-(-(xo + int(size[0]) + g) // xa) * xa, int(size[1]) + 2 * g,
            int(size[2]) + (2 * g if nd > 2 else 0))


def box_locals(params, size):
    """Local coordinates of every slot of a block's region, in storage order, and
    the mask of its padding slots."""
    g, nd = int(params["nghost"]), int(params["ndim"])
    gz = g if nd > 2 else 0
    s = [int(v) for v in size]
    if interior_first(params):
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
    n0, n1, n2 = box(params, size)
    xo = x_layout(params)[1]
    k, j, i = np.meshgrid(np.arange(n2), np.arange(n1), np.arange(n0), indexing="ij")
    x, y, z = i.ravel() - xo, j.ravel() - g, k.ravel() - gz
    pad = (x < -g) | (x >= s[0] + g)
    return x, y, z, pad


def _lut(key):
    params = dict(amr=key[0], precision=key[1], nghost=key[2], ndim=key[3])
    x, y, z, pad = box_locals(params, key[4:])
    return {(int(a), int(b), int(c)): q for q, (a, b, c) in enumerate(zip(x, y, z)) if not pad[q]}


_LUTS = {}


def pad_index(params, off_b, size, i, j, k):
    """Index in P of block-local position (i, j, k) (interior cell or ghost slot)."""
    key = (int(params.get("amr", 0)), int(params.get("precision", 0)), int(params["nghost"]),
           int(params["ndim"])) + tuple(int(v) for v in size)
    if key not in _LUTS:
        _LUTS[key] = _lut(key)
    lut = _LUTS[key]
    i, j, k = np.broadcast_arrays(np.asarray(i), np.asarray(j), np.asarray(k))
    out = np.array([lut[(int(a), int(b), int(c))] for a, b, c in zip(i.ravel(), j.ravel(), k.ravel())])
    out = int(off_b) + out.reshape(i.shape)
    return int(out) if out.ndim == 0 else out
