"""The padded state layout (the data contract of the library and the oracle),
restated for the tests: g ghost layers per side along y and z; along x the
interior starts at slot xo = roundup(g, A) of a row of roundup(xo + size + g, A)
slots, A = 16 for a double state (128-byte rows) and 1 for a float state (rows of
size + 2g); slots further than g from the interior along x are padding."""
import numpy as np


def x_layout(params):
    xa = 1 if int(params.get("precision", 0)) == 1 else 16
    g = int(params["nghost"])
    return xa, -(-g // xa) * xa


def origin(params):
    """Padded coordinates of local cell (0, 0, 0)."""
    g, nd = int(params["nghost"]), int(params["ndim"])
    return x_layout(params)[1], g, (g if nd > 2 else 0)


def box(params, size):
    g, nd = int(params["nghost"]), int(params["ndim"])
    xa, xo = x_layout(params)
    return (-(-(xo + int(size[0]) + g) // xa) * xa, int(size[1]) + 2 * g,
            int(size[2]) + (2 * g if nd > 2 else 0))


def pad_index(params, off_b, size, i, j, k):
    n0, n1, _ = box(params, size)
    o = origin(params)
    return int(off_b) + ((k + o[2]) * n1 + (j + o[1])) * n0 + (i + o[0])


def box_locals(params, size):
    """Local coordinates of every slot of a block's padded box, in storage order,
    and the mask of its padding slots."""
    n0, n1, n2 = box(params, size)
    o = origin(params)
    k, j, i = np.meshgrid(np.arange(n2), np.arange(n1), np.arange(n0), indexing="ij")
    x, y, z = i.ravel() - o[0], j.ravel() - o[1], k.ravel() - o[2]
    g = int(params["nghost"])
    pad = (x < -g) | (x >= int(size[0]) + g)
    return x, y, z, pad
