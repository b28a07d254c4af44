"""Small synthetic cases shared by the oracle pins and the GPU tests."""
import numpy as np

from paper_2108_12240_amd import inputs as I


def flat_tree_case(levels=3, ndim=3):
    """Flat periodic unit cube (square in 2-D) on the refinement pattern of the torus
    tree, with a smooth non-uniform state (density and pressure waves, a moving
    field)."""
    if ndim == 3:
        t = I.case_tree(n0=32, bs=8, levels=levels, precision=I.PREC_FP64)
    else:
        t = I.case_tree_2d(n0=64, bs=8, levels=levels, precision=I.PREC_FP64)
    params = dict(t.params, metric=I.METRIC_MINKOWSKI_CART, spin=0.0, x_lo=[0.0, 0.0, 0.0], x_hi=[1.0, 1.0, 1.0],
                  bc=[[I.BC_PERIODIC, I.BC_PERIODIC]] * 3)
    n0 = int(params["ncell0"][0])
    cols = []
    for blk in t.blocks:
        g0, g1, g2 = I._block_cells(blk)
        n = n0 * 2 ** int(blk[0])
        x, y = (g0 + 0.5) / n, (g1 + 0.5) / n
        z = (g2 + 0.5) / n if ndim == 3 else np.full(x.size, 0.25)
        q = np.zeros((9, x.size))
        q[0] = 1.0 + 0.3 * np.sin(2 * np.pi * x) * np.cos(2 * np.pi * y)
        q[1] = 0.2 * np.sin(2 * np.pi * z)
        q[2] = 0.1 * np.cos(2 * np.pi * x)
        q[3] = 0.05
        q[4] = 1.0 + 0.2 * np.cos(2 * np.pi * (x + z))
        q[5] = 0.3
        q[6] = 0.1 * np.sin(2 * np.pi * x)
        q[7] = 0.2
        cols.append(q)
    return params, t.blocks, np.concatenate(cols, axis=1)


def tree_volumes(blocks, n0, ndim=3):
    """Coordinate volume (area in 2-D) of every interior cell (block-major) of a
    unit-cube tree."""
    return np.concatenate([np.full(int(np.prod(b[1:4])), (1.0 / (n0 * 2 ** int(b[0]))) ** ndim) for b in blocks])
