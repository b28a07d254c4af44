"""Pins of the oracle's block-tree ghost rule (restriction / prolongation between
levels of a 2:1-balanced tree of equal-size blocks) and of the tree generator.

What fixes the answers independently of the oracle's code: a linear field is
reproduced exactly by both restriction (the mean of the children of a cell is the
value at its centre) and limited linear prolongation (on linear data both one-sided
differences equal the slope); the children of one coarse cell average back to it;
a limited prolongation stays within the range of the coarse cell and its
neighbours; on a single-level grid the rule is the same-level copy rule; and the
generated tree partitions the domain with neighbours at most one level apart,
checked by brute force over pairs of leaves.
"""
import itertools

import numpy as np
import pytest

from oracle import oracle as O
from paper_2108_12240_amd import inputs as I
from tests import layout as L
from tests.cases import flat_tree_case, tree_volumes


def ghost_positions(c, G):
    """Per padded cell: (block, level, global level-l index per axis, is_ghost);
    padding slots of the x rows count as neither interior nor ghost."""
    rows = []
    for b, blk in enumerate(c.blocks):
        lev, s = int(blk[0]), blk[1:4]
        org = blk[4:7]
        x, y, z, pad = L.box_locals(c.params, s)
        loc = [x, y, z]
        ghost = np.zeros(loc[0].size, bool)
        for e in range(3):
            ghost |= (loc[e] < 0) | (loc[e] >= s[e])
        ghost &= ~pad
        glob = [org[e] + loc[e] for e in range(3)]
        rows.append((b, lev, glob, ghost))
    return rows


def linear_field(c, G, coef):
    """P (padded) with every variable = a + b.x at cell centres (level-0 units)."""
    P = np.full((9, G.ncp), np.nan)
    out_ghost_exp = np.full(G.ncp, np.nan)
    for (b, lev, glob, ghost) in ghost_positions(c, G):
        x = [(glob[e] + 0.5) / 2.0 ** lev for e in range(3)]
        val = coef[0] + coef[1] * x[0] + coef[2] * x[1] + coef[3] * x[2]
        sl = slice(int(G.off[b]), int(G.off[b + 1]))
        P[:, sl] = np.where(ghost, np.nan, val)[None, :]
        out_ghost_exp[sl] = np.where(ghost, val, np.nan)
    return P, out_ghost_exp


def away_from_edges(c, margin=3):
    """Mask of padded cells whose global position is at least `margin` cells (of
    their level) inside the domain on every axis (no wrap, no clamp involved)."""
    n0 = c.params["ncell0"]
    masks = []
    for blk in c.blocks:
        lev, s, org = int(blk[0]), blk[1:4], blk[4:7]
        x, y, z, pad = L.box_locals(c.params, s)
        ok = ~pad
        for e, v in enumerate((x, y, z)):
            glob = org[e] + v
            N = n0[e] * 2 ** lev
            ok &= (glob >= margin) & (glob < N - margin)
        masks.append(ok)
    return np.concatenate(masks)


@pytest.fixture(scope="module")
def two_level():
    return I.case_tree(n0=32, bs=8, levels=2, precision=I.PREC_FP64)


@pytest.fixture(scope="module")
def three_level():
    return I.case_tree(n0=32, bs=8, levels=3, precision=I.PREC_FP64)


def test_tree_partitions_domain_and_is_balanced(three_level):
    c = three_level
    n0 = c.params["ncell0"]
    blk = c.blocks
    # volume: each leaf covers (s / (n0 2^l))^3 of the unit cube; no leaf inside another
    vol = sum(np.prod([b[1 + e] / (n0[e] * 2.0 ** b[0]) for e in range(3)]) for b in blk)
    assert vol == pytest.approx(1.0, rel=1e-12)
    boxes = []
    for b in blk:
        lo = np.array([b[4 + e] / (n0[e] * 2.0 ** b[0]) for e in range(3)])
        hi = lo + np.array([b[1 + e] / (n0[e] * 2.0 ** b[0]) for e in range(3)])
        boxes.append((int(b[0]), lo, hi))
    # pairwise: no overlap; touching leaves (face, edge or corner, phi periodic)
    # differ by at most one level
    for (la, loa, hia), (lb, lob, hib) in itertools.combinations(boxes, 2):
        for shift in (-1.0, 0.0, 1.0):
            lob2, hib2 = lob.copy(), hib.copy()
            lob2[2] += shift
            hib2[2] += shift
            inter = np.minimum(hia, hib2) - np.maximum(loa, lob2)
            assert not (inter > 1e-12).all()
            if (inter > -1e-12).all():
                assert abs(la - lb) <= 1


@pytest.mark.parametrize("bad", ["overlap", "mixed_size", "odd_size", "shallow"])
def test_tree_rejects_invalid_block_lists(two_level, bad):
    c = two_level
    blocks = c.blocks.copy()
    if bad == "overlap":
        # a level-1 block inside a level-0 leaf
        b0 = int(np.flatnonzero(blocks[:, 0] == 0)[0])
        extra = blocks[b0].copy()
        extra[0] = 1
        extra[4:7] = 2 * blocks[b0, 4:7]
        blocks = np.vstack([blocks, extra])
    elif bad == "mixed_size":
        blocks = blocks.copy()
        blocks[0, 1:4] = 16
        blocks[0, 4:7] = 0
    elif bad == "odd_size":
        blocks = np.array([[0, 7, 7, 7, 0, 0, 0]], dtype=np.int32)
    else:
        # ghost layers deeper than half a block could reach past the adjacent leaf
        blocks = np.array([[0, 4, 4, 4, 0, 0, 0]], dtype=np.int32)
    with pytest.raises(Exception):
        O.OracleGrid(c.params, blocks)


def test_single_level_tree_equals_same_level_rule():
    c = I.case_torus(2, n=(32, 32, 32), bs=8)
    p0 = dict(c.params, amr=0)
    p1 = dict(c.params, amr=1)
    rng = np.random.default_rng(5)
    G0 = O.OracleGrid(p0, c.blocks)
    G1 = O.OracleGrid(p1, c.blocks)
    # the two grids lay their blocks out differently: map every slot of the first
    # layout to the same block-local position in the second
    i0, i1 = [], []
    for b, blk in enumerate(c.blocks):
        x, y, z, pad = L.box_locals(p0, blk[1:4])
        i0.append(G0.off[b] + np.nonzero(~pad)[0])
        i1.append(L.pad_index(p1, G1.off[b], blk[1:4], x[~pad], y[~pad], z[~pad]))
    i0, i1 = np.concatenate(i0), np.concatenate(i1)
    A = rng.standard_normal((9, G0.ncp))
    B = np.zeros((9, G1.ncp))
    B[:, i1] = A[:, i0]
    G0.fill_ghosts(A)
    G1.fill_ghosts(B)
    assert np.array_equal(A[:, i0], B[:, i1])


@pytest.mark.parametrize("coef", [(0.7, 0.3, -0.2, 0.05), (-1.0, 0.0, 1.25, 0.5)])
def test_linear_field_is_reproduced_by_restriction_and_prolongation(two_level, coef):
    c = two_level
    G = O.OracleGrid(c.params, c.blocks)
    P, expect = linear_field(c, G, coef)
    G.fill_ghosts(P)
    sel = np.isfinite(expect) & away_from_edges(c, margin=4)
    assert sel.sum() > 1000
    err = np.abs(P[:, sel] - expect[None, sel])
    assert err.max() <= 1e-12 * max(1.0, np.abs(expect[sel]).max())
    # both directions of the cross-level rule took part
    lev = np.concatenate([np.full(int(G.off[b + 1] - G.off[b]), int(c.blocks[b, 0])) for b in range(len(c.blocks))])
    assert (sel & (lev == 0)).any() and (sel & (lev == 1)).any()


def test_constant_field_is_kept(three_level):
    c = three_level
    G = O.OracleGrid(c.params, c.blocks)
    P = np.full((9, G.ncp), 0.75)        # dyadic: sums of eight copies are exact
    rows = ghost_positions(c, G)
    for (b, _, _, ghost) in rows:
        sl = slice(int(G.off[b]), int(G.off[b + 1]))
        P[:, sl][:, ghost] = np.nan
    G.fill_ghosts(P)
    assert np.array_equal(P, np.full_like(P, 0.75))


def fine_ghosts_by_coarse_cell(c, G):
    """For level-1 blocks: ghost slots grouped by the level-0 cell holding them,
    when that cell lies in a level-0 leaf (prolongation sources)."""
    n0 = c.params["ncell0"]
    leaf0 = {tuple(b[4:7] // b[1:4]): i for i, b in enumerate(c.blocks) if b[0] == 0}
    s = int(c.blocks[0, 1])
    groups = {}
    for (b, lev, glob, ghost) in ghost_positions(c, G):
        if lev != 1:
            continue
        base = int(G.off[b])
        for q in np.flatnonzero(ghost):
            gl = [int(glob[e][q]) for e in range(3)]
            if not all(0 <= gl[e] < 2 * n0[e] for e in range(3)):
                continue
            cc = tuple(v // 2 for v in gl)
            if tuple(v // s for v in cc) in leaf0:
                groups.setdefault((cc, b), []).append(base + q)
    return groups


def test_prolongation_children_average_to_the_coarse_cell(two_level):
    c = two_level
    G = O.OracleGrid(c.params, c.blocks)
    rng = np.random.default_rng(11)
    P = rng.uniform(0.5, 1.5, size=(9, G.ncp))
    Pin = P.copy()
    G.fill_ghosts(P)
    s = int(c.blocks[0, 1])
    idx = {tuple(b[4:7] // b[1:4]): i for i, b in enumerate(c.blocks) if b[0] == 0}
    g = c.params["nghost"]
    full = 0
    for (cc, b), slots in fine_ghosts_by_coarse_cell(c, G).items():
        if len(slots) != 8:
            continue
        full += 1
        cb = idx[tuple(v // s for v in cc)]
        loc = [cc[e] - int(c.blocks[cb, 4 + e]) for e in range(3)]
        qc = Pin[:, L.pad_index(c.params, G.off[cb], c.blocks[cb, 1:4], *loc)]
        assert np.allclose(P[:, slots].mean(axis=1), qc, rtol=0, atol=1e-14)
    assert full > 50


def test_prolongation_is_limited(two_level):
    """Every prolonged value lies within [min, max] of its coarse cell and the coarse
    cell's six neighbours (minmod slopes cannot overshoot)."""
    c = two_level
    G = O.OracleGrid(c.params, c.blocks)
    rng = np.random.default_rng(12)
    P = rng.uniform(-1.0, 1.0, size=(9, G.ncp))
    Pin = P.copy()
    G.fill_ghosts(P)
    # coarse neighbour values as the rule defines them: the fill of the coarse
    # blocks' own ghosts supplies them (same-level copies or restrictions)
    s = int(c.blocks[0, 1])
    g = c.params["nghost"]
    idx = {tuple(b[4:7] // b[1:4]): i for i, b in enumerate(c.blocks) if b[0] == 0}
    checked = 0
    for (cc, b), slots in fine_ghosts_by_coarse_cell(c, G).items():
        cb = idx[tuple(v // s for v in cc)]
        loc = [cc[e] - int(c.blocks[cb, 4 + e]) for e in range(3)]

        def at(a):
            return P[:, L.pad_index(c.params, G.off[cb], c.blocks[cb, 1:4], *a)]

        vals = [Pin[:, L.pad_index(c.params, G.off[cb], c.blocks[cb, 1:4], *loc)]]
        for d in range(3):
            for sgn in (-1, 1):
                a = list(loc)
                a[d] += sgn
                vals.append(at(a))
        vals = np.array(vals)
        lo, hi = vals.min(axis=0), vals.max(axis=0)
        for q in slots:
            assert (P[:, q] >= lo - 1e-15).all() and (P[:, q] <= hi + 1e-15).all()
            checked += 1
    assert checked > 200


def test_uniform_state_on_a_flat_tree_is_preserved_bit_for_bit():
    """Flat space, uniform dyadic state on a three-level tree: after one RK2 step the
    conserved state is unchanged bit for bit and the primitives are one uniform
    state (cross-level ghosts are exact copies of the uniform value)."""
    t = I.case_tree(n0=32, bs=8, levels=3, precision=I.PREC_FP64)
    params = dict(t.params, metric=I.METRIC_MINKOWSKI_CART, x_lo=[0.0, 0.0, 0.0], x_hi=[1.0, 1.0, 1.0],
                  bc=[[I.BC_PERIODIC, I.BC_PERIODIC]] * 3)
    state = np.array([1.0, 0.25, -0.125, 0.5, 0.75, 0.5, 0.25, -0.25, 0.0])
    prim = np.repeat(state[:, None], int(t.ioff[-1]), axis=1)
    G = O.OracleGrid(params, t.blocks)
    U0, P0 = G.init(prim)
    U, P = G.rk2_step(U0.copy(), P0.copy())
    assert np.array_equal(U, U0)
    Pi = G.unpack(P)
    assert (Pi == Pi[:, :1]).all()
    assert np.allclose(Pi[:, 0], state, rtol=1e-13, atol=1e-15)


@pytest.mark.parametrize("ndim", [3, 2])
def test_flux_correction_conserves_across_levels(ndim):
    """With the coarse faces on level boundaries set to the mean of the fine faces,
    the volume-weighted totals of D, S, tau and B are conserved to rounding on a
    periodic flat three-level tree (no sources); without that correction they
    drift at the 1e-4 level."""
    params, blocks, prim = flat_tree_case(ndim=ndim)
    G = O.OracleGrid(params, blocks)
    U, P = G.init(prim)
    vol = tree_volumes(blocks, int(params["ncell0"][0]), ndim)
    idx = G.interior_index()

    def totals(U):
        Ui = U[:, idx] if U.shape[1] == G.ncp else U
        return np.array([np.sum(Ui[q] * vol) for q in range(8)]), np.array([np.sum(np.abs(Ui[q]) * vol)
                                                                              for q in range(8)])
    t0, scale = totals(U)
    for _ in range(2):
        G.rk2_step(U, P)
    t1, _ = totals(U)
    st = G.stats()
    assert st["c2p_fail"] == 0
    assert (np.abs(t1 - t0) <= 1e-13 * np.maximum(scale, 1e-300)).all(), (t1 - t0) / scale


def test_two_d_tree_partitions_the_domain():
    """The 2-D tree's leaves cover the (ln r, theta) domain exactly once, levels
    differ by at most one across faces, edges and corners, and a uniform flat
    state is preserved bit for bit."""
    c = I.case_tree_2d(n0=64, bs=8, levels=3)
    assert set(np.unique(c.blocks[:, 0])) == {0, 1, 2}
    # rasterise each leaf onto the finest level: every fine cell is covered once
    fine = 64 * 4
    cover = np.zeros((fine, fine), np.int32)
    lev = np.full((fine, fine), -1, np.int32)
    for l, s0, s1, s2, o0, o1, o2 in c.blocks:
        f = 4 >> int(l)
        assert s2 == 1 and o2 == 0
        cover[o0 * f:(o0 + s0) * f, o1 * f:(o1 + s1) * f] += 1
        lev[o0 * f:(o0 + s0) * f, o1 * f:(o1 + s1) * f] = l
    assert (cover == 1).all()
    # 2:1 balance across faces, edges and corners
    for d0, d1 in [(1, 0), (0, 1), (1, 1), (1, -1)]:
        a = lev[max(d0, 0):fine + min(d0, 0), max(d1, 0):fine + min(d1, 0)]
        b = lev[max(-d0, 0):fine + min(-d0, 0), max(-d1, 0):fine + min(-d1, 0)]
        assert np.abs(a - b).max() <= 1
    params = dict(c.params, metric=I.METRIC_MINKOWSKI_CART, x_lo=[0.0, 0.0, 0.0], x_hi=[1.0, 1.0, 1.0],
                  bc=[[I.BC_PERIODIC, I.BC_PERIODIC]] * 3)
    state = np.array([1.0, 0.25, -0.125, 0.5, 0.75, 0.5, 0.25, -0.25, 0.0])
    prim = np.repeat(state[:, None], int(c.ioff[-1]), axis=1)
    G = O.OracleGrid(params, c.blocks)
    U0, P0 = G.init(prim)
    U, P = G.rk2_step(U0.copy(), P0.copy())
    assert np.array_equal(U, U0)
