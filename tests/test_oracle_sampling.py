"""The sampled full-size parity method is exact: one RK2 step of sampled blocks computed
on their two-deep neighbourhood equals the same blocks of a whole-grid step, bit for bit."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2108_12240_amd import inputs as I
from tests.test_gpu_fullsize import neighbourhood


@pytest.mark.parametrize("make", [lambda: I.case_torus(2, n=(64, 48, 48)), lambda: I.case4(nblocks=96, n0=48)])
def test_neighbourhood_step_equals_full_step(make):
    c = make()
    dt = 2e-3
    G = O.OracleGrid(c.params, c.blocks)
    U, P = G.init(c.prim)
    G.set_dt(dt)
    G.rk2_step(U, P)
    sel = [0, c.nblocks // 3, c.nblocks - 1]
    n1 = neighbourhood(c.blocks, c.params, sel)
    n2 = neighbourhood(c.blocks, c.params, n1)
    lmax = int(c.blocks[:, 0].max())
    if not (c.blocks[n2, 0] == lmax).any():
        n2 = sorted(set(n2) | {int(np.flatnonzero(c.blocks[:, 0] == lmax)[0])})
    S = O.OracleGrid(c.params, c.blocks[n2])
    prim_sub = np.concatenate([c.prim[:, c.ioff[b]:c.ioff[b + 1]] for b in n2], axis=1)
    Us, Ps = S.init(prim_sub)
    S.set_dt(dt)
    pos = {b: q for q, b in enumerate(n2)}
    s1 = [pos[b] for b in n1]
    s0 = [pos[b] for b in sel]
    U1, P1 = np.zeros_like(Us), np.zeros_like(Ps)
    S.fill_ghosts(Ps, s1)
    S.substep(Us, Us, Ps, U1, P1, 0.0, 1.0, s1)
    S.fill_ghosts(P1, s0)
    S.substep(Us, U1, P1, Us, Ps, 0.5, 0.5, s0)
    for b in sel:
        q = pos[b]
        full = G.interior_index()[G.ioff[b]:G.ioff[b + 1]]
        part = S.interior_index()[S.ioff[q]:S.ioff[q + 1]]
        assert np.array_equal(U[:, full], Us[:, part])
        assert np.array_equal(P[:, full], Ps[:, part])
