"""GPU time-step state through a sequence of calls, against the oracle's.

The device keeps dt, dt_next, c_h and kappa; a substep with a = 0 latches dt (and
c_h, kappa) from the wave speeds of the substep before it, a fixed dt (set_dt > 0)
overrides the CFL value and set_dt(0) returns to it. The sequence mixes RK stages,
host reads between them, a fixed dt and the return to the CFL time step; after
every call the host-visible state must equal the oracle's (FP64, 2-D SRMHD block)."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2108_12240_amd import bhac as B
from paper_2108_12240_amd import inputs as I

pytestmark = pytest.mark.gpu

KEYS = ("dt", "dt_next", "ch", "kappa")


def test_time_step_state_follows_the_oracle():
    import torch
    c = I.case1()
    G = B.Grid(c.params, c.blocks)
    Og = O.OracleGrid(c.params, c.blocks)
    U, P = G.init(c.prim)
    Uo, Po = Og.init(c.prim)
    U1, P1 = G.new_state("U"), G.new_state("P")
    U1o, P1o = np.zeros_like(Uo), np.zeros_like(Po)

    def check(tag, read=True):
        if not read:
            return
        ts, so = G.timestep(), Og.stats()
        for k in KEYS:
            assert ts[k] == pytest.approx(so[k], rel=1e-12), (tag, k, ts[k], so[k])

    def stage(a):
        if a == 0.0:
            Og.fill_ghosts(Po)
            G.substep(U, U, P, U1, P1, 0.0, 1.0)
            Og.substep(Uo, Uo, Po, U1o, P1o, 0.0, 1.0)
        else:
            Og.fill_ghosts(P1o)
            G.substep(U, U1, P1, U, P, 0.5, 0.5)
            Og.substep(Uo, U1o, P1o, Uo, Po, 0.5, 0.5)

    check("init")
    stage(0.0)
    check("stage 1, read at once")
    stage(0.5)
    stage(0.0)                     # no read between: the latch finishes the pending maxima itself
    stage(0.5)
    check("two steps")
    G.set_dt(2.5e-3)
    Og.set_dt(2.5e-3)
    check("fixed dt set")
    stage(0.0)
    stage(0.5)
    check("step with fixed dt")
    G.set_dt(0.0)                  # back to the CFL time step, without a read before
    Og.set_dt(0.0)
    stage(0.0)
    check("latched after the switch")
    stage(0.5)
    stage(0.0)
    stage(0.5)
    check("CFL steps again")
    torch.cuda.synchronize()
    eU = np.abs(G.unpack(U) - Uo[:, Og.interior_index()]).max()
    G.close()
    assert eU <= 1e-12 * np.abs(Uo).max()
