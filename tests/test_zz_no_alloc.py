"""bhac_substep_noalloc (face-flux scratch in a static device array, no allocation)
against bhac_substep, through the C ABI: two grids built alike, one advanced by each
entry point, compared bit for bit; then a second, smaller grid (the static array
keeps the first call's contents, which must not leak into the second); and grids
whose face fluxes exceed the static array are rejected before any launch."""
import numpy as np
import pytest

from paper_2108_12240_amd import bhac as B
from paper_2108_12240_amd import inputs as I

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    import torch as T
    assert T.cuda.is_available(), "GPU tests need a ROCm device"
    return T


def advance(c, noalloc, steps=2):
    """`steps` SSP-RK2 steps with the CFL time step, every substep through the chosen
    entry point; returns the final U, P (host) and the time-step state."""
    import torch
    G = B.Grid(c.params, c.blocks)
    U, P = G.init(c.prim)
    U1, P1 = G.new_state("U"), G.new_state("P")
    sub = G.substep_noalloc if noalloc else G.substep
    for _ in range(steps):
        sub(U, U, P, U1, P1, 0.0, 1.0)
        sub(U, U1, P1, U, P, 0.5, 0.5)
    torch.cuda.synchronize()
    out = (G.unpack(U), G.unpack(P), G.timestep(), G.stats())
    G.close()
    return out


CASES = [
    ("torus_48x32x32_mixed", lambda: I.case_torus(2, n=(48, 32, 32)), I.PREC_MIXED),
    ("torus_32_fp64", lambda: I.case_torus(2, n=32), I.PREC_FP64),
    ("amr_like_24_mixed", lambda: I.case4(nblocks=24, n0=48), I.PREC_MIXED),
    ("case1_fp64", lambda: I.case1(), I.PREC_FP64),
]


@pytest.mark.parametrize("prec", [I.PREC_MIXED, I.PREC_FP64])
def test_noalloc_substep_equals_substep_on_two_calls(torch, prec):
    """A larger grid, then a smaller one: each equal to bhac_substep bit for bit."""
    for name, make in (("torus_48x32x32", lambda: I.case_torus(2, n=(48, 32, 32))),
                       ("torus_32x16x16", lambda: I.case_torus(2, n=(32, 16, 16)))):
        c = make()
        c.params = dict(c.params, precision=prec, fused=0)
        print(f"\n[noalloc] {name} prec={prec}", flush=True)
        ref = advance(c, False)
        got = advance(c, True)
        assert np.array_equal(got[0], ref[0]) and np.array_equal(got[1], ref[1])
        assert got[2] == ref[2] and got[3] == ref[3]


@pytest.mark.parametrize("name,make,prec", CASES)
def test_noalloc_substep_equals_substep(torch, name, make, prec):
    c = make()
    c.params = dict(c.params, precision=prec, fused=0)
    print(f"\n[noalloc] {name}", flush=True)
    ref = advance(c, False, steps=1)
    got = advance(c, True, steps=1)
    assert np.array_equal(got[0], ref[0]) and np.array_equal(got[1], ref[1])


def test_noalloc_rejects_grids_beyond_the_static_scratch(torch):
    # 128^3 in FP64: 3 x 9 x 2.2 M faces x 8 bytes, far beyond 64 MiB
    c = I.case_torus(2, n=128)
    c.params = dict(c.params, precision=I.PREC_FP64, fused=0)
    G = B.Grid(c.params, c.blocks)
    U, P = G.init(c.prim)
    U1, P1 = G.new_state("U"), G.new_state("P")
    with pytest.raises(B.BhacError) as ei:
        G.substep_noalloc(U, U, P, U1, P1, 0.0, 1.0)
    assert ei.value.code == B.BHAC_EINVAL and "static scratch" in str(ei.value)
    G.close()


def test_noalloc_rejects_the_block_tiled_path(torch):
    c = I.case_torus(2, n=(48, 32, 32))
    c.params = dict(c.params, precision=I.PREC_MIXED, fused=1)
    G = B.Grid(c.params, c.blocks)
    U, P = G.init(c.prim)
    U1, P1 = G.new_state("U"), G.new_state("P")
    with pytest.raises(B.BhacError) as ei:
        G.substep_noalloc(U, U, P, U1, P1, 0.0, 1.0)
    assert ei.value.code == B.BHAC_EUNSUPPORTED
    G.close()
