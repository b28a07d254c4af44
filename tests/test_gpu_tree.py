"""GPU parity on block trees (amr = 1): the cross-level ghost fill and whole steps
against the oracle."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2108_12240_amd import bhac as B
from paper_2108_12240_amd import inputs as I
from tests.cases import flat_tree_case, tree_volumes
from tests.parity import rel_l1

pytestmark = pytest.mark.gpu

FP64_TOL = 1e-11
MIXED_TOL = 1e-5


def banner(msg):
    print(f"\n[tree] {msg}", flush=True)


@pytest.fixture(scope="module")
def torch():
    import torch as T
    assert T.cuda.is_available(), "GPU tests need a ROCm device"
    return T


def tree(prec, ndim=3, levels=3):
    if ndim == 3:
        c = I.case_tree(n0=32, bs=8, levels=levels, precision=prec)
    else:
        c = I.case_tree_2d(n0=64, bs=8, levels=levels, precision=prec)
    c.params = dict(c.params, precision=prec, fused=0)
    return c


@pytest.mark.parametrize("ndim", [3, 2])
@pytest.mark.parametrize("prec", [I.PREC_FP64, I.PREC_MIXED])
def test_fill_matches_oracle_bitwise(torch, prec, ndim):
    """Every ghost slot (same-level copies, restrictions, prolongations, clamps)
    equals the oracle's value, rounded to the state's precision."""
    c = tree(prec, ndim)
    banner(f"fill {c.name} prec={prec}")
    G = B.Grid(c.params, c.blocks)
    Og = O.OracleGrid(c.params, c.blocks)
    rng = np.random.default_rng(21)
    vals = rng.uniform(0.5, 1.5, size=(9, G.ncp))
    if prec == I.PREC_MIXED:
        vals = vals.astype(np.float32).astype(np.float64)
    ref = vals.copy()
    Og.fill_ghosts(ref)
    P = torch.from_numpy(vals).to("cuda", G.pdtype)
    G.fill_ghosts(P)
    got = P.cpu().double().numpy()
    if prec == I.PREC_MIXED:
        ref = ref.astype(np.float32).astype(np.float64)
    diff = got != ref
    assert not diff.any(), f"{int(diff.sum())} values differ, first at {np.argwhere(diff)[:3]}"
    # the cross-level cases were exercised: some ghost values are not copies of any input value
    G.close()


@pytest.mark.parametrize("ndim", [3, 2])
@pytest.mark.parametrize("prec", [I.PREC_FP64, I.PREC_MIXED])
def test_substep_reads_only_cross_level_ghosts_it_writes(torch, prec, ndim):
    """With every ghost slot of P_stage poisoned, a substep gives bit-identical
    results: same-level halos come from neighbours, cross-level ones are rebuilt
    from interiors before use."""
    c = tree(prec, ndim)
    banner(f"halo {c.name} prec={prec}")
    G = B.Grid(c.params, c.blocks)
    U, P = G.init(c.prim)
    G.set_dt(1e-3)
    ghost = np.ones(G.ncp, bool)
    ghost[G.interior_index()] = False
    gmask = torch.from_numpy(ghost).to(P.device)
    outs = []
    for poison in (False, True):
        Pin = P.clone()
        if poison:
            Pin[:, gmask] = float("nan")
        U1 = G.new_state("U")
        P1 = G.new_state("P")
        G.substep(U, U, Pin, U1, P1, 0.0, 1.0)
        torch.cuda.synchronize()
        outs.append((U1.cpu().numpy(), P1[:, torch.from_numpy(G.interior_index()).to(P.device)].cpu().numpy()))
    assert np.array_equal(outs[0][0], outs[1][0])
    assert np.array_equal(outs[0][1], outs[1][1])
    assert np.isfinite(outs[1][0]).all()
    G.close()


@pytest.mark.parametrize("ndim", [3, 2])
@pytest.mark.parametrize("prec,tol", [(I.PREC_FP64, FP64_TOL), (I.PREC_MIXED, MIXED_TOL)])
def test_ten_steps_match_oracle(torch, prec, tol, ndim):
    c = tree(prec, ndim)
    banner(f"10 steps {c.name} prec={prec}")
    Og = O.OracleGrid(c.params, c.blocks)
    Uo, Po = Og.run(c.prim, 10)
    G = B.Grid(c.params, c.blocks)
    U, P = G.run(c.prim, 10)
    torch.cuda.synchronize()
    idx = Og.interior_index()
    eU = rel_l1(G.unpack(U), Uo[:, idx])
    eP = rel_l1(G.unpack(P), Po[:, idx])
    print(f"  rel-L1 U {eU}\n  rel-L1 P {eP}\n  gpu {G.stats()} oracle {Og.stats()}", flush=True)
    assert (eU <= tol).all(), eU
    assert (eP <= tol).all(), eP
    G.close()


def test_graph_replay_equals_eager_steps(torch):
    c = tree(I.PREC_MIXED)
    banner(f"graph {c.name}")
    res = []
    for graph in (False, True):
        G = B.Grid(c.params, c.blocks)
        U, P = G.init(c.prim)
        U1, P1 = G.new_state("U"), G.new_state("P")
        if graph:
            G.capture_rk2_step(U, P, U1, P1)
        for _ in range(3):
            if graph:
                G.launch_rk2_step()
            else:
                G.rk2_step(U, P, U1, P1)
            torch.cuda.synchronize()
        res.append((U.cpu().numpy(), G.unpack(P)))
        G.close()
    assert np.array_equal(res[0][0], res[1][0])
    assert np.array_equal(res[0][1], res[1][1])


def test_block_tiled_path_rejects_trees(torch):
    c = tree(I.PREC_MIXED)
    with pytest.raises(B.BhacError) as e:
        B.Grid(dict(c.params, fused=1), c.blocks)
    assert e.value.code == B.BHAC_EUNSUPPORTED


@pytest.mark.parametrize("ndim", [3, 2])
@pytest.mark.parametrize("prec,tol", [(I.PREC_FP64, 1e-13), (I.PREC_MIXED, 1e-6)])
def test_flux_correction_conserves_across_levels(torch, prec, tol, ndim):
    """Periodic flat three-level tree (square in 2-D), no sources: the
    volume-weighted totals of D, S, tau and B after two RK2 steps equal the
    initial ones (to rounding; in mixed precision each cell's flux difference is
    formed in float)."""
    params, blocks, prim = flat_tree_case(ndim=ndim)
    params = dict(params, precision=prec, fused=0)
    banner(f"conservation ndim={ndim} prec={prec}")
    G = B.Grid(params, blocks)
    U, P = G.init(prim)
    U1, P1 = G.new_state("U"), G.new_state("P")
    vol = tree_volumes(blocks, int(params["ncell0"][0]), ndim)
    U0 = U.cpu().numpy().copy()
    for _ in range(2):
        G.rk2_step(U, P, U1, P1)
    torch.cuda.synchronize()
    Un = U.cpu().numpy()
    for q in range(8):
        scale = np.sum(np.abs(U0[q]) * vol)
        assert abs(np.sum(Un[q] * vol) - np.sum(U0[q] * vol)) <= tol * scale, q
    assert G.stats()["c2p_fail"] == 0
    G.close()
