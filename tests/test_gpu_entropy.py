"""GPU parity of the entropy field and the entropy-based inversion backup (through
the C ABI) against the CPU oracle."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2108_12240_amd import bhac as B
from paper_2108_12240_amd import inputs as I
from tests.parity import rel_l1

pytestmark = pytest.mark.gpu

FP64_TOL = 1e-11
MIXED_TOL = 1e-5


def banner(msg):
    print(f"\n[entropy] {msg}", flush=True)


@pytest.fixture(scope="module")
def torch():
    import torch as T
    assert T.cuda.is_available(), "GPU tests need a ROCm device"
    return T


def case(prec, n=(48, 32, 32), cfg=2):
    c = I.with_entropy(I.case_torus(cfg, n=n))
    c.params = dict(c.params, precision=prec, fused=0)
    return c


@pytest.mark.parametrize("prec,tol", [(I.PREC_FP64, FP64_TOL), (I.PREC_MIXED, MIXED_TOL)])
def test_ten_steps_match_oracle(torch, prec, tol):
    c = case(prec)
    banner(f"10 steps {c.name} prec={prec}")
    Og = O.OracleGrid(c.params, c.blocks)
    Uo, Po = Og.run(c.prim, 10)
    G = B.Grid(c.params, c.blocks)
    assert G.nvar == 10
    U, P = G.run(c.prim, 10)
    torch.cuda.synchronize()
    idx = Og.interior_index()
    eU = rel_l1(G.unpack(U), Uo[:, idx])
    eP = rel_l1(G.unpack(P), Po[:, idx])
    print(f"  rel-L1 U {eU}\n  rel-L1 P {eP}\n  gpu {G.stats()} oracle {Og.stats()}", flush=True)
    assert eU.shape == (10,) and (eU <= tol).all(), eU
    assert (eP <= tol).all(), eP
    assert G.stats()["c2p_backup"] == Og.stats()["c2p_backup"]
    G.close()


@pytest.mark.parametrize("prec", [I.PREC_FP64, I.PREC_MIXED])
def test_entropy_field_leaves_the_grmhd_rows_unchanged(torch, prec):
    """Without backups the nine GRMHD rows are bit-identical to a run without the field."""
    c = case(prec)
    banner(f"passive {c.name} prec={prec}")
    outs = []
    for ent in (0, 1):
        params = dict(c.params, entropy=ent)
        G = B.Grid(params, c.blocks)
        U, P = G.run(c.prim if ent else c.prim[:9], 3)
        torch.cuda.synchronize()
        outs.append((G.unpack(U)[:9], G.unpack(P)[:9], G.stats()))
        G.close()
    assert outs[1][2]["c2p_backup"] == 0
    assert np.array_equal(outs[0][0], outs[1][0])
    assert np.array_equal(outs[0][1], outs[1][1])


def perturb(c, G, Og, U, Uo, every=37):
    """Lower the energy of every `every`-th interior cell far below what its density
    and momentum need, so that the energy inversion has no root there."""
    sel = np.arange(0, G.nci, every)
    idx = Og.interior_index()
    import torch
    t = torch.from_numpy(sel).to(U.device)
    U[4, t] = -0.5 * U[0, t]
    Uo[4, idx[sel]] = -0.5 * Uo[0, idx[sel]]
    return sel


@pytest.mark.parametrize("prec,tol", [(I.PREC_FP64, 1e-12), (I.PREC_MIXED, 1e-6)])
def test_con2prim_backup_matches_oracle(torch, prec, tol):
    c = case(prec, n=32)
    banner(f"con2prim backup {c.name} prec={prec}")
    G = B.Grid(c.params, c.blocks)
    Og = O.OracleGrid(c.params, c.blocks)
    U, P = G.init(c.prim)
    Uo, Po = Og.init(c.prim)
    sel = perturb(c, G, Og, U, Uo)
    G.reset_stats()
    fail = torch.zeros(G.nci, dtype=torch.int8, device=U.device)
    G.con2prim(U, P, fail)
    ofail = np.zeros(Og.ncp, dtype=np.int8)
    Og.con2prim(Uo, Po, ofail)
    torch.cuda.synchronize()
    idx = Og.interior_index()
    st = G.stats()
    print(f"  gpu {st} oracle {Og.stats()}", flush=True)
    assert st["c2p_backup"] == Og.stats()["c2p_backup"] == len(sel)
    assert np.array_equal(fail.cpu().numpy(), ofail[idx])
    got, ref = G.unpack(P), Po[:, idx]
    err = rel_l1(got[:, sel], ref[:, sel])
    assert (err <= tol).all(), err
    assert (rel_l1(got, ref) <= tol).all()
    G.close()


@pytest.mark.parametrize("prec,tol", [(I.PREC_FP64, FP64_TOL), (I.PREC_MIXED, MIXED_TOL)])
def test_substep_backup_matches_oracle(torch, prec, tol):
    """A substep from a state whose energy cannot be inverted in some cells: the update
    kernel takes the entropy root there and rewrites those cells' conserved state."""
    c = case(prec, n=32)
    banner(f"substep backup {c.name} prec={prec}")
    G = B.Grid(c.params, c.blocks)
    Og = O.OracleGrid(c.params, c.blocks)
    U, P = G.init(c.prim)
    Uo, Po = Og.init(c.prim)
    perturb(c, G, Og, U, Uo)
    G.set_dt(2e-3)
    Og.set_dt(2e-3)
    G.reset_stats()
    U1, P1 = G.new_state("U"), G.new_state("P")
    G.substep(U, U, P, U1, P1, 0.0, 1.0)
    U1o, P1o = np.zeros_like(Uo), np.zeros_like(Po)
    Og.substep(Uo, Uo, Po, U1o, P1o, 0.0, 1.0)
    torch.cuda.synchronize()
    idx = Og.interior_index()
    st = G.stats()
    print(f"  gpu {st} oracle {Og.stats()}", flush=True)
    assert st["c2p_backup"] > 0
    assert st["c2p_backup"] == Og.stats()["c2p_backup"] and st["c2p_fail"] == Og.stats()["c2p_fail"]
    eU = rel_l1(G.unpack(U1), U1o[:, idx])
    eP = rel_l1(G.unpack(P1), P1o[:, idx])
    print(f"  rel-L1 U {eU}\n  rel-L1 P {eP}", flush=True)
    assert (eU <= tol).all(), eU
    assert (eP <= tol).all(), eP
    G.close()


def test_graph_replay_equals_eager_steps(torch):
    c = case(I.PREC_MIXED, n=32)
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


def test_entropy_needs_the_unfused_path_on_patches(torch):
    c = case(I.PREC_MIXED, n=32)
    with pytest.raises(B.BhacError) as e:
        B.Grid(dict(c.params, fused=1), c.blocks)
    assert e.value.code == B.BHAC_EUNSUPPORTED
    t = I.case_tree(n0=32, bs=8, levels=2)
    with pytest.raises(B.BhacError) as e:
        B.Grid(dict(t.params, entropy=1, fused=0), t.blocks)
    assert e.value.code == B.BHAC_EUNSUPPORTED


@pytest.mark.parametrize("prec", [I.PREC_FP64, I.PREC_MIXED])
def test_every_schedule_gives_identical_entropy_results(torch, prec):
    """The entropy flux comes out of whichever face kernel a direction uses (face per
    thread, LDS-staged x1 rows, line march); two RK2 steps under each of them give
    bit-identical states, the entropy rows included."""
    from paper_2108_12240_amd import autotune
    c = case(prec)
    banner(f"schedules {c.name} prec={prec}")
    ref, seen = None, []
    for cand in autotune.candidates(c.params)[1:]:
        if cand["sched"]["march_faces"] != 17:
            continue
        G = B.Grid(dict(c.params, **cand), c.blocks)
        sch = G.schedule()
        if sch in seen:
            G.close()
            continue
        seen.append(sch)
        U, P = G.run(c.prim, 2)
        torch.cuda.synchronize()
        got = (U.cpu().numpy(), G.unpack(P))
        G.close()
        assert got[0].shape[0] == 10
        if ref is None:
            ref = got
            continue
        assert np.array_equal(ref[0], got[0]), sch
        assert np.array_equal(ref[1], got[1]), sch
    assert len(seen) >= 8
