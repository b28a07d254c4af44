"""GPU parity: the HIP path (through the C ABI) against the CPU oracle."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2108_12240_amd import bhac as B
from paper_2108_12240_amd import inputs as I
from tests import layout as L
from tests.parity import rel_l1, linf

pytestmark = pytest.mark.gpu

FP64_TOL = 1e-11     # relative L1 per field after 10 steps, FP64 path
MIXED_TOL = 1e-5     # relative L1 per field after 10 steps, mixed path


def banner(msg):
    print(f"\n[parity] {msg}", flush=True)


@pytest.fixture(scope="module")
def torch():
    import torch as T
    assert T.cuda.is_available(), "GPU tests need a ROCm device"
    return T


def with_prec(c, precision, fused=0):
    c.params = dict(c.params, precision=precision, fused=fused)
    return c


def test_fill_ghosts_bitwise(torch):
    for c in (I.case1(), I.case_torus(2, n=(48, 32, 32)), I.case4(nblocks=64, n0=48)):
        for prec in (I.PREC_FP64, I.PREC_MIXED):
            banner(f"fill {c.name} prec={prec}")
            c = with_prec(c, prec)
            G = B.Grid(c.params, c.blocks)
            Og = O.OracleGrid(c.params, c.blocks)
            ids = np.zeros((9, G.ncp))
            for q in range(9):
                ids[q] = (np.arange(G.ncp) % 1000003) + 1.5 * q   # exact in float32
            P = torch.from_numpy(ids).to("cuda", G.pdtype)
            G.fill_ghosts(P)
            ref = ids.copy()
            Og.fill_ghosts(ref)
            got = P.cpu().double().numpy()
            assert np.array_equal(got, ref)
            G.close()


@pytest.mark.parametrize("cfg", ["case1", "torus"])
def test_prim2con_con2prim_compute_dt(torch, cfg):
    c = I.case1() if cfg == "case1" else I.case_torus(2, n=32)
    banner(f"pointwise {c.name}")
    G = B.Grid(c.params, c.blocks)
    Og = O.OracleGrid(c.params, c.blocks)
    U0, P0 = Og.init(c.prim)
    Ud, Pd = G.init(c.prim)
    idx = Og.interior_index()
    assert np.allclose(G.unpack(Ud), U0[:, idx], rtol=1e-13, atol=1e-15 * np.abs(U0).max())
    assert G.timestep()["dt_next"] == pytest.approx(Og.state.dt_next, rel=1e-13)
    # inversion from a perturbed guess
    guess = c.prim.copy()
    guess[0] *= 1.01
    guess[4] *= 0.98
    Pg = G.pack(guess)
    G.con2prim(Ud, Pg)
    Po = Og.pack(guess)
    Og.con2prim(U0, Po)
    assert np.allclose(G.unpack(Pg), Po[:, idx], rtol=1e-12, atol=1e-14)
    G.close()


def run_both(c, steps):
    G = B.Grid(c.params, c.blocks)
    Og = O.OracleGrid(c.params, c.blocks)
    Uo, Po = Og.run(c.prim, steps)
    Ud, Pd = G.run(c.prim, steps)
    import torch
    torch.cuda.synchronize()
    idx = Og.interior_index()
    res = dict(U=rel_l1(G.unpack(Ud), Uo[:, idx]), P=rel_l1(G.unpack(Pd), Po[:, idx]),
               Uinf=linf(G.unpack(Ud), Uo[:, idx]), gpu_stats=G.stats(), cpu_stats=Og.stats(),
               gpu_dt=G.timestep(), cpu_dt=Og.stats()["dt_next"])
    G.close()
    return res


FP64_CASES = [
    ("case1_64", lambda: I.case1()),
    ("torus_32", lambda: I.case_torus(2, n=32)),
    ("torus_48x32x32", lambda: I.case_torus(2, n=(48, 32, 32))),
    ("amr_like_64", lambda: with_prec(I.case4(nblocks=64, n0=48), I.PREC_FP64, 0)),
]


@pytest.mark.parametrize("name,make", FP64_CASES)
def test_fp64_ten_steps(torch, name, make):
    c = with_prec(make(), I.PREC_FP64)
    banner(f"fp64 10 steps {name}")
    r = run_both(c, 10)
    print("  rel-L1 U", r["U"], "\n  rel-L1 P", r["P"], "\n  stats", r["gpu_stats"], r["cpu_stats"], flush=True)
    assert (r["U"] <= FP64_TOL).all(), r["U"]
    assert (r["P"] <= FP64_TOL).all(), r["P"]
    assert r["gpu_dt"]["dt_next"] == pytest.approx(r["cpu_dt"], rel=1e-9)
    assert r["gpu_stats"]["c2p_fail"] == r["cpu_stats"]["c2p_fail"]


MIXED_CASES = [
    ("case1_64", lambda: I.case1()),
    ("torus_32", lambda: I.case_torus(2, n=32)),
    ("turbulent_torus_48", lambda: I.case_torus(5, n=48)),
    ("amr_like_64", lambda: I.case4(nblocks=64, n0=48)),
]


@pytest.mark.parametrize("name,make", MIXED_CASES)
def test_mixed_ten_steps(torch, name, make):
    c = with_prec(make(), I.PREC_MIXED, 0)
    banner(f"mixed 10 steps {name}")
    r = run_both(c, 10)
    print("  rel-L1 U", r["U"], "\n  rel-L1 P", r["P"], flush=True)
    assert (r["U"] <= MIXED_TOL).all(), r["U"]
    assert (r["P"] <= MIXED_TOL).all(), r["P"]


FUSED_CASES = [
    ("torus_32", lambda: I.case_torus(2, n=32)),
    ("turbulent_torus_48", lambda: I.case_torus(5, n=48)),
    ("torus_48x32x32", lambda: I.case_torus(2, n=(48, 32, 32))),
    ("amr_like_64", lambda: I.case4(nblocks=64, n0=48)),
]


@pytest.mark.parametrize("name,make", FUSED_CASES)
def test_fused_mixed_ten_steps(torch, name, make):
    c = with_prec(make(), I.PREC_MIXED, 1)
    banner(f"fused mixed 10 steps {name}")
    r = run_both(c, 10)
    print("  rel-L1 U", r["U"], "\n  rel-L1 P", r["P"], "\n  stats", r["gpu_stats"], r["cpu_stats"], flush=True)
    assert (r["U"] <= MIXED_TOL).all(), r["U"]
    assert (r["P"] <= MIXED_TOL).all(), r["P"]
    assert r["gpu_dt"]["dt_next"] == pytest.approx(r["cpu_dt"], rel=1e-5)


def test_fused_rejects_unsupported(torch):
    c = with_prec(I.case1(), I.PREC_MIXED, 1)
    with pytest.raises(B.BhacError) as e:
        B.Grid(c.params, c.blocks)
    assert e.value.code == B.BHAC_EUNSUPPORTED
    c = with_prec(I.case_torus(2, n=32), I.PREC_FP64, 1)
    with pytest.raises(B.BhacError) as e:
        B.Grid(c.params, c.blocks)
    assert e.value.code == B.BHAC_EUNSUPPORTED


def test_uniform_state_bitwise_on_gpu(torch):
    for recon, flux in ((I.RECON_MC, I.FLUX_TVDLF), (I.RECON_PPM, I.FLUX_HLL)):
        c = I.uniform_state(n=(16, 16, 16), bs=(8, 8, 8), recon=recon, flux=flux)
        banner(f"uniform recon={recon}")
        G = B.Grid(c.params, c.blocks)
        U0, P0 = G.init(c.prim)
        U0 = U0.clone()
        U, P = G.run(c.prim, 10)
        assert torch.equal(U, U0)
        G.close()


def test_substep_rejects_aliasing_and_uninitialised_dt(torch):
    c = I.case1()
    G = B.Grid(c.params, c.blocks)
    P = G.pack(c.prim)
    U = G.new_state("U")
    with pytest.raises(B.BhacError) as e:
        G.substep(U, U, P, U, P, 0.0, 1.0)
    assert e.value.code == B.BHAC_EALIAS
    P2 = G.new_state("P")
    with pytest.raises(B.BhacError) as e:
        G.substep(U, U, P, U, P2, 0.0, 1.0)
    assert e.value.code == B.BHAC_EINVAL
    G.close()


def outside_count(c, G):
    """For every padded cell: how many of its coordinates lie outside its block
    (-1 for the padding slots of the x rows)."""
    params = dict(c.params, precision=1 if G.pdtype == G.torch.float32 else 0)
    nout = np.zeros(G.ncp, dtype=np.int64)
    for b, blk in enumerate(c.blocks):
        s = blk[1:4]
        x, y, z, pad = L.box_locals(params, s)
        cnt = sum(((v < 0) | (v >= s[e])).astype(np.int64) for e, v in enumerate((x, y, z)))
        cnt[pad] = -1
        nout[G.off[b]:G.off[b + 1]] = cnt
    return nout


@pytest.mark.parametrize("name,make,prec,fused", [
    ("case1_fp64", lambda: I.case1(), I.PREC_FP64, 0),
    ("torus_fp64", lambda: I.case_torus(2, n=(48, 32, 32)), I.PREC_FP64, 0),
    ("torus_mixed", lambda: I.case_torus(2, n=(48, 32, 32)), I.PREC_MIXED, 0),
    ("case4_mixed", lambda: I.case4(nblocks=64, n0=48), I.PREC_MIXED, 0),
    ("torus_mixed_fused", lambda: I.case_torus(2, n=(48, 32, 32)), I.PREC_MIXED, 1),
])
def test_substep_reads_no_ghost_slot(torch, name, make, prec, fused):
    """The substep takes its halo from the neighbouring blocks' interiors: with every
    ghost slot of P_stage poisoned (NaN) it gives bit-identical results, and it
    writes no ghost slot of P_out."""
    banner(f"substep halo {name}")
    c = with_prec(make(), prec, fused)
    G = B.Grid(c.params, c.blocks)
    U, P = G.init(c.prim)
    G.set_dt(1e-3)            # both calls latch the same dt
    nout = torch.from_numpy(outside_count(c, G)).to(P.device)
    ids = np.zeros((9, G.ncp))
    for q in range(9):
        ids[q] = (np.arange(G.ncp) % 1000003) + 1.5 * q     # exact in float32
    outs = []
    for poison in (False, True):
        if poison:
            P[:, nout > 0] = float("nan")
        U1 = G.new_state("U")
        P1 = torch.from_numpy(ids).to("cuda", G.pdtype)
        G.substep(U, U, P, U1, P1, 0.0, 1.0)
        torch.cuda.synchronize()
        outs.append((U1.cpu().numpy(), P1.cpu().double().numpy()))
    (Ua, Pa), (Ub, Pb) = outs
    assert np.array_equal(Ua, Ub)
    assert np.array_equal(Pa, Pb)
    ghost = outside_count(c, G) > 0
    assert np.array_equal(Pb[:, ghost], ids[:, ghost])
    assert np.isfinite(Ub).all()
    G.close()


def test_fill_ghost_faces_fills_exactly_the_face_slabs(torch):
    for c in (I.case_torus(2, n=(48, 32, 32)), I.case4(nblocks=64, n0=48)):
        banner(f"face fill {c.name}")
        G = B.Grid(c.params, c.blocks)
        Og = O.OracleGrid(c.params, c.blocks)
        ids = np.zeros((9, G.ncp))
        for q in range(9):
            ids[q] = (np.arange(G.ncp) % 1000003) + 1.5 * q     # exact in float32
        ref = ids.copy()
        Og.fill_ghosts(ref)
        P = torch.from_numpy(ids).to("cuda", G.pdtype)
        G.fill_ghost_faces(P)
        got = P.cpu().double().numpy()
        nout = outside_count(c, G)
        face = nout == 1
        assert np.array_equal(got[:, face], ref[:, face])
        assert np.array_equal(got[:, nout >= 2], ids[:, nout >= 2])
        assert np.array_equal(got[:, nout == 0], ids[:, nout == 0])
        assert np.array_equal(got[:, nout < 0], ids[:, nout < 0])
        G.close()
