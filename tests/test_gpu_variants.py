"""GPU parity beyond the benchmark configurations: the 2-D Kerr-Schild grid, and
the 3-D torus with every reconstruction / Riemann-solver pair under the face-kernel
and the line-march schedules, in both precisions."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2108_12240_amd import bhac as B
from paper_2108_12240_amd import inputs as I
from tests.parity import rel_l1

pytestmark = pytest.mark.gpu

TOL = {I.PREC_FP64: 1e-11, I.PREC_MIXED: 1e-5}
_ORACLE = {}


def banner(msg):
    print(f"\n[variants] {msg}", flush=True)


def oracle_run(key, params, blocks, prim, steps):
    if key not in _ORACLE:
        Og = O.OracleGrid(params, blocks)
        U, P = Og.run(prim, steps)
        idx = Og.interior_index()
        _ORACLE[key] = (U[:, idx], P[:, idx], Og.stats())
    return _ORACLE[key]


def check(c, params, key, steps=10):
    import torch
    Uo, Po, st = oracle_run(key, dict(params, precision=I.PREC_FP64, sched=None), c.blocks, c.prim, steps)
    G = B.Grid(params, c.blocks)
    U, P = G.run(c.prim, steps)
    torch.cuda.synchronize()
    eU, eP = rel_l1(G.unpack(U), Uo), rel_l1(G.unpack(P), Po)
    print(f"  schedule {G.schedule()}\n  rel-L1 U {eU}\n  rel-L1 P {eP}\n  gpu {G.stats()} oracle {st}", flush=True)
    tol = TOL[int(params["precision"])]
    assert (eU <= tol).all(), eU
    assert (eP <= tol).all(), eP
    assert G.stats()["c2p_fail"] == st["c2p_fail"]
    G.close()


@pytest.mark.parametrize("prec", [I.PREC_FP64, I.PREC_MIXED])
@pytest.mark.parametrize("recon,flux", [(I.RECON_PPM, I.FLUX_HLL), (I.RECON_MC, I.FLUX_TVDLF)])
def test_kerr_schild_2d(prec, recon, flux):
    c = I.case_torus_2d(n=(64, 64), bs=16)
    params = dict(c.params, precision=prec, recon=recon, flux=flux, fused=0)
    banner(f"{c.name} prec={prec} recon={recon} flux={flux}")
    check(c, params, ("2d", recon, flux))


SCHEDULES = {"faces": dict(march_mask=0, march_faces=17, x1_staged=1),
             "lines": dict(march_mask=7, march_faces=9, x1_staged=0)}


@pytest.mark.parametrize("sched", sorted(SCHEDULES))
@pytest.mark.parametrize("prec", [I.PREC_FP64, I.PREC_MIXED])
@pytest.mark.parametrize("recon,flux", [(I.RECON_MC, I.FLUX_HLL), (I.RECON_PPM, I.FLUX_TVDLF)])
def test_kerr_schild_3d_solver_pairs(prec, recon, flux, sched):
    c = I.case_torus(2, n=32, bs=16)
    params = dict(c.params, precision=prec, recon=recon, flux=flux, fused=0, sched=SCHEDULES[sched])
    banner(f"{c.name} prec={prec} recon={recon} flux={flux} schedule={sched}")
    check(c, params, ("3d", recon, flux))
