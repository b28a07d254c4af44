"""The autotuner times the substep implementations and schedules and caches its
choice; every schedule gives the same results."""
import numpy as np
import pytest

from paper_2108_12240_amd import autotune
from paper_2108_12240_amd import bhac as B
from paper_2108_12240_amd import inputs as I

pytestmark = pytest.mark.gpu


def test_tune_and_cache(tmp_path):
    c = I.case_torus(2, n=(48, 32, 32))
    params = dict(c.params, precision=I.PREC_MIXED)
    path = str(tmp_path / "tune.json")
    chosen, rep = autotune.tune(params, c.blocks, c.prim, steps=2, path=path)
    assert rep["cached"] is False
    assert chosen["fused"] in (0, 1)
    timed = [t for t in rep["timings"] if t["ms_per_step"] is not None]
    assert len(timed) >= 8 and all(t["ms_per_step"] > 0 for t in timed)
    again, rep2 = autotune.tune(params, c.blocks, c.prim, path=path)
    assert rep2["cached"] is True and again["fused"] == chosen["fused"]
    assert again.get("sched") == chosen.get("sched")


def test_unsupported_candidate_is_skipped(tmp_path):
    c = I.case_torus(2, n=32)
    params = dict(c.params, precision=I.PREC_FP64)        # block-tiled path is mixed-only
    chosen, rep = autotune.tune(params, c.blocks, c.prim, steps=1, path=str(tmp_path / "t.json"))
    assert chosen["fused"] == 0 and "sched" in chosen
    assert rep["timings"][0]["choice"] == {"fused": 1} and rep["timings"][0]["ms_per_step"] is None


@pytest.mark.parametrize("prec", [I.PREC_FP64, I.PREC_MIXED])
def test_every_schedule_gives_identical_results(prec):
    """Two RK2 steps under each distinct schedule give bit-identical states: the
    per-face arithmetic does not depend on how faces map to waves."""
    import torch
    c = I.case_torus(2, n=(48, 32, 32))
    params = dict(c.params, precision=prec, fused=0)
    print(f"\n[schedules] {c.name} prec={prec}", flush=True)
    ref, seen = None, []
    for cand in autotune.candidates(params)[1:]:
        G = B.Grid(dict(params, **cand), c.blocks)
        sch = G.schedule()
        if sch in seen:
            G.close()
            continue
        seen.append(sch)
        U, P = G.run(c.prim, 2)
        torch.cuda.synchronize()
        got = (U.cpu().numpy(), G.unpack(P))
        G.close()
        if ref is None:
            ref = got
            continue
        assert np.array_equal(ref[0], got[0]), sch
        assert np.array_equal(ref[1], got[1]), sch
    assert len(seen) >= 8


def test_exhaustive_search_times_every_distinct_schedule(tmp_path):
    c = I.case_torus(2, n=32)
    params = dict(c.params, precision=I.PREC_MIXED)
    chosen, rep = autotune.tune(params, c.blocks, c.prim, steps=1, path=str(tmp_path / "t.json"),
                                search="exhaustive")
    assert len(rep["timings"]) == len(autotune.candidates(params))
    ms = [t["ms_per_step"] for t in rep["timings"] if t["ms_per_step"] is not None]
    assert len(ms) >= 16
    best = [t for t in rep["timings"] if t["choice"] == rep["choice"]]
    assert len(best) == 1 and best[0]["ms_per_step"] == min(ms)
    assert chosen["fused"] == rep["choice"]["fused"] and chosen.get("sched") == rep["choice"].get("sched")


def test_x1_in_update_falls_back_where_the_grid_cannot_use_it():
    """x1_staged = 2 resolves to the staged face kernel on grids with the entropy
    field or a block tree, and to no x1 face mode at all where x1 is marched."""
    sched = dict(march_mask=6, march_faces=17, x1_staged=2)
    c = I.case_torus(2, n=32)
    G = B.Grid(dict(c.params, fused=0, sched=sched), c.blocks)
    assert G.schedule()["x1_staged"] == 2
    G.close()
    e = I.with_entropy(I.case_torus(2, n=32))
    G = B.Grid(dict(e.params, fused=0, sched=sched), e.blocks)
    assert G.schedule()["x1_staged"] == 1
    G.close()
    t = I.case_tree(n0=32, bs=8, levels=2)
    G = B.Grid(dict(t.params, fused=0, sched=sched), t.blocks)
    assert G.schedule()["x1_staged"] == 1
    G.close()
    G = B.Grid(dict(c.params, fused=0, sched=dict(sched, march_mask=7)), c.blocks)
    assert G.schedule()["x1_staged"] == 0
    G.close()
