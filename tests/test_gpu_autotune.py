"""The autotuner times the supported substep implementations and caches its choice."""
import pytest

from paper_2108_12240_amd import autotune
from paper_2108_12240_amd import inputs as I

pytestmark = pytest.mark.gpu


def test_tune_and_cache(tmp_path):
    c = I.case_torus(2, n=(48, 32, 32))
    params = dict(c.params, precision=I.PREC_MIXED)
    path = str(tmp_path / "tune.json")
    chosen, rep = autotune.tune(params, c.blocks, c.prim, steps=2, path=path)
    assert rep["cached"] is False
    assert chosen["fused"] in (0, 1)
    assert all(t["ms_per_step"] is not None and t["ms_per_step"] > 0 for t in rep["timings"])
    again, rep2 = autotune.tune(params, c.blocks, c.prim, path=path)
    assert rep2["cached"] is True and again["fused"] == chosen["fused"]


def test_unsupported_candidate_is_skipped(tmp_path):
    c = I.case_torus(2, n=32)
    params = dict(c.params, precision=I.PREC_FP64)        # block-tiled path is mixed-only
    chosen, rep = autotune.tune(params, c.blocks, c.prim, steps=1, path=str(tmp_path / "t.json"))
    assert chosen["fused"] == 0
    assert [t["ms_per_step"] is None for t in rep["timings"]] == [False, True]
