"""Host logic of the benchmark: the algorithmic byte model, the roofline figures
derived from kernel durations, the gating of stored counter figures on the kernel
sources, the one-GPU guard and the CPU-oracle baseline (no GPU needed)."""
import json
import os
import subprocess
import sys

import pytest

import bench
from paper_2108_12240_amd import inputs as I

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_update_bytes_per_cell():
    # U_stage 72 + U_base 72 in one stage of two + P 9R + six face fluxes 27R + U_out 72 + P_out 9R
    assert bench.bytes_per_unit("update", 8) == 540
    assert bench.bytes_per_unit("update", 4) == 360
    # the entropy field adds a row everywhere
    assert bench.bytes_per_unit("update", 8, 10) == 600
    assert bench.bytes_per_unit("update", 4, 10) == 400


def test_face_kernel_bytes_per_face():
    for fam in ("flux_x1", "flux_x2", "flux_x3"):
        assert bench.bytes_per_unit(fam, 8) == 144
        assert bench.bytes_per_unit(fam, 4, 10) == 80


def test_units_per_launch_count_faces_and_cells():
    c = I.case_torus(2, n=32)
    blk = c.blocks
    nface = [int(((blk[:, 1] + (d == 0)) * (blk[:, 2] + (d == 1)) * (blk[:, 3] + (d == 2))).sum()) for d in range(3)]
    info = dict(nface=nface, ncell=int(c.ioff[-1]), nvar=9, ghost_slots=0)
    # every block owns its faces: (s0 + 1) s1 s2 along x1, and so on
    assert nface[0] == sum(int((b[1] + 1) * b[2] * b[3]) for b in blk)
    assert bench.units_per_launch("flux_x1", info) == nface[0]
    assert bench.units_per_launch("flux_x2", info) == nface[1]
    assert bench.units_per_launch("update", info) == 32 ** 3


def fake_result(update_ms=0.25, launches=20):
    info = dict(nface=[2 ** 21 + 2 ** 17] * 3, ncell=2 ** 21, nvar=9, ghost_slots=0)
    kt = {"update": (launches, update_ms * launches), "flux_x1": (launches, 0.13 * launches),
          "step_begin": (10, 0.06), "step_end": (10, 0.06)}
    return dict(ktimes=kt, info=info)


def test_roofline_of_the_dominant_kernel():
    r = bench.roofline(fake_result(), 8, "no_such_workload")
    assert r["kernel"] == "update" and r["bound"] == "hbm" and r["unit"] == "GB/s"
    # the update moves the method's state: 260 B per zone-substep in FP64
    alg = 260 * 2 ** 21
    assert r["bytes_per_launch"] == alg
    assert r["achieved"] == pytest.approx(alg / 0.25e-3 / 1e9, rel=1e-6)
    assert r["frac"] == pytest.approx(r["achieved"] / 8000.0, abs=1e-4)
    # its own bytes (face fluxes, B and psi in P as well) beside it
    assert r["kernel_bytes_per_launch"] == 540 * 2 ** 21
    assert r["kernel_bytes_frac"] == pytest.approx(540 * 2 ** 21 / 0.25e-3 / 8e12, abs=1e-4)
    assert r["traffic"] is None                      # nothing stored for this workload
    assert bench.roofline(fake_result(), 4, "no_such_workload")["bytes_per_launch"] == 220 * 2 ** 21


def test_whole_substep_roofline():
    res = dict(fake_result(), ms_per_step=1.0)
    res["info"]["ncell"] = 2 ** 21
    s = bench.substep_roofline(res, 4, "ks_torus_128_mixed_plain")
    t = 0.5e-3
    assert s["hbm_frac"] == pytest.approx(220 * 2 ** 21 / t / 8e12, abs=1e-4)
    fl = bench.OPCOUNT["ks_torus_128"]["algorithmic"] * 2 ** 21
    assert s["alu_frac"] == pytest.approx(fl / t / 78.6e12, abs=1e-4)
    assert s["alu_floor_ms"] == pytest.approx(fl / 78.6e12 * 1e3, rel=1e-3)
    assert s["hbm_floor_ms"] == pytest.approx(220 * 2 ** 21 / 8e12 * 1e3, rel=1e-3)
    assert "alu_frac" not in bench.substep_roofline(res, 4, "no_such_workload")


def test_host_description():
    h = bench.host_info()
    assert h["logical_cpus"] >= 1 and 1 <= h["usable_cpus"] <= h["logical_cpus"]
    assert 1 <= h["threads_allowed"] <= h["usable_cpus"] and isinstance(h["cpu_model"], str)


def test_stored_traffic_is_used_only_with_matching_sources(monkeypatch):
    key = ("fake_workload", "update")
    monkeypatch.setitem(bench.TRAFFIC, key, (1.2e9, bench.source_digest()))
    r = bench.roofline(fake_result(), 8, "fake_workload")
    assert r["traffic"] == 1.2e9
    assert r["traffic_over_algorithmic"] == pytest.approx(1.2e9 / (260 * 2 ** 21), abs=1e-3)
    assert r["traffic_over_kernel_bytes"] == pytest.approx(1.2e9 / (540 * 2 ** 21), abs=1e-3)
    monkeypatch.setitem(bench.TRAFFIC, key, (1.2e9, "0000000000000000"))
    assert bench.roofline(fake_result(), 8, "fake_workload")["traffic"] is None


def test_stored_valu_counts_give_issue_rates(monkeypatch):
    monkeypatch.setitem(bench.VALU, ("fake_workload", "flux_x1"), (49e6, bench.source_digest()))
    rates = bench.valu_rates(fake_result(), "fake_workload")
    assert set(rates) == {"flux_x1"}
    expect = 49e6 * 64 / 0.13e-3
    assert rates["flux_x1"]["frac"] == pytest.approx(expect / bench.VALU_PEAK, abs=1e-3)


def test_more_than_one_gpu_is_refused():
    p = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, cwd=ROOT, timeout=300)
    assert p.returncode == 2
    msg = json.loads(p.stdout.strip().splitlines()[-1])
    assert "one GPU" in msg["error"]


def test_cpu_baseline_runs_the_oracle_on_a_bounded_sample():
    c = I.case_torus(2, n=32)
    c.params = dict(c.params, precision=I.PREC_FP64, fused=0)
    out = bench.cpu_baseline(c, 0.5)
    assert out["kind"] == "oracle" and out["cores"] == 1 and out["unit"] == "zone-updates/s"
    assert out["value"] > 0 and "blocks" in out["sample"]
    two = bench.cpu_baseline(c, 0.5, threads=2)
    assert two["cores"] == 2 and "2 thread(s)" in two["sample"]


def test_oracle_sample_is_the_neighbourhood_of_the_densest_block():
    c = I.case_torus(2, n=64)
    blocks, prim = bench._sample_case(c, 5)
    assert len(blocks) == 5 and prim.shape == (9, 5 * 16 ** 3)
    dens = [c.prim[0, c.ioff[b]:c.ioff[b + 1]].max() for b in range(c.nblocks)]
    densest = c.blocks[int(max(range(c.nblocks), key=lambda b: dens[b]))]
    assert any((b == densest).all() for b in blocks)


def test_bound_follows_the_larger_floor(monkeypatch):
    """With a stored VALU count whose issue time exceeds the HBM time of the
    kernel's algorithmic bytes, the roofline is taken against the VALU peak."""
    dig = bench.source_digest()
    hbm_floor = 260 * 2 ** 21 / 8e12                       # s per launch at 8 TB/s
    small = int(0.5 * hbm_floor * bench.VALU_PEAK / 64)     # issue time half the HBM floor
    monkeypatch.setitem(bench.VALU, ("fake_workload", "update"), (small, dig))
    assert bench.roofline(fake_result(), 8, "fake_workload")["bound"] == "hbm"
    big = int(2.0 * hbm_floor * bench.VALU_PEAK / 64)
    monkeypatch.setitem(bench.VALU, ("fake_workload", "update"), (big, dig))
    r = bench.roofline(fake_result(), 8, "fake_workload")
    assert r["bound"] == "alu" and r["unit"] == "Tlane-instr/s"
    assert r["frac"] == pytest.approx(big * 64 / 0.25e-3 / bench.VALU_PEAK, abs=1e-4)
    assert r["hbm_frac"] == pytest.approx(260 * 2 ** 21 / 0.25e-3 / 8e12, abs=1e-4)


def test_bytes_of_the_update_with_x1_faces_in_place():
    # as the update, without the x1 face fluxes: 9 (1.5 * 8 + R + 2R + 8 + R)
    assert bench.bytes_per_unit("update_x1", 8) == 468
    assert bench.bytes_per_unit("update_x1", 4) == 324


def test_source_digest_ignores_comments_only():
    src = 'int f(int a) { // a comment\n  /* another\n  one */ return a + 1; } const char *s = "//x";'
    assert bench._strip_comments(src) == bench._strip_comments(src.replace("a comment", "reworded"))
    assert bench._strip_comments(src) != bench._strip_comments(src.replace("a + 1", "a + 2"))
    assert '"//x"' in bench._strip_comments(src)
