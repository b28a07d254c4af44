"""Pins of the oracle's op counter (oracle/opcount.py, oracle/opcount.cpp).

* The op-count build computes exactly what the plain oracle computes (bit for bit).
* Its tallies equal hand counts of small functions read off their definitions.
* Counts are additive over blocks and independent of how the grid is split.
* The algorithmic flops per zone-substep stored in bench.py for the 128^3 torus are
  what the counter gives now on the same block sample.
"""
import math

import numpy as np
import pytest

from oracle import opcount as OC
from oracle import oracle as O
from paper_2108_12240_amd import inputs as I


@pytest.fixture(scope="module", autouse=True)
def built():
    OC.build(force=False)


def flops(counts, region):
    i = OC.REGIONS.index(region)
    return int(counts[i, [OC.KINDS.index(k) for k in OC.FLOP_KINDS]].sum())


def kind(counts, region, k):
    return int(counts[OC.REGIONS.index(region), OC.KINDS.index(k)])


def test_counting_build_is_bit_identical():
    c = I.case_torus(2, n=(32, 16, 16))
    res = OC.substep_counts(c.params, c.blocks, c.prim)
    Og = O.OracleGrid(c.params, c.blocks)
    U, P = Og.init(c.prim)
    U1, P1 = np.zeros_like(U), np.zeros_like(P)
    Og.substep(U, U, P, U1, P1, 0.0, 1.0)
    idx = Og.interior_index()
    assert np.array_equal(res["U1"][:, idx], U1[:, idx])
    assert np.array_equal(res["P1"][:, idx], P1[:, idx])


def test_mc_face_hand_count():
    """MC face states from q = (., 0, 1, 3, 4, .). Slope of (0, 1, 3): d- = 1 and d+ = 2
    (2 additions), the product test (1 multiplication), 2|d-| = 2 (1 multiplication),
    2|d+| = 4 (1, not smaller), |d- + d+|/2 = 1.5 (1 addition, 1 multiplication; smaller,
    recomputed when taken: 1 + 1): 4 additions, 5 multiplications, 4 comparisons, 4
    absolute values. Slope of (1, 3, 4): d- = 2, d+ = 1; 2|d-| = 4, 2|d+| = 2 (smaller,
    recomputed: 1 more multiplication), |d- + d+|/2 = 1.5 (smaller, recomputed): 4
    additions, 6 multiplications, 4 comparisons, 5 absolute values. Face values
    q_i + s/2 and q_{i+1} - s/2: 2 additions, 2 multiplications."""
    q = np.array([0.0, 0.0, 1.0, 3.0, 4.0, 0.0])
    out = np.zeros(2)
    with OC.counting() as L:
        OC.reset()
        L.orc_recon_face(0, q.ctypes.data_as(O._D), out.ctypes.data_as(O._D))
        counts, calls = OC.read()
    assert calls[OC.REGIONS.index("mc_slope")] == 2
    assert kind(counts, "mc_slope", "add") == 4 + 4
    assert kind(counts, "mc_slope", "mul") == 5 + 6
    assert kind(counts, "mc_slope", "cmp") == 4 + 4
    assert kind(counts, "mc_slope", "sign") == 4 + 5
    assert kind(counts, "mc_slope", "div") == 0
    assert kind(counts, "mc_face", "add") == 2 and kind(counts, "mc_face", "mul") == 2
    assert out[0] == 1.0 + 0.5 * 1.5 and out[1] == 3.0 - 0.5 * 1.5


def test_ppm_interface_hand_count():
    """A PPM face from smooth monotone data: per cell two interface values
    (q_a + q_b)/2 - (s_b - s_a)/6, i.e. 2 additions, 1 multiplication, 1 subtraction of
    slopes, 1 division and the final subtraction = 3 additions, 1 multiplication and
    1 division each; two cells per face."""
    q = np.array([0.0, 1.0, 2.0, 3.0, 4.0, 5.0]) ** 1.1
    out = np.zeros(2)
    with OC.counting() as L:
        OC.reset()
        L.orc_recon_face(1, q.ctypes.data_as(O._D), out.ctypes.data_as(O._D))
        counts, calls = OC.read()
    assert calls[OC.REGIONS.index("ppm_iface")] == 2
    assert calls[OC.REGIONS.index("mc_slope")] == 6
    assert kind(counts, "ppm_iface", "add") == 2 * 2 * 3
    assert kind(counts, "ppm_iface", "mul") == 2 * 2 * 1
    assert kind(counts, "ppm_iface", "div") == 2 * 2 * 1


def test_counts_are_additive_over_blocks():
    c = I.case4(nblocks=12, n0=48)
    a = OC.substep_counts(c.params, c.blocks, c.prim, sel=[0, 1, 2], dt=1e-3)
    b = OC.substep_counts(c.params, c.blocks, c.prim, sel=[3, 4], dt=1e-3)
    ab = OC.substep_counts(c.params, c.blocks, c.prim, sel=[0, 1, 2, 3, 4], dt=1e-3)
    # every part of the method is additive; "other" also holds the once-per-substep
    # time-step arithmetic (dt, c_h, kappa)
    assert np.array_equal(a["counts"][1:] + b["counts"][1:], ab["counts"][1:])
    assert np.array_equal(a["calls"][1:] + b["calls"][1:], ab["calls"][1:])
    assert a["zone_substeps"] + b["zone_substeps"] == ab["zone_substeps"]


def test_algorithmic_multiplicities():
    """Per zone-substep in 3-D with PPM: 27 slopes, 13.5 interface pairs, 27 limiters, 6
    face states, 3 Riemann combinations, and one each of sources, inversion and update;
    the oracle itself forms more slopes and limiters (it reconstructs each face from
    scratch) and one face more per block and direction."""
    c = I.case_torus(2, n=(32, 32, 32))
    res = OC.substep_counts(c.params, c.blocks, c.prim, sel=[0, 5], dt=1e-3)
    pz = OC.per_zone(c.params, res)["parts"]
    assert pz["mc_slope"]["min_calls_per_zone"] == 27
    assert pz["ppm_iface"]["min_calls_per_zone"] == 13.5
    assert pz["ppm_limit"]["min_calls_per_zone"] == 27
    assert pz["face_state"]["min_calls_per_zone"] == 6
    assert pz["riemann"]["min_calls_per_zone"] == 3
    s = 16
    assert pz["riemann"]["calls_per_zone"] == pytest.approx(3 * (s + 1) / s)
    assert pz["face_state"]["calls_per_zone"] == pytest.approx(6 * (s + 1) / s)
    assert pz["mc_slope"]["calls_per_zone"] == pytest.approx(27 * 6 * (s + 1) / s)
    assert pz["sources"]["calls_per_zone"] == 1 and pz["update"]["calls_per_zone"] == 1


def test_stored_benchmark_count_is_current():
    import bench
    name, stored = "ks_torus_128", bench.OPCOUNT["ks_torus_128"]
    case = I.case_torus(2, n=128)
    res = OC.substep_counts(case.params, case.blocks, case.prim, sel=OC.sample_blocks(case))
    pz = OC.per_zone(case.params, res)
    assert math.isclose(pz["algorithmic"], stored["algorithmic"], rel_tol=1e-9), (name, pz["algorithmic"])
    assert math.isclose(pz["computed"], stored["computed"], rel_tol=1e-9)
