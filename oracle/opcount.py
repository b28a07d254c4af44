"""Algorithmic operation counts of the GRMHD substep, from the oracle (test
infrastructure only: tests/ and the maintainer's measurement notes use it).

``opcount.cpp`` compiles the oracle unchanged with a counting arithmetic type and
tallies every floating-point operation in the part of the method the oracle marks
(metric, MC slope, PPM interface, PPM limiter, face state + flux + speeds, Riemann
combination, sources, inversion, prim->con, divergence + RK combine). Running a
substep of a workload through it gives, per part, the operations per call and the
calls per zone. Two totals per zone-substep follow:

* as computed by the oracle: its plain loops reconstruct every face from scratch
  (six MC slopes and two PPM limiters per face and variable) and evaluate the
  analytic metric at every cell and face;
* algorithmic: each part once per unit of the method -- per cell, direction and
  variable one MC slope, one PPM interface value (shared by the two cells of a
  face) and one limiter; per face two face states and one Riemann combination; per
  cell the sources, the inversion (the Newton steps it actually takes on the
  workload), the divergence and RK combine, and prim->con only where the inversion
  rewrote the cell. The metric is not counted (the GPU path reads precomputed
  tables, it is not part of the per-zone work).

Flops = additions/subtractions + multiplications + divisions + square roots +
transcendental calls. Comparisons and sign/absolute-value operations are reported
beside them but are not flops.

Usage: python -m oracle.opcount [workload] prints the table for a workload (a block
sample of the benchmark grids).
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
import sys
from contextlib import contextmanager

import numpy as np

from . import oracle as O

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "opcount.cpp")
LIB = os.path.join(HERE, "liboracle_opcount.so")

REGIONS = ("other", "metric", "mc_slope", "ppm_iface", "ppm_limit", "mc_face", "face_state", "riemann", "sources",
           "con2prim", "prim2con", "update")
KINDS = ("add", "mul", "div", "sqrt", "trans", "cmp", "sign")
FLOP_KINDS = ("add", "mul", "div", "sqrt", "trans")


def build(force: bool = True) -> str:
    """Compile the op-count build (also when either source is newer than the library)."""
    stale = not os.path.exists(LIB) or max(os.path.getmtime(SRC), os.path.getmtime(O.SRC)) > os.path.getmtime(LIB)
    if force or stale:
        tmp = LIB + ".tmp"
        subprocess.check_call(["g++", "-x", "c++", "-std=c++17", "-O2", "-ffp-contract=off", "-fno-fast-math",
                               "-fpermissive", "-w", "-fPIC", "-shared", "-I", HERE, "-o", tmp, SRC, "-lm"])
        os.replace(tmp, LIB)
    return LIB


_clib = None


def _counting_lib():
    global _clib
    if _clib is None:
        if not os.path.exists(LIB):
            build()
        L = O.load(LIB)
        L.orc_opcount_shape.argtypes = [C.POINTER(C.c_int), C.POINTER(C.c_int)]
        L.orc_opcount_read.argtypes = [C.POINTER(C.c_ulonglong), C.POINTER(C.c_ulonglong)]
        nr, nk = C.c_int(), C.c_int()
        L.orc_opcount_shape(C.byref(nr), C.byref(nk))
        assert (nr.value, nk.value) == (len(REGIONS), len(KINDS)), "region table out of date"
        _clib = L
    return _clib


@contextmanager
def counting():
    """Within the block, every oracle call (grids created inside included) runs in the
    op-count build; the plain build is restored afterwards."""
    L = _counting_lib()
    saved = O._lib
    O._lib = L
    try:
        L.orc_set_threads(1)
        yield L
    finally:
        O._lib = saved


def reset():
    _counting_lib().orc_opcount_reset()


def read():
    """(counts[region][kind], calls[region]) since the last reset."""
    cnt = (C.c_ulonglong * (len(REGIONS) * len(KINDS)))()
    calls = (C.c_ulonglong * len(REGIONS))()
    _counting_lib().orc_opcount_read(cnt, calls)
    return (np.array(cnt[:], dtype=np.int64).reshape(len(REGIONS), len(KINDS)),
            np.array(calls[:], dtype=np.int64))


def minimal_calls(params: dict, calls: np.ndarray, zone_substeps: int) -> dict:
    """Calls of each part per zone-substep when every part runs once per unit of the
    method (see the module docstring)."""
    nd, nv = int(params["ndim"]), 9
    ppm = int(params["recon"]) == 1
    r = {k: 0.0 for k in REGIONS}
    r["mc_slope"] = nd * nv
    if ppm:
        r["ppm_iface"] = nd * nv / 2.0        # one call forms the two interface values of a cell
        r["ppm_limit"] = nd * nv
    else:
        r["mc_face"] = nd * nv
    r["face_state"] = 2.0 * nd
    r["riemann"] = float(nd)
    r["sources"] = r["con2prim"] = r["update"] = 1.0
    r["prim2con"] = calls[REGIONS.index("prim2con")] / zone_substeps
    return r


def substep_counts(params: dict, blocks: np.ndarray, prim: np.ndarray, sel=None, dt=None) -> dict:
    """Counts of one substep (a = 0, b = 1) of the whole grid or of the block sample sel,
    from the state prim (ghosts filled, U from prim2con), with the CFL dt unless dt is
    given."""
    with counting():
        Og = O.OracleGrid(params, blocks)
        U, P = Og.init(prim)
        if dt is not None:
            Og.set_dt(dt)
        U1, P1 = np.zeros_like(U), np.zeros_like(P)
        reset()
        Og.substep(U, U, P, U1, P1, 0.0, 1.0, sel)
        counts, calls = read()
        zones = int(Og.nci) if sel is None else int(sum(Og.ioff[b + 1] - Og.ioff[b] for b in sel))
        out = dict(counts=counts, calls=calls, zone_substeps=zones, U1=U1, P1=P1, interior=Og.interior_index(),
                   stats=Og.stats())
        del Og
    return out


def per_zone(params: dict, res: dict) -> dict:
    """Flops (and comparisons, sign operations) per zone-substep, per part and in total,
    as the oracle computes them and with the algorithmic multiplicities."""
    counts, calls, zs = res["counts"], res["calls"], res["zone_substeps"]
    fl = [KINDS.index(k) for k in FLOP_KINDS]
    mins = minimal_calls(params, calls, zs)
    parts = {}
    tot_comp = tot_alg = 0.0
    for i, name in enumerate(REGIONS):
        flops = float(counts[i, fl].sum())
        per_call = flops / calls[i] if calls[i] else 0.0
        comp = flops / zs
        alg = per_call * mins[name] if name not in ("metric", "other") else 0.0
        parts[name] = dict(flops_per_call=per_call, calls_per_zone=calls[i] / zs, computed_per_zone=comp,
                           algorithmic_per_zone=alg, min_calls_per_zone=mins[name],
                           cmp_per_zone=counts[i, KINDS.index("cmp")] / zs,
                           sign_per_zone=counts[i, KINDS.index("sign")] / zs,
                           div_per_zone=counts[i, KINDS.index("div")] / zs,
                           sqrt_per_zone=counts[i, KINDS.index("sqrt")] / zs)
        if name not in ("metric", "other"):
            tot_comp += comp
            tot_alg += alg
    return dict(parts=parts, computed=tot_comp, algorithmic=tot_alg)


WORKLOADS = {
    # name: (case builder, block sample)
    "ks_torus_128": lambda I: (I.case_torus(2, n=128), "sample"),
    "ks_torus_192": lambda I: (I.case_torus(3, n=192), "sample"),
    "ks_turb_384": lambda I: (I.case_torus(5, n=384), "sample"),
    "case1_64": lambda I: (I.case1(), None),
}


def sample_blocks(case, k=32):
    """k blocks evenly spaced through the block list (every radius and angle band)."""
    nb = case.nblocks
    return sorted(set(int(b) for b in np.linspace(0, nb - 1, min(k, nb)).round()))


def main(argv=None):
    argv = sys.argv[1:] if argv is None else argv
    name = argv[0] if argv else "ks_torus_128"
    root = os.path.dirname(HERE)
    if root not in sys.path:
        sys.path.insert(0, root)
    from paper_2108_12240_amd import inputs as I
    case, samp = WORKLOADS[name](I)
    sel = sample_blocks(case) if samp == "sample" else None
    res = substep_counts(case.params, case.blocks, case.prim, sel)
    pz = per_zone(case.params, res)
    print(f"workload {name}: {res['zone_substeps']} zone-substeps counted"
          f"{'' if sel is None else f' (blocks {sel})'}")
    print(f"{'part':>11s} {'flops/call':>10s} {'calls/zone':>10s} {'computed':>9s} {'min calls':>9s} "
          f"{'algorithmic':>11s} {'div':>6s} {'sqrt':>6s} {'cmp':>7s} {'sign':>6s}")
    for k, v in pz["parts"].items():
        print(f"{k:>11s} {v['flops_per_call']:10.1f} {v['calls_per_zone']:10.2f} {v['computed_per_zone']:9.1f} "
              f"{v['min_calls_per_zone']:9.2f} {v['algorithmic_per_zone']:11.1f} {v['div_per_zone']:6.1f} "
              f"{v['sqrt_per_zone']:6.1f} {v['cmp_per_zone']:7.1f} {v['sign_per_zone']:6.1f}")
    print(f"total flops per zone-substep: as computed {pz['computed']:.1f}, algorithmic {pz['algorithmic']:.1f}")
    print(f"stored form: {name!r}: dict(algorithmic={float(pz['algorithmic'])!r}, computed={float(pz['computed'])!r})")
    return 0


if __name__ == "__main__":
    sys.exit(main())
