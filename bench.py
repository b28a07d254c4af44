#!/usr/bin/env python3
"""Benchmark of the GRMHD substep library on one MI355X.

Metric: zone-updates per second, counting interior cells times RK substeps (the
paper's "cellupdates", Section 4.2). One benchmark step is one SSP-RK2 step = two
substeps, each a full pass of the hot path (halo reads, reconstruction, face fluxes,
divergence, sources, RK combine, inversion, wave-speed reduction) over the whole
grid, with the CFL time step from the wave-speed reduction. Inputs are synthetic and
already resident in HBM when timing starts.

Headline: the 384^3 turbulent Kerr-Schild torus (13824 blocks of 16^3), mixed
precision, run for W warmup steps and then R timed segments of K steps each, one
continuous CFL-stepped run (W + R K steps; 105 with the defaults and with the
driver's K = 20); value = the median segment, with the best beside it. Beside it:
the plain FP64 path on the same grid (same protocol) and its speed-up, the 128^3
FP64 and 192^3 mixed torus grids, rooflines (HBM on the state bytes of the method,
VALU on its algorithmic flops) and the CPU oracle timed on the host's cores.
Prints ONE JSON line.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
FP_PEAK_TFLOPS = 78.6     # MI355X vector FP64 (and unpacked FP32), FMA = 2 flops
METRIC = "zone-updates/s per RK substep (FP64 vs mixed, 1 GPU) + % HBM roofline"

# Algorithmic HBM bytes per zone-substep: the state minimum of SSP-RK2 with the five
# hydrodynamic primitives stored (stage 1 reads U and P and writes them; stage 2 also
# reads U_base): 260 B with P in double, 220 B with P in float.
STATE_BYTES = {8: 260.0, 4: 220.0}
# Under constrained transport the state also holds the face field (three FP64 faces
# per cell): read at the stage, read at the base in half the stages, written.
CT_FACE_BYTES = 3 * 8 * 2.5

# Algorithmic flops per zone-substep (additions, multiplications, divisions, square
# roots, transcendental calls) of the method on each workload: the oracle's op
# counter (oracle/opcount.py: python -m oracle.opcount <name>, 32 evenly spaced
# blocks) with every part counted once per unit of the method (one MC slope, PPM
# interface and limiter per cell, direction and variable; two face states and one
# Riemann combination per face; sources, inversion with the Newton steps the
# workload takes, divergence and RK combine per cell; metric excluded). A test
# recomputes the 128^3 entry.
OPCOUNT = {
    "ks_torus_128": dict(algorithmic=3020.506254906748, computed=4091.952346801758),
    "ks_torus_192": dict(algorithmic=3012.2640030804805, computed=4084.5058059692383),
    "ks_turb_384": dict(algorithmic=3004.655625287224, computed=4091.6902465820312),
}
WORKLOAD_OPS = {"ks_torus_128_fp64_plain": "ks_torus_128", "ks_torus_128_mixed_plain": "ks_torus_128",
                "ks_torus_192_mixed_plain": "ks_torus_192", "ks_turb_384_mixed_plain": "ks_turb_384",
                "ks_turb_384_fp64_plain": "ks_turb_384"}

# Workloads: name -> (case builder kwargs, precision, fused)
WORKLOADS = {
    # 3-D GRMHD Kerr-Schild torus, 128^3 as 512 blocks of 16^3, PPM + HLL, plain FP64 path
    "ks_torus_128_fp64_plain": dict(cfg=2, n=128, precision=0, fused=0),
    "ks_torus_128_mixed_plain": dict(cfg=2, n=128, precision=1, fused=0),
    "ks_torus_192_mixed_plain": dict(cfg=3, n=192, precision=1, fused=0),
    # block-tiled (halo-gathering) mixed-precision path
    "ks_torus_128_mixed_fused": dict(cfg=2, n=128, precision=1, fused=1),
    "ks_torus_192_mixed_fused": dict(cfg=3, n=192, precision=1, fused=1),
    # AMR-like list: 4096 blocks of 8^3/12^3/16^3 on three levels, mixed precision
    "amr_like_4096_mixed_plain": dict(cfg=4, precision=1, fused=0),
    "amr_like_4096_mixed_fused": dict(cfg=4, precision=1, fused=1),
    # 384^3 torus with seeded turbulence, 13824 blocks of 16^3, mixed precision
    "ks_turb_384_mixed_plain": dict(cfg=5, n=384, precision=1, fused=0),
    "ks_turb_384_fp64_plain": dict(cfg=5, n=384, precision=0, fused=0),
    "ks_turb_384_mixed_fused": dict(cfg=5, n=384, precision=1, fused=1),
    # mixed precision, substep implementation chosen by the autotuner
    "ks_torus_128_fp64_auto": dict(cfg=2, n=128, precision=0, fused="auto"),
    "ks_torus_128_mixed_auto": dict(cfg=2, n=128, precision=1, fused="auto"),
    "ks_torus_192_mixed_auto": dict(cfg=3, n=192, precision=1, fused="auto"),
    "amr_like_4096_mixed_auto": dict(cfg=4, precision=1, fused="auto"),
    "ks_turb_384_mixed_auto": dict(cfg=5, n=384, precision=1, fused="auto"),
    # one GPU's share of the 384^3 turbulent torus sharded in eight phi-slabs:
    # 384 x 384 x 48 zones (1728 blocks of 16^3), phi ends joined periodically
    "ks_turb_384_slab8_mixed_plain": dict(cfg="slab", n=(384, 384, 48), precision=1, fused=0),
    # 2:1 block tree of 16^3 blocks on three levels around the torus (96^3 base,
    # 972 blocks, 4.0 M zones), with restriction / prolongation between levels
    "amr_tree_96_mixed_plain": dict(cfg="tree", n0=96, bs=16, levels=3, precision=1, fused=0),
    "amr_tree_96_fp64_plain": dict(cfg="tree", n0=96, bs=16, levels=3, precision=0, fused=0),
    # the same grid carrying the entropy field (inversion backup), FP64 and mixed
    "ks_torus_128_fp64_entropy": dict(cfg=2, n=128, precision=0, fused=0, entropy=1),
    "ks_torus_128_mixed_entropy": dict(cfg=2, n=128, precision=1, fused=0, entropy=1),
    "amr_tree_96_mixed_auto": dict(cfg="tree", n0=96, bs=16, levels=3, precision=1, fused="auto"),
    "amr_tree_96_fp64_auto": dict(cfg="tree", n0=96, bs=16, levels=3, precision=0, fused="auto"),
    # the same grid under staggered constrained transport (face field from the torus's
    # azimuthal potential), FP64 and mixed
    "ks_torus_128_fp64_ct": dict(cfg=2, n=128, precision=0, fused=0, ct=1),
    "ks_torus_128_mixed_ct": dict(cfg=2, n=128, precision=1, fused=0, ct=1),
    "ks_torus_128_fp64_x1u": dict(cfg=2, n=128, precision=0, fused=0,
                                  sched=dict(march_mask=6, march_faces=17, x1_staged=2)),
    "ks_torus_128_mixed_x1u": dict(cfg=2, n=128, precision=1, fused=0,
                                   sched=dict(march_mask=6, march_faces=17, x1_staged=2)),
}


# Measured HBM traffic per launch of the dominant kernel: rocprofv3 FETCH_SIZE and
# WRITE_SIZE (KiB per dispatch) scaled by what the same counters read for a plain
# 1 GiB device copy (FETCH_SIZE x2.0, WRITE_SIZE x1.0), averaged over the launches
# of one RK2 step. Each entry records the digest of the kernel sources it was taken
# on; with any other sources the field is reported as null.
TRAFFIC = {
    # (workload, kernel family): (bytes per launch, source digest)
    # profiles/update_ks_turb_384_hbm_traffic.md, update_ks_torus_192_mixed_128_fp64_hbm_traffic.md,
    # update_ks_torus_128_ct_hbm_traffic.md
    ("ks_turb_384_mixed_plain", "update"): (20828609478, "469e3e1370c9e273"),
    ("ks_turb_384_fp64_plain", "update_x1"): (30566730643, "469e3e1370c9e273"),
    ("ks_torus_192_mixed_plain", "update"): (2607481265, "469e3e1370c9e273"),
    ("ks_torus_128_fp64_plain", "update_x1"): (1133698907, "469e3e1370c9e273"),
    ("ks_torus_128_mixed_ct", "update"): (671370394, "469e3e1370c9e273"),
    ("ks_torus_128_fp64_ct", "update"): (983060125, "469e3e1370c9e273"),
    # profiles/update_amr_like_4096_hbm_traffic.md
    ("amr_like_4096_mixed_plain", "update"): (2569056062, "469e3e1370c9e273"),
}

# Measured VALU wave-instructions per launch (rocprofv3 SQ_INSTS_VALU, mean over the
# launches of two RK2 steps), with the digest of the sources they were counted on.
# With the HIP-event duration of the same kernel they give its VALU issue rate
# against 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz = 39.3e12 lane-instructions/s (one
# wave64 instruction takes 4 cycles of a 16-lane SIMD; FP64 and unpacked FP32 issue
# at the same rate). The counter includes transcendental instructions, which issue
# on a unit of their own, so float kernels heavy in reciprocals and square roots can
# read slightly above 1.
VALU = {
    # profiles/ks_turb_384_valu_counters.md, ks_torus_192_mixed_128_fp64_valu_counters.md,
    # ks_torus_128_ct_valu_counters.md
    ("ks_turb_384_fp64_plain", "flux_x2"): (750792543, "469e3e1370c9e273"),
    ("ks_turb_384_fp64_plain", "flux_x3"): (664407997, "469e3e1370c9e273"),
    ("ks_turb_384_mixed_plain", "flux_x2"): (632278966, "469e3e1370c9e273"),
    ("ks_turb_384_mixed_plain", "flux_x3"): (568482207, "469e3e1370c9e273"),
    ("ks_turb_384_mixed_plain", "flux_x1"): (1033852654, "469e3e1370c9e273"),
    ("ks_turb_384_mixed_plain", "update"): (1255450966, "469e3e1370c9e273"),
    ("ks_turb_384_fp64_plain", "update_x1"): (2592712348, "469e3e1370c9e273"),
    ("ks_torus_128_fp64_plain", "flux_x2"): (27779563, "469e3e1370c9e273"),
    ("ks_torus_128_fp64_plain", "flux_x3"): (24798987, "469e3e1370c9e273"),
    ("ks_torus_192_mixed_plain", "flux_x2"): (79490969, "469e3e1370c9e273"),
    ("ks_torus_192_mixed_plain", "flux_x3"): (71312299, "469e3e1370c9e273"),
    ("ks_torus_192_mixed_plain", "flux_x1"): (129381759, "469e3e1370c9e273"),
    ("ks_torus_192_mixed_plain", "update"): (158204683, "469e3e1370c9e273"),
    ("ks_torus_128_fp64_plain", "update_x1"): (96739932, "469e3e1370c9e273"),
    ("ks_torus_128_fp64_ct", "ct_edges"): (6303829, "469e3e1370c9e273"),
    ("ks_torus_128_mixed_ct", "ct_edges"): (6453333, "469e3e1370c9e273"),
    ("ks_torus_128_fp64_ct", "flux_x2"): (26931940, "469e3e1370c9e273"),
    ("ks_torus_128_fp64_ct", "flux_x3"): (24497943, "469e3e1370c9e273"),
    ("ks_torus_128_mixed_ct", "flux_x2"): (21784795, "469e3e1370c9e273"),
    ("ks_torus_128_mixed_ct", "flux_x3"): (19088117, "469e3e1370c9e273"),
    ("ks_torus_128_fp64_ct", "flux_x1"): (43389954, "469e3e1370c9e273"),
    ("ks_torus_128_mixed_ct", "flux_x1"): (34744871, "469e3e1370c9e273"),
    ("ks_torus_128_fp64_ct", "update"): (39467065, "469e3e1370c9e273"),
    ("ks_torus_128_mixed_ct", "update"): (40744997, "469e3e1370c9e273"),
}
VALU_PEAK = 39.3e12      # lane-instructions/s


def _strip_comments(src: str) -> str:
    """C/C++ source without its comments (string literals kept), so that a change of
    wording in a comment does not count as a change of the kernels."""
    import re
    pat = re.compile(r'"(?:\\.|[^"\\])*"|//[^\n]*|/\*.*?\*/', re.S)
    return pat.sub(lambda m: m.group(0) if m.group(0).startswith('"') else " ", src)


def source_digest(root: str = ROOT) -> str:
    """Digest of the library's sources (comments excluded)."""
    import hashlib
    h = hashlib.sha1()
    for d in (os.path.join(root, "paper_2108_12240_amd", "csrc"), os.path.join(root, "include")):
        for f in sorted(os.listdir(d)):
            if f.endswith((".hip", ".h", ".cpp")):
                with open(os.path.join(d, f), encoding="utf-8") as fh:
                    h.update(f.encode() + b"\0" + _strip_comments(fh.read()).encode())
    return h.hexdigest()[:16]


def bytes_per_unit(kernel: str, rsz: int, nv: int = 9) -> float:
    """Algorithmic HBM bytes per unit of work of each kernel family (unit in unit_of);
    nv rows of state (10 with the entropy field)."""
    u8 = 8
    if kernel == "fill_ghosts":            # per ghost slot: nv values read + nv written
        return 2 * nv * rsz
    if kernel.startswith("flux_x"):        # per face: one cell's nv primitives read, nv fluxes written
        return 2 * nv * rsz
    if kernel == "update":                 # per cell: U_stage, U_base (half the stages), P_stage,
        return nv * (u8 * 1.5 + rsz + 3 * rsz + u8 + rsz)   # 3 face fluxes, U_out, P_out
    if kernel == "update_x1":              # per cell: as update without the x1 faces (computed in place)
        return nv * (u8 * 1.5 + rsz + 2 * rsz + u8 + rsz)
    if kernel == "update_div":             # per cell: as update, with one stored divergence instead of fluxes
        return 9 * u8 * 1.5 + 9 * rsz + 9 * 4 + 9 * u8 + 9 * rsz
    if kernel == "block_flux":             # per zone: P_stage read once, divergence written once
        return 9 * rsz + 9 * 4
    return 0.0


def units_per_launch(kernel: str, info: dict) -> float:
    if kernel == "fill_ghosts":
        return info["ghost_slots"]
    if kernel.startswith("flux_x"):
        return info["nface"][int(kernel[-1]) - 1]
    if kernel in ("update", "update_x1", "update_div", "block_flux"):
        return info["ncell"]
    return 0.0


def grid_info(case, G):
    from paper_2108_12240_amd import bhac as B
    off, dst, _ = B.bhac_plan_ghosts(case.params, case.blocks)
    blk = case.blocks
    nface = [int(((blk[:, 1] + (d == 0)) * (blk[:, 2] + (d == 1)) * (blk[:, 3] + (d == 2))).sum()) for d in range(3)]
    return dict(ghost_slots=int(dst.size), nface=nface, ncell=int(G.nci), nvar=int(G.nvar))


def run_gpu(case, steps, warmup, repeats=1, graph=True, timing_steps=None, phi=None):
    """One continuous CFL-stepped run: `warmup` untimed RK2 steps, then `repeats`
    timed segments of `steps` steps each (HIP events on the launch stream around each
    segment). With graph=True the timed loop replays the captured step graph; the
    per-kernel durations then come from an eager pass of `timing_steps` further steps
    with HIP events around every launch (same kernels, same stream). phi: the face
    field of a constrained-transport grid (host), carried through every step."""
    import torch
    from paper_2108_12240_amd import bhac as B

    G = B.Grid(case.params, case.blocks, device="cuda:0")
    U1, P1 = G.new_state("U"), G.new_state("P")
    if phi is None:
        U, P = G.init(case.prim)
        if graph:
            G.capture_rk2_step(U, P, U1, P1)
        eager = lambda: G.rk2_step(U, P, U1, P1)
    else:
        U, P, ph = G.init_ct(case.prim, phi)
        ph1 = G.new_faces()
        if graph:
            G.capture_rk2_step_ct(U, P, U1, P1, ph, ph1)
        eager = lambda: G.rk2_step_ct(U, P, ph, U1, P1, ph1)
    step = G.launch_rk2_step if graph else eager
    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    B.bhac_get_timing(G.h)
    if not graph:
        B.bhac_set_timing(G.h, True)
    seg = []
    for _ in range(repeats):
        start, stop = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        start.record(stream)
        for _ in range(steps):
            step()
        stop.record(stream)
        torch.cuda.synchronize()
        seg.append(start.elapsed_time(stop))
    if graph:
        B.bhac_set_timing(G.h, True)
        for _ in range(timing_steps or steps):
            eager()
        torch.cuda.synchronize()
    B.bhac_set_timing(G.h, False)
    ktimes = B.bhac_get_timing(G.h)
    info = grid_info(case, G)
    stats = G.stats()
    ts = G.timestep()
    finite = bool(torch.isfinite(P).all().item())
    G.close()
    del U, P, U1, P1
    torch.cuda.empty_cache()
    med = sorted(seg)[len(seg) // 2] if len(seg) % 2 else 0.5 * sum(sorted(seg)[len(seg) // 2 - 1:len(seg) // 2 + 1])
    best = min(seg)
    zu = info["ncell"] * 2 * steps
    return dict(ms_total=sum(seg), ms_per_step=med / steps, ms_per_step_best=best / steps,
                segments_ms=[round(x, 4) for x in seg], value=zu / (med / 1e3), value_best=zu / (best / 1e3),
                ktimes=ktimes, info=info, stats=stats, dt=ts["dt"], finite=finite, graph=graph,
                steps_run=warmup + repeats * steps + (timing_steps or steps if graph else 0))


def valu_rates(res, workload):
    """VALU issue rate of each kernel family with a stored instruction count."""
    out = {}
    dig = source_digest()
    for fam, (launches, total_ms) in res["ktimes"].items():
        m = VALU.get((workload, fam))
        if not m or m[1] != dig or not launches:
            continue
        rate = m[0] * 64 / (total_ms / launches / 1e3)
        out[fam] = dict(bound="alu", achieved=round(rate / 1e12, 2), peak=VALU_PEAK / 1e12,
                        unit="Tlane-instr/s", frac=round(rate / VALU_PEAK, 3))
    return out


def autotune_summary(rep):
    """The autotuner's choice and the spread of the candidates it timed."""
    def label(ch):
        if ch["fused"]:
            return "block-tiled"
        sc = ch["sched"]
        return f"march{sc['march_mask']}/seg{sc['march_faces']}/x1stage{sc['x1_staged']}"
    ms = [t["ms_per_step"] for t in rep["timings"] if t["ms_per_step"] is not None]
    return dict(choice=label(rep["choice"]), cached=rep["cached"], timed=len(ms),
                best_ms=round(min(ms), 4), worst_ms=round(max(ms), 4))


UPDATE_FAMILIES = ("update", "update_x1", "update_div")


def state_bytes(rsz, ct=False):
    return STATE_BYTES[rsz] + (CT_FACE_BYTES if ct else 0.0)


def roofline(res, rsz, workload, ct=False):
    """Roofline of the dominant kernel (largest share of the timed kernels).

    The per-cell update is the kernel that moves the method's state (U_stage, U_base,
    P_stage in, U_out, P_out out); its algorithmic bytes per launch are the state
    bytes of one zone-substep (260 B FP64, 220 B mixed) times the zones. Its own
    traffic (which also reads the face fluxes, and B and psi from P as well as U) is
    reported beside it as kernel_bytes. Any other dominant kernel is measured on its
    own bytes. Where a VALU instruction count is stored for the dominant kernel (on
    the current sources) whose issue time at the chip's peak exceeds the HBM time of
    its bytes, the bound is the VALU peak instead."""
    kt = {k: v for k, v in res["ktimes"].items() if k not in ("step_begin", "step_end", "untimed")}
    dom = max(kt, key=lambda k: kt[k][1])
    launches, total_ms = kt[dom]
    avg_s = total_ms / launches / 1e3
    own = bytes_per_unit(dom, rsz, res["info"]["nvar"]) * units_per_launch(dom, res["info"])
    alg = state_bytes(rsz, ct) * res["info"]["ncell"] if dom in UPDATE_FAMILIES else own
    achieved = alg / avg_s / 1e9
    dig = source_digest()
    measured = TRAFFIC.get((workload, dom))
    traffic = measured[0] if measured and measured[1] == dig else None
    out = dict(kernel=dom, bound="hbm", achieved=round(achieved, 2), peak=HBM_PEAK_GBS, unit="GB/s",
               frac=round(achieved / HBM_PEAK_GBS, 4), traffic=traffic,
               traffic_over_algorithmic=round(traffic / alg, 3) if traffic else None,
               avg_launch_ms=round(total_ms / launches, 4), bytes_per_launch=alg,
               bytes_basis="state bytes per zone-substep x zones" if dom in UPDATE_FAMILIES else "kernel's own bytes",
               kernel_bytes_per_launch=own, kernel_bytes_frac=round(own / avg_s / 1e9 / HBM_PEAK_GBS, 4),
               traffic_over_kernel_bytes=round(traffic / own, 3) if traffic else None,
               share_of_step=round(total_ms / sum(v[1] for v in kt.values()), 3))
    counted = VALU.get((workload, dom))
    if counted and counted[1] == dig and counted[0] * 64 / VALU_PEAK > alg / (HBM_PEAK_GBS * 1e9):
        rate = counted[0] * 64 / avg_s
        out.update(bound="alu", achieved=round(rate / 1e12, 2), peak=VALU_PEAK / 1e12, unit="Tlane-instr/s",
                   frac=round(rate / VALU_PEAK, 4), hbm_frac=round(achieved / HBM_PEAK_GBS, 4))
    return out


def substep_roofline(res, rsz, workload, ct=False):
    """The whole substep against both ceilings: the state bytes at 8 TB/s and the
    method's algorithmic flops (oracle op counter) at the vector peak."""
    zones = res["info"]["ncell"]
    t = res["ms_per_step"] / 2 / 1e3
    sb = state_bytes(rsz, ct)
    hbm = sb * zones / t
    out = dict(ms=round(t * 1e3, 4), state_bytes_per_zone=sb,
               hbm_achieved_GBs=round(hbm / 1e9, 1), hbm_frac=round(hbm / (HBM_PEAK_GBS * 1e9), 4),
               hbm_floor_ms=round(sb * zones / (HBM_PEAK_GBS * 1e9) * 1e3, 4))
    ops = OPCOUNT.get(WORKLOAD_OPS.get(workload, ""))
    if ops:
        fl = ops["algorithmic"] * zones
        out.update(flops_per_zone=round(ops["algorithmic"], 1), alu_achieved_TFLOPs=round(fl / t / 1e12, 2),
                   alu_peak_TFLOPs=FP_PEAK_TFLOPS, alu_frac=round(fl / t / (FP_PEAK_TFLOPS * 1e12), 4),
                   alu_floor_ms=round(fl / (FP_PEAK_TFLOPS * 1e12) * 1e3, 4))
    return out


def host_info():
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        usable = len(os.sched_getaffinity(0))
    except (AttributeError, OSError):
        usable = os.cpu_count() or 1
    omp = int(os.environ.get("OMP_NUM_THREADS", "0") or 0)
    return dict(cpu_model=model, logical_cpus=os.cpu_count(), usable_cpus=usable,
                threads_allowed=min(usable, omp) if omp > 0 else usable)


def _sample_case(case, nblk):
    """The nblk blocks nearest (in level-0 cell units) to the block holding the densest
    cell, as a grid of their own: the same cells, scheme and state; where a sampled
    block's neighbour is not sampled, its halo follows the zero-gradient rule."""
    import numpy as np
    blk = np.asarray(case.blocks)
    scale = 2.0 ** blk[:, 0:1]
    centre = (blk[:, 4:7] + 0.5 * blk[:, 1:4]) / scale
    dens = np.array([case.prim[0, case.ioff[b]:case.ioff[b + 1]].max() for b in range(len(blk))])
    d = np.linalg.norm(centre - centre[int(dens.argmax())], axis=1)
    sel = np.sort(np.argsort(d, kind="stable")[:max(1, min(nblk, len(blk)))])
    prim = np.concatenate([case.prim[:, case.ioff[b]:case.ioff[b + 1]] for b in sel], axis=1)
    return blk[sel], prim


def cpu_baseline(case, seconds_hint: float, threads: int = 1):
    """The oracle as it stands on a bounded sample of the same workload (whole RK2 steps
    of a block sample, its ghost fills included), on `threads` host threads (the
    oracle's block loops; results are bit-identical to one thread)."""
    import numpy as np
    from oracle import oracle as O

    O.set_threads(threads)
    try:
        def steps_on(nblk, budget, max_steps):
            blocks, prim = _sample_case(case, nblk)
            Og = O.OracleGrid(case.params, blocks)
            U, P = Og.init(prim)
            U1, P1 = np.zeros_like(U), np.zeros_like(P)
            steps, el = 0, 0.0
            t0 = time.perf_counter()
            while steps == 0 or (el < budget and steps < max_steps):
                Og.rk2_step(U, P, U1, P1)
                steps += 1
                el = time.perf_counter() - t0
            return int(Og.nci), steps, el, len(blocks)

        nb = case.nblocks
        # probe: one step of a few blocks per thread gives the time per zone-update
        cells, steps, el, _ = steps_on(min(nb, 2 * threads), 0.0, 1)
        per_zu = el / (cells * 2 * steps)
        bs = case.ioff[-1] / nb
        nblk = int(max(1, min(nb, seconds_hint / 2.0 / (per_zu * 2 * bs))))
        cells, steps, el, nsel = steps_on(nblk, 0.8 * seconds_hint, 8)
    finally:
        O.set_threads(1)
    return dict(value=round(cells * 2 * steps / el, 1), unit="zone-updates/s", cores=threads, kind="oracle",
                sample=f"{steps} RK2 step(s) (2 substeps with ghost fills each) of {nsel} of the {nb} blocks "
                       f"({cells} zones; the blocks nearest the densest torus cell, as a grid of their own), "
                       f"{threads} thread(s), {el:.1f} s")


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def copy_bandwidth(nbytes: int = 1 << 30, repeats: int = 10) -> float:
    """Read-plus-write GB/s of a plain device-to-device copy of nbytes (the
    achievable streaming ceiling of this GPU, measured beside the HBM peak)."""
    import torch
    src = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda:0")
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    for _ in range(3):
        dst.copy_(src)
    torch.cuda.synchronize()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record()
    for _ in range(repeats):
        dst.copy_(src)
    b.record()
    torch.cuda.synchronize()
    gbs = 2 * nbytes * repeats / (a.elapsed_time(b) / 1e3) / 1e9
    del src, dst
    torch.cuda.empty_cache()
    return gbs


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20, help="SSP-RK2 steps (2 substeps each) per timed segment")
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--repeats", type=int, default=15, help="timed segments of one continuous run (median and best reported)")
    ap.add_argument("--workload", default="ks_turb_384_mixed_plain", choices=sorted(WORKLOADS))
    ap.add_argument("--compare", default="ks_turb_384_fp64_plain",
                    help="second path on the same grid reported beside the headline ('' to skip)")
    ap.add_argument("--extra", default="ks_torus_128_fp64_plain,ks_torus_192_mixed_plain,amr_like_4096_mixed_plain,"
                                       "ks_torus_128_fp64_ct",
                    help="further workloads timed with --extra-steps per segment ('' to skip)")
    ap.add_argument("--extra-steps", type=int, default=10)
    ap.add_argument("--cpu-seconds", type=float, default=12.0, help="target length of each oracle sample")
    ap.add_argument("--eager", action="store_true", help="time eager launches instead of the captured step graph")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--copy-probe", action="store_true",
                    help="only run a plain 1 GiB device-to-device copy (to calibrate HBM byte counters)")
    args = ap.parse_args(argv)

    if args.copy_probe:
        import torch
        torch.cuda.set_device(0)
        print(json.dumps(dict(copy_probe_bytes=1 << 30, repeats=13, read_plus_write_GBps=round(copy_bandwidth(), 1))),
              flush=True)
        return 0

    if args.gpus != 1:
        print(json.dumps(dict(error=f"this benchmark runs on exactly one GPU (asked for {args.gpus}); "
                                    "the multi-GPU halo exchange is not implemented in this library")), flush=True)
        return 2

    import torch
    from paper_2108_12240_amd import inputs as I

    assert torch.cuda.is_available(), "bench.py needs a ROCm GPU"
    torch.cuda.set_device(0)
    cases, faces = {}, {}

    def make(name):
        w = dict(WORKLOADS[name])
        kw = {k: w[k] for k in ("n", "n0", "bs", "levels") if k in w}
        key = (str(w["cfg"]), str(kw), bool(w.get("entropy")), bool(w.get("ct")))
        if key not in cases:
            log(f"inputs of {name}")
            c0 = I.make_case(w["cfg"], **kw)
            if w.get("ct"):
                c0, faces[key] = I.torus_with_face_field(c0)
            cases[key] = I.with_entropy(c0) if w.get("entropy") else c0
        c0 = cases[key]
        w["phi"] = faces.get(key)
        c = I.Case(c0.name, dict(c0.params), c0.blocks, c0.prim, c0.ioff, c0.steps)
        if w["fused"] == "auto":
            from paper_2108_12240_amd import autotune
            params, report = autotune.tune(dict(c.params, precision=w["precision"]), c.blocks, c.prim)
            w["fused"] = int(params["fused"])
            w["sched"] = params.get("sched")
            w["autotune"] = report
        c.params = dict(c.params, precision=w["precision"], fused=w["fused"])
        if w.get("sched"):
            c.params["sched"] = w["sched"]
        return c, w

    def measure(name, steps):
        c, w = make(name)
        log(f"timing {name}: {args.warmup} warmup + {args.repeats} x {steps} RK2 steps")
        r = run_gpu(c, steps, args.warmup, repeats=args.repeats, graph=not args.eager,
                    timing_steps=min(steps, 4), phi=w.get("phi"))
        rsz = 4 if w["precision"] == 1 else 8
        summary = dict(workload=name, value=round(r["value"], 1), value_best=round(r["value_best"], 1),
                       ms_per_step=round(r["ms_per_step"], 4), ms_per_step_best=round(r["ms_per_step_best"], 4),
                       segments_ms=r["segments_ms"], steps_per_segment=steps, dtype="f64" if rsz == 8 else "f32+f64",
                       zones=r["info"]["ncell"], roofline=roofline(r, rsz, name, bool(w.get("ct"))),
                       substep=substep_roofline(r, rsz, name, bool(w.get("ct"))),
                       kernel_ms={k: round(v[1] / max(v[0], 1), 4) for k, v in r["ktimes"].items()},
                       valu=valu_rates(r, name), c2p=r["stats"], finite=r["finite"], dt_last=r["dt"])
        if "autotune" in w:
            summary["autotune"] = autotune_summary(w["autotune"])
        return c, w, r, summary

    case, w, res, head = measure(args.workload, args.steps)
    copy_gbs = copy_bandwidth()
    head["roofline"]["copy_ceiling_GBs"] = round(copy_gbs, 1)
    if head["roofline"]["unit"] == "GB/s":
        head["roofline"]["frac_of_copy"] = round(head["roofline"]["achieved"] / copy_gbs, 4)
    head["substep"]["frac_of_copy"] = round(head["substep"]["hbm_achieved_GBs"] / copy_gbs, 4)
    rsz = 4 if w["precision"] == 1 else 8
    out = dict(metric=METRIC, value=head["value"], unit="zone-updates/s", n_gpus=1, steps=args.steps,
               warmup=args.warmup, ms_per_step=head["ms_per_step"], higher_is_better=True,
               scaling="weak", vs_baseline=None, dtype=head["dtype"],
               data="synthetic (seeded Kerr-Schild torus, no dataset)",
               config=dict(workload=args.workload, zones=res["info"]["ncell"], blocks=int(case.nblocks),
                           block_sizes=sorted(set(int(v) for v in case.blocks[:, 1])),
                           levels=sorted(set(int(v) for v in case.blocks[:, 0])), substeps_per_step=2,
                           recon="PPM", flux="HLL", time_step="CFL (lagged wave-speed reduction)",
                           fused=bool(w["fused"]), graph=res["graph"], repeats=args.repeats,
                           steps_run=res["steps_run"]),
               value_best=head["value_best"], ms_per_step_best=head["ms_per_step_best"],
               segments_ms=head["segments_ms"], roofline=head["roofline"], substep=head["substep"],
               kernel_ms=head["kernel_ms"], valu=head["valu"], c2p=head["c2p"], finite=head["finite"])
    if "autotune" in w:
        out["config"]["autotune"] = head["autotune"]
    if args.compare:
        _, _, r2, cmp_ = measure(args.compare, args.steps)
        cmp_["headline_speedup_over_this"] = round(res["value"] / r2["value"], 3)
        out["compare"] = cmp_
    if args.extra:
        out["configs"] = {}
        for name in [x for x in args.extra.split(",") if x]:
            _, _, _, ex = measure(name, args.extra_steps)
            out["configs"][name] = ex
    if not args.no_cpu_baseline:
        host = host_info()
        log(f"oracle on the host: {host}")
        base = cpu_baseline(case, args.cpu_seconds, threads=1)
        base["host"] = host
        if host["threads_allowed"] > 1:
            base["all_cores"] = cpu_baseline(case, args.cpu_seconds, threads=host["threads_allowed"])
        out["cpu_baseline"] = base
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
