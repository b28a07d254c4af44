"""Choose the substep implementation and kernel schedule for a workload by timing.

Candidates are the block-tiled kernels (``fused = 1``, where the grid supports
them) and the unfused kernels (``fused = 0``) under every schedule of the
``bhac_schedule`` search space: which directions take the line-march kernel and
which the face kernel, how long a march segment may be, and how the x1 faces are
computed where x1 is not marched (a face kernel reading memory, a face kernel
staging rows in LDS, or the update kernel itself). The default search is staged
(all march masks first, then segment lengths and the other x1 modes for the two
best); an exhaustive one times every candidate. Schedules that resolve to the
same kernels (an x1 mode the grid does not support, segment lengths longer than
every line) are timed once.
Each candidate advances a copy of the workload's initial state with replays of
the captured RK2-step graph; the fastest wins. Every schedule computes the same
fluxes, so the choice changes speed, not results. Choices are cached in a JSON
file keyed by the GPU architecture and a signature of the workload (metric,
dimensionality, reconstruction, flux, precision, block tree or not, entropy field
or not, and the histogram of block (level, size)) and of the library's sources,
so later runs skip the timing and a change of the kernels invalidates the choice. Everything
timed runs in the library's kernels.
"""
from __future__ import annotations

import hashlib
import json
import os

import numpy as np

from . import bhac as B

CACHE_ENV = "BHAC_AUTOTUNE_CACHE"
SEARCH_VERSION = 3
MARCH_FACES = (9, 17, 33)


def candidates(params: dict) -> list:
    """The search space: the block-tiled substep, then the unfused one under every
    schedule (march mask x x1 mode x segment length)."""
    out = [{"fused": 1}]
    ndim = int(params["ndim"])
    for mask in range(1 << ndim):
        for x1 in ((0,) if mask & 1 else (0, 1, 2)):
            for faces in (MARCH_FACES if mask else (MARCH_FACES[1],)):
                out.append({"fused": 0, "sched": {"march_mask": mask, "march_faces": faces, "x1_staged": x1}})
    return out


def cache_path() -> str:
    return os.environ.get(CACHE_ENV) or os.path.join(os.path.expanduser("~"), ".cache", "bhac_autotune.json")


def source_digest() -> str:
    """Digest of the library's kernel and interface sources (C/C++ comments
    excluded), so that a choice timed on other kernels is not reused."""
    import re
    pat = re.compile(r'"(?:\\.|[^"\\])*"|//[^\n]*|/\*.*?\*/', re.S)
    here = os.path.dirname(os.path.abspath(__file__))
    h = hashlib.sha1()
    for d in (os.path.join(here, "csrc"), os.path.join(os.path.dirname(here), "include")):
        for f in sorted(os.listdir(d)):
            if f.endswith((".hip", ".h", ".cpp")):
                with open(os.path.join(d, f), encoding="utf-8") as fh:
                    src = pat.sub(lambda m: m.group(0) if m.group(0).startswith('"') else " ", fh.read())
                h.update(f.encode() + b"\0" + src.encode())
    return h.hexdigest()[:16]


def signature(params: dict, blocks: np.ndarray) -> dict:
    keys = ("metric", "ndim", "recon", "flux", "precision", "nghost")
    hist = {}
    for blk in np.asarray(blocks):
        k = f"{int(blk[0])}:{int(blk[1])}x{int(blk[2])}x{int(blk[3])}"
        hist[k] = hist.get(k, 0) + 1
    return dict({k: int(params[k]) for k in keys}, amr=int(params.get("amr", 0)),
                entropy=int(params.get("entropy", 0)), search=SEARCH_VERSION, sources=source_digest(),
                blocks=dict(sorted(hist.items())))


def _key(arch: str, sig: dict) -> str:
    return arch + ":" + hashlib.sha1(json.dumps(sig, sort_keys=True).encode()).hexdigest()[:16]


def _load(path):
    try:
        with open(path) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def _time_candidate(params, blocks, prim, steps, warmup, seen):
    """ms per RK2 step of one candidate, or None where the grid rejects it or its
    resolved schedule was already timed."""
    import torch
    try:
        G = B.Grid(params, blocks)
    except B.BhacError as e:
        if e.code != B.BHAC_EUNSUPPORTED:
            raise
        return None, None
    try:
        resolved = None
        if not params["fused"]:
            resolved = G.schedule()
            if not any(resolved["march_mask"] & (1 << d) for d in range(int(params["ndim"]))):
                resolved["march_faces"] = 0          # unused when no direction marches
            if any(resolved == r for r in seen):
                return None, resolved
            seen.append(resolved)
        U, P = G.init(prim)
        U1, P1 = G.new_state("U"), G.new_state("P")
        G.capture_rk2_step(U, P, U1, P1)
        for _ in range(warmup):
            G.launch_rk2_step()
        torch.cuda.synchronize()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        for _ in range(steps):
            G.launch_rk2_step()
        b.record()
        torch.cuda.synchronize()
        return a.elapsed_time(b) / steps, resolved
    finally:
        G.close()


def _staged(params, blocks, prim, steps, warmup, seen, timings):
    """Two-stage search: every march mask at the middle segment length with the
    staged x1 face kernel where x1 is not marched (and the block-tiled kernels),
    then the other segment lengths and the other two x1 modes for the two fastest
    masks."""
    def run(cands):
        for cand in cands:
            ms, _ = _time_candidate(dict(params, **cand), blocks, prim, steps, warmup, seen)
            timings.append(dict(choice=cand, ms_per_step=ms))

    def sched(mask, faces, x1):
        return {"fused": 0, "sched": {"march_mask": mask, "march_faces": faces, "x1_staged": x1}}

    mid = MARCH_FACES[len(MARCH_FACES) // 2]
    run([{"fused": 1}] + [sched(m, mid, 0 if m & 1 else 1) for m in range(1 << int(params["ndim"]))])
    plain = sorted((t for t in timings if t["ms_per_step"] is not None and not t["choice"]["fused"]),
                   key=lambda t: t["ms_per_step"])
    second = []
    for t in plain[:2]:
        sc = t["choice"]["sched"]
        if sc["march_mask"]:
            second += [sched(sc["march_mask"], f, sc["x1_staged"]) for f in MARCH_FACES if f != mid]
        if not sc["march_mask"] & 1:
            second += [sched(sc["march_mask"], mid, x) for x in (0, 1, 2) if x != sc["x1_staged"]]
    run(second)


def tune(params: dict, blocks: np.ndarray, prim: np.ndarray, steps: int = 3, warmup: int = 1,
         path: str | None = None, refresh: bool = False, search: str = "staged"):
    """Return (params with the chosen variant, report). ``search`` is "staged" (about
    half the candidates, see _staged) or "exhaustive" (every candidate). The report
    lists each timed candidate's ms per RK2 step (None where the grid does not
    support it or an equal schedule was timed already)."""
    import torch
    if search not in ("staged", "exhaustive"):
        raise ValueError(f"unknown search {search!r}")
    path = path or cache_path()
    arch = torch.cuda.get_device_properties(0).gcnArchName.split(":")[0]
    sig = signature(params, blocks)
    key = _key(arch, sig) + ":" + search
    cache = _load(path)
    if not refresh and key in cache:
        entry = cache[key]
        return dict(params, **entry["choice"]), dict(entry, cached=True)
    timings, seen = [], []
    if search == "staged":
        _staged(params, blocks, prim, steps, warmup, seen, timings)
    else:
        for cand in candidates(params):
            ms, _ = _time_candidate(dict(params, **cand), blocks, prim, steps, warmup, seen)
            timings.append(dict(choice=cand, ms_per_step=ms))
    ok = [t for t in timings if t["ms_per_step"] is not None]
    best = min(ok, key=lambda t: t["ms_per_step"])
    entry = dict(arch=arch, signature=sig, search=search, choice=best["choice"], timings=timings)
    cache[key] = entry
    try:
        os.makedirs(os.path.dirname(path), exist_ok=True)
        tmp = path + ".tmp"
        with open(tmp, "w") as f:
            json.dump(cache, f, indent=1, sort_keys=True)
        os.replace(tmp, path)
    except OSError:
        pass
    return dict(params, **best["choice"]), dict(entry, cached=False)
