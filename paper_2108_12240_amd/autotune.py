"""Choose the faster substep implementation for a workload by timing it.

Candidates are the unfused kernels (``fused = 0``) and the block-tiled kernels
(``fused = 1``, where the grid supports them). Each candidate advances a copy of
the workload's initial state with replays of the captured RK2-step graph; the
fastest wins. Choices are cached in a JSON file keyed by the GPU architecture and
a signature of the workload (metric, dimensionality, reconstruction, flux,
precision, and the histogram of block (level, size)), so later runs skip the
timing. Everything timed runs in the library's kernels.
"""
from __future__ import annotations

import hashlib
import json
import os

import numpy as np

from . import bhac as B

CACHE_ENV = "BHAC_AUTOTUNE_CACHE"
CANDIDATES = ({"fused": 0}, {"fused": 1})


def cache_path() -> str:
    return os.environ.get(CACHE_ENV) or os.path.join(os.path.expanduser("~"), ".cache", "bhac_autotune.json")


def signature(params: dict, blocks: np.ndarray) -> dict:
    keys = ("metric", "ndim", "recon", "flux", "precision", "nghost")
    hist = {}
    for blk in np.asarray(blocks):
        k = f"{int(blk[0])}:{int(blk[1])}x{int(blk[2])}x{int(blk[3])}"
        hist[k] = hist.get(k, 0) + 1
    return dict({k: int(params[k]) for k in keys}, blocks=dict(sorted(hist.items())))


def _key(arch: str, sig: dict) -> str:
    return arch + ":" + hashlib.sha1(json.dumps(sig, sort_keys=True).encode()).hexdigest()[:16]


def _load(path):
    try:
        with open(path) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def _time_candidate(params, blocks, prim, steps, warmup):
    import torch
    G = B.Grid(params, blocks)
    try:
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
        return a.elapsed_time(b) / steps
    finally:
        G.close()


def tune(params: dict, blocks: np.ndarray, prim: np.ndarray, steps: int = 3, warmup: int = 1,
         path: str | None = None, refresh: bool = False):
    """Return (params with the chosen variant, report). The report lists each
    candidate's ms per RK2 step (None where the grid does not support it)."""
    import torch
    path = path or cache_path()
    arch = torch.cuda.get_device_properties(0).gcnArchName.split(":")[0]
    sig = signature(params, blocks)
    key = _key(arch, sig)
    cache = _load(path)
    if not refresh and key in cache:
        entry = cache[key]
        return dict(params, **entry["choice"]), dict(entry, cached=True)
    timings = []
    for cand in CANDIDATES:
        p = dict(params, **cand)
        try:
            ms = _time_candidate(p, blocks, prim, steps, warmup)
        except B.BhacError as e:
            if e.code != B.BHAC_EUNSUPPORTED:
                raise
            ms = None
        timings.append(dict(choice=cand, ms_per_step=ms))
    ok = [t for t in timings if t["ms_per_step"] is not None]
    best = min(ok, key=lambda t: t["ms_per_step"])
    entry = dict(arch=arch, signature=sig, choice=best["choice"], timings=timings)
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
