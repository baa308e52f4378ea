"""Autotuner for the acceleration structure and the traversal parameters.

For a given scene, set of views and render settings, it times candidate launch
configurations: node format, scheduler, LDS stack depth, resident waves per
CU, block size and the persistent lane-refill threshold.  Every candidate's
image must be bit-identical to the FP32 plain-scheduler image, since changing
these parameters must never change a hit.  The fastest configuration per
(node format, scheduler) is returned and cached in a JSON file keyed by the
device, the scene and the render settings.  `autotune_width` also chooses the
node width (2, 4 or 8 children per node), which needs one build per width.
"""
from __future__ import annotations

import hashlib
import itertools
import json
import os
import time
from typing import Dict, Iterable, List, Optional

import numpy as np

from . import RTQ_NODE_FP32, RTQ_NODE_Q8, SCHED_MEGAKERNEL, SCHED_PERSISTENT, SCHED_PLAIN, render

STACK_ENTRY_BYTES = 6  # LDS bytes per traversal-stack entry and lane
DEFAULT_CACHE = os.environ.get("RTQ_AUTOTUNE_CACHE", os.path.join(os.path.expanduser("~"), ".cache", "rtq",
                                                                   "autotune.json"))

GRID = {
    SCHED_PERSISTENT: dict(stack_depth=[12, 16, 20, 24], waves_per_cu=[16, 24, 32], block=[128, 256],
                           refill=[8, 16, 32]),
    SCHED_MEGAKERNEL: dict(stack_depth=[12, 16, 20, 24], waves_per_cu=[16, 24, 32], block=[128, 256],
                           refill=[8, 16, 32]),
    SCHED_PLAIN: dict(stack_depth=[12, 16, 20, 24], block=[64, 128, 256]),
}
QUICK_GRID = {
    SCHED_PERSISTENT: dict(stack_depth=[16, 20], waves_per_cu=[24, 32], block=[128, 256], refill=[8]),
    SCHED_MEGAKERNEL: dict(stack_depth=[16, 20], waves_per_cu=[24, 32], block=[256], refill=[8]),
    SCHED_PLAIN: dict(stack_depth=[12, 16], block=[64, 128]),
}


def _key(S, cams, settings) -> str:
    import torch
    h = hashlib.sha256()
    h.update(torch.cuda.get_device_name(0).encode())
    info = S.info()
    for k in ("n_instances", "n_prototypes", "n_unique_quads", "n_instanced_quads", "tlas_nodes", "blas_nodes"):
        h.update(str(info[k]).encode())
    for c in cams:
        h.update(repr((c.eye, c.look, c.up, c.vfov_deg, c.w, c.h)).encode())
    h.update(repr((settings.spp, settings.depth)).encode())
    return h.hexdigest()[:20]


def _candidates(grid: Dict[str, List[int]]) -> Iterable[dict]:
    keys = sorted(grid)
    for vals in itertools.product(*(grid[k] for k in keys)):
        yield dict(zip(keys, vals))


def autotune_render(S, cams, settings, formats=(RTQ_NODE_Q8, RTQ_NODE_FP32),
                    schedulers=(SCHED_PERSISTENT, SCHED_PLAIN), grid: Optional[dict] = None, reps: int = 2,
                    cache: Optional[str] = DEFAULT_CACHE, log=None) -> dict:
    """Returns {"<format>/<scheduler>": {"opts": {...}, "ms": t}, ...} plus "table"."""
    import torch
    grid = grid or GRID
    key = _key(S, cams, settings)
    if cache and os.path.exists(cache):
        try:
            stored = json.load(open(cache))
            if key in stored:
                return stored[key]
        except (OSError, ValueError):
            pass
    n_pix = sum(c.w * c.h for c in cams)
    img = torch.empty(n_pix, device="cuda")
    frame0 = settings.frame
    # reference: FP32 plain when the scene has FP32 nodes (4-wide), else quantized plain
    ref_fmt = RTQ_NODE_FP32 if S.info()["formats"] & RTQ_NODE_FP32 else RTQ_NODE_Q8
    render(S, cams, settings, images=img, node_format=ref_fmt, scheduler=SCHED_PLAIN)
    ref = img.clone()
    lim = torch.cuda.get_device_properties(0).shared_memory_per_block if hasattr(
        torch.cuda.get_device_properties(0), "shared_memory_per_block") else 65536
    result: Dict[str, dict] = {}
    table = []
    for fmt in formats:
        for sched in schedulers:
            best = None
            for cand in _candidates(grid[sched]):
                if cand["block"] * cand["stack_depth"] * STACK_ENTRY_BYTES > lim:
                    continue
                opts = dict(node_format=fmt, scheduler=sched, **cand)
                render(S, cams, settings, images=img, **opts)  # warm
                torch.cuda.synchronize()
                if not torch.equal(img.view(torch.int32), ref.view(torch.int32)):
                    raise RuntimeError(f"autotune: {opts} changed the image")
                t0 = time.perf_counter()
                for r in range(reps):
                    settings.frame = frame0 + 1 + r
                    render(S, cams, settings, images=img, **opts)
                torch.cuda.synchronize()
                ms = 1e3 * (time.perf_counter() - t0) / reps
                settings.frame = frame0
                table.append(dict(opts, ms=round(ms, 3)))
                if log:
                    log(f"autotune {opts}: {ms:.2f} ms")
                if best is None or ms < best[1]:
                    best = (opts, ms)
            result[f"{fmt}/{sched}"] = {"opts": best[0], "ms": round(best[1], 3)}
    result["table"] = table
    if cache:
        try:
            os.makedirs(os.path.dirname(cache), exist_ok=True)
            stored = json.load(open(cache)) if os.path.exists(cache) else {}
            stored[key] = result
            json.dump(stored, open(cache, "w"), indent=1)
        except (OSError, ValueError):
            pass
    return result


def autotune_trace(S, rays, formats=(RTQ_NODE_Q8, RTQ_NODE_FP32), schedulers=(SCHED_PERSISTENT, SCHED_PLAIN),
                   grid: Optional[dict] = None, reps: int = 3, log=None) -> dict:
    """Tune closest-hit queries on a fixed ray set; every candidate must return
    hits bit-identical to the FP32 plain reference."""
    import torch
    from . import trace_closest
    grid = grid or GRID
    lim = 65536
    ref = trace_closest(S, rays, node_format=RTQ_NODE_FP32, scheduler=SCHED_PLAIN)
    torch.cuda.synchronize()
    result: Dict[str, dict] = {}
    table = []
    for fmt in formats:
        for sched in schedulers:
            best = None
            for cand in _candidates(grid[sched]):
                if cand["block"] * cand["stack_depth"] * STACK_ENTRY_BYTES > lim:
                    continue
                opts = dict(node_format=fmt, scheduler=sched, **cand)
                h = trace_closest(S, rays, **opts)
                torch.cuda.synchronize()
                for k in ("t", "u", "v", "inst", "prim"):
                    if not torch.equal(getattr(h, k).view(torch.int32), getattr(ref, k).view(torch.int32)):
                        raise RuntimeError(f"autotune: {opts} changed the hits ({k})")
                t0 = time.perf_counter()
                for _ in range(reps):
                    trace_closest(S, rays, **opts)
                torch.cuda.synchronize()
                ms = 1e3 * (time.perf_counter() - t0) / reps
                table.append(dict(opts, ms=round(ms, 3)))
                if log:
                    log(f"autotune trace {opts}: {ms:.2f} ms")
                if best is None or ms < best[1]:
                    best = (opts, ms)
            result[f"{fmt}/{sched}"] = {"opts": best[0], "ms": round(best[1], 3)}
    result["table"] = table
    return result


def autotune_build(scene_arrays, cams, settings, widths=(4, 8, 2), open_pcts=(0,),
                   schedulers=(SCHED_PERSISTENT,), grid: Optional[dict] = None, reps: int = 2,
                   build_opts: Optional[dict] = None, rays=None, log=None) -> dict:
    """Choose the build: the node width and how many top-level entries
    opening instances adds (rtq_build_opts.open_pct; 0 is the library's
    default).  The scene (generator arrays) is built once per (width, opening)
    pair, the quantized-node launches of each are tuned, and the fastest pair
    is returned with its launch options.  Every build's frames (and closest
    hits of `rays`, an [n, 8] FP32 device tensor, when given) must equal the
    4-wide FP32 plain reference bit for bit.  The scenes are freed before
    returning.

    Returns {"best": {"node_width": w, "open_pct": p, "opts": {...}, "ms": t},
    "builds": {(w, p): {...}}}."""
    import torch
    from . import Scene, trace_closest
    build_opts = dict(build_opts or {})
    grid = grid or QUICK_GRID
    S4 = Scene(scene_arrays, **build_opts)
    n_pix = sum(c.w * c.h for c in cams)
    img = torch.empty(n_pix, device="cuda")
    render(S4, cams, settings, images=img, node_format=RTQ_NODE_FP32, scheduler=SCHED_PLAIN)
    ref = img.clone()
    ref_hits = trace_closest(S4, rays, node_format=RTQ_NODE_FP32, scheduler=SCHED_PLAIN) if rays is not None else None
    torch.cuda.synchronize()
    S4.close()
    builds = {}
    best = None
    for w in widths:
        for pct in open_pcts:
            S = Scene(scene_arrays, **dict(build_opts, node_width=w, open_pct=pct))
            render(S, cams, settings, images=img, node_format=RTQ_NODE_Q8, scheduler=SCHED_PERSISTENT)
            torch.cuda.synchronize()
            if not torch.equal(img.view(torch.int32), ref.view(torch.int32)):
                raise RuntimeError(f"autotune: node width {w}, opening {pct} changed the image")
            if ref_hits is not None:
                h = trace_closest(S, rays, node_format=RTQ_NODE_Q8, scheduler=SCHED_PERSISTENT)
                torch.cuda.synchronize()
                for k in ("t", "u", "v", "inst", "prim"):
                    if not torch.equal(getattr(h, k).view(torch.int32), getattr(ref_hits, k).view(torch.int32)):
                        raise RuntimeError(f"autotune: node width {w}, opening {pct} changed the hits ({k})")
            r = autotune_render(S, cams, settings, formats=(RTQ_NODE_Q8,), schedulers=schedulers, grid=grid,
                                reps=reps, cache=None, log=log)
            r.pop("table", None)
            info = S.info()
            top = min(r.values(), key=lambda x: x["ms"])
            builds[(w, pct)] = dict(top, nodes=info["tlas_nodes"] + info["blas_nodes"],
                                    depth=[info["tlas_depth"], info["blas_depth_max"]],
                                    top_entries=info["n_top_entries"])
            if log:
                log(f"autotune width {w}, opening {pct}: {builds[(w, pct)]}")
            if best is None or top["ms"] < best["ms"]:
                best = dict(node_width=w, open_pct=pct, opts=top["opts"], ms=top["ms"])
            S.close()
    return {"best": best, "builds": builds}


def autotune_width(scene_arrays, cams, settings, widths=(4, 8, 2), schedulers=(SCHED_PERSISTENT,),
                   grid: Optional[dict] = None, reps: int = 2, build_opts: Optional[dict] = None, rays=None,
                   log=None) -> dict:
    """autotune_build over node widths at the default opening.

    Returns {"best": {"node_width": w, "opts": {...}, "ms": t}, "widths": {w: {...}}}."""
    opening = (build_opts or {}).get("open_pct", 0)
    r = autotune_build(scene_arrays, cams, settings, widths=widths, open_pcts=(opening,), schedulers=schedulers,
                       grid=grid, reps=reps, build_opts={k: v for k, v in (build_opts or {}).items()
                                                         if k != "open_pct"}, rays=rays, log=log)
    return {"best": r["best"], "widths": {w: v for (w, _), v in r["builds"].items()}}
