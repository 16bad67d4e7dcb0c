"""Autotuner for the decomposition and tile parameters of the interaction kernels.

The kernels' LDS tiles are fixed at compile time, in a few variants chosen at
run time; what the tuner searches:
  - the decomposition: the size of the cells (``cell_target``: particles per
    top cell at the mean density, subject to edge >= max h; on the
    hierarchy, ``split_count``: the particle count above which a cell is
    split) and the slack on h when cells are built (``h_margin``);
  - the tiles: the work layout of the sweeps (``sweep``: sources split
    between the four wavefronts of a unit, or staged once and shared, with
    16 targets per wavefront), the density staging (``staging``: compact,
    four work-groups per CU, or wide, room for larger cells) and the cell
    size above which the force sweep takes 256 targets per unit
    (``shared_min``).
For a given workload the tuner times a captured pass (build, sort, density,
force) for each candidate, one group of parameters at a time (the best of a
group is kept while the next is searched), and keeps the fastest.  Results
are cached per (GPU architecture, precision, workload class) in a JSON
file, so a workload of the same class is not re-tuned.
"""
from __future__ import annotations

import json
import math
import os
import time
from typing import Callable, Optional

CANDIDATES = [
    {"cell_target": 24, "h_margin": 0.1},
    {"cell_target": 32, "h_margin": 0.1},
    {"cell_target": 48, "h_margin": 0.1},
    {"cell_target": 64, "h_margin": 0.1},
    {"cell_target": 96, "h_margin": 0.1},
    {"cell_target": 128, "h_margin": 0.1},
    {"cell_target": 64, "h_margin": 0.05},
    # a wider margin stages more of each source at once: fewer stagings again
    # when h starts far from its root (random sets solved from a uniform guess)
    {"cell_target": 32, "h_margin": 0.2},
    {"cell_target": 48, "h_margin": 0.2},
]

# tile groups searched after the decomposition (sph.SPH_SWEEP_* and
# sph.SPH_STAGING_* values: 2 split, 1 shared; 0 compact, 1 wide)
LAYOUT_CANDIDATES = [
    {"sweep": 2, "staging": 0},
    {"sweep": 2, "staging": 1},
    {"sweep": 1, "staging": 0},
]
SHARED_MIN_CANDIDATES = [{"shared_min": 128}, {"shared_min": 64}, {"shared_min": 256}]
STAGES = [CANDIDATES, LAYOUT_CANDIDATES, SHARED_MIN_CANDIDATES]

# hierarchical decomposition: leaf size (the split rule's count) for multi-resolution sets
TREE_CANDIDATES = [
    {"split_count": 64},
    {"split_count": 128},
    {"split_count": 256},
    {"split_count": 384},
    {"split_count": 512},
]

CACHE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "_tune", "autotune.json")


def workload_class(n_total: int, n_boxes: int, precision: str) -> str:
    """Workloads of the same class share a tuning: log2 buckets of the
    particles per box and of the box count."""
    ppb = max(1, n_total // max(1, n_boxes))
    return f"{precision}|ppb2^{int(math.log2(ppb))}|boxes2^{int(math.log2(max(1, n_boxes)))}"


def load_cache(path: str = CACHE) -> dict:
    try:
        with open(path) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def save_cache(cache: dict, path: str = CACHE) -> None:
    os.makedirs(os.path.dirname(path), exist_ok=True)
    tmp = path + ".tmp"
    with open(tmp, "w") as f:
        json.dump(cache, f, indent=1, sort_keys=True)
    os.replace(tmp, path)


class CandidateUnusable(Exception):
    """Raised by a timer for a candidate the workload cannot use: it is skipped."""


def _unusable(e: Exception) -> bool:
    """A candidate the workload cannot use: the timer says so, or the library
    refused it for capacity (a cell or grid beyond the kernels' limits), state
    or a grid too coarse for h in a periodic box.  Anything else (a HIP error,
    a wrong result, a bug) is raised."""
    if isinstance(e, CandidateUnusable):
        return True
    from . import sph
    return isinstance(e, sph.SPHError) and e.status in (sph.SPH_E_CAPACITY, sph.SPH_E_STATE,
                                                       sph.SPH_E_H_TOO_LARGE)


def choose(timings: dict) -> dict:
    """Fastest candidate (ties: the earlier one)."""
    best_key = min(timings, key=lambda k: (timings[k], list(timings).index(k)))
    return json.loads(best_key)


def tune(time_candidate: Callable[[dict], float], key: str, arch: str, candidates=None,
         cache_path: str = CACHE, force: bool = False) -> dict:
    """Return the best parameters for (arch, key), timing candidates if needed.

    time_candidate(params) -> seconds per pass (lower is better).  A candidate
    the workload cannot use (CandidateUnusable, or the library's capacity or
    state refusal) is skipped; every other exception propagates.
    """
    candidates = CANDIDATES if candidates is None else candidates
    cache = load_cache(cache_path)
    full = f"{arch}|{key}"
    if not force and full in cache:
        return dict(cache[full]["best"], cached=True)
    timings, skipped = {}, {}
    for c in candidates:
        try:
            timings[json.dumps(c, sort_keys=True)] = float(time_candidate(c))
        except Exception as e:
            if not _unusable(e):
                raise
            skipped[json.dumps(c, sort_keys=True)] = str(e)
    if not timings:
        raise RuntimeError("no autotune candidate ran")
    best = choose(timings)
    cache[full] = {"best": best, "timings": timings, "skipped": skipped, "when": time.time()}
    save_cache(cache, cache_path)
    return dict(best, cached=False)


def tune_staged(time_candidate: Callable[[dict], float], key: str, arch: str, stages=None,
                cache_path: str = CACHE, force: bool = False) -> dict:
    """Coordinate search over groups of parameters: each stage's candidates
    are timed on top of the best of the stages before (same timer contract
    and skipping rules as tune()); the final best is cached under (arch, key)."""
    stages = STAGES if stages is None else stages
    cache = load_cache(cache_path)
    full = f"{arch}|{key}|staged"
    if not force and full in cache:
        return dict(cache[full]["best"], cached=True)
    best: dict = {}
    timings, skipped = {}, {}
    for stage in stages:
        stage_t = {}
        for c in stage:
            cand = dict(best, **c)
            k = json.dumps(cand, sort_keys=True)
            if k in timings:
                stage_t[k] = timings[k]
                continue
            try:
                stage_t[k] = timings[k] = float(time_candidate(cand))
            except Exception as e:
                if not _unusable(e):
                    raise
                skipped[k] = str(e)
        if stage_t:
            best = choose(stage_t)
    if not timings:
        raise RuntimeError("no autotune candidate ran")
    cache[full] = {"best": best, "timings": timings, "skipped": skipped, "when": time.time()}
    save_cache(cache, cache_path)
    return dict(best, cached=False)


def gpu_timer(ps, precision: str, batch=None, reps: int = 3, arch: Optional[str] = None, h_init=None,
              fixed: Optional[dict] = None):
    """A time_candidate function for tune(): median of `reps` graph replays of
    the whole pass (build, sort, density from the initial h, force).  h_init
    (a device tensor) replaces the set's initial h; `fixed` holds parameters
    common to every candidate (for instance max_depth)."""
    import torch
    from . import sph

    def run(params: dict) -> float:
        parts = sph.Particles.from_numpy(ps, "cuda:0")
        h0 = parts.h.clone() if h_init is None else h_init.clone()
        ctx = sph.Context(ps.box, precision=precision, **dict(fixed or {}, **params))
        stream = torch.cuda.Stream()
        try:
            with torch.cuda.stream(stream):
                ctx.graph_capture(parts, batch, h_init=h0)
                ctx.check(allow_unconverged=False)
                times = []
                for _ in range(reps):
                    a = torch.cuda.Event(enable_timing=True)
                    b = torch.cuda.Event(enable_timing=True)
                    a.record()
                    ctx.graph_launch()
                    b.record()
                    b.synchronize()
                    times.append(a.elapsed_time(b) * 1e-3)
                ctx.check()
        finally:
            ctx.close()
        times.sort()
        return times[len(times) // 2]

    return run
