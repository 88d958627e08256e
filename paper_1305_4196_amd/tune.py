"""Autotuner for the brick-task launch configuration.

The cell tasks of Sec. II.D.2 are blocked by a tunable b_x x b_y x b_z and the
paper picks the blocking by benchmark; here the same choice (plus the
workgroup size) is made per system by timing the candidates on the GPU.

Candidates come from a score of every shape of 1..4 cells per axis on 128..512
threads (lanes that hold an atom for a brick two standard deviations above
the mean, wavefronts per CU the LDS stage allows, halo candidates staged per
atom); the best-scored few are timed (one list build amortised over
`rebuild_interval` steps plus one force launch) and the fastest is applied
and cached in a JSON file keyed by the system's signature.
"""
from __future__ import annotations

import json
import math
import os
from typing import Dict, List, Optional, Tuple

import numpy as np

from . import binding as B

CACHE_ENV = "MD_TUNE_CACHE"
DEFAULT_CACHE = os.path.join(os.path.expanduser("~"), ".cache", "mdgpu_tune.json")
LDS_PER_CU = 160 * 1024


def record_stride(halo: int, cells: int) -> int:
    return (8 + 3 * halo + 2 * cells + 2 + 3) // 4 * 4


def score(shape: Tuple[int, int, int], threads: int, occ: float, wgpc: int = 8,
          lds_max: int = LDS_PER_CU) -> float:
    """Estimated efficiency of a brick shape and workgroup size for the mean
    occupancy `occ` of the non-empty cells (0 if the LDS stage does not fit)."""
    bx, by, bz = shape
    cells = bx * by * bz
    halo = (bx + 2) * (by + 2) * (bz + 2)
    atoms = occ * cells
    rounds = math.ceil((atoms + 2.0 * math.sqrt(atoms)) / threads)
    eff = atoms / (rounds * threads)
    lds = 24.0 * 1.1 * occ * halo + 4.0 * record_stride(halo, cells) + 512
    blocks = min(wgpc, math.floor(LDS_PER_CU / lds))
    if blocks < 1 or lds > lds_max:
        return 0.0
    waves = min(16.0, min(32.0, blocks * threads / 64))
    return eff * (waves / 16.0) * (1.0 - 0.01 * halo / cells)


def candidates(occ: float, top: int = 6) -> List[Tuple[Tuple[int, int, int], int]]:
    scored = []
    for bz in range(1, 5):
        for by in range(1, 5):
            for bx in range(1, 5):
                for t in range(128, 513, 64):
                    sc = score((bx, by, bz), t, occ)
                    if sc > 0:
                        scored.append((sc, (bx, by, bz), t))
    scored.sort(key=lambda v: -v[0])
    out, seen = [], set()
    for sc, shape, t in scored:
        if (shape, t) in seen:
            continue
        seen.add((shape, t))
        out.append((shape, t))
        if len(out) == top:
            break
    return out


def occupancy(counts: np.ndarray) -> float:
    """Mean occupancy of the non-empty cells."""
    return float(counts.sum() / max(int((counts > 0).sum()), 1))


def signature(system) -> str:
    """Cache key: atoms, replicas, cells, occupancy of the non-empty cells, potential."""
    cs, _ = B.md_get_cells(system.ctx)
    counts = np.diff(cs)
    return f"{system.pot.kind}-n{system.n}-r{system.R}-c{counts.size}-occ{occupancy(counts):.2f}"


def load_cache(path: Optional[str] = None) -> Dict[str, dict]:
    path = path or os.environ.get(CACHE_ENV, DEFAULT_CACHE)
    if not os.path.exists(path):
        return {}
    with open(path) as f:
        return json.load(f)


def save_cache(cache: Dict[str, dict], path: Optional[str] = None):
    path = path or os.environ.get(CACHE_ENV, DEFAULT_CACHE)
    os.makedirs(os.path.dirname(path) or ".", exist_ok=True)
    tmp = path + ".tmp"
    with open(tmp, "w") as f:
        json.dump(cache, f, indent=1, sort_keys=True)
    os.replace(tmp, path)


def apply(system, shape: Tuple[int, int, int], threads: int):
    B.md_set_tuning(system.ctx, 3, shape[0] | shape[1] << 8 | shape[2] << 16)
    B.md_set_tuning(system.ctx, 4, threads)


def _time_config(system, shape, threads, precision, kind, rebuild_interval, reps) -> float:
    import torch
    apply(system, shape, threads)
    system.build(kind)                      # sizes the list and the LDS stage
    F = torch.empty_like(system.pos)
    B.md_compute_forces(system.ctx, system.dpot, precision, F, None, None)
    torch.cuda.synchronize()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(4)]
    best = float("inf")
    for _ in range(reps):
        ev[0].record()
        B.md_build_neighbor_list(system.ctx, kind)
        ev[1].record()
        B.md_compute_forces(system.ctx, system.dpot, precision, F, None, None)
        ev[2].record()
        torch.cuda.synchronize()
        t_list = ev[0].elapsed_time(ev[1])
        t_force = ev[1].elapsed_time(ev[2])
        best = min(best, t_force + t_list / rebuild_interval)
    code = B.md_get_status(system.ctx)[0]
    if code != B.MD_OK:
        raise B.MDError(code, "tuning run failed")
    return best


def tune(system, precision: int = B.MD_MIXED, kind: int = B.MD_LIST_FULL, rebuild_interval: float = 9.0,
         top: int = 6, reps: int = 3, cache_path: Optional[str] = None, use_cache: bool = True) -> dict:
    """Pick and apply the fastest brick shape / workgroup size for `system`
    (an MDSystem whose cells are built); returns the chosen entry."""
    B.md_build_cells(system.ctx, system.pos, system.boxes, system.pot.rc, system.skin)
    key = f"{signature(system)}-p{precision}-k{kind}"
    cache = load_cache(cache_path) if use_cache else {}
    if key in cache:
        e = cache[key]
        apply(system, tuple(e["shape"]), e["threads"])
        return e
    cs, _ = B.md_get_cells(system.ctx)
    occ = occupancy(np.diff(cs))
    results = []
    for shape, t in candidates(occ, top):
        ms = _time_config(system, shape, t, precision, kind, rebuild_interval, reps)
        results.append({"shape": list(shape), "threads": t, "ms": ms})
    results.sort(key=lambda e: e["ms"])
    best = dict(results[0], candidates=results)
    apply(system, tuple(best["shape"]), best["threads"])
    if use_cache:
        cache[key] = best
        save_cache(cache, cache_path)
    return best
