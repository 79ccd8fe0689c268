"""Autotuner of query plans, with a JSON cache of its choices.

A plan's launch choices change no result (tested): the plan form (one
launch per stage across indexes, or one chain per group), the stream or
chain count, the projection kernel's vectors per wave (its tile height: 4 or
16; 0 lets the launcher pick by launch size), the vote kernel (single- or
multi-pass) and the single-pass vote kernel's workgroup (8 or 16 waves,
which sets how much LDS its repeat queue, the candidate buffer of the
reruns, gets).  tune() times a plan for every candidate on the caller's
batches and keeps the fastest.  The choice is stored under a key made of the
GPU architecture, the precision arm and, for every group of batches with one
(index, k, v), the tuple (d, T, depth, k, v, nq bucket) with nq rounded up
to a power of two; a later tune() with the same key returns the stored
choice without timing.

The cache file is MRPT_TUNING_CACHE if set, else
~/.cache/mrpt_amd/plan_tuning.json.  Entries are plain JSON.
"""
import json
import os
import time
from typing import Callable, Dict, Iterable, List, Optional, Sequence, Tuple

DEFAULT_CANDIDATES = {
    "fused": (1, 0),
    "branches": (1, 2, 4, 8),
    "proj_rows": (0, 16),
    "vote_kernel": (0, 2),
    "vote_waves": (0, 16),
}


def cache_path() -> str:
    env = os.environ.get("MRPT_TUNING_CACHE")
    if env:
        return env
    return os.path.join(os.path.expanduser("~"), ".cache", "mrpt_amd", "plan_tuning.json")


def arch() -> str:
    import torch
    props = torch.cuda.get_device_properties(torch.cuda.current_device())
    return getattr(props, "gcnArchName", props.name).split(":")[0]


def nq_bucket(nq: int) -> int:
    b = 1
    while b < nq:
        b *= 2
    return b


def signature(batches: Sequence[Tuple], precision: int) -> str:
    """batches: (Index, Q, k, v) as mrpt.Plan takes them."""
    groups: Dict[Tuple, int] = {}
    for ix, Q, k, v in batches:
        key = (id(ix), int(k), int(v))
        groups.setdefault(key, 0)
        groups[key] += int(Q.shape[0])
    byix = {id(ix): ix for ix, _, _, _ in batches}
    parts = []
    for (ixid, k, v), nq in groups.items():
        info = byix[ixid].info
        parts.append((int(info.d), int(info.T), int(info.depth), k, v, nq_bucket(nq)))
    parts.sort()
    return json.dumps({"arch": arch(), "precision": int(precision), "groups": parts}, separators=(",", ":"))


def _load(path: str) -> dict:
    try:
        with open(path) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def _store(path: str, data: dict) -> None:
    os.makedirs(os.path.dirname(os.path.abspath(path)), exist_ok=True)
    tmp = path + ".tmp"
    with open(tmp, "w") as f:
        json.dump(data, f, indent=1, sort_keys=True)
    os.replace(tmp, path)


def candidates(grid: Optional[Dict[str, Iterable[int]]] = None) -> List[Dict[str, int]]:
    g = dict(DEFAULT_CANDIDATES)
    if grid:
        g.update({k: tuple(v) for k, v in grid.items()})
    out = []
    for f in g["fused"]:
        for b in g["branches"]:
            for pr in g["proj_rows"]:
                for vk in g["vote_kernel"]:
                    for vw in g["vote_waves"]:
                        out.append({"fused": f, "branches": b, "proj_rows": pr, "vote_kernel": vk,
                                    "vote_waves": vw})
    return out


def tune(batches: Sequence[Tuple], precision: int, time_plan: Callable[[object], float],
         grid: Optional[Dict[str, Iterable[int]]] = None, retune: bool = False, path: Optional[str] = None,
         log: Callable[[str], None] = lambda s: None):
    """Returns (choice, timings, from_cache).  time_plan(plan) -> ms per launch.

    choice is a dict of mrpt.Plan keyword arguments; timings maps every
    candidate timed in this call to its ms (empty on a cache hit)."""
    from paper_1509_06957_amd import mrpt
    path = path or cache_path()
    key = signature(batches, precision)
    data = _load(path)
    if not retune and key in data:
        log(f"tuning cache hit ({path})")
        return dict(data[key]["choice"]), {}, True
    timings = {}
    best = None
    for c in candidates(grid):
        plan = mrpt.Plan(batches, precision=precision, **c)
        try:
            ms = time_plan(plan)
        finally:
            plan.close()
        name = ",".join(f"{k}={v}" for k, v in c.items())
        timings[name] = round(ms, 4)
        log(f"{name}: {ms:.3f} ms per launch")
        if best is None or ms < best[1]:
            best = (c, ms)
    data = _load(path)
    data[key] = {"choice": best[0], "ms": round(best[1], 4), "timings": timings, "tuned_at": time.time()}
    _store(path, data)
    return dict(best[0]), timings, False
