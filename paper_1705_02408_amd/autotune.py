"""Autotuner for the search's free parameters.

None of the tuned settings changes a result: the fronts are the same for any
group factor (lambda), near-scan length, LDS staging size of a front (the
bucket stage), workgroup size, single-wave threshold and merges by halves
(the tile of one merge: a workgroup, half a workgroup or a wave).  They
trade the number of Explore iterations (grid barriers) against wasted
expansions, scan work against staging, and large merges against many small
ones.  The tuner times the search launch with its device clock over one
setting at a time (coordinate descent in the order lambda, near-scan,
workgroup size, single-wave threshold, LDS stage, merges by halves), keeps
the fastest, and caches the choice in a JSON file keyed by device and a
workload class (dimension mix, objective count and a size bucket).
"""
from __future__ import annotations

import dataclasses
import json
import math
import os
import time

from . import mpap

DEFAULT_CACHE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tuning_cache.json")

LAMBDAS = (0.25, 0.5, 1.0, 2.0, 4.0, 8.0)
NEAR_SCANS = (8, 16, 32)
BLOCK_THREADS = (1024, 512)
# default threshold, never, every iteration, iterations of at least 4,096,
# 16,384 or 32,768 targets (these also choose the single-wave build where the
# default would not, as on roadmaps of many tiny fronts)
WAVE_MIN_TARGETS = (0, -1, 1, 4096, 16384, 32768)
STAGE_CAPS = (0, 2048)          # 0 = all the LDS holds
MERGE_HALVES = (0, -1, 8192)    # by roadmap size, never, always

# the tuned fields of mpap_search_params, in descent order
FIELDS = ("lambda_", "near_scan", "block_threads", "wave_min_targets", "stage_cap",
          "merge_halves")


@dataclasses.dataclass
class Choice:
    lam: float
    near_scan: int
    kernel_ms: float
    tried: list
    block_threads: int = 0
    wave_min_targets: int = 0
    stage_cap: int = 0
    merge_halves: int = 0

    def fields(self) -> dict:
        return dict(lambda_=self.lam, near_scan=self.near_scan, block_threads=self.block_threads,
                    wave_min_targets=self.wave_min_targets, stage_cap=self.stage_cap,
                    merge_halves=self.merge_halves)


def workload_key(device: str, dims, n_obj: int, nodes: int) -> str:
    bucket = int(round(math.log2(max(nodes, 1))))
    dims = "".join(sorted({str(d) for d in dims}))
    return f"{device}|d{dims}|o{n_obj}|n2^{bucket}"


def _device_name() -> str:
    try:
        import torch
        return torch.cuda.get_device_properties(0).gcnArchName.split(":")[0]
    except Exception:  # pragma: no cover - informational only
        return "gfx950"


def _time(graph, params, repeats: int) -> float:
    best = math.inf
    for _ in range(repeats):
        res = mpap.mpap_search_batch(graph, params)
        best = min(best, res.stats()["gpu_ms"])
        res.close()
    return best


def _copy(p, **over):
    q = mpap.mpap_search_params()
    for f, _ in mpap.mpap_search_params._fields_:
        setattr(q, f, getattr(p, f))
    for k, v in over.items():
        setattr(q, k, v)
    return q


def tune(graph, base_params, dims, n_obj: int, cache_path: str | None = DEFAULT_CACHE,
         repeats: int = 2, lambdas=LAMBDAS, near_scans=NEAR_SCANS,
         block_threads=BLOCK_THREADS, wave_min_targets=WAVE_MIN_TARGETS,
         stage_caps=STAGE_CAPS, merge_halves=MERGE_HALVES, use_cache: bool = True,
         log=None) -> Choice:
    """Pick the settings for ``graph`` searched with ``base_params`` (one
    mpap_search_params, or one per query; their tuned fields are overridden).
    Returns the choice; the cache is updated.  ``log`` (optional) receives one
    line per timed setting."""
    nodes = graph.info()["n"]
    key = workload_key(_device_name(), dims, n_obj, nodes)
    cache = {}
    if cache_path and os.path.exists(cache_path):
        with open(cache_path) as f:
            cache = json.load(f)
    if use_cache and key in cache:
        c = cache[key]
        return Choice(c["lam"], c["near_scan"], c["kernel_ms"], c.get("tried", []),
                      c.get("block_threads", 0), c.get("wave_min_targets", 0),
                      c.get("stage_cap", 0), c.get("merge_halves", 0))
    base = base_params if isinstance(base_params, list) else [base_params]
    cur = dict(lambda_=0.5, near_scan=16, block_threads=1024, wave_min_targets=0, stage_cap=0,
               merge_halves=0)
    grid = dict(lambda_=lambdas, near_scan=near_scans, block_threads=block_threads,
                wave_min_targets=wave_min_targets, stage_cap=stage_caps,
                merge_halves=merge_halves)
    tried = []
    seen = {}

    def measure(setting):
        k = tuple(setting[f] for f in FIELDS)
        if k not in seen:
            ms = _time(graph, [_copy(p, **setting) for p in base], repeats)
            seen[k] = ms
            tried.append(dict(setting, kernel_ms=ms))
            if log:
                log("# autotune " + " ".join(f"{f.rstrip('_')} {setting[f]}" for f in FIELDS) +
                    f": {ms:.1f} ms")
        return seen[k]

    _time(graph, [_copy(p, **cur) for p in base], 1)  # warm the workspace (capacities)
    for f in FIELDS:
        best_v, best_ms = cur[f], measure(cur)
        for v in grid[f]:
            ms = measure(dict(cur, **{f: v}))
            if ms < best_ms:
                best_v, best_ms = v, ms
        cur[f] = best_v
    choice = Choice(cur["lambda_"], cur["near_scan"], seen[tuple(cur[f] for f in FIELDS)], tried,
                    cur["block_threads"], cur["wave_min_targets"], cur["stage_cap"],
                    cur["merge_halves"])
    if cache_path:
        cache[key] = dict(lam=choice.lam, near_scan=choice.near_scan,
                          block_threads=choice.block_threads,
                          wave_min_targets=choice.wave_min_targets, stage_cap=choice.stage_cap,
                          merge_halves=choice.merge_halves,
                          kernel_ms=choice.kernel_ms, tried=tried, when=time.time())
        tmp = cache_path + f".tmp{os.getpid()}"
        with open(tmp, "w") as fh:
            json.dump(cache, fh, indent=1, sort_keys=True)
        os.replace(tmp, cache_path)
    return choice


def apply(params, choice: Choice):
    """Copies of ``params`` (one or a list) with the tuned settings."""
    single = not isinstance(params, list)
    out = [_copy(p, **choice.fields()) for p in ([params] if single else params)]
    return out[0] if single else out
