"""Autotuner for the search's free parameters.

None of the tuned settings changes a result (the fronts are the same for any
group factor, near-scan length or LDS staging size); they only trade the
number of Explore iterations (grid barriers) against wasted expansions, and
scan work against staging.  The tuner times a small grid of settings on the
caller's graph (or batch) with the device clock of the search launch, keeps
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

LAMBDAS = (0.25, 0.5, 1.0, 2.0)
NEAR_SCANS = (8, 16, 32)


@dataclasses.dataclass
class Choice:
    lam: float
    near_scan: int
    kernel_ms: float
    tried: list


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


def tune(graph, base_params, dims, n_obj: int, cache_path: str | None = DEFAULT_CACHE,
         repeats: int = 2, lambdas=LAMBDAS, near_scans=NEAR_SCANS, use_cache: bool = True,
         log=None) -> Choice:
    """Pick (lambda, near_scan) for ``graph`` searched with ``base_params`` (one
    mpap_search_params, or one per query; their lambda/near_scan fields are
    overridden).  Returns the choice; the cache is updated.  ``log`` (optional)
    receives one line per timed setting."""
    nodes = graph.info()["n"]
    key = workload_key(_device_name(), dims, n_obj, nodes)
    cache = {}
    if cache_path and os.path.exists(cache_path):
        with open(cache_path) as f:
            cache = json.load(f)
    if use_cache and key in cache:
        c = cache[key]
        return Choice(c["lam"], c["near_scan"], c["kernel_ms"], c.get("tried", []))
    base = base_params if isinstance(base_params, list) else [base_params]

    def with_(lam, ns):
        out = []
        for p in base:
            q = mpap.mpap_search_params()
            for f, _ in mpap.mpap_search_params._fields_:
                setattr(q, f, getattr(p, f))
            q.lambda_ = lam
            q.near_scan = ns
            out.append(q)
        return out

    tried = []
    _time(graph, with_(0.5, 16), 1)  # warm the workspace (capacities)
    for lam in lambdas:
        ms = _time(graph, with_(lam, 16), repeats)
        tried.append(dict(lam=lam, near_scan=16, kernel_ms=ms))
        if log:
            log(f"# autotune lambda {lam} near_scan 16: {ms:.1f} ms")
    best_lam = min(tried, key=lambda r: r["kernel_ms"])["lam"]
    for ns in near_scans:
        if ns == 16:
            continue
        ms = _time(graph, with_(best_lam, ns), repeats)
        tried.append(dict(lam=best_lam, near_scan=ns, kernel_ms=ms))
        if log:
            log(f"# autotune lambda {best_lam} near_scan {ns}: {ms:.1f} ms")
    best = min(tried, key=lambda r: r["kernel_ms"])
    choice = Choice(best["lam"], best["near_scan"], best["kernel_ms"], tried)
    if cache_path:
        cache[key] = dict(lam=choice.lam, near_scan=choice.near_scan,
                          kernel_ms=choice.kernel_ms, tried=tried, when=time.time())
        tmp = cache_path + f".tmp{os.getpid()}"
        with open(tmp, "w") as f:
            json.dump(cache, f, indent=1, sort_keys=True)
        os.replace(tmp, cache_path)
    return choice


def apply(params, choice: Choice):
    """Copies of ``params`` (one or a list) with the tuned settings."""
    single = not isinstance(params, list)
    out = []
    for p in ([params] if single else params):
        q = mpap.mpap_search_params()
        for f, _ in mpap.mpap_search_params._fields_:
            setattr(q, f, getattr(p, f))
        q.lambda_ = choice.lam
        q.near_scan = choice.near_scan
        out.append(q)
    return out[0] if single else out
