"""Benchmark: useful label expansions per second of the wavefront multiobjective
search on one MI355X, plus queries per second of the batched serving load.

Headline step: one whole search (Alg. 3 Explore to an empty open set, then
the goal front and its copy to the host) on a device-resident roadmap: the 3D
workspace with 20,000 free samples, ~40 neighbours, 100 boxes, 80 feature
blobs, three objectives (cost, drift, max drift so far), drift bound 0.25.
The roadmap is built on the GPU before timing (it equals the oracle's
roadmap bit for bit, and the search on it the whole oracle run, both checked
by the GPU tests).  `value` = X / step wall time, X = sum over nodes of the
final front size (an instance property).

Also measured: the 2D (2,000 samples) and 6D double-integrator (50,000
states) single-query workloads, and the batched serving load (256 queries of
uneven size in one recorded launch, on the learned drift judged by the
library with the analytic fallback, against the same batch on the analytic
drift recomputed inside the recorded launch and against one launch per
query).

Prints one JSON line.  Only one GPU is supported: --gpus N > 1 exits.
"""
from __future__ import annotations

import argparse
import json
import os
import statistics
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E
TICK_MS = 1e-5         # the device's 100 MHz wall clock


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def alg_bytes(X: int, R: int, n_obj: int) -> int:
    """Least bytes the search must move: one 12-byte in-edge record per useful
    relaxation, one read of each expanded label (s bytes) and its arena write,
    bucket slot and frontier index (s + 4 bytes); s = 16 (two objectives) or
    20 (three)."""
    s = 16 if n_obj == 2 else 20
    return 12 * R + s * X + (s + 4) * X


def search_source_hash() -> str:
    """First 16 hex digits of the SHA-256 of the search kernel sources."""
    import hashlib
    csrc = os.path.join(ROOT, "paper_1705_02408_amd", "csrc")
    h = hashlib.sha256()
    for f in ("search_kernels.hip", "search_kernels.h", "device_common.h"):
        with open(os.path.join(csrc, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def search_kernel(st: dict) -> str:
    """Name of the search build that ran (from a result's statistics)."""
    if st.get("wave_build"):
        base = "k_search_wave"
    else:
        base = "k_search_halves" if st.get("half_front_cap", 0) > 0 else "k_search"
    o = st.get("build_objectives", 0)
    return f"{base}_o{o}" if o in (2, 3) else base


def measured_traffic(profile: str = "k_search_halves_o3_plain3d_n20000.md"):
    """HBM bytes per search launch from a committed rocprofv3 counter summary
    under profiles/, or None when the kernel sources have changed since the
    counters were taken."""
    path = os.path.join(ROOT, "profiles", profile)
    try:
        with open(path) as f:
            line = next(l for l in f if l.startswith("traffic:"))
    except (OSError, StopIteration):
        return None
    kv = dict(t.split("=", 1) for t in line.split()[1:])
    if kv.get("source_sha256_16") != search_source_hash():
        return None
    return int(1024 * (float(kv["fetch_kib"]) * float(kv["fetch_scale"]) +
                       float(kv["write_kib"]) * float(kv["write_scale"])))


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    import platform
    return platform.processor() or platform.machine()


def host_cores() -> int:
    try:
        return len(os.sched_getaffinity(0))
    except AttributeError:  # pragma: no cover
        return os.cpu_count() or 1


# ------------------------------------------------------------ single queries
def measure_tuned(dg, env, steps: int, ref_front):
    """The same searches with the autotuner's settings for this roadmap
    (chosen here, not read from a cache): times, the choice, and whether the
    goal front is the default settings' bit for bit."""
    import numpy as np
    from paper_1705_02408_amd import autotune, mpap
    base = mpap.search_params(env.beta, env.n_obj, env.radius, env.lam)
    t0 = time.perf_counter()
    ch = autotune.tune(dg, base, [env.dim], env.n_obj, cache_path=None, repeats=2)
    tune_s = time.perf_counter() - t0
    f = ch.fields()
    kw = dict(near_scan=f["near_scan"], block_threads=f["block_threads"],
              wave_min_targets=f["wave_min_targets"], stage_cap=f["stage_cap"],
              merge_halves=f["merge_halves"])
    times, kms, same = [], [], True
    for i in range(steps + 1):
        ts = time.perf_counter()
        res = mpap.mpap_search(dg, env.beta, env.n_obj, env.radius, f["lambda_"], **kw)
        fr = res.goal_front()
        st = res.stats()
        res.close()
        if i == 0:
            continue  # the first call sizes the workspace for the new settings
        times.append(time.perf_counter() - ts)
        kms.append(st["gpu_ms"])
        same = same and np.array_equal(fr.vecs.view(np.uint32), ref_front.vecs.view(np.uint32))
    total = sum(times)
    out = {"choice": {k.rstrip("_"): v for k, v in f.items()}, "tune_s": tune_s,
           "ms_per_step": 1000.0 * total / steps, "labels_per_s": st["front_labels"] * steps / total,
           "kernel_ms_mean": statistics.mean(kms), "kernel_ms_min": min(kms),
           "waves": st["waves"], "kernel": search_kernel(st), "X_front_labels": st["front_labels"],
           "same_goal_front": bool(same)}
    log(f"# {env.name} autotuned: {out}")
    return out


def measure_single(env, steps: int, warmup: int, with_trace: bool = True, tune: bool = False):
    """Whole searches of one roadmap built on the GPU: returns a dict of the
    step and kernel times, counts and per-phase device times (and, with
    ``tune``, the same for the autotuner's settings)."""
    import numpy as np
    import torch
    from paper_1705_02408_amd import mpap
    t0 = time.perf_counter()
    dg = mpap.mpap_build_graph(env)
    torch.cuda.synchronize()
    build_s = time.perf_counter() - t0
    ginfo = dg.info()
    log(f"# {env.name}: graph built on GPU in {build_s:.3f}s: {ginfo}")
    trace = {}

    def step():
        res = mpap.mpap_search(dg, env.beta, env.n_obj, env.radius, env.lam)
        fr = res.goal_front()
        st = res.stats()
        if with_trace:
            trace["t"] = res.wave_trace()
        res.close()
        return fr, st

    for i in range(warmup):
        fr, st = step()
        log(f"# warmup {i}: {st}")
    torch.cuda.synchronize()
    times, kms, stats = [], [], []
    t_start = time.perf_counter()
    for i in range(steps):
        ts = time.perf_counter()
        fr, st = step()
        times.append(time.perf_counter() - ts)
        kms.append(st["gpu_ms"])
        stats.append(st)
    torch.cuda.synchronize()
    total = time.perf_counter() - t_start
    tuned = measure_tuned(dg, env, steps, fr) if tune else None
    dg.close()
    st = stats[-1]
    X, R = st["front_labels"], st["relaxations"]
    k_ms = statistics.mean(kms)
    B = alg_bytes(X, R, env.n_obj)
    out = {
        "workload": f"{env.name}: {env.dim}D roadmap, {ginfo['n']} nodes, {ginfo['e']} directed "
                    f"edges, {env.box_lo.shape[0]} boxes, {env.blob_mu.shape[0]} blobs, "
                    f"{env.n_obj} objectives, beta {env.beta}, lambda {env.lam}",
        "nodes": ginfo["n"], "edges": ginfo["e"], "graph_build_s": build_s,
        "steps": steps, "total_s": total, "ms_per_step": 1000.0 * total / steps,
        "labels_per_s": X * steps / total, "queries_per_s": steps / total,
        "X_front_labels": X, "R_relaxations": R, "labels_expanded_gpu": st["labels_expanded"],
        "waves": st["waves"], "merges": st["merges"], "candidates": st["candidates"],
        "goal_front": int(fr.vecs.shape[0]), "kernel_ms_mean": k_ms, "kernel_ms_min": min(kms),
        "step_ms_median": 1000 * statistics.median(times), "blocks": st["blocks"],
        "lds_front_cap": st["lds_front_cap"], "max_front": st["max_front"],
        "wave_build": st["wave_build"], "kernel": search_kernel(st),
        "half_merges": st["half_merges"], "half_backouts": st["half_backouts"],
        "alg_bytes_per_launch": B,
        "achieved_GBps": B / (k_ms * 1e-3) / 1e9,
    }
    if tuned is not None:
        out["autotuned"] = tuned
    if with_trace and "t" in trace:
        tr = trace["t"].astype(np.float64)
        out["phases"] = {
            "count_ms": float(((tr[:, 1] - tr[:, 0]) * TICK_MS).sum()),
            "select_ms": float(((tr[:, 2] - tr[:, 1]) * TICK_MS).sum()),
            "merge_ms": float(((tr[:, 3] - tr[:, 2]) * TICK_MS).sum()),
            "merge_busiest_block_ms": float((tr[:, 6] * TICK_MS).sum()),
            "merge_mean_block_ms": float((tr[:, 7] * TICK_MS).sum() / max(1, st["blocks"])),
            "max_group": int(tr[:, 4].max()) if tr.shape[0] else 0,
            "max_targets": int(tr[:, 5].max()) if tr.shape[0] else 0,
        }
    return out


def golden_whole_search():
    """The stored whole-oracle run of the 3D workload (written by
    tests/golden/make_plain3d_golden.py): its own wall time and CPU."""
    path = os.path.join(ROOT, "tests", "golden", "plain3d_s0_front.json")
    try:
        with open(path) as f:
            s = json.load(f)
    except OSError:
        return None
    return {"value": s["oracle_labels_per_s"], "unit": "labels/s", "cores": s["oracle_cores"],
            "seconds": s["oracle_seconds"], "X": s["X"], "cpu": s["oracle_cpu"],
            "source": "tests/golden/plain3d_s0_front.json (whole search, timed by the script "
                      "that wrote it)"}


def cpu_prefix_baseline(env, seconds: float):
    """The oracle on a bounded sample of the headline search: labels are made
    permanent in ascending cost order, so the sample is the cheap start of
    the search (small fronts), which makes its rate an upper bound of the
    whole search's rate."""
    from oracle import graph as ograph, search as osearch
    t1 = time.perf_counter()
    g = ograph.build_graph(env)
    gb = time.perf_counter() - t1
    labels, secs, finished = osearch.timed_sample(g, env.beta, env.n_obj, 150000)
    target = int(150000 * max(1.0, seconds / max(secs, 1e-3)) ** 0.5)
    if not finished and target > labels:
        labels, secs, finished = osearch.timed_sample(g, env.beta, env.n_obj, target)
    return {"value": labels / secs, "unit": "labels/s", "cores": 1, "kind": "oracle",
            "sample": (f"sequential label-setting oracle (one thread) on the headline workload's "
                       f"own roadmap, the first {labels} labels it makes permanent "
                       f"({'the whole search' if finished else 'a prefix: the cheapest labels, small fronts; an upper bound of the whole-search rate'}), "
                       f"{secs:.2f}s; oracle roadmap build {gb:.1f}s not counted"),
            "cpu": cpu_model(), "host_cores": host_cores(),
            "whole_search_reference": golden_whole_search()}


def cpu_whole_search(env):
    """The oracle's whole search of a small workload (one thread)."""
    from oracle import graph as ograph, search as osearch
    g = ograph.build_graph(env)
    res = osearch.search(g, env.beta, env.n_obj)
    return {"value": res.X / res.seconds, "unit": "labels/s", "cores": 1, "kind": "oracle",
            "seconds": res.seconds, "X": res.X,
            "sample": "the whole search of the same workload (oracle roadmap, one thread)"}


# ------------------------------------------------------------ online update
def measure_update(env, reps: int = 3):
    """Obstacles found after the search (Sec. 3, online implementation): five
    boxes added to the roadmap (only the new collision checks), the search
    continued from the earlier labels, against a fresh search of the changed
    roadmap (wall times of the whole calls, fronts compared)."""
    import numpy as np
    import torch
    from paper_1705_02408_amd import mpap, synth
    lo, hi = synth.discovered_boxes(env, 4, 5)
    g0 = mpap.mpap_build_graph(env)
    r0 = mpap.mpap_search(g0, env.beta, env.n_obj, env.radius, env.lam)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    g1 = mpap.mpap_graph_add_boxes(g0, lo, hi)
    torch.cuda.synchronize()
    add_ms = 1e3 * (time.perf_counter() - t0)
    upd_ms, fresh_ms = [], []
    for _ in range(reps + 1):
        ts = time.perf_counter()
        upd = mpap.mpap_search_update(r0, g1, env.beta, env.n_obj, env.radius, env.lam)
        upd_ms.append(1e3 * (time.perf_counter() - ts))
        ts = time.perf_counter()
        fresh = mpap.mpap_search(g1, env.beta, env.n_obj, env.radius, env.lam)
        fresh_ms.append(1e3 * (time.perf_counter() - ts))
        same = np.array_equal(upd.goal_front().vecs.view(np.uint32),
                              fresh.goal_front().vecs.view(np.uint32))
        su, sf = upd.stats(), fresh.stats()
        upd.close()
        fresh.close()
    out = {"workload": f"{env.name} + 5 boxes found after the search",
           "edges_removed": g0.info()["e"] - g1.info()["e"], "add_boxes_ms": add_ms,
           "update_ms": statistics.median(upd_ms[1:]), "fresh_search_ms": statistics.median(fresh_ms[1:]),
           "update_kernel_ms": su["gpu_ms"], "fresh_kernel_ms": sf["gpu_ms"],
           "update_labels_expanded": su["labels_expanded"],
           "fresh_labels_expanded": sf["labels_expanded"],
           "same_goal_front": bool(same), "front_labels": sf["front_labels"]}
    out["speedup"] = out["fresh_search_ms"] / out["update_ms"]
    r0.close()
    g1.close()
    g0.close()
    log(f"# online update: {out}")
    return out


# --------------------------------------------------------- MC verification
def measure_mc(env, flights: int = 262144, cpu_flights: int = 256):
    """Monte Carlo verification of two plans of the goal front (the cheapest,
    P_soln, and the one of least largest drift): GPU flights/s, the outcome
    rates, and the oracle on a bounded sample of flights on one host core."""
    import numpy as np
    from oracle import mcverify as omc
    from paper_1705_02408_amd import mpap
    dg = mpap.mpap_build_graph(env)
    res = mpap.mpap_search(dg, env.beta, env.n_obj, env.radius, env.lam)
    fr = res.goal_front()
    out = {"workload": f"{env.name}: goal front {fr.vecs.shape[0]} plans",
           "model": dict(mpap.MC_DEFAULTS, rollouts=flights), "plans": {}}
    picks = {"least_cost": 0, "least_max_drift": int(np.argmin(fr.vecs[:, 2]))}
    for name, k in picks.items():
        path = res.path(int(fr.label[k]))
        mpap.mpap_mc_verify(dg, path, with_samples=False, rollouts=1024)  # warm
        st, _, _ = mpap.mpap_mc_verify(dg, path, with_samples=False, rollouts=flights)
        out["plans"][name] = {
            "cost_drift_maxdrift": [float(x) for x in fr.vecs[k]], "nodes": len(path),
            "steps": st["steps"], "flight_s": st["duration"], "gpu_ms": st["gpu_ms"],
            "flights_per_s": flights / (st["gpu_ms"] * 1e-3),
            "flight_steps_per_s": flights * st["steps"] / (st["gpu_ms"] * 1e-3),
            "within_bound": st["within_bound"] / flights,
            "collision_free": st["collision_free"] / flights,
            "success": st["success"] / flights, "mean_max_err": st["mean_max_err"]}
    # the oracle on a bounded sample of the cheapest plan's flights
    path = res.path(int(fr.label[0]))
    mp = omc.MCParams(rollouts=cpu_flights)
    p, v, a = omc.nominal_segments(env.pos[path], mp.f64("speed"), mp.f64("dt"))
    t0 = time.perf_counter()
    omc.rollouts(p, v, a, mp, env.blob_mu, env.blob_sigma, env.blob_amp, env.box_lo, env.box_hi)
    cpu_s = time.perf_counter() - t0
    out["cpu_baseline"] = {"value": cpu_flights / cpu_s, "unit": "flights/s", "cores": 1,
                           "kind": "oracle",
                           "sample": f"{cpu_flights} flights of the cheapest plan, numpy float64 "
                                     f"vectorised over flights, one core, {cpu_s:.2f} s"}
    res.close()
    dg.close()
    log(f"# MC verification: {out['plans']}")
    return out


# ------------------------------------------------------------------- batch
def surrogate_error_stats(ana, sur, held, beta):
    import numpy as np
    floor = 1e-3 * beta
    rel = np.abs(sur[held] - ana[held]).astype(np.float64) / np.maximum(ana[held], floor)
    return {"heldout_edges": int(held.size), "p50": float(np.percentile(rel, 50)),
            "p90": float(np.percentile(rel, 90)), "p99": float(np.percentile(rel, 99)),
            "max": float(rel.max())}


def train_surrogates(seed: int):
    """One surrogate per dimension, trained on roadmaps that are not part of
    the measured batch (other seeds)."""
    import numpy as np
    from paper_1705_02408_amd import mpap, synth
    models = {}
    for dim, env in ((2, synth.make_env(10_000 + seed, 2, 50000, 20, 30, 20.0, 0.3, 2,
                                        blob_amp=0.3)),
                     (3, synth.make_env(20_000 + seed, 3, 30000, 100, 80, 40.0, 0.25, 2,
                                        blob_amp=0.4))):
        g = mpap.mpap_build_graph(env)
        e = g.info()["e"]
        n_train = min(1 << 20, (e // 4096) * 4096)
        perm = np.random.default_rng(seed + dim).permutation(e)
        edges = perm[:n_train]
        s = mpap.Surrogate(seed=seed * 10 + dim)
        t0 = time.perf_counter()
        loss = s.train(g, edges, epochs=8, batch=4096, lr=2e-3)
        dt = time.perf_counter() - t0
        s.score(g)
        ana = mpap.mpap_graph_drift(g, 0)
        sur = mpap.mpap_graph_drift(g, 1)
        _, base = mpap.mpap_edge_features(g, with_base=True)
        cost = g.export()["cost"]
        only_base = (cost.astype(np.float64) * np.clip(base, 0, 1)).astype(np.float32)
        held = perm[n_train:]
        err = surrogate_error_stats(ana, sur, held, env.beta)
        err_base = surrogate_error_stats(ana, only_base, held, env.beta)
        log(f"# surrogate {dim}D: {n_train} edges, {dt:.2f}s, loss {loss[0]:.4g} -> "
            f"{loss[-1]:.4g}; held-out rel err p50 {err['p50']:.3g} p99 {err['p99']:.3g} "
            f"(8-point base alone p50 {err_base['p50']:.3g} p99 {err_base['p99']:.3g})")
        models[dim] = dict(model=s, train_s=dt, loss_first=float(loss[0]),
                           loss_last=float(loss[-1]), n_train=int(n_train),
                           heldout_rel_err=err, heldout_rel_err_base_only=err_base)
        g.close()
    return models


def _cpu_batch_worker(args):
    env, = args
    from oracle import graph as ograph, search as osearch
    g = ograph.build_graph(env)
    if g["goal"].sum() == 0:
        return None
    res = osearch.search(g, env.beta, env.n_obj)
    return res.X, res.seconds


def cpu_batch_baseline(envs, X_batch: int, seconds: float):
    """The oracle over whole queries of the batch on every host core (one
    query per process): a seeded sample of the batch's queries below 4,000
    samples, as many as finish in about `seconds` of wall time.  The label
    rate over the sample (aggregate over the cores) is scaled to queries/s
    with the batch's own mean labels per query; the sample's small fronts
    make it an upper bound of the rate on the whole batch."""
    import multiprocessing as mp

    import numpy as np
    cores = min(host_cores(), 16)  # a one-GPU machine's share of the host
    small = [k for k, e in enumerate(envs) if e.n_nodes <= 4000]
    order = [small[i] for i in np.random.default_rng(0).permutation(len(small))]
    done_labels, done_q, cpu_s = 0, 0, 0.0
    t0 = time.perf_counter()
    ctx = mp.get_context("spawn")  # fresh interpreters: nothing of the GPU state
    with ctx.Pool(cores) as pool:
        pending = [pool.apply_async(_cpu_batch_worker, ((envs[k],),)) for k in order]
        for r in pending:
            left = seconds - (time.perf_counter() - t0)
            if left <= 0:
                break
            try:
                out = r.get(timeout=left)
            except mp.TimeoutError:
                break
            if out is None:
                continue
            done_labels += out[0]
            cpu_s += out[1]
            done_q += 1
        pool.terminate()
    wall = time.perf_counter() - t0
    if done_q == 0 or cpu_s <= 0:
        return None
    rate = done_labels / cpu_s * cores  # labels/s over all cores (search time only)
    mean_x = X_batch / max(len(envs), 1)
    return {"value": rate / mean_x, "unit": "queries/s", "cores": cores, "kind": "oracle",
            "labels_per_s": rate,
            "sample": (f"whole oracle searches of {done_q} queries of the batch (seeded sample of "
                       f"the queries below 4,000 samples), one per process on {cores} cores, "
                       f"{done_labels} labels in {cpu_s:.1f} s of search time ({wall:.1f} s wall "
                       f"with the oracle roadmap builds); labels/s x cores scaled by the batch's "
                       f"mean {mean_x:.0f} labels per query (small queries: an upper bound)"),
            "cpu": cpu_model()}


def measure_batch(args, with_surrogate: bool = True):
    """Serving-style load: args.queries independent queries of uneven size in
    one persistent launch recorded as a HIP graph (a) on the learned drift,
    judged by the library with the analytic fallback, (b) on the analytic
    drift recomputed inside the recorded launch, (c) one launch per query on
    the precomputed analytic drift."""
    import numpy as np
    import torch
    from paper_1705_02408_amd import autotune, mpap, synth

    t0 = time.perf_counter()
    envs, parts = [], []
    q = 0
    while len(parts) < args.queries:
        e = synth.batch_query(args.seed, q)
        q += 1
        try:
            parts.append(mpap.mpap_build_graph(e))
            envs.append(e)
        except mpap.MpapError as ex:  # no sample in the goal ball: draw the next query
            if ex.status != mpap.MPAP_ERR_NOGOAL:
                raise
    torch.cuda.synchronize()
    build_s = time.perf_counter() - t0
    nq = len(envs)
    ana_ms = sum(mpap.mpap_analytic_drift(p) for p in parts)
    out = {"queries": nq, "build_s": build_s, "analytic_drift_ms": ana_ms}
    models = None
    if with_surrogate:
        models = train_surrogates(args.seed)
        sur_ms = sum(models[e.dim]["model"].score(p) for e, p in zip(envs, parts))
        out["surrogate"] = {f"{d}d": {k: v for k, v in m.items() if k != "model"}
                            for d, m in models.items()}
        out["surrogate_score_ms"] = sur_ms
    union = mpap.mpap_graph_concat(parts)
    info = union.info()
    log(f"# {nq} roadmaps ({info}) built in {build_s:.2f}s; analytic drift {ana_ms:.1f} ms")
    base = [mpap.search_params(e.beta, e.n_obj, e.radius, e.lam) for e in envs]
    # tuned on the whole batch: a subset of queries has fewer merge targets per
    # iteration and picks other merge tiles (a 32-query subset chose
    # workgroup-only merges, which are 1.7x slower on all 256 queries)
    t0 = time.perf_counter()
    choice = autotune.tune(union, base, sorted({e.dim for e in envs}), 2, repeats=1,
                           lambdas=(0.5, 1.0), log=log)
    out["autotune"] = {"s": time.perf_counter() - t0, **{k.rstrip("_"): v for k, v in
                                                         choice.fields().items()}}
    log(f"# autotuned {choice.fields()} in {out['autotune']['s']:.1f}s")

    def params(heur):
        return autotune.apply([mpap.search_params(e.beta, e.n_obj, e.radius, e.lam,
                                                  heuristic=heur) for e in envs], choice)

    def timed_plan(plan, judge: bool, label: str):
        for _ in range(min(args.warmup, 1)):
            r = plan.run()
            if judge:
                r.judge(1e-2, fallback=True)
            r.close()
        torch.cuda.synchronize()
        walls, stats, lats = [], [], []
        for _ in range(args.batch_steps):
            ts = time.perf_counter()
            res = plan.run()
            if judge:
                res.judge(1e-2, fallback=True)
            for k in range(nq):
                res.goal_front(k)
            walls.append(time.perf_counter() - ts)
            st = res.stats()
            stats.append(st)
            lats.append([res.query_info(k)["latency_ms"] for k in range(nq)])
            res.close()
            log(f"# {label}: {walls[-1]:.3f}s, kernel {st['gpu_ms']:.1f} ms, rejected "
                f"{st['judged_failed']}, fallback {st['fallback_ms']:.1f} ms")
        wall = statistics.mean(walls)
        lat = np.array(lats[-1])
        st = stats[-1]
        return {"queries_per_s": nq / wall, "step_wall_s": wall,
                "label_expansions_per_s": st["front_labels"] / wall,
                "kernel_ms_mean": statistics.mean(s_["gpu_ms"] for s_ in stats),
                "judge_rejected": st["judged_failed"], "fallback_ms": st["fallback_ms"],
                "latency_ms": {"p50": float(np.percentile(lat, 50)),
                               "p99": float(np.percentile(lat, 99)), "max": float(lat.max())},
                "X_front_labels": st["front_labels"], "R_relaxations": st["relaxations"],
                "waves": st["waves"], "wave_build": st["wave_build"],
                "half_front_cap": st["half_front_cap"],
                "build_objectives": st["build_objectives"], "kernel": search_kernel(st)}

    res_sur = None
    if with_surrogate:
        t0 = time.perf_counter()
        plan = mpap.Plan(union, params(1), parts=parts,
                         models=[models[e.dim]["model"] for e in envs])
        log(f"# surrogate plan recorded in {time.perf_counter() - t0:.2f}s")
        res_sur = timed_plan(plan, True, "batched+surrogate")
        res_sur["plan"] = plan.info()
        plan.close()
    plan = mpap.Plan(union, params(0), parts=parts, analytic=True)
    res_ana = timed_plan(plan, False, "batched+analytic")
    res_ana["plan"] = plan.info()
    plan.close()

    log("# plain: one launch per query")
    seq, Xp, per_q = 0.0, 0, []
    for k, (p, e) in enumerate(zip(parts, envs)):
        ts = time.perf_counter()
        r1 = mpap.mpap_search(p, e.beta, e.n_obj, e.radius, e.lam)
        r1.goal_front()
        Xp += r1.stats()["front_labels"]
        r1.close()
        dt = time.perf_counter() - ts
        per_q.append(dt)
        seq += dt
        if (k + 1) % 64 == 0:
            log(f"# plain: {k + 1}/{nq} queries, {seq:.1f}s")
    head = res_sur if res_sur is not None else res_ana
    X = res_ana["X_front_labels"]
    B = alg_bytes(X, res_ana["R_relaxations"], 2)
    k_ms = res_ana["kernel_ms_mean"]
    out.update({
        "queries_per_s": head["queries_per_s"],
        "batched_surrogate": res_sur,
        "batched_analytic": res_ana,
        "plain_one_launch_per_query": {"queries_per_s": nq / seq, "wall_s": seq,
                                       "label_expansions_per_s": Xp / seq,
                                       "latency_ms_p50": 1e3 * float(np.percentile(per_q, 50)),
                                       "latency_ms_p99": 1e3 * float(np.percentile(per_q, 99))},
        "speedup_surrogate_vs_analytic_batched": (res_sur["queries_per_s"] /
                                                  res_ana["queries_per_s"]) if res_sur else None,
        "speedup_batched_vs_plain": head["queries_per_s"] / (nq / seq),
        "nodes": info["n"], "edges": info["e"],
        "roofline": {"bound": "hbm", "achieved": B / (k_ms * 1e-3) / 1e9, "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": B / (k_ms * 1e-3) / 1e9 / HBM_PEAK_GBS,
                     "kernel": search_kernel(res_ana),
                     "alg_bytes_per_launch": B,
                     "traffic": measured_traffic("k_search_wave_o2_batch256.md")
                     if args.queries == 256 and args.seed == 0 else None},
    })
    if not args.no_cpu_baseline:
        log("# batch CPU baseline (oracle, all cores)")
        out["cpu_baseline"] = cpu_batch_baseline(envs, X, args.cpu_seconds)
    union.close()
    for p in parts:
        p.close()
    if models:
        for m in models.values():
            m["model"].close()
    return out


def run_copy(args):
    """A plain device copy of 1 GiB, K times: per launch 2^30 bytes read and
    2^30 bytes written.  Profiled with the same counters as the search, it
    gives the counters' bytes-per-unit scale on this device."""
    import torch
    nbytes = 1 << 30
    src = torch.empty(nbytes // 4, dtype=torch.float32, device="cuda").uniform_()
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        dst.copy_(src)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / max(args.steps, 1)
    print(json.dumps({"metric": "copy GB/s (read + write)", "value": 2 * nbytes / dt / 1e9,
                      "unit": "GB/s", "n_gpus": 1, "steps": args.steps, "warmup": 0,
                      "ms_per_step": 1e3 * dt, "bytes_read_per_launch": nbytes,
                      "bytes_written_per_launch": nbytes}), flush=True)


def run_batch(args):
    b = measure_batch(args, with_surrogate=not args.no_surrogate)
    out = {
        "metric": ("queries/s (batched, learned drift judged per query, exact fallback)"
                   if b["batched_surrogate"] else "queries/s (batched, analytic drift)"),
        "value": b["queries_per_s"], "unit": "queries/s", "n_gpus": 1,
        "steps": args.batch_steps, "warmup": args.warmup,
        "ms_per_step": 1000.0 * (b["batched_surrogate"] or b["batched_analytic"])["step_wall_s"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic (seeded generator)",
        "config": {"workload": f"batch of {b['queries']} queries, 2D/3D even odds, sizes "
                               f"log-uniform 2000-50000 samples, two objectives",
                   "queries_per_step": b["queries"], "parallelism": "single GPU"},
        "batched_serving": b, "roofline": b["roofline"],
        "cpu_baseline": b.get("cpu_baseline"),
    }
    print(json.dumps(out), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--n", type=int, default=20000)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--workload", choices=["plain3d", "plain2d", "plain6d", "batch", "copy"],
                    default="plain3d",
                    help="copy: a plain 1 GiB device copy, the reference for the HBM "
                         "traffic counters")
    ap.add_argument("--queries", type=int, default=256, help="batch workload: query count")
    ap.add_argument("--batch-steps", type=int, default=2, help="timed batches")
    ap.add_argument("--no-batch", action="store_true",
                    help="skip the batched serving measurement of the default run")
    ap.add_argument("--no-configs", action="store_true",
                    help="skip the 2D and 6D single-query rows of the default run")
    ap.add_argument("--no-surrogate", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=20.0,
                    help="time budget of each CPU-baseline sample")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-tune", action="store_true",
                    help="skip the autotuned leg of the single-query workloads")
    args = ap.parse_args()

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU only; the search of one "
                                   "roadmap is not sharded across GPUs",
                          "n_gpus": args.gpus}), flush=True)
        sys.exit(2)

    import torch
    from paper_1705_02408_amd import mpap, synth  # noqa: F401  (fails loudly if not built)

    if not torch.cuda.is_available():
        print(json.dumps({"error": "no GPU visible"}), flush=True)
        sys.exit(1)
    torch.cuda.init()

    if args.workload == "batch":
        return run_batch(args)
    if args.workload == "copy":
        return run_copy(args)
    env = {"plain3d": lambda: synth.plain3d(args.seed, n=args.n),
           "plain2d": lambda: synth.plain2d(args.seed, n=args.n),
           "plain6d": lambda: synth.plain6d(args.seed, n=args.n)}[args.workload]()
    head = measure_single(env, args.steps, args.warmup, tune=not args.no_tune)
    for k in ("phases",):
        log(f"# {k} {head.get(k)}")
    headline_3d = args.workload == "plain3d" and args.n == 20000 and args.seed == 0
    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_prefix_baseline(env, args.cpu_seconds)
    out = {
        "metric": "label expansions/s (useful, oracle-exact front)",
        "value": head["labels_per_s"],
        "unit": "labels/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": head["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic (seeded generator), roadmap built on the GPU",
        "config": {"workload": head["workload"], "queries_per_step": 1,
                   "parallelism": "single GPU"},
        "queries_per_s": head["queries_per_s"],
        "search": {k: v for k, v in head.items() if k not in ("workload",)},
        "roofline": {"bound": "hbm", "achieved": head["achieved_GBps"], "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": head["achieved_GBps"] / HBM_PEAK_GBS,
                     "traffic": measured_traffic() if headline_3d else None,
                     "traffic_unit": "bytes per launch (rocprofv3 FETCH_SIZE + WRITE_SIZE, "
                                     "scaled by a plain copy's counts)",
                     "kernel": head["kernel"],
                     "alg_bytes_per_launch": head["alg_bytes_per_launch"]},
        "cpu_baseline": cpu,
    }
    if headline_3d and not args.no_configs:
        rows = {}
        for name, env2 in (("plain2d_n2000", synth.plain2d(0)), ("plain6d_n50000",
                                                                synth.plain6d(0))):
            r = measure_single(env2, args.steps, args.warmup, with_trace=False,
                               tune=not args.no_tune)
            if not args.no_cpu_baseline and env2.dim == 2:
                r["cpu_baseline"] = cpu_whole_search(env2)
            rows[name] = r
        out["configs"] = rows
    if headline_3d and not args.no_configs:
        out["online_update"] = measure_update(env)
        out["mc_verification"] = measure_mc(env)
    if not args.no_batch and headline_3d:
        out["batched_serving"] = measure_batch(args, with_surrogate=not args.no_surrogate)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
