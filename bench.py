"""Benchmark: useful label expansions per second of the wavefront multiobjective
search on one MI355X.

A step is one whole search (Alg. 3 Explore to an empty open set, then the
goal front) on a device-resident roadmap: the 3D workspace with 20,000 free
samples, ~40 neighbours, 100 boxes, 80 feature blobs, three objectives (cost,
drift, max drift so far), drift bound 0.25.  The roadmap is built on the GPU
before timing.  `value` counts useful expansions X = sum over nodes of the
final front size (an instance property) per second of step wall time.

Prints one JSON line (rank 0).  Only one GPU is supported: --gpus N > 1 exits.
"""
from __future__ import annotations

import argparse
import json
import os
import platform
import statistics
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E


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
    csrc = os.path.join(os.path.dirname(os.path.abspath(__file__)), "paper_1705_02408_amd", "csrc")
    h = hashlib.sha256()
    for f in ("search_kernels.hip", "search_kernels.h", "device_common.h"):
        with open(os.path.join(csrc, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic():
    """HBM bytes per k_search launch on the benchmark workload from the
    committed rocprofv3 counter summary, or None when the kernel sources have
    changed since the counters were taken."""
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "profiles",
                        "k_search_plain3d_n20000.md")
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


def cpu_count_used() -> int:
    return 1


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--n", type=int, default=20000)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--workload", choices=["plain3d", "plain2d", "batch", "copy"],
                    default="plain3d",
                    help="copy: a plain 1 GiB device copy, the reference for the HBM "
                         "traffic counters")
    ap.add_argument("--queries", type=int, default=256, help="batch workload: query count")
    ap.add_argument("--batch-steps", type=int, default=2, help="timed batches")
    ap.add_argument("--no-batch", action="store_true",
                    help="skip the batched serving measurement of the default run")
    ap.add_argument("--no-surrogate", action="store_true")
    ap.add_argument("--cpu-labels", type=int, default=150000,
                    help="labels the oracle makes permanent in the CPU baseline sample")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    args = ap.parse_args()

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU only; the search of one "
                                   "roadmap is not sharded across GPUs",
                          "n_gpus": args.gpus}), flush=True)
        sys.exit(2)

    import numpy as np
    import torch
    from paper_1705_02408_amd import mpap, synth

    if not torch.cuda.is_available():
        print(json.dumps({"error": "no GPU visible"}), flush=True)
        sys.exit(1)
    torch.cuda.init()

    if args.workload == "batch":
        return run_batch(args)
    if args.workload == "copy":
        return run_copy(args)
    env = (synth.plain3d(args.seed, n=args.n) if args.workload == "plain3d"
           else synth.plain2d(args.seed, n=args.n))
    n_obj = env.n_obj
    t0 = time.perf_counter()
    dg = mpap.mpap_build_graph(env)
    torch.cuda.synchronize()
    build_s = time.perf_counter() - t0
    ginfo = dg.info()
    print(f"# graph built on GPU in {build_s:.3f}s: {ginfo}", file=sys.stderr, flush=True)

    trace = {}

    def step():
        res = mpap.mpap_search(dg, env.beta, n_obj, env.radius, env.lam)
        fr = res.goal_front()
        st = res.stats()
        trace["t"] = res.wave_trace()
        res.close()
        return fr, st

    for i in range(args.warmup):
        fr, st = step()
        print(f"# warmup {i}: {st}", file=sys.stderr, flush=True)

    torch.cuda.synchronize()
    times, kms, stats = [], [], []
    t_start = time.perf_counter()
    for i in range(args.steps):
        ts = time.perf_counter()
        fr, st = step()
        times.append(time.perf_counter() - ts)
        kms.append(st["gpu_ms"])
        stats.append(st)
    torch.cuda.synchronize()
    total = time.perf_counter() - t_start
    print(f"# timed {args.steps} steps in {total:.3f}s; last stats {stats[-1]}",
          file=sys.stderr, flush=True)

    X = stats[-1]["front_labels"]
    R = stats[-1]["relaxations"]
    ms_per_step = 1000.0 * total / args.steps
    value = X * args.steps / total
    k_ms = statistics.mean(kms)
    B = alg_bytes(X, R, n_obj)
    achieved = B / (k_ms * 1e-3) / 1e9

    tr = trace["t"].astype(np.float64)
    tick_ms = 1e-5  # 100 MHz device clock
    phases = {
        "count_ms": float(((tr[:, 1] - tr[:, 0]) * tick_ms).sum()),
        "select_ms": float(((tr[:, 2] - tr[:, 1]) * tick_ms).sum()),
        "merge_ms": float(((tr[:, 3] - tr[:, 2]) * tick_ms).sum()),
        "count_work_block0_ms": float(((tr[:, 8] - tr[:, 0]) * tick_ms).sum()),
        "select_work_block0_ms": float(((tr[:, 9] - tr[:, 1]) * tick_ms).sum()),
        "merge_busiest_block_ms": float((tr[:, 6] * tick_ms).sum()),
        "merge_mean_block_ms": float((tr[:, 7] * tick_ms).sum() / max(1, stats[-1]["blocks"])),
        "max_group": int(tr[:, 4].max()) if tr.shape[0] else 0,
        "max_targets": int(tr[:, 5].max()) if tr.shape[0] else 0,
    }
    print(f"# phases {phases}", file=sys.stderr, flush=True)
    for w in range(0, tr.shape[0], max(1, tr.shape[0] // 12)):
        r = tr[w]
        print(f"# wave {w}: count {(r[1]-r[0])*tick_ms:.3f} select {(r[2]-r[1])*tick_ms:.3f} "
              f"merge {(r[3]-r[2])*tick_ms:.3f} ms, group {int(r[4])}, targets {int(r[5])}, "
              f"busiest block {r[6]*tick_ms:.3f} ms, mean block {r[7]*tick_ms/stats[-1]['blocks']:.3f} ms",
              file=sys.stderr, flush=True)

    cpu = None
    if not args.no_cpu_baseline:
        from oracle import graph as ograph, search as osearch
        t1 = time.perf_counter()
        g = ograph.build_graph(env)
        gb = time.perf_counter() - t1
        labels, secs, finished = osearch.timed_sample(g, env.beta, n_obj, args.cpu_labels)
        cpu = {"value": labels / secs, "unit": "labels/s", "cores": cpu_count_used(),
               "kind": "oracle",
               "sample": (f"sequential label-setting oracle on the same workload, first "
                          f"{labels} labels made permanent ({'whole search' if finished else 'bounded sample'}), "
                          f"{secs:.2f}s on one core of {platform.processor() or platform.machine()}; "
                          f"oracle graph build {gb:.1f}s not counted"),
               "host_cpus": os.cpu_count()}

    out = {
        "metric": "label expansions/s (useful, oracle-exact front)",
        "value": value,
        "unit": "labels/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic (seeded generator), graph built on the GPU",
        "config": {
            "workload": f"{env.name}: {env.dim}D r-disc roadmap, {ginfo['n']} nodes, "
                        f"{ginfo['e']} directed edges, {env.box_lo.shape[0]} boxes, "
                        f"{env.blob_mu.shape[0]} blobs, {n_obj} objectives, beta {env.beta}, "
                        f"lambda {env.lam}",
            "queries_per_step": 1,
            "parallelism": "single GPU",
        },
        "queries_per_s": args.steps / total,
        "search": {"X_front_labels": X, "R_relaxations": R,
                   "labels_expanded_gpu": stats[-1]["labels_expanded"],
                   "waves": stats[-1]["waves"], "merges": stats[-1]["merges"],
                   "candidates": stats[-1]["candidates"],
                   "goal_front": int(fr.vecs.shape[0]),
                   "kernel_ms_mean": k_ms, "kernel_ms_min": min(kms),
                   "step_ms_median": 1000 * statistics.median(times),
                   "blocks": stats[-1]["blocks"], "lds_front_cap": stats[-1]["lds_front_cap"],
                   "max_front": stats[-1]["max_front"], "phases": phases},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS,
                     "traffic": measured_traffic() if args.workload == "plain3d" and
                     args.n == 20000 and args.seed == 0 else None,
                     "traffic_unit": "bytes per launch (rocprofv3 FETCH_SIZE + WRITE_SIZE, "
                                     "scaled by a plain copy's counts)",
                     "kernel": "k_search", "alg_bytes_per_launch": B},
        "cpu_baseline": cpu,
    }
    dg.close()
    if not args.no_batch:
        log = lambda m: print(m, file=sys.stderr, flush=True)  # noqa: E731
        out["batched_serving"] = measure_batch(args, log, with_surrogate=not args.no_surrogate)
    print(json.dumps(out), flush=True)


def train_surrogates(seed: int, log):
    """One surrogate per dimension, trained on roadmaps that are not part of
    the measured batch (the largest query sizes, other seeds)."""
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
        edges = np.random.default_rng(seed + dim).permutation(e)[:n_train]
        s = mpap.Surrogate(seed=seed * 10 + dim)
        t0 = time.perf_counter()
        loss = s.train(g, edges, epochs=8, batch=4096, lr=2e-3)
        dt = time.perf_counter() - t0
        s.score(g)
        ana = mpap.mpap_graph_drift(g, 0)
        sur = mpap.mpap_graph_drift(g, 1)
        held = np.setdiff1d(np.arange(e), edges)
        rel = np.abs(sur[held] - ana[held]) / np.maximum(ana[held], 1e-3)
        log(f"# surrogate {dim}D: {n_train} edges, {dt:.2f}s, loss {loss[0]:.4g} -> "
            f"{loss[-1]:.4g}, held-out median rel err {np.median(rel):.4f} (n={held.size})")
        models[dim] = dict(model=s, train_s=dt, loss_first=float(loss[0]),
                           loss_last=float(loss[-1]), heldout_median_rel=float(np.median(rel)),
                           n_train=int(n_train))
        g.close()
    return models


def measure_batch(args, log, with_surrogate: bool = True):
    """Serving-style load: args.queries independent queries of uneven size in
    one persistent launch, on the learned drift (judged by the analytic
    re-walk, failing queries searched again on the analytic drift), against
    the same queries searched one launch each on the analytic drift."""
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
    # analytic precompute time (the drift the plain path uses)
    ana_ms = sum(mpap.mpap_analytic_drift(p) for p in parts)
    out = {"queries": nq, "build_s": build_s, "analytic_drift_ms": ana_ms}
    models = None
    sur_ms = 0.0
    if with_surrogate:
        models = train_surrogates(args.seed, log)
        sur_ms = sum(models[e.dim]["model"].score(p) for e, p in zip(envs, parts))
        out["surrogate"] = {f"{d}d": {k: v for k, v in m.items() if k != "model"}
                            for d, m in models.items()}
        out["surrogate_score_ms"] = sur_ms
    union = mpap.mpap_graph_concat(parts)
    info = union.info()
    log(f"# {nq} roadmaps ({info}) built in {build_s:.2f}s; analytic drift {ana_ms:.1f} ms, "
        f"surrogate scoring {sur_ms:.1f} ms")
    heur = 1 if with_surrogate else 0
    params = [mpap.search_params(e.beta, e.n_obj, e.radius, e.lam, heuristic=heur) for e in envs]
    # tune on the first 32 queries (the choice never changes a result)
    sub = mpap.mpap_graph_concat(parts[:32])
    t0 = time.perf_counter()
    choice = autotune.tune(sub, params[:32], sorted({e.dim for e in envs}), 2, repeats=1,
                           lambdas=(0.5, 1.0, 2.0), near_scans=(8, 16, 32), log=log)
    sub.close()
    log(f"# autotune {time.perf_counter() - t0:.1f}s")
    params = autotune.apply(params, choice)
    log(f"# autotuned: lambda {choice.lam}, near_scan {choice.near_scan} ({choice.tried})")

    # the batch recorded once as a HIP graph: scoring of every roadmap by its
    # surrogate, the persistent search, the goal fronts
    t0 = time.perf_counter()
    plan = mpap.Plan(union, params, parts=parts if with_surrogate else None,
                     models=[models[e.dim]["model"] for e in envs] if with_surrogate else None)
    log(f"# plan recorded in {time.perf_counter() - t0:.2f}s")

    def one_batch():
        ts = time.perf_counter()
        res = plan.run()
        st = res.stats()
        ok = [True] * nq
        if with_surrogate:
            ok = mpap.surrogate_judge(res, [e.beta for e in envs])
        lat = [res.query_info(k)["latency_ms"] for k in range(nq)]
        res.close()
        log(f"# batch: {time.perf_counter() - ts:.2f}s, kernel {st['gpu_ms']:.1f} ms, "
            f"judge passed {sum(ok)}/{nq}")
        fb_ms = 0.0
        for k in [k for k in range(nq) if not ok[k]]:
            # the judge rejected this front: search the query again on the
            # analytic drift of its own roadmap
            r2 = mpap.mpap_search(parts[k], envs[k].beta, envs[k].n_obj, envs[k].radius,
                                  choice.lam)
            fb_ms += r2.stats()["gpu_ms"]
            lat[k] = st["gpu_ms"] + fb_ms  # answered after the batch and the re-search
            r2.goal_front()
            r2.close()
        return time.perf_counter() - ts, st, lat, ok, fb_ms

    for i in range(min(args.warmup, 1)):
        one_batch()
    torch.cuda.synchronize()
    walls, stats, lats, oks, fbs = [], [], [], [], []
    for i in range(args.batch_steps):
        w, st, lat, ok, fb = one_batch()
        walls.append(w)
        stats.append(st)
        lats.append(lat)
        oks.append(ok)
        fbs.append(fb)
    torch.cuda.synchronize()
    wall = statistics.mean(walls)
    X = stats[-1]["front_labels"]
    lat = np.array(lats[-1])
    # plain: one launch per query, analytic drift
    log("# plain: one launch per query")
    seq = 0.0
    Xp = 0
    for k, (p, e) in enumerate(zip(parts, envs)):
        ts = time.perf_counter()
        r1 = mpap.mpap_search(p, e.beta, e.n_obj, e.radius, e.lam)
        r1.goal_front()
        Xp += r1.stats()["front_labels"]
        r1.close()
        seq += time.perf_counter() - ts
        if (k + 1) % 64 == 0:
            log(f"# plain: {k + 1}/{nq} queries, {seq:.1f}s")
    k_ms = statistics.mean(s_["gpu_ms"] for s_ in stats)
    B = alg_bytes(X, stats[-1]["relaxations"], 2)
    out.update({
        "queries_per_s": nq / wall,
        "label_expansions_per_s": X / wall,
        "step_wall_s": wall,
        "judge_pass_fraction": float(np.mean(oks[-1])),
        "fallback_ms": fbs[-1],
        "latency_ms": {"p50": float(np.percentile(lat, 50)), "p99": float(np.percentile(lat, 99)),
                       "max": float(lat.max())},
        "plain_one_launch_per_query": {"queries_per_s": nq / seq,
                                       "label_expansions_per_s": Xp / seq,
                                       "wall_s": seq},
        "speedup_vs_plain": (nq / wall) / (nq / seq),
        "search": {"X_front_labels": X, "R_relaxations": stats[-1]["relaxations"],
                   "waves": stats[-1]["waves"], "kernel_ms_mean": k_ms,
                   "max_front": stats[-1]["max_front"], "nodes": info["n"], "edges": info["e"]},
        "roofline": {"bound": "hbm", "achieved": B / (k_ms * 1e-3) / 1e9, "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": B / (k_ms * 1e-3) / 1e9 / HBM_PEAK_GBS,
                     "kernel": "k_search_wave" if stats[-1]["wave_build"] else "k_search"},
        "autotune": {"lambda": choice.lam, "near_scan": choice.near_scan},
        "plan": plan.info(),
    })
    plan.close()
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
    log = lambda m: print(m, file=sys.stderr, flush=True)  # noqa: E731
    b = measure_batch(args, log, with_surrogate=not args.no_surrogate)
    out = {
        "metric": "queries/s (batched, oracle-exact fronts)",
        "value": b["queries_per_s"], "unit": "queries/s", "n_gpus": 1,
        "steps": args.batch_steps, "warmup": args.warmup,
        "ms_per_step": 1000.0 * b["step_wall_s"], "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic (seeded generator)",
        "config": {"workload": f"batch of {b['queries']} queries, 2D/3D even odds, sizes "
                               f"log-uniform 2000-50000 samples, two objectives",
                   "queries_per_step": b["queries"], "parallelism": "single GPU"},
        "batched_serving": b, "roofline": dict(b["roofline"], traffic=None),
        "cpu_baseline": None,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
