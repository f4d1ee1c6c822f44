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


def cpu_count_used() -> int:
    return 1


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--n", type=int, default=20000)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--workload", choices=["plain3d", "plain2d", "batch"], default="plain3d")
    ap.add_argument("--queries", type=int, default=256, help="batch workload: query count")
    ap.add_argument("--cpu-labels", type=int, default=150000,
                    help="labels the oracle makes permanent in the CPU baseline sample")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    args = ap.parse_args()

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU only; the search of one "
                                   "roadmap is not sharded across GPUs (see DESIGN.md)",
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
                     "frac": achieved / HBM_PEAK_GBS, "traffic": None,
                     "kernel": "k_search", "alg_bytes_per_launch": B},
        "cpu_baseline": cpu,
    }
    dg.close()
    print(json.dumps(out), flush=True)


def run_batch(args):
    """Serving-style load: args.queries independent queries of uneven size in
    one persistent launch; compared with the same queries searched one by one."""
    import numpy as np
    import torch
    from paper_1705_02408_amd import mpap, synth

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
    union = mpap.mpap_graph_concat(parts)
    torch.cuda.synchronize()
    build_s = time.perf_counter() - t0
    info = union.info()
    print(f"# {len(parts)} roadmaps built on GPU in {build_s:.2f}s: {info}", file=sys.stderr,
          flush=True)
    params = [mpap.search_params(e.beta, e.n_obj, e.radius, e.lam) for e in envs]

    def step():
        res = mpap.mpap_search_batch(union, params)
        st = res.stats()
        lat = [res.query_info(k)["latency_ms"] for k in range(len(envs))]
        fronts = [res.goal_front(k).vecs.shape[0] for k in range(len(envs))]
        res.close()
        return st, lat, fronts

    for i in range(args.warmup):
        st, lat, fr = step()
        print(f"# warmup {i}: {st}", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    times, stats, lats = [], [], []
    ts0 = time.perf_counter()
    for i in range(args.steps):
        ts = time.perf_counter()
        st, lat, fr = step()
        times.append(time.perf_counter() - ts)
        stats.append(st)
        lats.append(lat)
    torch.cuda.synchronize()
    total = time.perf_counter() - ts0
    nq = len(envs)
    X = stats[-1]["front_labels"]
    lat = np.array(lats[-1])
    # the plain alternative: the same queries, one launch each
    seq = []
    for p, e in zip(parts, envs):
        ts = time.perf_counter()
        r1 = mpap.mpap_search(p, e.beta, e.n_obj, e.radius, e.lam)
        r1.goal_front()
        r1.close()
        seq.append(time.perf_counter() - ts)
    seq_total = sum(seq)
    k_ms = statistics.mean(s_["gpu_ms"] for s_ in stats)
    R = stats[-1]["relaxations"]
    B = alg_bytes(X, R, 2)
    out = {
        "metric": "queries/s (batched, oracle-exact fronts)",
        "value": nq * args.steps / total,
        "unit": "queries/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": 1000.0 * total / args.steps,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic (seeded generator), roadmaps built on the GPU",
        "config": {"workload": f"batch of {nq} queries, 2D/3D even odds, sizes log-uniform "
                               f"2000-50000 samples ({info['n']} nodes, {info['e']} edges), "
                               f"two objectives", "queries_per_step": nq,
                   "parallelism": "single GPU, one persistent launch"},
        "label_expansions_per_s": X * args.steps / total,
        "latency_ms": {"p50": float(np.percentile(lat, 50)), "p99": float(np.percentile(lat, 99)),
                       "max": float(lat.max())},
        "plain_one_launch_per_query": {"queries_per_s": nq / seq_total,
                                       "label_expansions_per_s": X / seq_total},
        "search": {"X_front_labels": X, "R_relaxations": R, "waves": stats[-1]["waves"],
                   "kernel_ms_mean": k_ms, "max_front": stats[-1]["max_front"]},
        "roofline": {"bound": "hbm", "achieved": B / (k_ms * 1e-3) / 1e9, "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": B / (k_ms * 1e-3) / 1e9 / HBM_PEAK_GBS,
                     "traffic": None, "kernel": "k_search", "alg_bytes_per_launch": B},
        "cpu_baseline": None,
    }
    union.close()
    for p in parts:
        p.close()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
