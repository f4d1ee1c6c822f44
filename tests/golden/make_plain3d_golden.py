"""Write the stored expected result of the whole 3D benchmark search.

Calls only the oracle (``oracle/``) and the seeded input generator: the
roadmap of the 3D workspace workload (20,000 samples, 100 boxes, 80 blobs,
three objectives, bound 0.25, seed 0) is built by ``oracle.graph`` and the
sequential label-setting oracle runs Alg. 3's search to its end (every
per-node front exact, Sec. 3 RemoveDominated under weak dominance).  Nothing
here comes from the HIP library.

Outputs (beside this script):
* ``plain3d_s0_fronts.npz``: per node, the front size and an 8-byte BLAKE2b
  digest of the front's float32 bit patterns (rows (c, d, m) in ascending
  lexicographic order, little-endian), plus per-array digests of the roadmap
  the oracle searched (so a test can first confirm it rebuilt the same
  roadmap);
* ``plain3d_s0_front.json``: X (sum of front sizes), R (sum of front size
  times out-degree), the goal front as float32 bit patterns, the oracle's own
  wall time, the CPU it ran on.

Run: ``python tests/golden/make_plain3d_golden.py`` (about 25 minutes on one
core).
"""
from __future__ import annotations

import hashlib
import json
import os
import platform
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

from oracle import graph as ograph, search as osearch  # noqa: E402
from paper_1705_02408_amd import synth  # noqa: E402

STEM = "plain3d_s0"


def front_digest(v: np.ndarray) -> bytes:
    """8-byte BLAKE2b of a front's (c, d, m) float32 rows sorted lexicographically."""
    v = np.ascontiguousarray(v, dtype=np.float32).reshape(-1, 3)
    if v.shape[0]:
        v = v[np.lexsort((v[:, 2], v[:, 1], v[:, 0]))]
    return hashlib.blake2b(np.ascontiguousarray(v).astype("<f4").tobytes(),
                           digest_size=8).digest()


def array_digest(a: np.ndarray) -> str:
    return hashlib.blake2b(np.ascontiguousarray(a).tobytes(), digest_size=16).hexdigest()


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return platform.processor() or platform.machine()


def main():
    env = synth.plain3d(0)
    t0 = time.perf_counter()
    g = ograph.build_graph(env)
    build_s = time.perf_counter() - t0
    n = g["row_ptr"].shape[0] - 1
    print(f"oracle roadmap: {n} nodes, {int(g['row_ptr'][-1])} edges, {build_s:.1f}s",
          flush=True)
    res = osearch.search(g, env.beta, env.n_obj)
    print(f"oracle search: X={res.X} R={res.R} {res.seconds:.1f}s "
          f"violations={res.violations}", flush=True)
    assert res.violations == 0
    counts = np.diff(res.front_off).astype(np.int32)
    dig = np.zeros((n, 8), dtype=np.uint8)
    for v in range(n):
        dig[v] = np.frombuffer(front_digest(res.node_front(v)), dtype=np.uint8)
    vecs, gnode, _ = osearch.goal_front(res, g["goal"])
    graph_digests = {k: array_digest(g[k]) for k in
                     ("row_ptr", "col", "cost", "drift", "reset", "goal")}
    np.savez_compressed(os.path.join(HERE, f"{STEM}_fronts.npz"), count=counts, digest=dig)
    summary = {
        "source": "whole sequential label-setting oracle (oracle/mosearch.c) on the oracle's "
                  "own roadmap (oracle/graph.py) of the 3D workspace workload, seed 0; "
                  "written by tests/golden/make_plain3d_golden.py",
        "workload": env.name, "n_obj": env.n_obj, "beta": env.beta,
        "nodes": n, "edges": int(g["row_ptr"][-1]),
        "X": int(res.X), "R": int(res.R), "arena_labels": int(res.c.shape[0]),
        "goal_front_bits": np.ascontiguousarray(vecs, np.float32).view(np.uint32).tolist(),
        "goal_front_nodes": gnode.tolist(),
        "graph_digests": graph_digests,
        "oracle_seconds": res.seconds, "oracle_cores": 1, "oracle_cpu": cpu_model(),
        "oracle_labels_per_s": res.X / res.seconds,
        "graph_build_seconds": build_s,
        "digest": "blake2b-8 of the front's (c, d, m) float32 rows in ascending "
                  "lexicographic order, little-endian",
    }
    with open(os.path.join(HERE, f"{STEM}_front.json"), "w") as f:
        json.dump(summary, f, indent=1)
        f.write("\n")
    print(json.dumps({k: v for k, v in summary.items() if k != "goal_front_bits"}), flush=True)


if __name__ == "__main__":
    main()
