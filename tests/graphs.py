"""Helpers shared by tests: graph fixtures from edge lists and golden files."""
from __future__ import annotations

import json
import os

import numpy as np

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def from_edges(n, edges, reset, goal):
    """CSR dict from [(u, v, cost, drift), ...], rows sorted by target."""
    edges = sorted(edges, key=lambda e: (e[0], e[1]))
    row_ptr = np.zeros(n + 1, dtype=np.int32)
    for u, _, _, _ in edges:
        row_ptr[u + 1] += 1
    row_ptr = np.cumsum(row_ptr).astype(np.int32)
    col = np.array([e[1] for e in edges], dtype=np.int32)
    cost = np.array([e[2] for e in edges], dtype=np.float32)
    drift = np.array([e[3] for e in edges], dtype=np.float32)
    return dict(row_ptr=row_ptr, col=col, cost=cost, drift=drift,
                reset=np.asarray(reset, dtype=np.uint8), goal=np.asarray(goal, dtype=np.uint8))


def load_golden(name):
    with open(os.path.join(GOLDEN, name)) as f:
        spec = json.load(f)
    g = from_edges(spec["nodes"], [tuple(e) for e in spec["edges"]], spec["reset"], spec["goal"])
    return spec, g


def as_vecs(rows):
    return np.array(rows, dtype=np.float32).reshape(-1, 3)


def load_plain3d_golden():
    """Stored whole-oracle result of the 3D benchmark workload (seed 0):
    (summary dict, per-node front sizes int32 [n], per-node 8-byte digests
    uint8 [n, 8]).  Written by tests/golden/make_plain3d_golden.py."""
    with open(os.path.join(GOLDEN, "plain3d_s0_front.json")) as f:
        summary = json.load(f)
    z = np.load(os.path.join(GOLDEN, "plain3d_s0_fronts.npz"))
    return summary, z["count"], z["digest"]


def front_digest(v) -> bytes:
    """8-byte BLAKE2b of a front's (c, d, m) float32 rows sorted
    lexicographically (the digest of the stored whole-oracle result)."""
    import hashlib
    v = np.ascontiguousarray(v, dtype=np.float32).reshape(-1, 3)
    if v.shape[0]:
        v = v[np.lexsort((v[:, 2], v[:, 1], v[:, 0]))]
    return hashlib.blake2b(np.ascontiguousarray(v).astype("<f4").tobytes(),
                           digest_size=8).digest()


def array_digest(a) -> str:
    import hashlib
    return hashlib.blake2b(np.ascontiguousarray(a).tobytes(), digest_size=16).hexdigest()
