"""Independent references that pin the oracle search.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).  None of these share code
with mosearch.c; each reaches (part of) the same result by another route.

* ``brute_fronts``: exhaustive enumeration of walks on tiny graphs, followed
  by the plain Pareto-minimum of Sec. 3 (RemoveDominated, weak reading).
  Only walks that cannot be optimal are skipped, by two facts of the label
  fold: inside a stretch of the walk that passes no relocalising node, a
  repeated node closes a cycle whose removal lowers or keeps every component;
  and a relocalising node reached twice yields (c2, 0, m2) after (c1, 0, m1)
  with c1 < c2, m1 <= m2, so the second visit is dominated as well.  The root
  label (0, 0, 0) is the least vector, so the root is never re-entered.
* ``dijkstra``: scalar shortest-path distances for one additive float32
  objective (minimum-cost end of the front when the bound is off).
* ``bellman_ford_drift``: least reachable drift with relocalisation, by
  repeated relaxation of the monotone maps d -> reset ? 0 : d + delta.
* ``weighted_sum_search``: the single-label foil of Sec. 3 (Fig. 1 argument):
  one label per node, ranked by c + w d, with the same cutoff.
"""
from __future__ import annotations

import heapq

import numpy as np

F32 = np.float32


class _Front:
    """Pareto set of float32 vectors at one node (weak dominance, dedupe)."""

    def __init__(self, use):
        self.use = use
        self.v = np.zeros((0, 3), dtype=np.float32)

    def insert(self, x):
        x = np.asarray(x, dtype=np.float32)
        if self.v.shape[0]:
            A = self.v[:, : self.use]
            xs = x[: self.use]
            if np.any(np.all(A <= xs, axis=1)):
                return
            keep = ~np.all(xs <= A, axis=1)
            self.v = self.v[keep]
        self.v = np.concatenate([self.v, x[None, :]], axis=0)


def brute_fronts(g: dict, beta: float, n_obj: int, root: int = 0,
                 max_steps: int = 5_000_000):
    """Per-node Pareto fronts by enumerating every walk that could be optimal.

    Returns a list of float32 [k, 3] arrays (lexicographically sorted)."""
    rp, col = g["row_ptr"], g["col"]
    cost, drift, reset = g["cost"], g["drift"], g["reset"]
    n = rp.shape[0] - 1
    use = 3 if n_obj >= 3 else 2
    fronts = [_Front(use) for _ in range(n)]
    beta = F32(beta)
    fronts[root].insert((0.0, 0.0, 0.0))
    steps = 0
    # stack entries: (node, c, d, m, segment-set, visited-reset-set)
    stack = [(root, F32(0), F32(0), F32(0), frozenset([root]), frozenset([root]))]
    while stack:
        u, c, d, m, seg, rs = stack.pop()
        steps += 1
        if steps > max_steps:
            raise RuntimeError("walk enumeration budget exceeded")
        for e in range(rp[u], rp[u + 1]):
            v = int(col[e])
            if v == root:
                continue
            c2 = F32(c + cost[e])
            dpre = F32(d + drift[e])
            if not dpre <= beta:
                continue
            if reset[v]:
                if v in rs:
                    continue
                d2 = F32(0.0)
                seg2 = frozenset([v])
                rs2 = rs | {v}
            else:
                if v in seg:
                    continue
                d2 = dpre
                seg2 = seg | {v}
                rs2 = rs
            m2 = max(m, dpre) if n_obj >= 3 else F32(0.0)
            fronts[v].insert((c2, d2, m2))
            stack.append((v, c2, d2, m2, seg2, rs2))
    out = []
    for f in fronts:
        v = f.v
        if v.shape[0]:
            v = v[np.lexsort((v[:, 2], v[:, 1], v[:, 0]))]
        out.append(v.astype(np.float32))
    return out


def dijkstra(g: dict, weight: np.ndarray, root: int = 0):
    """Least float32 fold of ``weight`` over walks from root (additive,
    non-negative weights): textbook Dijkstra with float32 sums."""
    rp, col = g["row_ptr"], g["col"]
    n = rp.shape[0] - 1
    dist = np.full(n, np.inf, dtype=np.float32)
    dist[root] = F32(0)
    done = np.zeros(n, dtype=bool)
    h = [(0.0, root)]
    while h:
        du, u = heapq.heappop(h)
        if done[u]:
            continue
        done[u] = True
        for e in range(rp[u], rp[u + 1]):
            v = int(col[e])
            nd = F32(dist[u] + weight[e])
            if nd < dist[v]:
                dist[v] = nd
                heapq.heappush(h, (float(nd), v))
    return dist


def bellman_ford_drift(g: dict, root: int = 0):
    """Least drift reachable at every node with relocalisation and no bound:
    repeat d[v] <- min(d[v], reset[v] ? 0 : d[u] + delta_e) to a fixpoint."""
    rp, col = g["row_ptr"], g["col"]
    drift, reset = g["drift"], g["reset"]
    n = rp.shape[0] - 1
    d = np.full(n, np.inf, dtype=np.float32)
    d[root] = F32(0)
    for _ in range(n + 1):
        changed = False
        for u in range(n):
            if not np.isfinite(d[u]):
                continue
            for e in range(rp[u], rp[u + 1]):
                v = int(col[e])
                nd = F32(0) if reset[v] else F32(d[u] + drift[e])
                if nd < d[v]:
                    d[v] = nd
                    changed = True
        if not changed:
            break
    return d


def weighted_sum_search(g: dict, beta: float, w: float, root: int = 0):
    """One label per node, the one with least c + w*d (Sec. 3, the combined
    cost foil of Fig. 1), with the same drift cutoff and relocalisation.

    Returns float32 [n, 2] (c, d) of the kept label per node (inf if none)."""
    rp, col = g["row_ptr"], g["col"]
    cost, drift, reset = g["cost"], g["drift"], g["reset"]
    n = rp.shape[0] - 1
    best = np.full(n, np.inf)
    lab = np.full((n, 2), np.inf, dtype=np.float32)
    lab[root] = (0.0, 0.0)
    best[root] = 0.0
    h = [(0.0, root)]
    done = np.zeros(n, dtype=bool)
    while h:
        _, u = heapq.heappop(h)
        if done[u]:
            continue
        done[u] = True
        c, d = lab[u]
        for e in range(rp[u], rp[u + 1]):
            v = int(col[e])
            c2 = F32(c + cost[e])
            dpre = F32(d + drift[e])
            if not dpre <= F32(beta):
                continue
            d2 = F32(0) if reset[v] else dpre
            s = float(c2) + w * float(d2)
            if s < best[v] and not done[v]:
                best[v] = s
                lab[v] = (c2, d2)
                heapq.heappush(h, (s, v))
    return lab
