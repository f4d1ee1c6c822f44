"""Alg. 3 (Explore) of the paper, step by step, in plain Python.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

This is the group loop of Sec. 3 as the paper writes it, with the readings
used throughout the repository (weak Pareto dominance per head node with one
copy of equal vectors, the bound tested on the pre-relocalisation drift,
float32 label sums in path order):

* P_open holds the root plan (x_init, no path, cost 0, heuristic 0), P(x_init)
  the same plan, the group G the same plan, i = 0;
* while P_open is not empty -- and, in the paper's early-stop mode, while no
  plan of G has its head in the goal set (every plan satisfies the bound, so
  "feasible" adds nothing) --
  - every plan p of G is extended to every out-neighbour x of its head: the
    child's cost and heuristic, kept when the heuristic is within the bound,
    added to P(x) and to P_open;
  - RemoveDominated over the plans sharing a head;
  - P_open loses G; i grows by one; G becomes the open plans of cost at most
    i * lambda * r_n (float32 product of the float32 step lambda * r_n).
  An iteration whose G is empty changes nothing but i, so i jumps to the first
  index whose threshold reaches the least open cost.
* P_candidates are the plans at goal nodes; the goal front is their Pareto
  minimum, whose first entry in (c, d, m) order is P_soln (the minimum-cost
  plan).

Run to an empty P_open the per-node sets are the exact Pareto fronts the
label-setting oracle (mosearch.c) computes; with the early stop they are the
state at the iteration the loop ends.  Tie rule for equal vectors at a node:
the plan made first stays (plans are numbered in the order the loops above
make them: G in ascending plan number, out-edges in CSR order).
"""
from __future__ import annotations

import dataclasses

import numpy as np

F32 = np.float32


def _fold(c, d, m, ce, de, reset_x, n_obj):
    """Child of a plan along one edge (Alg. 3 child line): float32 sums;
    None when the pre-relocalisation drift exceeds the bound is decided by
    the caller."""
    c2 = F32(c + ce)
    dpre = F32(d + de)
    d2 = F32(0.0) if reset_x else dpre
    m2 = F32(max(m, dpre)) if n_obj == 3 else F32(0.0)
    return c2, dpre, d2, m2


def _weakly_dominates(a, b):
    return a[0] <= b[0] and a[1] <= b[1] and a[2] <= b[2]


def _first_reaching_step(cmin, delta):
    """Least i >= 0 with float32(i * delta) >= cmin."""
    i = max(0, int(np.floor(float(cmin) / float(delta))) - 2)
    while F32(F32(i) * delta) < cmin:
        i += 1
    return i


@dataclasses.dataclass
class ExploreResult:
    vec: list            # per plan (c, d, m) float32
    node: list           # per plan head
    parent: list         # per plan parent plan (-1 for the root)
    fronts: list         # per node, plan numbers alive at the end
    groups: int          # groups expanded (non-empty iterations)
    stopped: bool        # the early stop ended the loop
    last_i: int          # iteration index of the group the loop ended on

    def node_front(self, v: int) -> np.ndarray:
        rows = np.array([self.vec[p] for p in self.fronts[v]], dtype=np.float32).reshape(-1, 3)
        if rows.shape[0]:
            rows = rows[np.lexsort((rows[:, 2], rows[:, 1], rows[:, 0]))]
        return rows

    def goal_front(self, goal) -> np.ndarray:
        """Pareto minimum of P_candidates (plans at goal nodes), ascending
        (c, d, m); entry 0 is P_soln."""
        cand = [self.vec[p] for v in np.nonzero(np.asarray(goal))[0] for p in self.fronts[v]]
        keep = []
        for a in cand:
            if any(_weakly_dominates(b, a) and b != a for b in cand):
                continue
            if a not in keep:
                keep.append(a)
        rows = np.array(keep, dtype=np.float32).reshape(-1, 3)
        if rows.shape[0]:
            rows = rows[np.lexsort((rows[:, 2], rows[:, 1], rows[:, 0]))]
        return rows


def explore(g: dict, beta: float, n_obj: int, lam: float, radius: float, root: int = 0,
            early_stop: bool = False, max_iter: int = 1 << 30) -> ExploreResult:
    """Alg. 3 on graph ``g`` (CSR dict with cost, drift, reset, goal)."""
    rp, col = g["row_ptr"], g["col"]
    cost = np.asarray(g["cost"], np.float32)
    drift = np.asarray(g["drift"], np.float32)
    reset = np.asarray(g["reset"])
    goal = np.asarray(g["goal"])
    n = rp.shape[0] - 1
    beta = F32(beta)
    delta = F32(F32(lam) * F32(radius))

    vec = [(F32(0.0), F32(0.0), F32(0.0))]
    node = [root]
    parent = [-1]
    P = [[] for _ in range(n)]
    P[root].append(0)
    alive = [True]
    open_ = {0}
    G = [0]
    i = 0
    groups = 0
    stopped = False
    while open_:
        if early_stop and any(goal[node[p]] for p in G):
            stopped = True
            break
        if groups >= max_iter:
            raise RuntimeError("iteration cap reached")
        touched = []
        for p in G:                                   # forall p in G
            u = node[p]
            c, d, m = vec[p]
            for e in range(rp[u], rp[u + 1]):         # forall x in N(p.head)
                x = int(col[e])
                c2, dpre, d2, m2 = _fold(c, d, m, cost[e], drift[e], reset[x], n_obj)
                if dpre <= beta:                      # heuristic cutoff
                    q = len(vec)
                    vec.append((c2, d2, m2))
                    node.append(x)
                    parent.append(p)
                    alive.append(True)
                    P[x].append(q)
                    open_.add(q)
                    touched.append(x)
        groups += 1
        # RemoveDominated: per head node, weak dominance, first-made copy of
        # equal vectors stays
        for x in sorted(set(touched)):
            keep = []
            for q in P[x]:
                a = vec[q]
                dead = False
                for r in P[x]:
                    b = vec[r]
                    if r != q and _weakly_dominates(b, a) and (b != a or r < q):
                        dead = True
                        break
                if dead:
                    alive[q] = False
                    open_.discard(q)
                else:
                    keep.append(q)
            P[x] = keep
        open_.difference_update(G)                    # P_open <- P_open \ G
        if not open_:
            G = []
            break
        i += 1
        T = F32(F32(i) * delta)
        G = sorted(p for p in open_ if vec[p][0] <= T)
        if not G:                                     # empty groups change nothing but i
            i = _first_reaching_step(min(vec[p][0] for p in open_), delta)
            T = F32(F32(i) * delta)
            G = sorted(p for p in open_ if vec[p][0] <= T)
    return ExploreResult(vec=vec, node=node, parent=parent, fronts=P, groups=groups,
                         stopped=stopped, last_i=i)
