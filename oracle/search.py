"""ctypes wrapper around the sequential label-setting oracle (mosearch.c).

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

``search`` returns the exact per-node Pareto fronts of the float32 label fold
described in mosearch.c, and ``goal_front`` the Pareto-minimal labels over the
goal set, P_candidates of Sec. 3 Alg. 3 kept whole instead of reduced to its
minimum-cost member.
"""
from __future__ import annotations

import ctypes
import dataclasses
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "mosearch.c")
_LIB = os.path.join(_HERE, "_mosearch.so")
_lib = None


def build(force: bool = False) -> str:
    """Compile mosearch.c with IEEE float32 semantics (no FMA contraction)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + f".tmp{os.getpid()}"
        subprocess.check_call(["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math",
                               "-fPIC", "-shared", "-o", tmp, _SRC])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        lib = ctypes.CDLL(build())
        P = ctypes.c_void_p
        lib.mo_run.restype = P
        lib.mo_run.argtypes = [ctypes.c_int32, P, P, P, P, P, ctypes.c_float, ctypes.c_int32,
                               ctypes.c_int32, ctypes.c_int64, ctypes.POINTER(ctypes.c_int32)]
        lib.mo_num_labels.restype = ctypes.c_int64
        lib.mo_num_labels.argtypes = [P]
        lib.mo_copy_arena.argtypes = [P, P, P, P, P, P]
        lib.mo_copy_fronts.argtypes = [P, P, P]
        lib.mo_counters.argtypes = [P, P]
        lib.mo_free.argtypes = [P]
        _lib = lib
    return _lib


def _ptr(a):
    return a.ctypes.data_as(ctypes.c_void_p)


@dataclasses.dataclass
class OracleResult:
    n_obj: int
    beta: float
    # arena of permanent labels
    c: np.ndarray
    d: np.ndarray
    m: np.ndarray
    node: np.ndarray
    parent: np.ndarray
    # per-node fronts as arena indices
    front_off: np.ndarray
    front_lab: np.ndarray
    X: int            # sum of per-node front sizes
    violations: int
    pushes: int
    pops: int
    R: int = 0        # sum over front labels of the head's out-degree
    seconds: float = 0.0
    complete: bool = True
    cut: float = float("inf")  # fronts are exact for costs below this

    def node_front(self, v: int) -> np.ndarray:
        """float32 [k, 3] vectors (c, d, m) at node v, lexicographic order."""
        idx = self.front_lab[self.front_off[v]:self.front_off[v + 1]]
        out = np.stack([self.c[idx], self.d[idx], self.m[idx]], axis=1)
        return sort_lex(out)

    def path(self, label: int) -> list[int]:
        nodes = []
        a = int(label)
        while a >= 0:
            nodes.append(int(self.node[a]))
            a = int(self.parent[a])
        return nodes[::-1]


def sort_lex(v: np.ndarray) -> np.ndarray:
    if v.shape[0] == 0:
        return v.reshape(0, 3).astype(np.float32)
    order = np.lexsort((v[:, 2], v[:, 1], v[:, 0]))
    return v[order]


def search(g: dict, beta: float, n_obj: int, root: int = 0,
           max_labels: int = 0, allow_partial: bool = False) -> OracleResult:
    """Exact per-node fronts for graph ``g`` (CSR dict), bound beta.

    With ``max_labels`` > 0 and ``allow_partial`` the run stops once that many
    labels are permanent.  Labels become permanent in lexicographic order, so
    the partial fronts are then exactly the final fronts restricted to costs
    below ``cut`` (the cost of the last permanent label): ``complete`` tells
    which case holds."""
    import time
    lib = _load()
    rp = np.ascontiguousarray(g["row_ptr"], dtype=np.int32)
    col = np.ascontiguousarray(g["col"], dtype=np.int32)
    cost = np.ascontiguousarray(g["cost"], dtype=np.float32)
    drift = np.ascontiguousarray(g["drift"], dtype=np.float32)
    reset = np.ascontiguousarray(g["reset"], dtype=np.uint8)
    n = rp.shape[0] - 1
    st = ctypes.c_int32(0)
    t0 = time.perf_counter()
    h = lib.mo_run(n, _ptr(rp), _ptr(col), _ptr(cost), _ptr(drift), _ptr(reset),
                   ctypes.c_float(np.float32(beta)), n_obj, root, max_labels,
                   ctypes.byref(st))
    secs = time.perf_counter() - t0
    if not h:
        raise RuntimeError(f"oracle failed, status {st.value}")
    try:
        if st.value != 0 and not (st.value == 1 and allow_partial):
            raise RuntimeError(f"oracle stopped, status {st.value}")
        L = lib.mo_num_labels(h)
        c = np.empty(L, np.float32)
        d = np.empty(L, np.float32)
        m = np.empty(L, np.float32)
        node = np.empty(L, np.int32)
        parent = np.empty(L, np.int32)
        lib.mo_copy_arena(h, _ptr(c), _ptr(d), _ptr(m), _ptr(node), _ptr(parent))
        cnt = np.zeros(5, np.int64)
        lib.mo_counters(h, _ptr(cnt))
        off = np.empty(n + 1, np.int64)
        lab = np.empty(int(cnt[0]), np.int32)
        lib.mo_copy_fronts(h, _ptr(off), _ptr(lab))
    finally:
        lib.mo_free(h)
    outdeg = np.diff(rp).astype(np.int64)
    sizes = np.diff(off)
    R = int((sizes * outdeg).sum())
    complete = st.value == 0
    cut = float("inf") if complete else float(c[-1])
    return OracleResult(n_obj=n_obj, beta=float(np.float32(beta)), c=c, d=d, m=m, node=node,
                        parent=parent, front_off=off, front_lab=lab, X=int(cnt[0]),
                        violations=int(cnt[2]), pushes=int(cnt[3]), pops=int(cnt[4]), R=R,
                        seconds=secs, complete=complete, cut=cut)


def pareto_min(vecs: np.ndarray, n_obj: int) -> np.ndarray:
    """Indices of the Pareto-minimal rows of vecs [k, 3] under weak dominance;
    among equal rows the first is kept.  Plain O(k^2) definition."""
    k = vecs.shape[0]
    keep = []
    use = 3 if n_obj >= 3 else 2
    for i in range(k):
        dom = False
        for j in range(k):
            if j == i:
                continue
            le = all(vecs[j, a] <= vecs[i, a] for a in range(use))
            if not le:
                continue
            eq = all(vecs[j, a] == vecs[i, a] for a in range(use))
            if not eq or j < i:
                dom = True
                break
        if not dom:
            keep.append(i)
    return np.array(keep, dtype=np.int64)


def goal_front(res: OracleResult, goal: np.ndarray):
    """Goal front: Pareto-minimal vectors over the labels at goal nodes, sorted
    lexicographically by (c, d, m).  Witness of each vector: the first label
    with that vector in (goal node id, permanence order).

    Returns (vecs float32 [k, 3], goal_node int32 [k], label int32 [k])."""
    gidx = np.nonzero(np.asarray(goal) != 0)[0]
    labs = []
    for v in gidx:
        labs.extend(res.front_lab[res.front_off[v]:res.front_off[v + 1]].tolist())
    labs = np.array(labs, dtype=np.int64)
    if labs.size == 0:
        return (np.zeros((0, 3), np.float32), np.zeros(0, np.int32), np.zeros(0, np.int32))
    vecs = np.stack([res.c[labs], res.d[labs], res.m[labs]], axis=1)
    keep = pareto_min(vecs, res.n_obj)
    vecs, labs = vecs[keep], labs[keep]
    order = np.lexsort((vecs[:, 2], vecs[:, 1], vecs[:, 0]))
    vecs, labs = vecs[order], labs[order]
    return vecs.astype(np.float32), res.node[labs].astype(np.int32), labs.astype(np.int32)


def rewalk(g: dict, nodes: list[int], beta: float, n_obj: int):
    """Fold a label along an explicit walk (Alg. 3 child step), float32.

    Returns (c, d, m, feasible)."""
    rp, col = g["row_ptr"], g["col"]
    c = np.float32(0.0)
    d = np.float32(0.0)
    m = np.float32(0.0)
    ok = True
    for u, v in zip(nodes[:-1], nodes[1:]):
        row = col[rp[u]:rp[u + 1]]
        j = np.nonzero(row == v)[0]
        if j.size == 0:
            return None
        e = rp[u] + int(j[0])
        c = np.float32(c + g["cost"][e])
        dpre = np.float32(d + g["drift"][e])
        if not dpre <= np.float32(beta):
            ok = False
        d = np.float32(0.0) if g["reset"][v] else dpre
        if n_obj >= 3:
            m = max(m, dpre)
    return c, d, m, ok


def timed_sample(g: dict, beta: float, n_obj: int, max_labels: int, root: int = 0):
    """Run the oracle until it has made ``max_labels`` labels permanent (or
    finished) and time it.  Returns (labels made permanent, seconds, finished).
    Used only to quote a CPU rate on a bounded piece of a large search."""
    import time
    lib = _load()
    rp = np.ascontiguousarray(g["row_ptr"], dtype=np.int32)
    col = np.ascontiguousarray(g["col"], dtype=np.int32)
    cost = np.ascontiguousarray(g["cost"], dtype=np.float32)
    drift = np.ascontiguousarray(g["drift"], dtype=np.float32)
    reset = np.ascontiguousarray(g["reset"], dtype=np.uint8)
    st = ctypes.c_int32(0)
    t0 = time.perf_counter()
    h = lib.mo_run(rp.shape[0] - 1, _ptr(rp), _ptr(col), _ptr(cost), _ptr(drift), _ptr(reset),
                   ctypes.c_float(np.float32(beta)), n_obj, root, int(max_labels),
                   ctypes.byref(st))
    secs = time.perf_counter() - t0
    if not h:
        raise RuntimeError(f"oracle failed, status {st.value}")
    try:
        labels = int(lib.mo_num_labels(h))
    finally:
        lib.mo_free(h)
    return labels, secs, st.value == 0
