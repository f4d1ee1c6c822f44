"""Seeded synthetic workloads for the multiobjective search.

This module only draws random numbers and lays them out: sample positions,
axis-aligned box obstacles, Gaussian feature blobs, start and goal.  It holds
none of the search or graph arithmetic (no neighbour test, no drift, no
perception quality), so that both the HIP library and the CPU checker can take
their inputs from here without sharing any of the method's code.

The generator is counter-based SplitMix64: draw ``i`` of a stream with key
``k`` is ``mix64(k + (i + 1) * GAMMA)`` (Steele, Lea and Flood, "Fast
splittable pseudorandom number generators", OOPSLA 2014).  A stream key is
``mix64(seed * GAMMA ^ tag)`` for a per-entity tag.  A uniform float32 in
[0, 1) is ``(u >> 40) * 2**-24`` (exact in float32).

The environments stand in for the paper's simulation scenes (Sec. 4): sampled
roadmaps over a unit workspace with axis-aligned box obstacles (Sec. 4.2) and a
mapped set of perception features whose density drives a drift heuristic
(Sec. 4.1).  The paper's own scenes and building data are not used.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

GAMMA = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)

# entity tags
TAG_BOXES = 1
TAG_BLOBS = 2
TAG_SAMPLES = 3
TAG_QUERY = 4
TAG_BATCH = 5
TAG_VEL = 6
TAG_EDGES = 7
TAG_DISCOVER = 8


def mix64(z):
    """SplitMix64 finaliser on uint64 scalars or arrays (wrapping arithmetic)."""
    z = np.asarray(z, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = (z ^ (z >> np.uint64(30))) * _M1
        z = (z ^ (z >> np.uint64(27))) * _M2
    return z ^ (z >> np.uint64(31))


class Stream:
    """One counter-based SplitMix64 stream; draws are consumed in order."""

    def __init__(self, seed: int, tag: int):
        with np.errstate(over="ignore"):
            k = np.uint64(seed & 0xFFFFFFFFFFFFFFFF) * GAMMA
        self.key = mix64(k ^ np.uint64(tag))
        self.pos = 0

    def u64(self, n: int) -> np.ndarray:
        i = np.arange(self.pos + 1, self.pos + n + 1, dtype=np.uint64)
        self.pos += n
        with np.errstate(over="ignore"):
            return mix64(self.key + i * GAMMA)

    def uniform(self, n: int) -> np.ndarray:
        """n float32 values in [0, 1)."""
        return ((self.u64(n) >> np.uint64(40)).astype(np.float32)
                * np.float32(2.0 ** -24))


@dataclasses.dataclass
class Env:
    """A planning instance: roadmap samples plus the mapped environment.

    ``pos[0]`` is the initial state (node 0); rows 1..n are free samples.
    ``vel`` is set only for the double-integrator state space (dim 6: position
    and velocity in 3D, boxes/blobs/goal in the 3D workspace); ``k_out`` and
    ``horizon`` are that roadmap's out-degree and steering time.
    """
    dim: int
    pos: np.ndarray            # float32 [n_nodes, dim]
    box_lo: np.ndarray         # float32 [n_boxes, dim]
    box_hi: np.ndarray         # float32 [n_boxes, dim]
    blob_mu: np.ndarray        # float32 [n_blobs, dim]
    blob_sigma: np.ndarray     # float32 [n_blobs]
    blob_amp: np.ndarray       # float32 [n_blobs]
    goal: np.ndarray           # float32 [dim]
    goal_radius: float
    radius: float              # r_n of the r-disc graph
    beta: float                # perception-heuristic bound
    n_obj: int                 # 2: (cost, drift); 3: (cost, drift, max drift)
    lam: float = 0.5           # group cost factor (Sec. 4.2 uses 0.5)
    check_step: float = 0.005  # collision / drift sub-step length
    reset_q: float = 0.8       # relocalisation threshold on q
    name: str = ""
    seed: int = 0
    vel: np.ndarray | None = None
    k_out: int = 0
    horizon: float = 0.0
    traj_steps: int = 0

    @property
    def n_nodes(self) -> int:
        return int(self.pos.shape[0])

    @property
    def wdim(self) -> int:
        """Dimension of the workspace (positions, boxes, blobs, goal)."""
        return 3 if self.dim == 6 else self.dim


def _point_in_any_box(p, lo, hi):
    """p [m, d]; closed boxes.  Returns bool [m]."""
    if lo.shape[0] == 0:
        return np.zeros(p.shape[0], dtype=bool)
    inside = np.ones((p.shape[0], lo.shape[0]), dtype=bool)
    for a in range(p.shape[1]):
        inside &= (p[:, None, a] >= lo[None, :, a]) & (p[:, None, a] <= hi[None, :, a])
    return inside.any(axis=1)


def _boxes(seed, dim, count, hmin, hmax, init, goal, goal_r):
    """Axis-aligned boxes with uniform centres and half-extents; boxes that
    cover the start or touch the goal ball are redrawn."""
    s = Stream(seed, TAG_BOXES)
    lo_l, hi_l = [], []
    goal64 = goal.astype(np.float64)
    while len(lo_l) < count:
        u = s.uniform(2 * dim)
        c = u[:dim]
        h = np.float32(hmin) + np.float32(hmax - hmin) * u[dim:]
        lo = (c - h).astype(np.float32)
        hi = (c + h).astype(np.float32)
        if np.all(init >= lo) and np.all(init <= hi):
            continue
        near = np.clip(goal64, lo.astype(np.float64), hi.astype(np.float64))
        if float(np.sum((near - goal64) ** 2)) <= float(goal_r) ** 2:
            continue
        lo_l.append(lo)
        hi_l.append(hi)
    return (np.array(lo_l, dtype=np.float32).reshape(count, dim),
            np.array(hi_l, dtype=np.float32).reshape(count, dim))


def _blobs(seed, dim, count, amp):
    s = Stream(seed, TAG_BLOBS)
    mu = s.uniform(count * dim).reshape(count, dim)
    sig = np.float32(0.05) + np.float32(0.10) * s.uniform(count)
    amp = np.full(count, amp, dtype=np.float32)
    return mu.astype(np.float32), sig.astype(np.float32), amp


def _free_samples(seed, dim, n, lo, hi):
    """n uniform samples of [0,1)^dim outside every (closed) box, in draw order."""
    s = Stream(seed, TAG_SAMPLES)
    out = []
    have = 0
    while have < n:
        m = max(1024, 2 * (n - have))
        p = s.uniform(m * dim).reshape(m, dim)
        ok = ~_point_in_any_box(p, lo, hi)
        p = p[ok]
        out.append(p[: n - have])
        have += min(p.shape[0], n - have)
    return np.concatenate(out, axis=0).astype(np.float32)


def disc_radius(dim: int, n: int, mean_degree: float) -> float:
    """Radius giving ``mean_degree`` expected neighbours for n uniform samples."""
    if dim == 2:
        return math.sqrt(mean_degree / (math.pi * n))
    if dim == 3:
        return (3.0 * mean_degree / (4.0 * math.pi * n)) ** (1.0 / 3.0)
    raise ValueError(dim)


def make_env(seed: int, dim: int, n: int, n_boxes: int, n_blobs: int,
             mean_degree: float, beta: float, n_obj: int,
             hmin: float = 0.02, hmax: float = 0.08,
             init=None, goal=None, goal_radius: float = 0.05,
             lam: float = 0.5, blob_amp: float = 0.3, name: str = "") -> Env:
    init = np.full(dim, 0.1, dtype=np.float32) if init is None else np.asarray(init, np.float32)
    goal = np.full(dim, 0.9, dtype=np.float32) if goal is None else np.asarray(goal, np.float32)
    lo, hi = _boxes(seed, dim, n_boxes, hmin, hmax, init, goal, goal_radius)
    mu, sig, amp = _blobs(seed, dim, n_blobs, blob_amp)
    samples = _free_samples(seed, dim, n, lo, hi)
    pos = np.concatenate([init[None, :], samples], axis=0).astype(np.float32)
    r = np.float32(disc_radius(dim, n, mean_degree))
    return Env(dim=dim, pos=pos, box_lo=lo, box_hi=hi, blob_mu=mu, blob_sigma=sig,
               blob_amp=amp, goal=goal, goal_radius=float(np.float32(goal_radius)),
               radius=float(r), beta=float(np.float32(beta)), n_obj=n_obj,
               lam=float(np.float32(lam)), name=name, seed=seed)


def discovered_boxes(env: Env, seed: int, count: int, hmin: float = 0.03,
                     hmax: float = 0.08):
    """Obstacles found after the roadmap was built (online updates): boxes
    with uniform centres in the middle of the workspace ([0.25, 0.75] per
    axis) and uniform half-extents, redrawn if they cover the start or touch
    the goal ball.  Returns (lo, hi) float32 [count, dim]."""
    s = Stream(seed, TAG_DISCOVER)
    d = env.wdim
    init = env.pos[0][:d]
    goal64 = np.asarray(env.goal, np.float64)
    lo_l, hi_l = [], []
    while len(lo_l) < count:
        u = s.uniform(2 * d)
        c = np.float32(0.25) + np.float32(0.5) * u[:d]
        h = np.float32(hmin) + np.float32(hmax - hmin) * u[d:]
        lo = (c - h).astype(np.float32)
        hi = (c + h).astype(np.float32)
        if np.all(init >= lo) and np.all(init <= hi):
            continue
        near = np.clip(goal64, lo.astype(np.float64), hi.astype(np.float64))
        if float(np.sum((near - goal64) ** 2)) <= float(env.goal_radius) ** 2:
            continue
        lo_l.append(lo)
        hi_l.append(hi)
    return (np.array(lo_l, dtype=np.float32).reshape(count, d),
            np.array(hi_l, dtype=np.float32).reshape(count, d))


def with_boxes(env: Env, lo, hi) -> Env:
    """The same instance (same samples) with the boxes added to its map."""
    return dataclasses.replace(env, box_lo=np.concatenate([env.box_lo, lo]).astype(np.float32),
                               box_hi=np.concatenate([env.box_hi, hi]).astype(np.float32),
                               name=env.name + f"_plus{lo.shape[0]}boxes")


def plain2d(seed: int = 0, n: int = 2000) -> Env:
    """Unit square, n uniform free samples, ~20 neighbours, 20 rectangles,
    30 feature blobs of amplitude 0.3, start (0.1, 0.1), goal ball r=0.05 at
    (0.9, 0.9), drift bound 0.3, two objectives (cost, drift)."""
    return make_env(seed, 2, n, 20, 30, 20.0, 0.3, 2, name=f"plain2d_n{n}_s{seed}")


def plain3d(seed: int = 0, n: int = 20000) -> Env:
    """Unit cube, n uniform free samples, ~40 neighbours, 100 boxes, 80 blobs
    of amplitude 0.4, start (0.1,0.1,0.1), goal ball r=0.05 at (0.9,0.9,0.9),
    drift bound 0.25, three objectives (cost, drift, max drift so far)."""
    return make_env(seed, 3, n, 100, 80, 40.0, 0.25, 3, blob_amp=0.4,
                    name=f"plain3d_n{n}_s{seed}")


def _unit_ball(seed: int, n: int) -> np.ndarray:
    """n velocities uniform in the open unit ball, by rejection from the cube
    [-1, 1)^3 (draw order kept)."""
    s = Stream(seed, TAG_VEL)
    out, have = [], 0
    while have < n:
        m = max(1024, 2 * (n - have))
        v = (np.float32(2.0) * s.uniform(3 * m).reshape(m, 3) - np.float32(1.0)).astype(np.float32)
        v = v[(v.astype(np.float64) ** 2).sum(axis=1) < 1.0]
        out.append(v[: n - have])
        have += min(v.shape[0], n - have)
    return np.concatenate(out, axis=0).astype(np.float32)


def plain6d(seed: int = 0, n: int = 50000) -> Env:
    """Double-integrator roadmap: states (position, velocity), positions
    uniform free in the unit cube (150 boxes, half-extents 0.02-0.06),
    velocities uniform in the unit ball; start at rest at (0.1, 0.1, 0.1), goal
    ball r=0.05 at (0.9, 0.9, 0.9) in position (any velocity); 100 feature
    blobs of amplitude 0.4; 30 out-edges per node under a steering time of
    0.5 with 100 check steps; drift bound 0.3, two objectives."""
    init = np.full(3, 0.1, dtype=np.float32)
    goal = np.full(3, 0.9, dtype=np.float32)
    lo, hi = _boxes(seed, 3, 150, 0.02, 0.06, init, goal, 0.05)
    mu, sig, amp = _blobs(seed, 3, 100, 0.4)
    pos = np.concatenate([init[None, :], _free_samples(seed, 3, n, lo, hi)], axis=0)
    vel = np.concatenate([np.zeros((1, 3), np.float32), _unit_ball(seed, n)], axis=0)
    return Env(dim=6, pos=pos.astype(np.float32), box_lo=lo, box_hi=hi, blob_mu=mu,
               blob_sigma=sig, blob_amp=amp, goal=goal, goal_radius=float(np.float32(0.05)),
               radius=1.0, beta=float(np.float32(0.3)), n_obj=2, name=f"plain6d_n{n}_s{seed}",
               seed=seed, vel=vel, k_out=30, horizon=0.5, traj_steps=100)


def tiny_random_graph(seed: int, n: int = 30, p_reset: float = 0.2,
                      mean_degree: float = 4.0, integer_costs: bool = False,
                      zero_drift_frac: float = 0.1):
    """A small directed graph with arbitrary per-edge (cost, drift) and reset
    flags, for exhaustive checks.  Node positions are only used to pick a
    neighbourhood structure; edge weights are drawn independently.

    Returns dict(row_ptr, col, cost, drift, reset, goal) with CSR rows sorted by
    target id.  ``integer_costs`` draws costs and drifts from small dyadic sets
    so that equal label vectors (ties) arise often.
    """
    s = Stream(seed, TAG_EDGES)
    pts = s.uniform(2 * n).reshape(n, 2)
    pts[0] = (0.05, 0.05)
    # neighbourhood: k nearest in draw space (generator-level structure only)
    k = max(1, int(round(mean_degree)))
    rows = []
    for u in range(n):
        d2 = ((pts - pts[u]) ** 2).sum(axis=1)
        d2[u] = np.inf
        nb = np.argsort(d2, kind="stable")[:k]
        rows.append(sorted(int(v) for v in nb))
    # symmetrise (both directions), keep sorted, unique
    adj = [set(r) for r in rows]
    for u in range(n):
        for v in rows[u]:
            adj[v].add(u)
    row_ptr = np.zeros(n + 1, dtype=np.int32)
    col = []
    for u in range(n):
        nb = sorted(adj[u])
        col.extend(nb)
        row_ptr[u + 1] = row_ptr[u] + len(nb)
    col = np.array(col, dtype=np.int32)
    e = col.shape[0]
    if integer_costs:
        cost = (1.0 + np.floor(s.uniform(e) * 3.0)).astype(np.float32) * np.float32(0.25)
        drift = np.floor(s.uniform(e) * 4.0).astype(np.float32) * np.float32(0.125)
    else:
        cost = (np.float32(0.05) + np.float32(0.95) * s.uniform(e)).astype(np.float32)
        drift = (np.float32(0.3) * s.uniform(e)).astype(np.float32)
        z = s.uniform(e) < np.float32(zero_drift_frac)
        drift[z] = np.float32(0.0)
    reset = (s.uniform(n) < np.float32(p_reset)).astype(np.uint8)
    reset[0] = 0
    goal = np.zeros(n, dtype=np.uint8)
    # goal set: the nodes farthest from node 0 in draw space (two of them)
    far = np.argsort(-((pts - pts[0]) ** 2).sum(axis=1), kind="stable")[:2]
    goal[far] = 1
    return dict(row_ptr=row_ptr, col=col, cost=cost, drift=drift, reset=reset, goal=goal)


def _free_point(s: Stream, dim: int, lo, hi):
    while True:
        p = s.uniform(dim).astype(np.float32)
        if not _point_in_any_box(p[None, :], lo, hi)[0]:
            return p


def batch_query(batch_seed: int, q: int, nmin: int = 2000, nmax: int = 50000,
                n_obj3: int = 2) -> Env:
    """Query q of a serving-style batch: dimension 2 or 3 (even odds), sample
    count log-uniform in [nmin, nmax], per-query seeded boxes, blobs, start and
    goal centre (uniform, at least 0.5 apart).  Scene densities follow the
    single-query workloads of that dimension; the goal radius grows for small
    roadmaps so that about ten samples fall in the goal ball (never below
    0.05).  ``n_obj3`` sets the objective count of 3D queries."""
    s = Stream(batch_seed * 1000003 + q, TAG_BATCH)
    u = s.uniform(2)
    dim = 2 if u[0] < np.float32(0.5) else 3
    n = int(round(math.exp(math.log(nmin) + float(u[1]) * (math.log(nmax) - math.log(nmin)))))
    seed = int(s.u64(1)[0] & np.uint64(0x7FFFFFFF))
    qs = Stream(seed, TAG_QUERY)
    while True:
        init = qs.uniform(dim).astype(np.float32)
        goal = qs.uniform(dim).astype(np.float32)
        if float(np.sum((init.astype(np.float64) - goal) ** 2)) >= 0.25:
            break
    if dim == 2:
        gr = max(0.05, math.sqrt(10.0 / (math.pi * n)))
        env = make_env(seed, 2, n, 20, 30, 20.0, 0.3, 2, init=init, goal=goal,
                       goal_radius=gr, blob_amp=0.3)
    else:
        gr = max(0.05, (10.0 * 3.0 / (4.0 * math.pi * n)) ** (1.0 / 3.0))
        env = make_env(seed, 3, n, 100, 80, 40.0, 0.25, n_obj3, init=init, goal=goal,
                       goal_radius=gr, blob_amp=0.4)
    env.name = f"batch{batch_seed}_q{q}_{dim}d_n{n}"
    return env
