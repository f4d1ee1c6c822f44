"""Oracle roadmap for the double-integrator state space (position and velocity
in 3D, the dynamics class of the quadrotor experiments, Sec. 4.1 and Sec. 5),
built as BuildGraph does (Sec. 3, Alg. 2) with a steering cost in place of the
Euclidean distance, plus the per-edge drift inputs (Alg. 1 step 2).

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

Definitions (the paper names the dynamics, not the numerics; these readings
are fixed for every consumer of a 6D roadmap):

* Steering x0 = (p0, v0) -> x1 = (p1, v1) in fixed time T is the
  minimum-energy control of the double integrator (minimise the integral of
  |u|^2 with p'' = u).  Per axis, with a = (p1 - p0) - v0 T and b = v1 - v0,
  the optimal control is u(t) = c0 + c1 t with
      c0 = 6a/T^2 - 2b/T,   c1 = (6bT - 12a)/T^3,
  and its energy is J = 12a^2/T^3 - 12ab/T^2 + 4b^2/T.  The edge cost is J
  summed over the axes.  Everything is float32 with each operation rounded
  separately, in the order written in ``steer`` (T is a power of two, so the
  divisions by T, T^2 and T^3 are exact scalings).
* The trajectory is checked at t_k = (k T)/K, k = 0..K:
  p(t) = p0 + t (v0 + t (c0/2 + t c1/6)), v(t) = v0 + t (c0 + t c1/2)
  (float32, Horner order).  An edge is reachable iff at every t_k the
  position lies in the closed unit cube and in no closed box, and
  |v(t_k)|^2 <= 1.
* Out-edges of u: of all v != u in ascending (J, v) order, the first k_out
  reachable ones (directed; rows sorted by target id).
* Drift increment: sum over the K chords of the checked polyline of
  chord length times (1 - q(chord midpoint)), in float64 on the float32 check
  points, rounded once to float32 (the length-weighted midpoint rule of the
  2D/3D roadmaps along the trajectory).
* Relocalisation and goal as in oracle.graph: q(p_v) > the float32 reset_q,
  and the position in the goal ball (any velocity).
"""
from __future__ import annotations

import numpy as np

from .graph import goal_mask, quality

F32 = np.float32


def steer(p0, v0, p1, v1, T):
    """float32 (J, c0, c1) of the minimum-energy steer; inputs broadcast over
    leading axes, last axis = 3 spatial axes; J drops that axis."""
    T = F32(T)
    T2 = T * T
    T3 = T2 * T
    a = (p1 - p0) - v0 * T
    b = v1 - v0
    ja = ((F32(12) * a) * a) / T3 - ((F32(12) * a) * b) / T2 + ((F32(4) * b) * b) / T
    J = (ja[..., 0] + ja[..., 1]) + ja[..., 2]
    c0 = (F32(6) * a) / T2 - (F32(2) * b) / T
    c1 = ((F32(6) * b) * T - F32(12) * a) / T3
    return J.astype(F32), c0.astype(F32), c1.astype(F32)


def check_times(T, K):
    return ((np.arange(K + 1, dtype=F32) * F32(T)) / F32(K)).astype(F32)


def trajectory(p0, v0, c0, c1, T, K):
    """float32 positions and velocities [m, K+1, 3] at the check times."""
    t = check_times(T, K)[None, :, None]
    h2 = (c0 * F32(0.5))[:, None, :]
    h3 = (c1 / F32(6))[:, None, :]
    g1 = (c1 * F32(0.5))[:, None, :]
    p = p0[:, None, :] + t * (v0[:, None, :] + t * (h2 + t * h3))
    v = v0[:, None, :] + t * (c0[:, None, :] + t * g1)
    return p.astype(F32), v.astype(F32)


def reachable(p, v, box_lo, box_hi):
    """Edge reachability from its check points (see the module docstring)."""
    inside = np.all((p >= F32(0)) & (p <= F32(1)), axis=(1, 2))
    sp = (v[..., 0] * v[..., 0] + v[..., 1] * v[..., 1]) + v[..., 2] * v[..., 2]
    ok = inside & np.all(sp <= F32(1), axis=1)
    if box_lo.shape[0] == 0 or p.shape[0] == 0:
        return ok
    # only boxes that meet the bounding box of an edge's points can hold one
    lo = p.min(axis=1)
    hi = p.max(axis=1)
    ov = np.all((hi[:, None, :] >= box_lo[None]) & (lo[:, None, :] <= box_hi[None]), axis=2)
    ei, bj = np.nonzero(ov & ok[:, None])
    if ei.size:
        hit = np.all((p[ei] >= box_lo[bj][:, None, :]) & (p[ei] <= box_hi[bj][:, None, :]),
                     axis=2).any(axis=1)
        ok[ei[hit]] = False
    return ok


def traj_drift(p, mu, sigma, amp):
    """Per edge: sum_k |p_{k+1} - p_k| (1 - q((p_k + p_{k+1})/2)), float64 on
    the float32 points, rounded once to float32."""
    P = p.astype(np.float64)
    seg = P[:, 1:, :] - P[:, :-1, :]
    ln = np.sqrt((seg * seg).sum(axis=2))
    mid = 0.5 * (P[:, 1:, :] + P[:, :-1, :])
    m, K = ln.shape
    q = quality(mid.reshape(-1, 3), mu, sigma, amp).reshape(m, K)
    acc = np.zeros(m, dtype=np.float64)
    for k in range(K):
        acc += ln[:, k] * (1.0 - q[:, k])
    return acc.astype(F32)


def out_edges(pos, vel, u, k_out, T, K, box_lo, box_hi, batch=64):
    """The first k_out reachable targets of u in ascending (J, v) order.
    Returns (targets, J, c0, c1) in that order."""
    n = pos.shape[0]
    J, c0, c1 = steer(pos[u][None, :], vel[u][None, :], pos, vel, T)
    J = J.copy()
    order = np.argsort(J, kind="stable")  # ties by node id
    order = order[order != u]
    keep = []
    s = 0
    while s < order.size and len(keep) < k_out:
        cand = order[s:s + batch]
        p, v = trajectory(np.repeat(pos[u][None, :], cand.size, 0),
                          np.repeat(vel[u][None, :], cand.size, 0), c0[cand], c1[cand], T, K)
        ok = reachable(p, v, box_lo, box_hi)
        keep.extend(cand[ok].tolist())
        s += cand.size
        batch *= 2  # candidates in order, in growing slices
    keep = np.array(keep[:k_out], dtype=np.int64)
    return keep, J[keep], c0[keep], c1[keep]


def _first_reachable_block(pos, vel, rows, k_out, T, K, box_lo, box_hi, width):
    """out_edges for a block of sources at once, looking at the first `width`
    candidates of each; a source with fewer than k_out reachable among them is
    returned as None (the caller falls back to out_edges)."""
    P0, V0 = pos[rows], vel[rows]
    J, c0, c1 = steer(P0[:, None, :], V0[:, None, :], pos[None, :, :], vel[None, :, :], T)
    J[np.arange(rows.size), rows] = np.inf  # v != u
    order = np.argsort(J, axis=1, kind="stable")[:, :width]
    r = np.repeat(np.arange(rows.size), width)
    cand = order.reshape(-1)
    p, v = trajectory(P0[r], V0[r], c0[r, cand], c1[r, cand], T, K)
    ok = reachable(p, v, box_lo, box_hi).reshape(rows.size, width)
    out = []
    for i in range(rows.size):
        sel = order[i][ok[i]][:k_out]
        if sel.size < k_out:
            out.append(None)
            continue
        out.append((sel, J[i, sel], c0[i, sel], c1[i, sel]))
    return out


def build_graph6d(env, block=32, width=64):
    """The directed 6D roadmap of ``env`` (synth.plain6d): dict of CSR arrays
    like oracle.graph.build_graph (row_ptr, col sorted per row, cost = J,
    drift, reset, goal, q)."""
    pos = np.ascontiguousarray(env.pos, F32)
    vel = np.ascontiguousarray(env.vel, F32)
    n = pos.shape[0]
    T, K, k_out = float(env.horizon), int(env.traj_steps), int(env.k_out)
    cols, costs, drifts = [], [], []
    row_ptr = np.zeros(n + 1, dtype=np.int32)
    for u0 in range(0, n, block):
        rows = np.arange(u0, min(n, u0 + block))
        blk = _first_reachable_block(pos, vel, rows, k_out, T, K, env.box_lo, env.box_hi,
                                     min(width, n - 1))
        src, tg, jj, cc0, cc1 = [], [], [], [], []
        for i, u in enumerate(rows):
            found = blk[i]
            if found is None:
                found = out_edges(pos, vel, int(u), k_out, T, K, env.box_lo, env.box_hi)
            tgt, J, c0, c1 = found
            o = np.argsort(tgt, kind="stable")
            src.append(np.full(tgt.size, u, dtype=np.int64))
            tg.append(tgt[o]); jj.append(J[o]); cc0.append(c0[o]); cc1.append(c1[o])
            row_ptr[u + 1] = row_ptr[u] + tgt.size
        src = np.concatenate(src)
        if src.size == 0:
            continue
        c0, c1 = np.concatenate(cc0), np.concatenate(cc1)
        p, _ = trajectory(pos[src], vel[src], c0, c1, T, K)
        cols.append(np.concatenate(tg).astype(np.int32))
        costs.append(np.concatenate(jj).astype(F32))
        drifts.append(traj_drift(p, env.blob_mu, env.blob_sigma, env.blob_amp))
    q = quality(pos, env.blob_mu, env.blob_sigma, env.blob_amp)
    empty = [np.zeros(0, np.int32)]
    return dict(row_ptr=row_ptr, col=np.concatenate(cols or empty),
                cost=np.concatenate(costs or [np.zeros(0, F32)]),
                drift=np.concatenate(drifts or [np.zeros(0, F32)]),
                reset=(q > float(np.float32(env.reset_q))).astype(np.uint8),
                goal=goal_mask(pos, env.goal, env.goal_radius), q=q)


def edge_features6d(env, g):
    """Inputs of the learned drift surrogate for the edges of a 6D roadmap
    (forward CSR order): p_u (3), p_v (3), trajectory length (sum of the
    chords of the check points), 1 - q at t = (k + 1/2) T / 8, k = 0..7, on
    the trajectory, 1 - q(p_v); float32 values before the bfloat16 rounding.
    Also returns base = the speed-weighted mean of the eight 1 - q values
    (sum s_k w_k / sum s_k with s_k = |v(t_k)|, the arc-length weighting of
    the drift integral), float64 rounded to float32."""
    pos = np.ascontiguousarray(env.pos, F32)
    vel = np.ascontiguousarray(env.vel, F32)
    row_ptr, col = g["row_ptr"], g["col"]
    n = row_ptr.shape[0] - 1
    src = np.repeat(np.arange(n), np.diff(row_ptr))
    T, K = float(env.horizon), int(env.traj_steps)
    _, c0, c1 = steer(pos[src], vel[src], pos[col], vel[col], T)
    p, _ = trajectory(pos[src], vel[src], c0, c1, T, K)
    P = p.astype(np.float64)
    seg = P[:, 1:, :] - P[:, :-1, :]
    elen = np.sqrt((seg * seg).sum(axis=2)).sum(axis=1)
    e = col.shape[0]
    f = np.zeros((e, 16), dtype=F32)
    f[:, 0:3] = pos[src]
    f[:, 3:6] = pos[col]
    f[:, 6] = elen
    t = ((np.arange(8, dtype=F32) + F32(0.5)) * F32(T) / F32(8)).astype(F32)
    h2, h3, g1 = c0 * F32(0.5), c1 / F32(6), c1 * F32(0.5)
    sw = np.zeros(e)
    ss = np.zeros(e)
    for k in range(8):
        tk = t[k]
        pk = pos[src] + tk * (vel[src] + tk * (h2 + tk * h3))
        vk = vel[src] + tk * (c0 + tk * g1)
        w = 1.0 - quality(pk.astype(F32), env.blob_mu, env.blob_sigma, env.blob_amp)
        sp = np.sqrt((vk.astype(np.float64) ** 2).sum(axis=1))
        f[:, 7 + k] = w
        sw += sp * w
        ss += sp
    f[:, 15] = 1.0 - quality(pos[col], env.blob_mu, env.blob_sigma, env.blob_amp)
    mean_w = f[:, 7:15].astype(np.float64).mean(axis=1)
    base = np.where(ss > 0, sw / np.where(ss > 0, ss, 1.0), mean_w)
    return f, base.astype(F32), elen.astype(F32)
