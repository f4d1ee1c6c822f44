"""Oracle graph construction: BuildGraph (Sec. 3, Alg. 2) plus the per-edge
drift inputs of the perception heuristic (Sec. 3, Alg. 1 step 2).

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

Definitions used (the paper leaves the numerics open; these are the readings
this project fixes, applied identically by every consumer of a graph):

* Cost(u, v) is the Euclidean length, evaluated in float32 as
  sqrt((dx*dx + dy*dy) [+ dz*dz]) with every operation rounded separately
  (no fused multiply-add), dx = x_v - x_u.
* Near(V \\ {v}, v, r_n) keeps u != v with Cost(v, u) < r_n, strictly, as in
  the primitive list of Sec. 3.
* Collision(u, v) checks the points x_a + t_k (x_b - x_a), t_k = k / K,
  k = 0..K, K = ceil(Cost / step), against closed axis-aligned boxes
  (Sec. 4.2 uses axis-aligned boxes), all in float32, where (a, b) is the pair
  ordered by node id so that the test is symmetric.
* Perception quality q(x) = clamp(sum_j a_j exp(-|x - mu_j|^2 / (2 s_j^2)),
  0, 1) over the feature blobs, in float64.  The drift increment of an edge is
  the edge length times one minus the mean of q at the K sub-step midpoints
  (a continuous-rate reading of the per-time-step drift heuristic of
  Sec. 4.1), summed in float64 and rounded once to float32.
* A node relocalises (its drift resets to zero on arrival) iff q(x_v) > the
  float32 threshold (0.8 as a float32 number, the value a float32 parameter
  carries).
* Goal membership: (dx*dx + dy*dy [+ dz*dz]) <= r_g*r_g in float32.
"""
from __future__ import annotations

import math

import numpy as np

F32 = np.float32


def _sqdist_rows(pos, rows):
    """float32 squared distances from pos[rows] to every node, per-op rounding."""
    diff = pos[None, :, :] - pos[rows][:, None, :]
    sq = diff[..., 0] * diff[..., 0]
    for a in range(1, pos.shape[1]):
        sq = sq + diff[..., a] * diff[..., a]
    return sq


def near_pairs(pos, r, chunk=256):
    """All ordered pairs (u, v), u != v, with Cost(u, v) < r (Alg. 2, Near).

    Returns (src, dst, cost) with rows sorted by (src, dst)."""
    n = pos.shape[0]
    r = F32(r)
    src_l, dst_l, c_l = [], [], []
    for u0 in range(0, n, chunk):
        rows = np.arange(u0, min(n, u0 + chunk))
        cost = np.sqrt(_sqdist_rows(pos, rows))
        mask = cost < r
        mask[np.arange(rows.shape[0]), rows] = False
        ru, vv = np.nonzero(mask)
        src_l.append(rows[ru].astype(np.int32))
        dst_l.append(vv.astype(np.int32))
        c_l.append(cost[ru, vv].astype(np.float32))
    return (np.concatenate(src_l), np.concatenate(dst_l), np.concatenate(c_l))


def substeps(cost, step):
    """K = ceil(Cost / step) in float32 (at least 1)."""
    k = np.ceil(cost.astype(np.float32) / F32(step)).astype(np.int64)
    return np.maximum(k, 1)


def collides(pos, a, b, cost, box_lo, box_hi, step):
    """Collision(a, b) for pairs a < b (Alg. 2 with closed axis-aligned boxes).

    Points x_a + (k/K) (x_b - x_a), k = 0..K, float32 with separate rounding."""
    m = a.shape[0]
    hit = np.zeros(m, dtype=bool)
    if box_lo.shape[0] == 0 or m == 0:
        return hit
    K = substeps(cost, step)
    xa = pos[a]
    xb = pos[b]
    diff = (xb - xa).astype(np.float32)
    seg_lo = np.minimum(xa, xb) - F32(1e-5)
    seg_hi = np.maximum(xa, xb) + F32(1e-5)
    for j in range(box_lo.shape[0]):
        lo = box_lo[j]
        hi = box_hi[j]
        cand = np.all((seg_hi >= lo) & (seg_lo <= hi), axis=1) & ~hit
        idx = np.nonzero(cand)[0]
        if idx.size == 0:
            continue
        for kv in np.unique(K[idx]):
            sel = idx[K[idx] == kv]
            t = (np.arange(kv + 1, dtype=np.float32) / F32(kv)).astype(np.float32)
            p = xa[sel][:, None, :] + (t[None, :, None] * diff[sel][:, None, :])
            inside = np.all((p >= lo) & (p <= hi), axis=2).any(axis=1)
            hit[sel[inside]] = True
    return hit


def quality(x, mu, sigma, amp):
    """q(x) = clamp(sum_j a_j exp(-|x - mu_j|^2 / (2 sigma_j^2)), 0, 1), float64."""
    x = np.asarray(x, dtype=np.float64)
    acc = np.zeros(x.shape[0], dtype=np.float64)
    for j in range(mu.shape[0]):
        d2 = np.zeros(x.shape[0], dtype=np.float64)
        for a in range(x.shape[1]):
            t = x[:, a] - float(mu[j, a])
            d2 += t * t
        acc += float(amp[j]) * np.exp(-d2 / (2.0 * float(sigma[j]) ** 2))
    return np.clip(acc, 0.0, 1.0)


def edge_drift(pos, a, b, cost, mu, sigma, amp, step):
    """Drift increment of edge (a, b): len * (1 - mean q over K midpoints).

    Evaluated in float64 as sum_j (len/K) (1 - q(x_a + (j+1/2)/K (x_b - x_a)))
    and rounded once to float32."""
    K = substeps(cost, step)
    out = np.zeros(a.shape[0], dtype=np.float64)
    xa = pos[a].astype(np.float64)
    xb = pos[b].astype(np.float64)
    ln = cost.astype(np.float64)
    for kv in np.unique(K):
        sel = np.nonzero(K == kv)[0]
        s = (np.arange(kv, dtype=np.float64) + 0.5) / kv
        pts = xa[sel][:, None, :] + s[None, :, None] * (xb[sel] - xa[sel])[:, None, :]
        q = quality(pts.reshape(-1, pos.shape[1]), mu, sigma, amp).reshape(sel.size, kv)
        acc = np.zeros(sel.size, dtype=np.float64)
        for j in range(kv):
            acc += (ln[sel] / kv) * (1.0 - q[:, j])
        out[sel] = acc
    return out.astype(np.float32)


def goal_mask(pos, goal, goal_radius):
    g = np.asarray(goal, dtype=np.float32)
    d = (pos - g[None, :]).astype(np.float32)
    sq = d[:, 0] * d[:, 0]
    for a in range(1, pos.shape[1]):
        sq = sq + d[:, a] * d[:, a]
    r = F32(goal_radius)
    return (sq <= r * r).astype(np.uint8)


def build_graph(env):
    """BuildGraph (Alg. 2) and per-edge drift for an r-disc roadmap.

    Returns a dict of CSR arrays: row_ptr int32[n+1], col int32[E] (targets
    sorted per row), cost float32[E], drift float32[E], reset uint8[n],
    goal uint8[n], plus q float64[n] (node quality, for diagnostics)."""
    pos = np.ascontiguousarray(env.pos, dtype=np.float32)
    n = pos.shape[0]
    src, dst, cost = near_pairs(pos, env.radius)
    # undirected pairs a < b carry the collision test and the drift value
    und = src < dst
    a, b, c = src[und], dst[und], cost[und]
    hit = collides(pos, a, b, c, env.box_lo, env.box_hi, env.check_step)
    a, b, c = a[~hit], b[~hit], c[~hit]
    dr = edge_drift(pos, a, b, c, env.blob_mu, env.blob_sigma, env.blob_amp, env.check_step)
    # both directions
    s2 = np.concatenate([a, b])
    d2 = np.concatenate([b, a])
    c2 = np.concatenate([c, c])
    r2 = np.concatenate([dr, dr])
    order = np.lexsort((d2, s2))
    s2, d2, c2, r2 = s2[order], d2[order], c2[order], r2[order]
    row_ptr = np.zeros(n + 1, dtype=np.int64)
    np.add.at(row_ptr, s2.astype(np.int64) + 1, 1)
    row_ptr = np.cumsum(row_ptr).astype(np.int32)
    q = quality(pos, env.blob_mu, env.blob_sigma, env.blob_amp)
    reset = (q > float(np.float32(env.reset_q))).astype(np.uint8)
    goal = goal_mask(pos, env.goal, env.goal_radius)
    return dict(row_ptr=row_ptr, col=d2.astype(np.int32), cost=c2.astype(np.float32),
                drift=r2.astype(np.float32), reset=reset, goal=goal, q=q)


def graph_stats(g):
    n = g["row_ptr"].shape[0] - 1
    e = int(g["row_ptr"][-1])
    return dict(n=n, e=e, mean_degree=e / max(n, 1),
                reset_frac=float(g["reset"].mean()), n_goal=int(g["goal"].sum()),
                min_cost=float(g["cost"].min()) if e else math.inf)


def edge_features(pos, row_ptr, col, cost, mu, sigma, amp):
    """Inputs of the learned drift surrogate per edge (forward CSR order), from
    the id-ordered pair (a, b): x_a (3), x_b (3, zero z in 2D), the length,
    1 - q at x_a + (k + 1/2)/8 (x_b - x_a) for k = 0..7, and 1 - q(x_b)
    (float64 q, complement in float64), as float32 values before the bfloat16
    rounding of the model.  Also returns base = the mean of the eight 1 - q
    values (float64, rounded to float32): the 8-point midpoint estimate of
    drift / length that the network corrects."""
    n = row_ptr.shape[0] - 1
    src = np.repeat(np.arange(n), np.diff(row_ptr))
    a = np.minimum(src, col)
    b = np.maximum(src, col)
    pa = pos[a].astype(np.float32)
    pb = pos[b].astype(np.float32)
    e = col.shape[0]
    f = np.zeros((e, 16), dtype=np.float32)
    d = pos.shape[1]
    f[:, 0:d] = pa
    f[:, 3:3 + d] = pb
    f[:, 6] = cost
    diff = (pb - pa).astype(np.float32)
    acc = np.zeros(e, dtype=np.float64)
    for k in range(8):
        s = np.float32((k + 0.5) / 8.0)
        pts = (pa + s * diff).astype(np.float32)
        w = 1.0 - quality(pts, mu, sigma, amp)
        f[:, 7 + k] = w
        acc += w
    f[:, 15] = 1.0 - quality(pb, mu, sigma, amp)
    return f, (acc / 8.0).astype(np.float32)
