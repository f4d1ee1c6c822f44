"""Pins for the oracle's roadmap and drift inputs (oracle/graph.py): each part
checked against geometry, closed forms or quadrature, never against itself.

* Near (Alg. 2): float64 distances decide every pair away from the radius;
  exact dyadic pairs at the radius are excluded (strict test), self excluded,
  symmetric, rows sorted.
* Collision (Alg. 2, closed axis-aligned boxes of Sec. 4.2): a float64 slab
  test of the continuous segment bounds the sampled test from both sides; a
  hand-placed box touched only at a face is hit, one crossed between two
  samples is missed.
* Quality q and the drift increment (Sec. 4.1 drift reading): closed forms (no
  blobs, a blob centre, one standard deviation away, clamping, a constant
  field) and the midpoint-rule error bound against adaptive quadrature of the
  drift integral.
* Learned-heuristic inputs: endpoint order, length, closed forms of the
  quality samples, and the 8-point base against quadrature.
"""
import math

import numpy as np
import pytest

from oracle import graph
from paper_1705_02408_amd import synth

F32 = np.float32
quad = pytest.importorskip("scipy.integrate").quad


def env_of(pos, boxes=(), blobs=(), radius=0.25, step=0.005, reset_q=0.8,
           goal=None, goal_radius=0.05):
    """A hand-made environment: pos [n, d]; boxes [(lo, hi)]; blobs
    [(mu, sigma, amp)]."""
    pos = np.asarray(pos, F32)
    d = pos.shape[1]
    lo = np.array([b[0] for b in boxes], F32).reshape(-1, d)
    hi = np.array([b[1] for b in boxes], F32).reshape(-1, d)
    mu = np.array([b[0] for b in blobs], F32).reshape(-1, d)
    sg = np.array([b[1] for b in blobs], F32).reshape(-1)
    am = np.array([b[2] for b in blobs], F32).reshape(-1)
    g = np.full(d, 0.9, F32) if goal is None else np.asarray(goal, F32)
    return synth.Env(dim=d, pos=pos, box_lo=lo, box_hi=hi, blob_mu=mu, blob_sigma=sg,
                     blob_amp=am, goal=g, goal_radius=goal_radius, radius=radius, beta=0.3,
                     n_obj=2, check_step=step, reset_q=reset_q)


# ------------------------------------------------------------------- Near
@pytest.mark.parametrize("dim,n,r", [(2, 400, 0.08), (3, 500, 0.15)])
def test_near_against_float64_distances(dim, n, r):
    rng = np.random.default_rng(dim)
    pos = rng.uniform(0, 1, (n, dim)).astype(F32)
    src, dst, cost = graph.near_pairs(pos, r)
    got = set(zip(src.tolist(), dst.tolist()))
    d64 = np.sqrt(((pos[:, None, :].astype(np.float64) - pos[None, :, :]) ** 2).sum(axis=2))
    sure_in = (d64 < r * (1 - 1e-6)) & ~np.eye(n, dtype=bool)
    sure_out = (d64 > r * (1 + 1e-6)) | np.eye(n, dtype=bool)
    want_in = set(zip(*np.nonzero(sure_in)))
    assert want_in <= got
    assert not any(sure_out[u, v] for u, v in got)
    assert all(u != v for u, v in got)
    assert got == {(v, u) for u, v in got}                    # symmetric
    order = np.lexsort((dst, src))
    assert np.array_equal(order, np.arange(src.size))         # rows sorted
    # the float32 length is the float64 distance within a few float32 ulp
    ref = d64[src, dst]
    assert np.all(np.abs(cost - ref) <= 4 * np.finfo(F32).eps * ref)


@pytest.mark.parametrize("dim", [2, 3])
def test_near_is_strict_at_the_radius(dim):
    """Dyadic coordinates make the lengths exact: a pair at exactly r_n is
    not a neighbour, one inside is."""
    p = np.zeros((4, dim), F32)
    p[1, -1] = 0.25      # |p1 - p0| = 0.25 = r
    p[2, 0] = 0.125      # 0.125 < r
    p[3, 0] = 0.625      # far from everything
    src, dst, cost = graph.near_pairs(p, 0.25)
    pairs = set(zip(src.tolist(), dst.tolist()))
    assert (0, 1) not in pairs and (1, 0) not in pairs
    assert (0, 2) in pairs and (2, 0) in pairs
    assert not any(3 in pr for pr in pairs)
    assert cost[(src == 0) & (dst == 2)][0] == F32(0.125)


# -------------------------------------------------------------- Collision
def slab_interval(xa, xb, lo, hi):
    """Parameter interval [t0, t1] of the continuous segment inside the
    closed box (float64 slab method); None if it misses."""
    t0, t1 = 0.0, 1.0
    for k in range(xa.shape[0]):
        a, b = float(xa[k]), float(xb[k])
        dk = b - a
        if dk == 0.0:
            if a < lo[k] or a > hi[k]:
                return None
            continue
        u0, u1 = (float(lo[k]) - a) / dk, (float(hi[k]) - a) / dk
        if u0 > u1:
            u0, u1 = u1, u0
        t0, t1 = max(t0, u0), min(t1, u1)
        if t0 > t1:
            return None
    return t0, t1


@pytest.mark.parametrize("dim", [2, 3])
def test_collision_bounded_by_the_continuous_segment(dim):
    """Sampled collision sits between two exact statements: a segment whose
    continuous path misses a slightly grown box is never hit, and one that
    stays inside a slightly shrunk box for more than one sample spacing is
    always hit."""
    rng = np.random.default_rng(10 + dim)
    m = 3000
    pos = rng.uniform(0, 1, (2 * m, dim)).astype(F32)
    a = np.arange(0, 2 * m, 2)
    b = a + 1
    # short segments, like roadmap edges
    pos[b] = (pos[a] + rng.uniform(-0.08, 0.08, (m, dim))).astype(F32)
    d = pos[b].astype(np.float64) - pos[a]
    cost = np.sqrt((d * d).sum(axis=1)).astype(F32)
    ctr = rng.uniform(0, 1, (40, dim))
    half = rng.uniform(0.01, 0.06, (40, dim))
    lo, hi = (ctr - half).astype(F32), (ctr + half).astype(F32)
    step = 0.005
    hit = graph.collides(pos, a, b, cost, lo, hi, step)
    K = graph.substeps(cost, step)
    n_sure_hit = n_sure_miss = 0
    for i in range(m):
        xa, xb = pos[a[i]].astype(np.float64), pos[b[i]].astype(np.float64)
        grown = [slab_interval(xa, xb, lo[j].astype(np.float64) - 1e-6,
                               hi[j].astype(np.float64) + 1e-6) for j in range(40)]
        if all(iv is None for iv in grown):
            assert not hit[i], i
            n_sure_miss += 1
        shrunk = [slab_interval(xa, xb, lo[j].astype(np.float64) + 1e-6,
                                hi[j].astype(np.float64) - 1e-6) for j in range(40)]
        if any(iv is not None and iv[1] - iv[0] > 1.0 / K[i] + 1e-6 for iv in shrunk):
            assert hit[i], i
            n_sure_hit += 1
    assert n_sure_hit > 50 and n_sure_miss > 1000


def test_collision_closed_faces_and_gaps_between_samples():
    """Dyadic geometry: step 0.125 and a segment of length 0.375 give the
    samples t = 0, 1/3, 2/3, 1 at x = 0, 0.125, 0.25, 0.375."""
    pos = np.array([[0.0, 0.5], [0.375, 0.5]], F32)
    a, b = np.array([0]), np.array([1])
    cost = np.array([0.375], F32)

    def hits(lo, hi):
        return bool(graph.collides(pos, a, b, cost, np.array([lo], F32), np.array([hi], F32),
                                   0.125)[0])
    assert graph.substeps(cost, 0.125)[0] == 3
    assert hits([0.25, 0.5], [0.3, 0.6])          # sample x = 0.25 on the lower face
    assert hits([0.3, 0.25], [0.375, 0.5])        # end point on a corner edge
    assert not hits([0.15, 0.4], [0.2, 0.6])      # crossed between two samples
    assert not hits([0.0, 0.5 + 2 ** -10], [0.375, 0.75])  # just above the segment


# ------------------------------------------------------------ quality, drift
def test_quality_closed_forms():
    mu = np.array([[0.5, 0.5, 0.5]], F32)
    sg = np.array([0.1], F32)
    am = np.array([0.75], F32)
    x = np.array([[0.5, 0.5, 0.5], [0.6, 0.5, 0.5], [5.0, 5.0, 5.0]], F32)
    q = graph.quality(x, mu, sg, am)
    assert q[0] == 0.75                                       # exp(0) = 1
    s = float(sg[0])
    dx = float(F32(0.6)) - float(F32(0.5))
    assert q[1] == pytest.approx(0.75 * math.exp(-dx * dx / (2 * s * s)), rel=1e-14)
    assert q[2] == 0.0
    # no blobs: zero quality everywhere
    assert np.all(graph.quality(x, mu[:0], sg[:0], am[:0]) == 0.0)
    # clamped to [0, 1]
    assert graph.quality(x[:1], mu, sg, np.array([1.5], F32))[0] == 1.0
    assert graph.quality(x[:1], mu, sg, np.array([-0.5], F32))[0] == 0.0
    # additive below the clamp
    two = graph.quality(x, np.concatenate([mu, mu]), np.concatenate([sg, sg]),
                        np.array([0.25, 0.5], F32))
    assert np.allclose(two, graph.quality(x, mu, sg, np.array([0.75], F32)), rtol=1e-15)


def test_drift_closed_forms():
    rng = np.random.default_rng(3)
    pos = rng.uniform(0.2, 0.8, (60, 3)).astype(F32)
    a = np.arange(0, 60, 2)
    b = a + 1
    d = pos[b].astype(np.float64) - pos[a]
    cost = np.sqrt((d * d).sum(axis=1)).astype(F32)
    none = graph.edge_drift(pos, a, b, cost, np.zeros((0, 3), F32), np.zeros(0, F32),
                            np.zeros(0, F32), 0.005)
    assert np.array_equal(none, cost)                         # q = 0: drift = length
    mu = np.array([[0.5, 0.5, 0.5]], F32)
    full = graph.edge_drift(pos, a, b, cost, mu, np.array([1e4], F32),
                            np.array([2.0], F32), 0.005)
    assert np.all(full == 0.0)                                # q = 1: no drift
    const = graph.edge_drift(pos, a, b, cost, mu, np.array([1e4], F32),
                             np.array([0.375], F32), 0.005)
    assert np.allclose(const, cost * (1 - 0.375), rtol=1e-6)  # q = 0.375 everywhere


@pytest.mark.parametrize("seed", range(4))
def test_drift_is_the_midpoint_rule_of_the_drift_integral(seed):
    """drift = integral over the edge of (1 - q) to within the midpoint rule's
    bound L * max|f''| / (24 K^2), f(s) = L (1 - q(x_a + s (x_b - x_a))), with
    |q''| <= sum_j a_j L^2 / sigma_j^2 for Gaussian blobs (no clamping: the
    amplitudes sum below 1).  A left- or right-end rule, a dropped length
    factor or a wrong sub-step count is off by far more."""
    rng = np.random.default_rng(100 + seed)
    dim = 2 + seed % 2
    n_e = 40
    pos = rng.uniform(0.3, 0.7, (2 * n_e, dim)).astype(F32)
    a = np.arange(0, 2 * n_e, 2)
    b = a + 1
    pos[b] = (pos[a] + rng.uniform(-0.06, 0.06, (n_e, dim))).astype(F32)
    d = pos[b].astype(np.float64) - pos[a]
    cost = np.sqrt((d * d).sum(axis=1)).astype(F32)
    mu = rng.uniform(0.3, 0.7, (3, dim)).astype(F32)
    sg = rng.uniform(0.05, 0.15, 3).astype(F32)
    am = np.array([0.3, 0.3, 0.3], F32)
    dr = graph.edge_drift(pos, a, b, cost, mu, sg, am, 0.005).astype(np.float64)
    K = graph.substeps(cost, 0.005)

    def q_exact(x):
        return sum(float(am[j]) * math.exp(-float(((x - mu[j].astype(np.float64)) ** 2).sum())
                                           / (2 * float(sg[j]) ** 2)) for j in range(3))
    for i in range(n_e):
        xa, xb = pos[a[i]].astype(np.float64), pos[b[i]].astype(np.float64)
        L = float(cost[i])
        I, _ = quad(lambda s: L * (1.0 - q_exact(xa + s * (xb - xa))), 0.0, 1.0,
                    epsabs=1e-14, epsrel=1e-13)
        qpp = sum(float(am[j]) * L * L / float(sg[j]) ** 2 for j in range(3))
        bound = L * qpp / (24.0 * K[i] ** 2) + 2 * np.finfo(F32).eps * L
        assert abs(dr[i] - I) <= bound, (i, dr[i], I, bound)


def test_relocalisation_threshold_is_strict():
    """A node at a blob centre has q equal to the amplitude: q = 0.8 does not
    relocalise (q > 0.8 is required), the next float32 amplitude does."""
    pos = np.array([[0.1, 0.1], [0.5, 0.5], [0.9, 0.9]], F32)
    for amp, want in ((F32(0.8), 0), (np.nextafter(F32(0.8), F32(1)), 1)):
        env = env_of(pos, blobs=[((0.5, 0.5), 0.05, amp)], radius=0.7)
        g = graph.build_graph(env)
        assert g["reset"][1] == want


def test_roadmap_is_symmetric_with_one_drift_per_edge():
    env = synth.plain2d(2, n=500)
    g = graph.build_graph(env)
    rp, col = g["row_ptr"], g["col"]
    n = rp.shape[0] - 1
    src = np.repeat(np.arange(n), np.diff(rp))
    fwd = {(int(u), int(v)): (g["cost"][e], g["drift"][e]) for e, (u, v) in
           enumerate(zip(src, col))}
    for (u, v), cd in fwd.items():
        assert fwd[(v, u)] == cd
    # every box-free straight edge keeps its Near length
    d = env.pos[col].astype(np.float64) - env.pos[src]
    assert np.allclose(g["cost"], np.sqrt((d * d).sum(axis=1)), rtol=1e-6)


# ------------------------------------------------------ learned-heuristic inputs
def test_edge_features_layout_and_closed_forms():
    rng = np.random.default_rng(5)
    pos = rng.uniform(0.3, 0.7, (30, 3)).astype(F32)
    n = pos.shape[0]
    rp = np.arange(0, 2 * n + 1, 2, dtype=np.int32)[: n + 1]
    col = np.array([(u + k) % n for u in range(n) for k in (1, 7)], np.int32)
    src = np.repeat(np.arange(n), 2)
    d = pos[col].astype(np.float64) - pos[src]
    cost = np.sqrt((d * d).sum(axis=1)).astype(F32)
    e0 = np.zeros((0, 3), F32)
    f, base = graph.edge_features(pos, rp, col, cost, e0, np.zeros(0, F32), np.zeros(0, F32))
    lo, hi = np.minimum(src, col), np.maximum(src, col)
    assert np.array_equal(f[:, 0:3], pos[lo]) and np.array_equal(f[:, 3:6], pos[hi])
    assert np.array_equal(f[:, 6], cost)
    assert np.all(f[:, 7:16] == 1.0) and np.all(base == 1.0)  # no blobs: 1 - q = 1
    # a blob centred on the id-larger endpoint: its 1 - q is exactly 1 - a
    mu = pos[hi[:1]]
    f1, _ = graph.edge_features(pos, rp[:2], col[:2], cost[:2], mu, np.array([0.05], F32),
                                np.array([0.625], F32))
    assert f1[0, 15] == F32(1 - 0.625)


def test_feature_base_is_the_eight_point_midpoint_rule():
    """base * length equals the drift integral to within the midpoint rule's
    bound with 8 sub-steps."""
    rng = np.random.default_rng(6)
    n = 40
    pos = rng.uniform(0.3, 0.7, (n, 3)).astype(F32)
    rp = np.arange(n + 1, dtype=np.int32)
    col = np.array([(u + 1) % n for u in range(n)], np.int32)
    src = np.arange(n)
    d = pos[col].astype(np.float64) - pos[src]
    cost = np.sqrt((d * d).sum(axis=1)).astype(F32)
    mu = rng.uniform(0.3, 0.7, (2, 3)).astype(F32)
    sg = np.array([0.2, 0.3], F32)
    am = np.array([0.4, 0.4], F32)
    _, base = graph.edge_features(pos, rp, col, cost, mu, sg, am)
    for i in range(n):
        ia, ib = min(i, int(col[i])), max(i, int(col[i]))
        xa, xb = pos[ia].astype(np.float64), pos[ib].astype(np.float64)
        L = float(cost[i])

        def one_minus_q(s):
            x = xa + s * (xb - xa)
            return 1.0 - sum(float(am[j]) * math.exp(-float(((x - mu[j]) ** 2).sum())
                                                     / (2 * float(sg[j]) ** 2))
                             for j in range(2))
        I, _ = quad(one_minus_q, 0.0, 1.0, epsabs=1e-14, epsrel=1e-13)
        qpp = sum(float(am[j]) * L * L / float(sg[j]) ** 2 for j in range(2))
        assert abs(float(base[i]) - I) <= qpp / (24 * 64) + 1e-6, i
