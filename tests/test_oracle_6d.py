"""Pins of the double-integrator roadmap oracle (oracle/graph6d.py) against
what the mathematics fixes: the steering energy against direct quadrature of
the optimal control, boundary conditions, optimality against perturbed
controls, the neighbour selection against a brute-force loop, and the drift
of a straight constant-velocity trajectory against the 2D/3D edge drift."""
import numpy as np
import pytest

from oracle import graph as ograph, graph6d
from paper_1705_02408_amd import synth

F32 = np.float32


def states(seed, m):
    rng = np.random.default_rng(seed)
    p0 = rng.uniform(0.2, 0.8, (m, 3)).astype(F32)
    p1 = rng.uniform(0.2, 0.8, (m, 3)).astype(F32)
    v0 = rng.uniform(-0.5, 0.5, (m, 3)).astype(F32)
    v1 = rng.uniform(-0.5, 0.5, (m, 3)).astype(F32)
    return p0, v0, p1, v1


def control_energy(c0, c1, T, steps=20000):
    """Integral over [0, T] of |c0 + c1 t|^2 by the midpoint rule, float64."""
    t = (np.arange(steps) + 0.5) * (T / steps)
    u = c0.astype(np.float64)[:, None, :] + c1.astype(np.float64)[:, None, :] * t[None, :, None]
    return (u * u).sum(axis=2).sum(axis=1) * (T / steps)


@pytest.mark.parametrize("T", [0.5, 0.25, 1.0])
def test_steer_energy_is_the_integral_of_the_control(T):
    p0, v0, p1, v1 = states(1, 200)
    J, c0, c1 = graph6d.steer(p0, v0, p1, v1, T)
    assert np.allclose(J, control_energy(c0, c1, T), rtol=2e-5, atol=1e-6)


def test_steer_meets_both_boundary_states():
    p0, v0, p1, v1 = states(2, 200)
    T, K = 0.5, 100
    _, c0, c1 = graph6d.steer(p0, v0, p1, v1, T)
    p, v = graph6d.trajectory(p0, v0, c0, c1, T, K)
    assert np.array_equal(p[:, 0], p0) and np.array_equal(v[:, 0], v0)
    assert np.allclose(p[:, -1], p1, atol=2e-5)
    assert np.allclose(v[:, -1], v1, atol=2e-5)


def test_steer_is_the_minimum_energy_control():
    """Adding a control that leaves both end states unchanged (zero mean and
    zero first moment over [0, T]) raises the energy."""
    p0, v0, p1, v1 = states(3, 50)
    T = 0.5
    J, c0, c1 = graph6d.steer(p0, v0, p1, v1, T)
    steps = 4000
    t = (np.arange(steps) + 0.5) * (T / steps)
    # Legendre-like shape orthogonal to 1 and t on [0, T]
    s = t / T
    du = 6 * s * s - 6 * s + 1
    rng = np.random.default_rng(4)
    for _ in range(5):
        eps = rng.normal(0, 0.3, (50, 3))
        u = (c0.astype(np.float64)[:, None, :] + c1.astype(np.float64)[:, None, :] * t[None, :, None]
             + eps[:, None, :] * du[None, :, None])
        # end states unchanged: integral of du and of (T - t) du vanish
        assert abs((du * (T / steps)).sum()) < 1e-7
        assert abs(((T - t) * du * (T / steps)).sum()) < 1e-7
        Jp = (u * u).sum(axis=2).sum(axis=1) * (T / steps)
        assert np.all(Jp > J.astype(np.float64) * (1 - 1e-5))
        assert np.all(Jp - J > 0.5 * (eps ** 2).sum(axis=1) * (du ** 2).mean() * T)


def brute_out_edges(env, u):
    """The first k_out reachable targets of u in (J, id) order: a plain loop
    over candidates and check points, each box tested on its own."""
    pos, vel = env.pos.astype(F32), env.vel.astype(F32)
    T, K = env.horizon, env.traj_steps
    J, c0, c1 = graph6d.steer(pos[u][None], vel[u][None], pos, vel, T)
    order = sorted((float(J[v]), v) for v in range(pos.shape[0]) if v != u)
    keep = []
    for _, v in order:
        p, vv = graph6d.trajectory(pos[u][None], vel[u][None], c0[v][None], c1[v][None], T, K)
        ok = True
        for k in range(K + 1):
            x, w = p[0, k], vv[0, k]
            if np.any(x < 0) or np.any(x > 1):
                ok = False
            if (w[0] * w[0] + w[1] * w[1]) + w[2] * w[2] > F32(1):
                ok = False
            for j in range(env.box_lo.shape[0]):
                if np.all(x >= env.box_lo[j]) and np.all(x <= env.box_hi[j]):
                    ok = False
            if not ok:
                break
        if ok:
            keep.append(v)
        if len(keep) == env.k_out:
            break
    return sorted(keep)


def test_neighbour_selection_matches_brute_force():
    env = synth.plain6d(5, n=120)
    env.k_out = 6
    env.traj_steps = 20
    g = graph6d.build_graph6d(env, block=16, width=8)
    for u in range(0, env.n_nodes, 7):
        row = g["col"][g["row_ptr"][u]:g["row_ptr"][u + 1]].tolist()
        assert row == brute_out_edges(env, u), u


def test_straight_trajectory_drift_matches_the_segment_drift():
    """A steer with a = b = 0 is the straight line at constant velocity, so its
    check points are evenly spaced and the chord drift is the segment drift of
    the 2D/3D roadmaps with K sub-steps."""
    env = synth.plain6d(6, n=50)
    rng = np.random.default_rng(7)
    T, K = 0.5, 40
    # dyadic states: p0 + v T is exact, so a = b = 0 exactly
    p0 = (rng.integers(300, 500, (20, 3)) / 1024.0).astype(F32)
    v = (rng.integers(-300, 300, (20, 3)) / 1024.0).astype(F32)
    p1 = (p0 + v * F32(T)).astype(F32)
    _, c0, c1 = graph6d.steer(p0, v, p1, v, T)
    assert np.all(c0 == 0) and np.all(c1 == 0)
    p, _ = graph6d.trajectory(p0, v, c0, c1, T, K)
    d6 = graph6d.traj_drift(p, env.blob_mu, env.blob_sigma, env.blob_amp).astype(np.float64)
    pts = np.concatenate([p0, p[:, -1]], axis=0)
    ln = np.sqrt(((p[:, -1].astype(np.float64) - p0) ** 2).sum(axis=1))
    a = np.arange(20)
    d3 = ograph.edge_drift(pts, a, a + 20, ln.astype(F32), env.blob_mu, env.blob_sigma,
                           env.blob_amp, float(ln.max()) / K * 1.000001)
    # edge_drift picks K = ceil(len / step) sub-steps; compare where that is K
    Kd = ograph.substeps(ln.astype(F32), float(ln.max()) / K * 1.000001)
    sel = Kd == K
    assert sel.sum() >= 1
    assert np.allclose(d6[sel], d3[sel].astype(np.float64), rtol=1e-5, atol=1e-7)


def test_features_base_is_the_weighted_mean():
    env = synth.plain6d(8, n=200)
    env.goal_radius = 0.3
    g = graph6d.build_graph6d(env)
    f, base, elen = graph6d.edge_features6d(env, g)
    w = f[:, 7:15].astype(np.float64)
    assert np.all(base >= w.min(axis=1) - 1e-6) and np.all(base <= w.max(axis=1) + 1e-6)
    # trajectory length at least the straight distance between the end points
    d = np.sqrt(((f[:, 3:6].astype(np.float64) - f[:, 0:3]) ** 2).sum(axis=1))
    assert np.all(elen >= d * (1 - 1e-5))
