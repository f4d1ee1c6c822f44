"""Pins for the Monte Carlo verification oracle (oracle/mcverify.py), each
against something other than itself:

* Philox4x32-10 against the known-answer vectors published with the
  generator (Random123);
* the normals against the standard normal law (moments, Kolmogorov-Smirnov);
* the LQR gain against scipy's discrete algebraic Riccati solver;
* the polyline nominal against its closed form (end points, points on the
  segments, rest at the nodes, the peak speed, velocity integrating to the
  motion), the cubic nominal against the steering of the 6D
  roadmap (both states met, its energy equal to the closed-form cost J);
* dead reckoning: without fixes or other noise the final estimation error
  has the closed-form variance of twice-summed accelerometer noise;
* special cases: no noise gives zero error, a box on the path is hit, fixes
  everywhere shrink the error.
"""
import math

import numpy as np
import pytest
import scipy.linalg
import scipy.stats

from oracle import graph6d, mcverify as mc


@pytest.mark.parametrize("ctr,key,want", [
    ((0, 0, 0, 0), (0, 0), (0x6627e8d5, 0xe169c58d, 0xbc57ac4c, 0x9b00dbd8)),
    ((0xffffffff,) * 4, (0xffffffff,) * 2, (0x408f276d, 0x41c83b0e, 0xa20bc7c6, 0x6d5451fd)),
    ((0x243f6a88, 0x85a308d3, 0x13198a2e, 0x03707344), (0xa4093822, 0x299f31d0),
     (0xd16cfe09, 0x94fdcceb, 0x5001e420, 0x24126ea1)),
])
def test_philox_known_answers(ctr, key, want):
    got = mc.philox4x32_10(np.array(ctr, np.uint32), np.array(key, np.uint32))
    assert [int(x) for x in got] == list(want)


def test_normals_are_standard():
    z = mc.normals(7, np.arange(2000)[:, None], np.arange(25)[None, :], 3).ravel()
    assert z.shape[0] == 100000
    assert abs(z.mean()) < 0.015 and abs(z.std() - 1.0) < 0.015
    assert scipy.stats.kstest(z, "norm").pvalue > 1e-4
    # the counter decides the draw: other seeds, steps, flights give other numbers
    a = mc.normals(7, 3, 5, 0)
    assert not np.array_equal(a, mc.normals(8, 3, 5, 0))
    assert not np.array_equal(a, mc.normals(7, 4, 5, 0))
    assert not np.array_equal(a, mc.normals(7, 3, 6, 0))
    assert not np.array_equal(a, mc.normals(7, 3, 5, 1))


@pytest.mark.parametrize("dt,qp,qv,ru", [(0.01, 100.0, 20.0, 1.0), (0.005, 10.0, 1.0, 0.1),
                                         (0.02, 1.0, 0.0, 2.0)])
def test_lqr_gain_solves_the_riccati_equation(dt, qp, qv, ru):
    kp, kv, P = mc.lqr_gain(dt, qp, qv, ru)
    A = np.array([[1.0, dt], [0.0, 1.0]])
    B = np.array([[0.5 * dt * dt], [dt]])
    Ps = scipy.linalg.solve_discrete_are(A, B, np.diag([qp, qv]), np.array([[ru]]))
    assert np.abs(P - Ps).max() <= 1e-9 * np.abs(Ps).max()
    K = np.linalg.solve(np.array([[ru]]) + B.T @ Ps @ B, B.T @ Ps @ A)
    assert np.allclose([kp, kv], K.ravel(), rtol=1e-9)
    assert np.all(np.abs(np.linalg.eigvals(A - B @ K)) < 1.0)


def test_polyline_nominal():
    pts = np.array([[0.1, 0.1, 0.1], [0.4, 0.2, 0.1], [0.45, 0.6, 0.3], [0.9, 0.9, 0.9]],
                   np.float32)
    speed, dt = 0.8, 0.001
    p, v, a = mc.nominal_segments(pts, speed, dt)
    P = pts.astype(np.float64)
    lengths = np.sqrt(((P[1:] - P[:-1]) ** 2).sum(axis=1))
    total = 1.5 * lengths.sum() / speed
    assert p.shape[0] == math.ceil(total / dt) + 1
    assert np.allclose(p[0], P[0], atol=0) and np.allclose(p[-1], P[-1], atol=1e-12)
    # every sample lies on one of the segments
    for x in p[::7]:
        dist = []
        for i in range(3):
            s = np.clip(np.dot(x - P[i], P[i + 1] - P[i]) / np.dot(P[i + 1] - P[i], P[i + 1] - P[i]),
                        0, 1)
            dist.append(np.linalg.norm(P[i] + s * (P[i + 1] - P[i]) - x))
        assert min(dist) < 1e-12
    # at rest at every node, the peak speed on each segment (its middle) is
    # `speed`, and the velocity integrates to the motion (trapezoid rule)
    tau = np.concatenate([[0.0], np.cumsum(1.5 * lengths / speed)])
    for i in range(3):
        k0 = int(math.ceil(tau[i] / dt - 1e-9))
        assert np.linalg.norm(v[k0]) < 2 * speed * 6 * dt / (1.5 * lengths[i] / speed)
        km = int(round(0.5 * (tau[i] + tau[i + 1]) / dt))
        assert np.linalg.norm(v[km]) == pytest.approx(speed, rel=1e-3)
    moved = np.cumsum(0.5 * (v[1:] + v[:-1]) * dt, axis=0)
    assert np.allclose(P[0] + moved[-1], P[-1], atol=1e-4)


def test_cubic_nominal_is_the_steering_trajectory():
    rng = np.random.default_rng(3)
    P = rng.uniform(0.2, 0.8, (4, 3)).astype(np.float32)
    V = rng.uniform(-0.4, 0.4, (4, 3)).astype(np.float32)
    T, dt = 0.5, 0.001
    p, v, a = mc.nominal_cubic(P, V, T, dt)
    per = int(round(T / dt))
    for i in range(4):
        k = i * per
        assert np.allclose(p[k], P[i], atol=1e-12) and np.allclose(v[k], V[i], atol=1e-12)
    for i in range(3):
        # a is linear in time on each edge [iT, (i+1)T) (the sample at (i+1)T
        # belongs to the next edge): its value at the edge's end by
        # extrapolation from two samples inside, then the exact integral of a
        # linear function squared; the energy equals the steering cost J
        a0, al = a[i * per], a[i * per + per - 1]
        a1 = a0 + (al - a0) * (T / ((per - 1) * dt))
        energy = T * (a0 @ a0 + a0 @ a1 + a1 @ a1) / 3.0
        J = float(graph6d.steer(P[i], V[i], P[i + 1], V[i + 1], np.float32(T))[0])
        assert energy == pytest.approx(J, rel=1e-5)


def test_dead_reckoning_variance():
    """No fixes (q_min above 1), no applied noise, exact start: the final
    position error per axis is sum_k B1 sigma_a eta_k propagated by A, whose
    variance is sigma_a^2 dt^4 sum_{m<K} (m + 1/2)^2."""
    pts = np.array([[0.1, 0.1], [0.9, 0.1]], np.float32)
    mp = mc.MCParams(rollouts=20000, sigma_w=0.0, sigma0=0.0, q_min=2.0, sigma_a=1.0, seed=5)
    dt = mp.f64("dt")
    p, v, a = mc.nominal_segments(pts, mp.f64("speed"), dt)
    r = mc.rollouts(p, v, a, mp, np.zeros((0, 2), np.float32), np.zeros(0, np.float32),
                    np.zeros(0, np.float32), np.zeros((0, 2)), np.zeros((0, 2)))
    K = r.steps
    want = mp.f64("sigma_a") ** 2 * dt ** 4 * sum((m + 0.5) ** 2 for m in range(K))
    for axis in range(2):
        got = r.final_err[:, axis].var()
        assert got == pytest.approx(want, rel=0.05), (axis, got, want)
    assert not r.collided.any()


def test_special_cases():
    pts = np.array([[0.1, 0.1], [0.5, 0.5], [0.9, 0.2]], np.float32)
    none = np.zeros((0, 2))
    quiet = mc.MCParams(rollouts=64, sigma_w=0.0, sigma_a=0.0, sigma0=0.0, sigma_v=1e-3)
    p, v, a = mc.nominal_segments(pts, quiet.f64("speed"), quiet.f64("dt"))
    r = mc.rollouts(p, v, a, quiet, np.zeros((0, 2), np.float32), np.zeros(0, np.float32),
                    np.zeros(0, np.float32), none, none)
    assert np.all(r.max_err == 0.0) and not r.collided.any()
    # a box around the middle node is entered by every flight
    r = mc.rollouts(p, v, a, quiet, np.zeros((0, 2), np.float32), np.zeros(0, np.float32),
                    np.zeros(0, np.float32), np.array([[0.48, 0.48]]), np.array([[0.52, 0.52]]))
    assert r.collided.all()
    # fixes everywhere (quality clamped to 1) against none
    noisy = mc.MCParams(rollouts=2000, seed=9)
    p, v, a = mc.nominal_segments(pts, noisy.f64("speed"), noisy.f64("dt"))
    blob = (np.array([[0.5, 0.5]], np.float32), np.array([5.0], np.float32),
            np.array([10.0], np.float32))
    with_fix = mc.rollouts(p, v, a, noisy, *blob, none, none)
    without = mc.rollouts(p, v, a, noisy, np.zeros((0, 2), np.float32), np.zeros(0, np.float32),
                          np.zeros(0, np.float32), none, none)
    assert with_fix.max_err.mean() < 0.5 * without.max_err.mean()
