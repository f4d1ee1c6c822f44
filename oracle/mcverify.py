"""Monte Carlo verification of a plan (Sec. 3, final phase; the system and
localisation models of Sec. 4.1), plain numpy in float64.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

The paper estimates, by sampling, the probability that the plan P_soln keeps
the localisation error within a bound when it is flown: a double integrator
tracks the nominal trajectory with an LQR controller, an accelerometer with
noise drives the prediction of a Kalman filter, and position fixes from the
mapped features correct it.  The paper gives the structure, not the numbers,
so the model is fixed here (the same one the library's kernels run):

* nominal trajectory: 2D/3D roadmaps -- the plan's polyline flown from rest
  to rest along every segment (the minimum-energy cubic between the two
  nodes at zero velocity, over 1.5 length / speed, so the peak speed is
  ``speed``; a double integrator cannot follow a corner at speed);
  6D roadmaps -- per edge the cubic through both states over the steering
  time T (the fixed-time minimum-energy trajectory of a double integrator),
  with its velocity and acceleration; sampled at t_k = k dt, k = 0..K with
  K = ceil(duration / dt), the last sample clamped to the end;
* per axis (identical axes) x = (p, v), x_{k+1} = A x_k + B a_k with
  A = [[1, dt], [0, 1]], B = [dt^2/2, dt]; applied acceleration
  a_k = u_k + sigma_w xi_k;
* control u_k = (v_nom,k+1 - v_nom,k) / dt - k_p (p_hat_k - p_nom,k)
  - k_v (v_hat_k - v_nom,k): the feed-forward is the nominal velocity change
  over the step (the discrete double integrator then keeps the nominal
  velocity exactly), the feedback the steady-state discrete LQR gain for
  Q = diag(q_p, q_v), R = r_u (Riccati recursion from P = Q, a fixed 20,000
  steps);
* Kalman filter: prediction with the measured acceleration a_k + sigma_a eta_k
  and process covariance sigma_a^2 B B^T; a position fix at the new true
  position when the feature quality there is q >= q_min, with noise variance
  sigma_v^2 / q (q = the clamped blob sum of the drift model, float64);
* start: true position p_nom,0 + sigma_0 xi_0, velocity v_nom,0; estimate the
  nominal state, covariance diag(sigma_0^2, 0);
* per rollout: the largest localisation error max_k |p_k - p_hat_k| over
  k = 0..K and whether any true position p_k lies in a (closed) box.

Random numbers: Philox4x32-10 (Salmon, Moraes, Dror, Shaw, "Parallel random
numbers: as easy as 1, 2, 3", SC 2011) keyed by the seed (low word, high
word) with counter (step, rollout, draw, 0) -- step 0xffffffff for the start
-- giving two 64-bit words; each word's top 53 bits plus one half make a
uniform in (0, 1), and the pair gives two normals by the Box-Muller
transform.  Per step 3 * dim normals in the order xi, eta, zeta (draws
0, 1, 2, ... of two normals each).
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

M0, M1 = np.uint64(0xD2511F53), np.uint64(0xCD9E8D57)
W0, W1 = np.uint32(0x9E3779B9), np.uint32(0xBB67AE85)
MASK32 = np.uint64(0xFFFFFFFF)
START_STEP = 0xFFFFFFFF


def philox4x32_10(ctr, key):
    """Philox4x32 with 10 rounds.  ctr: uint32 [..., 4]; key: uint32 [..., 2]
    (broadcast).  Returns uint32 [..., 4]."""
    c = [np.asarray(ctr[..., i], np.uint32) for i in range(4)]
    k0 = np.asarray(key[..., 0], np.uint32).copy()
    k1 = np.asarray(key[..., 1], np.uint32).copy()
    for r in range(10):
        if r > 0:
            k0 = ((k0.astype(np.uint64) + np.uint64(W0)) & MASK32).astype(np.uint32)
            k1 = ((k1.astype(np.uint64) + np.uint64(W1)) & MASK32).astype(np.uint32)
        p0 = M0 * c[0].astype(np.uint64)
        p1 = M1 * c[2].astype(np.uint64)
        hi0, lo0 = (p0 >> np.uint64(32)).astype(np.uint32), (p0 & MASK32).astype(np.uint32)
        hi1, lo1 = (p1 >> np.uint64(32)).astype(np.uint32), (p1 & MASK32).astype(np.uint32)
        c = [hi1 ^ c[1] ^ k0, lo1, hi0 ^ c[3] ^ k1, lo0]
    return np.stack(c, axis=-1)


def normals(seed: int, step, rollout, draw):
    """Two standard normals per (step, rollout, draw) counter: float64 [..., 2]."""
    step, rollout, draw = np.broadcast_arrays(np.asarray(step, np.uint64),
                                              np.asarray(rollout, np.uint64),
                                              np.asarray(draw, np.uint64))
    ctr = np.stack([step.astype(np.uint32), rollout.astype(np.uint32), draw.astype(np.uint32),
                    np.zeros(step.shape, np.uint32)], axis=-1)
    key = np.array([seed & 0xFFFFFFFF, (seed >> 32) & 0xFFFFFFFF], np.uint32)
    w = philox4x32_10(ctr, key).astype(np.uint64)
    a = (w[..., 0] << np.uint64(32)) | w[..., 1]
    b = (w[..., 2] << np.uint64(32)) | w[..., 3]
    u1 = ((a >> np.uint64(11)).astype(np.float64) + 0.5) * 2.0 ** -53
    u2 = ((b >> np.uint64(11)).astype(np.float64) + 0.5) * 2.0 ** -53
    r = np.sqrt(-2.0 * np.log(u1))
    t = 2.0 * math.pi * u2
    return np.stack([r * np.cos(t), r * np.sin(t)], axis=-1)


def lqr_gain(dt: float, q_p: float, q_v: float, r_u: float, steps: int = 20000):
    """Steady-state discrete LQR gain (k_p, k_v) of the per-axis double
    integrator, by the Riccati recursion from P = Q."""
    A = np.array([[1.0, dt], [0.0, 1.0]])
    B = np.array([[0.5 * dt * dt], [dt]])
    Q = np.diag([q_p, q_v])
    P = Q.copy()
    for _ in range(steps):
        S = r_u + (B.T @ P @ B)[0, 0]
        K = (B.T @ P @ A) / S
        P = Q + A.T @ P @ A - (A.T @ P @ B) @ K
    S = r_u + (B.T @ P @ B)[0, 0]
    K = (B.T @ P @ A) / S
    return float(K[0, 0]), float(K[0, 1]), P


def nominal_segments(pts, speed: float, dt: float):
    """The polyline through pts (float32 [m, d]) flown from rest to rest along
    every segment: per segment the cubic between the two nodes at zero
    velocity (the cubic of nominal_cubic with v0 = v1 = 0) over the time
    1.5 length / speed, so that the peak speed (at mid-segment) is ``speed``;
    p, v, a float64 [K+1, d] at t_k = k dt (clamped to the end)."""
    P = np.asarray(pts, np.float64)
    seg = P[1:] - P[:-1]
    length = np.sqrt((seg * seg).sum(axis=1))
    dur = 1.5 * length / speed
    tau = np.concatenate([[0.0], np.cumsum(dur)])
    total = tau[-1]
    K = max(1, int(math.ceil(total / dt)))
    t = np.minimum(np.arange(K + 1) * dt, total)
    i = np.clip(np.searchsorted(tau, t, side="right") - 1, 0, len(dur) - 1)
    s = (t - tau[i])[:, None]
    T = dur[i][:, None]
    p0, p1 = P[i], P[i + 1]
    c2 = (3.0 * (p1 - p0)) / (T * T)
    c3 = (2.0 * (p0 - p1)) / (T * T * T)
    p = p0 + c2 * s * s + c3 * s * s * s
    v = 2.0 * c2 * s + 3.0 * c3 * s * s
    a = 2.0 * c2 + 6.0 * c3 * s
    return p, v, a


def nominal_cubic(states_p, states_v, horizon: float, dt: float):
    """Per edge the cubic between consecutive states over time T: p, v, a
    float64 [K+1, 3] at t_k = k dt (clamped to the end)."""
    P = np.asarray(states_p, np.float64)
    V = np.asarray(states_v, np.float64)
    T = float(horizon)
    m = P.shape[0] - 1
    total = m * T
    K = max(1, int(math.ceil(total / dt)))
    t = np.minimum(np.arange(K + 1) * dt, total)
    i = np.clip(np.floor(t / T).astype(np.int64), 0, m - 1)
    s = t - i * T
    p0, p1, v0, v1 = P[i], P[i + 1], V[i], V[i + 1]
    c2 = (3.0 * (p1 - p0) - (2.0 * v0 + v1) * T) / (T * T)
    c3 = (2.0 * (p0 - p1) + (v0 + v1) * T) / (T * T * T)
    s_ = s[:, None]
    p = p0 + v0 * s_ + c2 * s_ * s_ + c3 * s_ * s_ * s_
    v = v0 + 2.0 * c2 * s_ + 3.0 * c3 * s_ * s_
    a = 2.0 * c2 + 6.0 * c3 * s_
    return p, v, a


def quality(x, mu, sig, amp):
    """Clamped blob sum at points x [R, d], float64, blobs in order."""
    acc = np.zeros(x.shape[0])
    for j in range(mu.shape[0]):
        d2 = np.zeros(x.shape[0])
        for k in range(x.shape[1]):
            t = x[:, k] - np.float64(mu[j, k])
            d2 = d2 + t * t
        s = np.float64(sig[j])
        acc = acc + np.float64(amp[j]) * np.exp(-d2 / (2.0 * (s * s)))
    return np.clip(acc, 0.0, 1.0)


@dataclasses.dataclass
class MCParams:
    """Model constants (float32 values, as the library takes them)."""
    rollouts: int = 4096
    dt: float = 0.005
    speed: float = 0.5
    sigma_w: float = 0.1
    sigma_a: float = 0.1
    sigma_v: float = 0.005
    q_min: float = 0.8
    sigma0: float = 0.002
    err_bound: float = 0.05
    q_p: float = 100.0
    q_v: float = 20.0
    r_u: float = 1.0
    seed: int = 1

    def f64(self, name):
        """The float32 parameter widened to float64."""
        return float(np.float32(getattr(self, name)))


@dataclasses.dataclass
class MCResult:
    max_err: np.ndarray     # float64 [R]
    collided: np.ndarray    # bool [R]
    final_err: np.ndarray   # float64 [R, d]: p - p_hat at the last step
    steps: int
    gain: tuple


def rollouts(p_nom, v_nom, a_nom, mp: MCParams, mu, sig, amp, box_lo, box_hi,
             rollout_ids=None):
    """The rollouts of the plan's nominal trajectory (p_nom, v_nom, a_nom
    float64 [K+1, d]); rollout_ids (optional) picks which counters to run."""
    dt = mp.f64("dt")
    sw, sa, sv, s0, qmin = (mp.f64(k) for k in ("sigma_w", "sigma_a", "sigma_v", "sigma0",
                                                "q_min"))
    d = p_nom.shape[1]
    K = p_nom.shape[0] - 1
    kp, kv, _ = lqr_gain(dt, mp.f64("q_p"), mp.f64("q_v"), mp.f64("r_u"))
    ids = np.arange(mp.rollouts) if rollout_ids is None else np.asarray(rollout_ids)
    R = ids.shape[0]
    half = 0.5 * dt * dt
    lo = np.asarray(box_lo, np.float64)
    hi = np.asarray(box_hi, np.float64)

    def inside(x):
        if lo.shape[0] == 0:
            return np.zeros(x.shape[0], bool)
        return np.any(np.all((x[:, None, :] >= lo[None]) & (x[:, None, :] <= hi[None]), axis=2),
                      axis=1)

    nd = (d + 1) // 2  # draws of two normals for d values
    xi0 = np.concatenate([normals(mp.seed, START_STEP, ids[:, None], j) for j in range(nd)],
                         axis=-1).reshape(R, -1)[:, :d]
    p = p_nom[0][None, :] + s0 * xi0
    v = np.repeat(v_nom[0][None, :], R, axis=0)
    ph = np.repeat(p_nom[0][None, :], R, axis=0)
    vh = np.repeat(v_nom[0][None, :], R, axis=0)
    P00 = np.full(R, s0 * s0)
    P01 = np.zeros(R)
    P11 = np.zeros(R)
    err = np.sqrt(((p - ph) ** 2).sum(axis=1))
    max_err = err.copy()
    hit = inside(p)
    nz = (3 * d + 1) // 2
    for k in range(K):
        z = np.concatenate([normals(mp.seed, k, ids[:, None], j) for j in range(nz)],
                           axis=-1).reshape(R, -1)
        xi, eta, zeta = z[:, :d], z[:, d:2 * d], z[:, 2 * d:3 * d]
        ff = (v_nom[k + 1] - v_nom[k]) / dt
        u = ff[None, :] - kp * (ph - p_nom[k][None, :]) - kv * (vh - v_nom[k][None, :])
        a = u + sw * xi
        p = p + v * dt + half * a
        v = v + dt * a
        am = a + sa * eta
        # prediction: x_hat = A x_hat + B a_meas, P = A P A^T + sigma_a^2 B B^T
        ph = ph + vh * dt + half * am
        vh = vh + dt * am
        q_a = sa * sa
        n00 = P00 + 2.0 * dt * P01 + dt * dt * P11 + q_a * half * half
        n01 = P01 + dt * P11 + q_a * half * dt
        n11 = P11 + q_a * dt * dt
        P00, P01, P11 = n00, n01, n11
        # position fix where the features are good enough
        q = quality(p, mu, sig, amp)
        fix = q >= qmin
        qs = np.where(fix, q, 1.0)
        Rv = sv * sv / qs
        zpos = p + (sv / np.sqrt(qs))[:, None] * zeta
        S = P00 + Rv
        K0 = P00 / S
        K1 = P01 / S
        innov = zpos - ph
        ph = np.where(fix[:, None], ph + K0[:, None] * innov, ph)
        vh = np.where(fix[:, None], vh + K1[:, None] * innov, vh)
        u00 = (1.0 - K0) * P00
        u01 = (1.0 - K0) * P01
        u11 = P11 - K1 * P01
        P00 = np.where(fix, u00, P00)
        P01 = np.where(fix, u01, P01)
        P11 = np.where(fix, u11, P11)
        err = np.sqrt(((p - ph) ** 2).sum(axis=1))
        max_err = np.maximum(max_err, err)
        hit = hit | inside(p)
    return MCResult(max_err=max_err, collided=hit, final_err=p - ph, steps=K, gain=(kp, kv))
