"""Monte Carlo verification on the GPU (mpap_mc_verify) against the oracle
(oracle/mcverify.py) on the same plan -- the witness of P_soln in the
oracle's own search of the oracle's roadmap, which the library builds bit for
bit -- and the same counter-based normals: every flight's largest
localisation error agrees to 1e-9 relative (float64 on both sides; the
transcendental functions of the two math libraries may differ in the last
bit), every collision flag and the success counts agree.  2D, 3D and the 6D
steering cubics.  Then what the estimate says about the front: on the 3D
workload the plans of lower drift fly with smaller localisation errors.
"""
import numpy as np
import pytest

from oracle import graph as ograph, graph6d as og6, mcverify as mc, search as osearch
from paper_1705_02408_amd import synth

pytestmark = pytest.mark.gpu
mpap = pytest.importorskip("paper_1705_02408_amd.mpap")


def oracle_plan(env, g, k=0):
    """Node path of goal-front entry k of the oracle's search."""
    ref = osearch.search(g, env.beta, env.n_obj)
    vecs, gnode, lab = osearch.goal_front(ref, g["goal"])
    assert vecs.shape[0] > k
    return ref.path(int(lab[k])), vecs


def compare(env, g, path, rollouts=2048, **kw):
    mp = mc.MCParams(rollouts=rollouts, **kw)
    if env.dim == 6:
        p, v, a = mc.nominal_cubic(env.pos[path], env.vel[path], np.float32(env.horizon),
                                   mp.f64("dt"))
    else:
        p, v, a = mc.nominal_segments(env.pos[path], mp.f64("speed"), mp.f64("dt"))
    want = mc.rollouts(p, v, a, mp, env.blob_mu, env.blob_sigma, env.blob_amp, env.box_lo,
                       env.box_hi)
    dg = mpap.mpap_build_graph(env)
    st, got, col = mpap.mpap_mc_verify(dg, path, **{f: getattr(mp, f) for f in (
        "rollouts", "dt", "speed", "sigma_w", "sigma_a", "sigma_v", "q_min", "sigma0",
        "err_bound", "q_p", "q_v", "r_u", "seed")})
    dg.close()
    assert st["steps"] == want.steps
    assert st["gain_p"] == pytest.approx(want.gain[0], rel=1e-12)
    assert st["gain_v"] == pytest.approx(want.gain[1], rel=1e-12)
    rel = np.abs(got - want.max_err) / np.maximum(want.max_err, 1e-300)
    assert rel.max() <= 1e-9, (rel.max(), int(rel.argmax()))
    assert np.array_equal(col, want.collided)
    bound = mp.f64("err_bound")
    near = np.abs(want.max_err - bound) <= 1e-9 * bound
    within = want.max_err <= bound
    assert abs(st["within_bound"] - int(within.sum())) <= int(near.sum())
    assert st["collision_free"] == int((~want.collided).sum())
    print(f"{env.name}: {len(path)} nodes, {want.steps} steps, within bound "
          f"{st['within_bound']}/{rollouts}, collision free {st['collision_free']}, "
          f"mean max error {st['mean_max_err']:.4g}, {st['gpu_ms']:.2f} ms", flush=True)
    return st


def test_mc_2d_matches_the_oracle():
    env = synth.plain2d(0)
    g = ograph.build_graph(env)
    path, _ = oracle_plan(env, g)
    compare(env, g, path)


def test_mc_3d_matches_the_oracle():
    env = synth.plain3d(3, n=1500)
    g = ograph.build_graph(env)
    path, vecs = oracle_plan(env, g)
    compare(env, g, path, seed=11, sigma_a=0.5)
    # the goal-front entry of least drift too
    k = int(np.argmin(vecs[:, 1]))
    path2, _ = oracle_plan(env, g, k)
    compare(env, g, path2, seed=12)


def test_mc_6d_matches_the_oracle():
    env = synth.plain6d(0, n=1200)
    g = og6.build_graph6d(env)
    ref = osearch.search(g, env.beta, env.n_obj)
    vecs, gnode, lab = osearch.goal_front(ref, g["goal"])
    assert vecs.shape[0] > 0
    compare(env, g, ref.path(int(lab[0])), rollouts=1024, dt=0.005)


def test_mc_noise_free_and_errors():
    env = synth.plain2d(0, n=500)
    dg = mpap.mpap_build_graph(env)
    res = mpap.mpap_search(dg, env.beta, env.n_obj, env.radius, env.lam)
    fr = res.goal_front()
    path = res.path(int(fr.label[0]))
    st, me, col = mpap.mpap_mc_verify(dg, path, rollouts=300, sigma_w=0.0, sigma_a=0.0,
                                      sigma0=0.0)
    mp = mc.MCParams(rollouts=4, sigma_w=0.0, sigma_a=0.0, sigma0=0.0)
    p, v, a = mc.nominal_segments(env.pos[path], mp.f64("speed"), mp.f64("dt"))
    want = mc.rollouts(p, v, a, mp, env.blob_mu, env.blob_sigma, env.blob_amp, env.box_lo,
                       env.box_hi)
    print("noise-free:", path, st, int(col.sum()), want.collided, flush=True)
    assert not want.collided.any()
    assert np.all(me == 0.0) and st["within_bound"] == 300 and st["collision_free"] == 300
    with pytest.raises(mpap.MpapError):
        mpap.mpap_mc_verify(dg, path[:1])
    with pytest.raises(mpap.MpapError):
        mpap.mpap_mc_verify(dg, path, dt=0.0)
    res.close()
    dg.close()


def test_lower_drift_plans_fly_with_smaller_errors():
    """The perception heuristic against the estimate: over the goal front of
    the 20,000-sample 3D workload, the mean largest localisation error of a
    plan rises with its largest drift (rank correlation), and the front's
    plan of least drift keeps the error bound more often than its cheapest
    plan."""
    import scipy.stats
    env = synth.plain3d(0)
    dg = mpap.mpap_build_graph(env)
    res = mpap.mpap_search(dg, env.beta, 3, env.radius, env.lam)
    fr = res.goal_front()
    ks = np.unique(np.linspace(0, fr.vecs.shape[0] - 1, 24).astype(int))
    errs, within = [], []
    for k in ks:
        st, _, _ = mpap.mpap_mc_verify(dg, res.path(int(fr.label[k])), with_samples=False,
                                       rollouts=8192, seed=100 + int(k))
        errs.append(st["mean_max_err"])
        within.append(st["within_bound"] / st["rollouts"])
        print(f"plan {k}: (c, d, m) {fr.vecs[k]}, {st['steps']} steps, mean max error "
              f"{st['mean_max_err']:.4f}, within bound {within[-1]:.3f}, collision free "
              f"{st['collision_free'] / st['rollouts']:.3f}, {st['gpu_ms']:.1f} ms", flush=True)
    rho = scipy.stats.spearmanr(fr.vecs[ks, 2], errs).correlation
    lo_d = int(np.argmin(fr.vecs[ks, 2]))
    print(f"front of {fr.vecs.shape[0]}: {len(ks)} plans, Spearman(max drift, mean MC error) "
          f"{rho:.3f}; within bound at least cost {within[0]:.3f}, at least max drift "
          f"{within[lo_d]:.3f}", flush=True)
    assert rho > 0.5
    assert within[lo_d] > within[0]
    res.close()
    dg.close()
