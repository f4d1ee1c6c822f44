"""Learned per-edge drift surrogate on the matrix cores: forward and gradients
against the float64 reference on the same bfloat16 tensors, inputs against the
oracle's features, training, scoring, and the analytic re-walk that judges a
search on the surrogate's drift (with fallback to the analytic search)."""
import numpy as np
import pytest

from oracle import graph as ograph, mlp, search as osearch
from paper_1705_02408_amd import synth

pytestmark = pytest.mark.gpu
mpap = pytest.importorskip("paper_1705_02408_amd.mpap")


def bits(a):
    return np.ascontiguousarray(a, dtype=np.float32).view(np.uint32)


def rel_fro(a, b):
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-30))


def random_inputs(seed, n):
    rng = np.random.default_rng(seed)
    X = rng.uniform(0, 1, (n, 16)).astype(np.float32)
    Xb = mlp.bf16_round(X)
    return Xb, mlp.bf16_bits(Xb), rng.uniform(0, 1, n).astype(np.float32)


def trained_like_params(seed):
    rng = np.random.default_rng(seed)
    p = mlp.init_params(seed)
    p["b1"] = rng.normal(0, 0.2, 64).astype(np.float32)
    p["b2"] = rng.normal(0, 0.2, 64).astype(np.float32)
    p["b3"] = np.array([0.1], np.float32)
    return p


@pytest.mark.parametrize("n", [32, 1000, 4096])
def test_forward_matches_reference(n):
    p = trained_like_params(0)
    Xf, Xbits, _ = random_inputs(1, n)
    s = mpap.Surrogate()
    s.set_params(mlp.flat(p))
    y = s.forward(Xbits)
    ref, _ = mlp.forward(p, Xf)
    assert rel_fro(y, ref) <= 1e-3
    s.close()


@pytest.mark.parametrize("n", [64, 1024, 4096])
def test_gradient_matches_reference(n):
    p = trained_like_params(2)
    Xf, Xbits, t = random_inputs(3, n)
    s = mpap.Surrogate()
    s.set_params(mlp.flat(p))
    g, y = s.gradient(Xbits, t)
    yref, gref = mlp.backward(p, Xf, t)
    assert rel_fro(y, yref) <= 1e-3
    gd = mlp.unflat(g)
    for k in ("W1", "b1", "W2", "b2", "w3", "b3"):
        assert rel_fro(gd[k], gref[k]) <= 1e-3, (k, rel_fro(gd[k], gref[k]))
    s.close()


@pytest.fixture(scope="module")
def road3d():
    env = synth.plain3d(0, n=3000)
    dg = mpap.mpap_build_graph(env)
    yield env, dg
    dg.close()


def test_edge_features_match_oracle(road3d):
    env, dg = road3d
    g = dg.export()
    X = mpap.mpap_edge_features(dg)
    ref = ograph.edge_features(env.pos, g["row_ptr"], g["col"], g["cost"], env.blob_mu,
                               env.blob_sigma, env.blob_amp)
    refb = mlp.bf16_bits(mlp.bf16_round(ref))
    # positions and length: the same float32 values, rounded the same way
    assert np.array_equal(X[:, :7], refb[:, :7])
    # q: float32 device exp vs float64 -> at most one bfloat16 step apart
    dq = np.abs(X[:, 7:].astype(np.int32) - refb[:, 7:].astype(np.int32))
    assert dq.max() <= 1


def test_training_learns_the_analytic_drift(road3d):
    env, dg = road3d
    e = dg.info()["e"]
    rng = np.random.default_rng(4)
    edges = rng.permutation(e)[: (e // 2048) * 2048]
    s = mpap.Surrogate(seed=5)
    loss = s.train(dg, edges, epochs=12, batch=1024, lr=2e-3)
    assert np.all(np.isfinite(loss))
    assert loss[-1] < 0.2 * loss[0]
    s.score(dg)
    ana = mpap.mpap_graph_drift(dg, 0)
    sur = mpap.mpap_graph_drift(dg, 1)
    rel = np.abs(sur - ana) / np.maximum(ana, 1e-3)
    assert np.median(rel) < 0.05
    s.close()


def test_surrogate_search_is_judged_and_falls_back(road3d):
    env, dg = road3d
    e = dg.info()["e"]
    edges = np.random.default_rng(6).permutation(e)[: (e // 2048) * 2048]
    s = mpap.Surrogate(seed=7)
    s.train(dg, edges, epochs=12, batch=1024, lr=2e-3)
    s.score(dg)
    res = mpap.mpap_search(dg, env.beta, 3, env.radius, env.lam, heuristic=1)
    fr = res.goal_front()
    rs = mpap.mpap_rescore_front(res, 0)
    # the re-walk reproduces the cost exactly (cost does not use the surrogate)
    assert np.array_equal(bits(rs["cost"]), bits(fr.vecs[:, 0]))
    ok = mpap.surrogate_front_ok(res, 0, env.beta)
    res.close()
    # corrupted weights: the judge must reject the surrogate's front
    bad = mlp.flat(mlp.init_params(1))
    bad[mlp.flat(mlp.init_params(1)).shape[0] - 1] = -5.0  # output bias: drift clamps to 0
    s.set_params(bad)
    s.score(dg)
    res2 = mpap.mpap_search(dg, env.beta, 3, env.radius, env.lam, heuristic=1)
    assert not mpap.surrogate_front_ok(res2, 0, env.beta)
    res2.close()
    # the fallback is the analytic search, exact against the oracle
    g = dg.export()
    ref = osearch.search(g, env.beta, 3)
    rv, _, _ = osearch.goal_front(ref, g["goal"])
    res3 = mpap.mpap_search(dg, env.beta, 3, env.radius, env.lam, heuristic=0)
    assert np.array_equal(bits(res3.goal_front().vecs), bits(rv))
    res3.close()
    s.close()
    assert ok in (True, False)


def test_surrogate_gain_on_fine_drift_integration():
    """The analytic drift integrates q at every collision sub-step; the
    surrogate needs 9 q values per edge whatever the edge length.  With a fine
    sub-step (0.001) the surrogate scores a roadmap several times faster."""
    env = synth.plain3d(1, n=3000)
    env.check_step = 0.001
    dg = mpap.mpap_build_graph(env)
    s = mpap.Surrogate(seed=9)
    for _ in range(2):
        t_ana = mpap.mpap_analytic_drift(dg)
        t_sur = s.score(dg)
    assert t_ana > 2.0 * t_sur, (t_ana, t_sur)
    s.close()
    dg.close()
