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
    """Gradients of the matrix-core kernels against the exact float64
    gradients of the same bfloat16 model, entry by entry, within the bound of
    the kernels' own roundings: the two output gradients rounded to bfloat16
    (relative 2^-9 each), one bfloat16 step of h1 where the float32 and the
    float64 first layer round differently (2 * 2^-9), and float32 sums of n
    terms (n * 2^-24), all relative to the entry's absolute-term sum."""
    p = trained_like_params(2)
    Xf, Xbits, t = random_inputs(3, n)
    s = mpap.Surrogate()
    s.set_params(mlp.flat(p))
    g, y = s.gradient(Xbits, t)
    yref, gref = mlp.backward(p, Xf, t)
    assert rel_fro(y, yref) <= 1e-3
    absg = mlp.gradient_abs_terms(p, Xf, t)
    u = 2.0 ** -9
    tol = 4 * u + n * 2.0 ** -24
    gd = mlp.unflat(g)
    for k in ("W1", "b1", "W2", "b2", "w3", "b3"):
        err = np.abs(gd[k].astype(np.float64) - gref[k])
        bound = tol * absg[k] + 1e-30
        assert np.all(err <= bound), (k, float((err / bound).max()))
        # and the whole block close in the Frobenius sense
        assert rel_fro(gd[k], gref[k]) <= 4 * u, (k, rel_fro(gd[k], gref[k]))
    s.close()


@pytest.fixture(scope="module")
def road3d():
    env = synth.plain3d(0, n=3000)
    dg = mpap.mpap_build_graph(env)
    yield env, dg
    dg.close()


def test_edge_features_match_oracle(road3d):
    env, dg = road3d
    g = ograph.build_graph(env)
    got = dg.export()
    assert np.array_equal(got["col"], g["col"]) and np.array_equal(bits(got["cost"]), bits(g["cost"]))
    X, base = mpap.mpap_edge_features(dg, with_base=True)
    ref, ref_base = ograph.edge_features(env.pos, g["row_ptr"], g["col"], g["cost"],
                                         env.blob_mu, env.blob_sigma, env.blob_amp)
    refb = mlp.bf16_bits(mlp.bf16_round(ref))
    # positions and length: the same float32 values, rounded the same way
    assert np.array_equal(X[:, :7], refb[:, :7])
    # 1 - q: float32 device exp vs float64, so at most one bfloat16 step apart
    # (plus the float32 error of q itself where 1 - q is tiny)
    xv = (X[:, 7:].astype(np.uint32) << 16).view(np.float32)
    rv = ref[:, 7:]
    assert np.all(np.abs(xv - rv) <= 2.0 ** -8 * np.abs(rv) + 2e-6)
    # the float32 8-point base against the float64 one
    assert np.all(np.abs(base - ref_base) <= 1e-6 + 1e-5 * ref_base)


def test_training_learns_the_analytic_drift(road3d):
    env, dg = road3d
    e = dg.info()["e"]
    rng = np.random.default_rng(4)
    edges = rng.permutation(e)[: (e // 2048) * 2048]
    s = mpap.Surrogate(seed=5)
    loss = s.train(dg, edges, epochs=12, batch=1024, lr=2e-3)
    assert np.all(np.isfinite(loss))
    # the training target is 256 (drift/length - 8-point base); the untrained
    # network (zero output layer) has the loss of the base alone
    ana = mpap.mpap_graph_drift(dg, 0)
    _, base = mpap.mpap_edge_features(dg, with_base=True)
    g = dg.export()
    t = 256.0 * (ana / g["cost"] - base).astype(np.float64)[edges]
    loss_base = float(np.mean(t * t))
    print(f"loss of the base alone {loss_base:.3g}; after each epoch {loss}")
    assert loss[-1] < 0.5 * loss_base
    s.score(dg)
    sur = mpap.mpap_graph_drift(dg, 1)
    rel = np.abs(sur - ana) / np.maximum(ana, 1e-3)
    assert np.median(rel) < 0.01
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
    # the trained network passes the judge (1e-2 relative drift after the
    # analytic re-walk, bound kept)
    assert not res.judge(1e-2, fallback=False)[0]
    res.close()
    # corrupted weights: the judge must reject the surrogate's front, and the
    # library's fallback answers with the analytic search, exact against the
    # oracle on the oracle's own roadmap (the library's roadmap equals it)
    bad = mlp.flat(mlp.init_params(1))
    bad[mlp.flat(mlp.init_params(1)).shape[0] - 1] = -500.0  # output bias: drift clamps to 0
    s.set_params(bad)
    s.score(dg)
    res2 = mpap.mpap_search(dg, env.beta, 3, env.radius, env.lam, heuristic=1)
    assert res2.judge(1e-2, fallback=True)[0]
    g = ograph.build_graph(env)
    ref = osearch.search(g, env.beta, 3)
    rv, _, _ = osearch.goal_front(ref, g["goal"])
    assert np.array_equal(bits(res2.goal_front().vecs), bits(rv))
    assert res2.stats()["judged_failed"] == 1
    res2.close()
    s.close()


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


def test_network_improves_on_the_eight_point_base(road3d):
    """What the trained network adds: on held-out edges its prediction
    (base + network) is closer to the analytic drift than the 8-point base
    alone (the estimate the network corrects), in the median and in the root
    mean square.  Trained on only 65,536 edges of this 3,000-sample roadmap
    its p99 is worse than the base's (0.059 against 0.039); the tail at the
    training size of the batched workload is asserted separately below."""
    env, dg = road3d
    e = dg.info()["e"]
    perm = np.random.default_rng(8).permutation(e)
    n_tr = (int(0.7 * e) // 1024) * 1024
    train, held = perm[:n_tr], perm[n_tr:]
    s = mpap.Surrogate(seed=3)
    s.train(dg, train, epochs=16, batch=1024, lr=2e-3)
    s.score(dg)
    ana = mpap.mpap_graph_drift(dg, 0).astype(np.float64)
    sur = mpap.mpap_graph_drift(dg, 1).astype(np.float64)
    _, base = mpap.mpap_edge_features(dg, with_base=True)
    g = dg.export()
    only_base = g["cost"].astype(np.float64) * np.clip(base.astype(np.float64), 0.0, 1.0)
    floor = 1e-3 * env.beta
    err_net = np.abs(sur - ana)[held] / np.maximum(ana[held], floor)
    err_base = np.abs(only_base - ana)[held] / np.maximum(ana[held], floor)
    print(f"held-out median rel err: base {np.median(err_base):.3g}, "
          f"base + network {np.median(err_net):.3g}; p99 {np.percentile(err_base, 99):.3g} "
          f"-> {np.percentile(err_net, 99):.3g}")
    rms = lambda x: float(np.sqrt(np.mean(x * x)))  # noqa: E731
    rms_net = rms((sur - ana)[held]) / rms(ana[held])
    rms_base = rms((only_base - ana)[held]) / rms(ana[held])
    print(f"held-out relative rms error: base {rms_base:.3g}, base + network {rms_net:.3g}")
    # the network lowers both the typical and the root-mean-square error of
    # the 8-point estimate
    assert np.median(err_net) < 0.5 * np.median(err_base)
    assert rms_net < 0.7 * rms_base
    s.close()


@pytest.mark.parametrize("dim", [2, 3])
def test_network_tail_at_training_scale(dim):
    """The held-out tail of the relative drift error at the size the networks
    are trained at for the batched workload (2^20 edges, 8 epochs, the
    training roadmaps of that workload): the network's p99 stays below the
    1e-2 gate of the front judge and within 1.25x of the 8-point base's p99
    (measured: 2D 0.63x, 3D 1.02x).  The tail edges are those whose quality
    peaks lie between the nine sample points the features carry; weighting
    the training towards small-drift edges did not lower it."""
    if dim == 2:
        env = synth.make_env(10_000, 2, 50000, 20, 30, 20.0, 0.3, 2, blob_amp=0.3)
    else:
        env = synth.make_env(20_000, 3, 30000, 100, 80, 40.0, 0.25, 2, blob_amp=0.4)
    dg = mpap.mpap_build_graph(env)
    e = dg.info()["e"]
    n_train = min(1 << 20, (e // 4096) * 4096)
    perm = np.random.default_rng(dim).permutation(e)
    held = perm[n_train:]
    assert held.size > 50000
    s = mpap.Surrogate(seed=dim)
    s.train(dg, perm[:n_train], epochs=8, batch=4096, lr=2e-3)
    s.score(dg)
    ana = mpap.mpap_graph_drift(dg, 0).astype(np.float64)
    sur = mpap.mpap_graph_drift(dg, 1).astype(np.float64)
    _, base = mpap.mpap_edge_features(dg, with_base=True)
    only_base = dg.export()["cost"].astype(np.float64) * np.clip(base.astype(np.float64), 0, 1)
    floor = 1e-3 * env.beta
    err_net = np.abs(sur - ana)[held] / np.maximum(ana[held], floor)
    err_base = np.abs(only_base - ana)[held] / np.maximum(ana[held], floor)
    p_net, p_base = np.percentile(err_net, 99), np.percentile(err_base, 99)
    print(f"{dim}D held-out p99: base {p_base:.3g}, base + network {p_net:.3g} "
          f"(ratio {p_net / p_base:.2f}); p50 {np.median(err_base):.3g} -> "
          f"{np.median(err_net):.3g}", flush=True)
    assert p_net < 1e-2
    assert p_net <= 1.25 * p_base
    assert np.median(err_net) < np.median(err_base)
    s.close()
    dg.close()
