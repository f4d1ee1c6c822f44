"""The search entry point that allocates nothing (mpap_search_noalloc, a
fixed per-device scratch array) against mpap_search + mpap_goal_front on the
same roadmaps: two calls in a row, the second on a smaller roadmap (the
scratch keeps the first call's contents), then a third repeating the first.
Goal fronts are compared bit for bit, goal nodes exactly (both run the same
deterministic kernels in the same launch shape)."""
import numpy as np
import pytest

from oracle import graph as ograph, search as osearch
from paper_1705_02408_amd import synth

pytestmark = pytest.mark.gpu
mpap = pytest.importorskip("paper_1705_02408_amd.mpap")


def bits(a):
    return np.ascontiguousarray(a, dtype=np.float32).view(np.uint32)


def load(env):
    g = ograph.build_graph(env)
    dg = mpap.mpap_graph_from_csr(g["row_ptr"], g["col"], g["cost"], g["drift"], g["reset"],
                                  g["goal"])
    return g, dg


def check_against_search(env, dg, g=None):
    ref = mpap.mpap_search(dg, env.beta, env.n_obj, env.radius, env.lam)
    want = ref.goal_front()
    ref.close()
    got = mpap.mpap_search_noalloc(dg, env.beta, env.n_obj, env.radius, env.lam)
    print(f"{env.name}: goal front {got.vecs.shape[0]} labels", flush=True)
    assert got.vecs.shape == want.vecs.shape
    assert np.array_equal(bits(got.vecs), bits(want.vecs))
    assert np.array_equal(got.goal_node, want.goal_node)
    if g is not None:  # and the oracle's goal front
        res = osearch.search(g, env.beta, env.n_obj)
        of, _, _ = osearch.goal_front(res, g["goal"])
        assert np.array_equal(bits(got.vecs), bits(of))
    return got


def test_noalloc_matches_search_twice_second_smaller():
    env1 = synth.plain2d(0)            # 2,001 nodes, two objectives
    env2 = synth.plain3d(3, n=1500)    # 1,501 nodes, three objectives
    g1, d1 = load(env1)
    g2, d2 = load(env2)
    f1 = check_against_search(env1, d1, g1)
    f2 = check_against_search(env2, d2, g2)
    assert f1.vecs.shape[0] > 0 and f2.vecs.shape[0] > 0
    f3 = check_against_search(env1, d1)   # the first roadmap again, after the smaller one
    assert np.array_equal(bits(f3.vecs), bits(f1.vecs))
    d1.close()
    d2.close()


def test_noalloc_early_stop_matches_search():
    env = synth.plain2d(1, n=600)
    g, dg = load(env)
    for lam in (0.5, 2.0):
        ref = mpap.mpap_search(dg, env.beta, env.n_obj, env.radius, lam, early_stop=1)
        want = ref.goal_front()
        ref.close()
        got = mpap.mpap_search_noalloc(dg, env.beta, env.n_obj, env.radius, lam, early_stop=1)
        assert np.array_equal(bits(got.vecs), bits(want.vecs)), lam
        assert np.array_equal(got.goal_node, want.goal_node), lam
    dg.close()


def test_noalloc_capacity_and_size_limits():
    env = synth.plain2d(2, n=800)
    g, dg = load(env)
    full = mpap.mpap_search_noalloc(dg, env.beta, env.n_obj, env.radius, env.lam)
    k = full.vecs.shape[0]
    assert k >= 2
    with pytest.raises(mpap.MpapError) as ei:
        mpap.mpap_search_noalloc(dg, env.beta, env.n_obj, env.radius, env.lam, capacity=k - 1)
    assert ei.value.status == mpap.MPAP_ERR_CAPACITY
    dg.close()
    # a roadmap whose per-node state alone exceeds the scratch is refused up
    # front (a path of 1,000,000 nodes)
    n = 1_000_000
    row_ptr = np.arange(n + 1, dtype=np.int32)
    row_ptr[-1] = n - 1
    col = np.arange(1, n, dtype=np.int32)
    big = mpap.mpap_graph_from_csr(row_ptr, col, np.ones(n - 1, np.float32),
                                   np.zeros(n - 1, np.float32), np.zeros(n, np.uint8),
                                   np.eye(1, n, n - 1, dtype=np.uint8).ravel())
    with pytest.raises(mpap.MpapError) as ei:
        mpap.mpap_search_noalloc(big, 1.0, 2, 1.0, 0.5)
    assert ei.value.status == mpap.MPAP_ERR_INVAL
    assert "too large" in str(ei.value)
    big.close()
