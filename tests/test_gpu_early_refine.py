"""Bound refinement from one three-objective search, and the paper's early
stop of Alg. 3, on the GPU through the C ABI.

* mpap_refine_front: for every tighter bound beta' the refined front equals,
  bit for bit, the goal front of a search run at beta' (two and three
  objectives) and the oracle's at beta';
* early_stop = 1 (Alg. 3's loop condition): where the loop ends, the goal
  front P_candidates reduces to, and every per-node front at that point equal
  the plain Alg. 3 oracle (oracle/explore.py) for several group cost factors,
  single queries and a batch with mixed modes; the hand-worked instance of
  tests/golden/early_stop_spread.json.
"""
import numpy as np
import pytest

from oracle import explore, graph as ograph, search as osearch
from paper_1705_02408_amd import synth
from tests.graphs import as_vecs, load_golden

pytestmark = pytest.mark.gpu
mpap = pytest.importorskip("paper_1705_02408_amd.mpap")


def bits(a):
    return np.ascontiguousarray(a, dtype=np.float32).view(np.uint32)


def upload(g):
    return mpap.mpap_graph_from_csr(g["row_ptr"], g["col"], g["cost"], g["drift"], g["reset"],
                                    g["goal"])


# ----------------------------------------------------------------- refinement
@pytest.mark.parametrize("which", ["2d", "3d"])
def test_refined_fronts_equal_searches_at_the_tighter_bound(which):
    env = synth.plain2d(0) if which == "2d" else synth.plain3d(3, n=1500)
    g = ograph.build_graph(env)
    dg = upload(g)
    full = mpap.mpap_search(dg, env.beta, 3, env.radius, env.lam)
    fb = float(np.float32(env.beta))
    for frac in (1.0, 0.9, 0.75, 0.6, 0.5, 0.35, 0.2, 0.1, 0.0):
        bp = float(np.float32(fb * frac))
        for n_obj in (2, 3):
            got = full.refine(bp, n_obj)
            one = mpap.mpap_search(dg, bp, n_obj, env.radius, env.lam)
            want = one.goal_front()
            one.close()
            assert np.array_equal(bits(got.vecs), bits(want.vecs)), (which, bp, n_obj)
            assert all(g["goal"][v] for v in got.goal_node)
        if frac in (0.75, 0.35):
            ref = osearch.search(g, bp, 2)
            rv, _, _ = osearch.goal_front(ref, g["goal"])
            assert np.array_equal(bits(full.refine(bp, 2).vecs), bits(rv)), (which, bp)
    # witnesses of a refined front re-walk within the tighter bound
    bp = float(np.float32(fb * 0.5))
    fr = full.refine(bp, 3)
    for k in range(fr.vecs.shape[0]):
        c, d, m, ok = osearch.rewalk(g, full.path(int(fr.label[k])), bp, 3)
        assert ok and bits([c, d, m]).tolist() == bits(fr.vecs[k]).tolist()
    with pytest.raises(mpap.MpapError) as ei:
        full.refine(fb * 1.5, 2)
    assert ei.value.status == mpap.MPAP_ERR_INVAL
    full.close()
    two = mpap.mpap_search(dg, env.beta, 2, env.radius, env.lam)
    with pytest.raises(mpap.MpapError):
        two.refine(fb * 0.5, 2)
    two.close()
    dg.close()


# ----------------------------------------------------------------- early stop
def check_early(g, beta, n_obj, lam, radius, res=None, query=0, off=0):
    ex = explore.explore(g, beta, n_obj, lam, radius, early_stop=True)
    own = res is None
    if own:
        dg = upload(g)
        res = mpap.mpap_search(dg, beta, n_obj, radius, lam, early_stop=1)
    assert res.stop(query) == (ex.groups if ex.stopped else -1), (lam, ex.groups, ex.stopped)
    assert np.array_equal(bits(res.goal_front(query).vecs), bits(ex.goal_front(g["goal"])))
    n = g["row_ptr"].shape[0] - 1
    for v in range(n):
        a = res.node_front(off + v)
        a = a[np.lexsort((a[:, 2], a[:, 1], a[:, 0]))] if a.shape[0] else a.reshape(0, 3)
        assert np.array_equal(bits(a), bits(ex.node_front(v))), (lam, v)
    if own:
        res.close()
        dg.close()
    return ex


def test_early_stop_golden():
    spec, g = load_golden("early_stop_spread.json")
    dg = upload(g)
    for case in spec["cases"]:
        res = mpap.mpap_search(dg, spec["beta"], spec["n_obj"], case["radius"], case["lam"],
                               early_stop=1)
        assert res.stop() == case["groups"]
        assert np.array_equal(bits(res.goal_front().vecs), bits(as_vecs(case["goal_front"])))
        for v, rows in case["node_fronts"].items():
            a = res.node_front(int(v))
            a = a[np.lexsort((a[:, 2], a[:, 1], a[:, 0]))] if a.shape[0] else a.reshape(0, 3)
            assert np.array_equal(bits(a), bits(as_vecs(rows))), (case, v)
        res.close()
        exact = mpap.mpap_search(dg, spec["beta"], spec["n_obj"], case["radius"], case["lam"])
        assert exact.stop() == -1
        assert np.array_equal(bits(exact.goal_front().vecs),
                              bits(as_vecs(spec["exact_goal_front"])))
        exact.close()
    dg.close()


@pytest.mark.parametrize("seed,n_obj,ints", [(0, 2, False), (1, 3, False), (2, 2, True),
                                             (3, 3, True)])
@pytest.mark.parametrize("lam", [0.02, 0.25, 1.0, 4.0])
def test_early_stop_tiny_graphs_match_alg3(seed, n_obj, ints, lam):
    g = synth.tiny_random_graph(seed, n=30, p_reset=0.2, mean_degree=3.0, integer_costs=ints)
    check_early(g, 0.9, n_obj, lam, 1.0)


@pytest.mark.parametrize("lam", [0.25, 0.5, 2.0])
def test_early_stop_small_roadmaps_match_alg3(lam):
    for env in (synth.plain2d(0, n=300), synth.plain3d(3, n=400)):
        g = ograph.build_graph(env)
        ex = check_early(g, env.beta, env.n_obj, lam, env.radius)
        ref = osearch.search(g, env.beta, env.n_obj)
        rv, _, _ = osearch.goal_front(ref, g["goal"])
        got = ex.goal_front(g["goal"])
        if rv.shape[0]:
            assert got.shape[0] and got[0, 0] >= rv[0, 0]


def test_early_stop_per_query_in_a_batch():
    envs = [synth.batch_query(5, q, nmin=200, nmax=600) for q in range(8)]
    graphs = [ograph.build_graph(e) for e in envs]
    keep = [k for k, g in enumerate(graphs) if g["goal"].sum() > 0]
    envs = [envs[k] for k in keep]
    graphs = [graphs[k] for k in keep]
    parts = [upload(g) for g in graphs]
    union = mpap.mpap_graph_concat(parts)
    off = mpap.mpap_graph_queries(union)
    # every other query stops early; the others run to an empty P_open
    ps = [mpap.search_params(e.beta, e.n_obj, e.radius, e.lam, early_stop=k % 2)
          for k, e in enumerate(envs)]
    res = mpap.mpap_search_batch(union, ps)
    for k, (e, g) in enumerate(zip(envs, graphs)):
        if k % 2:
            check_early(g, e.beta, e.n_obj, e.lam, e.radius, res=res, query=k, off=int(off[k]))
        else:
            assert res.stop(k) == -1
            ref = osearch.search(g, e.beta, e.n_obj)
            rv, _, _ = osearch.goal_front(ref, g["goal"])
            assert np.array_equal(bits(res.goal_front(k).vecs), bits(rv)), k
    res.close()
    union.close()
    for p in parts:
        p.close()
