"""Batched search: many independent queries (the disjoint union of their
roadmaps) in one persistent launch must give, per query, exactly the fronts
of the oracle and of a single-query search."""
import numpy as np
import pytest

from oracle import graph as ograph, search as osearch
from paper_1705_02408_amd import synth

pytestmark = pytest.mark.gpu
mpap = pytest.importorskip("paper_1705_02408_amd.mpap")


def bits(a):
    return np.ascontiguousarray(a, dtype=np.float32).view(np.uint32)


@pytest.fixture(scope="module")
def small_batch():
    envs = [synth.batch_query(7, q, nmin=300, nmax=2500) for q in range(10)]
    graphs = [ograph.build_graph(e) for e in envs]
    keep = [i for i, g in enumerate(graphs) if g["goal"].sum() > 0]
    envs = [envs[i] for i in keep]
    graphs = [graphs[i] for i in keep]
    parts = [mpap.mpap_graph_from_csr(g["row_ptr"], g["col"], g["cost"], g["drift"], g["reset"],
                                      g["goal"]) for g in graphs]
    union = mpap.mpap_graph_concat(parts)
    yield envs, graphs, parts, union
    union.close()
    for p in parts:
        p.close()


def params_of(envs):
    return [mpap.search_params(e.beta, e.n_obj, e.radius, e.lam) for e in envs]


def test_concat_partition(small_batch):
    envs, graphs, parts, union = small_batch
    off = mpap.mpap_graph_queries(union)
    sizes = [g["row_ptr"].shape[0] - 1 for g in graphs]
    assert off.tolist() == np.concatenate([[0], np.cumsum(sizes)]).tolist()
    assert union.info()["e"] == sum(int(g["row_ptr"][-1]) for g in graphs)


def test_batch_matches_oracle_per_query(small_batch):
    envs, graphs, parts, union = small_batch
    res = mpap.mpap_search_batch(union, params_of(envs))
    off = mpap.mpap_graph_queries(union)
    for q, (e, g) in enumerate(zip(envs, graphs)):
        ref = osearch.search(g, e.beta, e.n_obj)
        rv, _, _ = osearch.goal_front(ref, g["goal"])
        fr = res.goal_front(q)
        assert np.array_equal(bits(fr.vecs), bits(rv)), q
        assert all(g["goal"][v] for v in fr.goal_node)
        # every node front of the query, in the union's numbering
        for v in range(0, g["row_ptr"].shape[0] - 1, 3):
            a = res.node_front(int(off[q]) + v)
            a = a[np.lexsort((a[:, 2], a[:, 1], a[:, 0]))] if a.shape[0] else a
            assert np.array_equal(bits(a), bits(ref.node_front(v))), (q, v)
        # witnesses re-walk inside the query
        for k in range(min(3, fr.vecs.shape[0])):
            path = [x - int(off[q]) for x in res.path(int(fr.label[k]))]
            c, d, m, ok = osearch.rewalk(g, path, e.beta, e.n_obj)
            assert ok and bits([c, d, m]).tolist() == bits(fr.vecs[k]).tolist()
        info = res.query_info(q)
        assert info["latency_ms"] > 0 and info["last_wave"] >= 0
    res.close()


def test_batch_matches_single_searches(small_batch):
    envs, graphs, parts, union = small_batch
    res = mpap.mpap_search_batch(union, params_of(envs))
    for q, (e, p) in enumerate(zip(envs, parts)):
        one = mpap.mpap_search(p, e.beta, e.n_obj, e.radius, e.lam)
        assert np.array_equal(bits(one.goal_front().vecs), bits(res.goal_front(q).vecs))
        one.close()
    res.close()


def test_batch_one_param_set_for_all(small_batch):
    envs, graphs, parts, union = small_batch
    e = envs[0]
    res = mpap.mpap_search_batch(union, mpap.search_params(0.3, 2, e.radius, 0.5))
    for q, p in enumerate(parts):
        one = mpap.mpap_search(p, 0.3, 2, e.radius, 0.5)
        assert np.array_equal(bits(one.goal_front().vecs), bits(res.goal_front(q).vecs))
        one.close()
    res.close()


def test_near_scan_setting_does_not_change_results(small_batch):
    envs, graphs, parts, union = small_batch
    outs = []
    for ns in (1, 4, 64):
        res = mpap.mpap_search_batch(union, [mpap.search_params(e.beta, e.n_obj, e.radius,
                                                                e.lam, near_scan=ns)
                                             for e in envs])
        outs.append([bits(res.goal_front(q).vecs).tobytes() for q in range(len(envs))])
        res.close()
    assert outs[0] == outs[1] == outs[2]


def test_rewalk_of_all_queries(small_batch):
    """The re-walk of every goal front in one launch equals the per-query
    re-walks, and on an analytic search reproduces the fronts bit for bit (the
    same float32 fold along the same edges)."""
    envs, graphs, parts, union = small_batch
    res = mpap.mpap_search_batch(union, params_of(envs))
    allq = mpap.mpap_rescore_front(res, -1)
    o = 0
    for q in range(len(envs)):
        fr = res.goal_front(q)
        one = mpap.mpap_rescore_front(res, q)
        k = fr.vecs.shape[0]
        for key in ("cost", "drift", "maxdrift", "feasible"):
            assert np.array_equal(allq[key][o:o + k], one[key]), (q, key)
        assert np.array_equal(bits(one["cost"]), bits(fr.vecs[:, 0])), q
        assert np.array_equal(bits(one["drift"]), bits(fr.vecs[:, 1])), q
        assert np.array_equal(bits(one["maxdrift"]), bits(fr.vecs[:, 2])), q
        assert one["feasible"].all(), q
        o += k
    assert o == allq["cost"].shape[0]
    res.close()


@pytest.mark.parametrize("halves", [8192, -1])
def test_mixed_objective_counts_in_one_launch(small_batch, halves):
    """Two- and three-objective queries in one launch run the builds that
    read the objective count per query: merges by halves forced
    (`k_search_halves`) or whole workgroups only (`k_search`), single-wave
    merges off.  Every goal front against the oracle; a group factor of 2
    (the fronts do not depend on it) gives iterations with enough targets for
    the halves."""
    envs, graphs, parts, union = small_batch
    nobj = [3 if e.dim == 3 else 2 for e in envs]
    assert 2 in nobj and 3 in nobj
    ps = [mpap.search_params(e.beta, k, e.radius, 2.0, wave_min_targets=-1, merge_halves=halves)
          for e, k in zip(envs, nobj)]
    res = mpap.mpap_search_batch(union, ps)
    st = res.stats()
    print({k: st[k] for k in ("gpu_ms", "wave_build", "build_objectives", "half_front_cap",
                              "half_merges", "merges")}, flush=True)
    assert st["wave_build"] == 0 and st["build_objectives"] == 0
    if halves > 0:
        assert st["half_front_cap"] > 0 and st["half_merges"] > 0
    else:
        assert st["half_front_cap"] == 0 and st["half_merges"] == 0
    for q, (e, g, k) in enumerate(zip(envs, graphs, nobj)):
        ref = osearch.search(g, e.beta, k)
        rv, _, _ = osearch.goal_front(ref, g["goal"])
        assert np.array_equal(bits(res.goal_front(q).vecs), bits(rv)), q
    res.close()
