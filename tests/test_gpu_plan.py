"""Captured batches (mpap_plan_*): the recorded graph of scoring -> search ->
goal fronts must give, on every launch, exactly what the eager batched search
gives (and the oracle's fronts for the plain drift), with the program's own
eager work between launches."""
import numpy as np
import pytest

from oracle import graph as ograph, search as osearch
from paper_1705_02408_amd import synth

pytestmark = pytest.mark.gpu
mpap = pytest.importorskip("paper_1705_02408_amd.mpap")


def bits(a):
    return np.ascontiguousarray(a, dtype=np.float32).view(np.uint32)


def same_result(a, b, nq):
    for q in range(nq):
        fa, fb = a.goal_front(q), b.goal_front(q)
        assert np.array_equal(bits(fa.vecs), bits(fb.vecs)), q
        assert np.array_equal(fa.goal_node, fb.goal_node), q
    sa, sb = a.stats(), b.stats()
    for k in ("waves", "labels_expanded", "front_labels", "relaxations", "max_front"):
        assert sa[k] == sb[k], k


@pytest.fixture(scope="module")
def oracle_batch():
    envs = [synth.batch_query(11, q, nmin=300, nmax=2500) for q in range(8)]
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


def test_plan_matches_oracle_and_eager(oracle_batch):
    envs, graphs, parts, union = oracle_batch
    nq = len(envs)
    params = [mpap.search_params(e.beta, e.n_obj, e.radius, e.lam) for e in envs]
    plan = mpap.Plan(union, params)
    eager = mpap.mpap_search_batch(union, params)
    refs = []
    for e, g in zip(envs, graphs):
        ref = osearch.search(g, e.beta, e.n_obj)
        refs.append(osearch.goal_front(ref, g["goal"])[0])
    other = mpap.mpap_graph_from_csr(graphs[0]["row_ptr"], graphs[0]["col"], graphs[0]["cost"],
                                     graphs[0]["drift"], graphs[0]["reset"], graphs[0]["goal"])
    for launch in range(3):
        res = plan.run()
        same_result(res, eager, nq)
        for q in range(nq):
            assert np.array_equal(bits(res.goal_front(q).vecs), bits(refs[q])), (launch, q)
        # per-node fronts read the plan's workspace until the next launch
        off = mpap.mpap_graph_queries(union)
        v = int(off[nq - 1])
        assert np.array_equal(bits(res.node_front(v)), bits(eager.node_front(v)))
        res.close()
        # the program's own eager work between launches
        r2 = mpap.mpap_search(other, envs[0].beta, envs[0].n_obj, envs[0].radius, envs[0].lam)
        assert np.array_equal(bits(r2.goal_front().vecs), bits(refs[0]))
        r2.close()
    info = plan.info()
    assert info == {"launches": 3, "records": 1, "fallbacks": 0}, info
    eager.close()
    other.close()
    plan.close()


def test_plan_with_surrogate_scoring():
    """Scoring inside the graph gives the same drift as eager scoring, so the
    fronts equal those of score + concat + batched search; a model changed
    between launches is picked up by the next launch."""
    envs, parts = [], []
    q = 0
    while len(parts) < 6:
        e = synth.batch_query(5, q, nmin=500, nmax=3000)
        q += 1
        try:
            parts.append(mpap.mpap_build_graph(e))
            envs.append(e)
        except mpap.MpapError as ex:
            if ex.status != mpap.MPAP_ERR_NOGOAL:
                raise
    models = {}
    for d in (2, 3):
        models[d] = mpap.Surrogate(seed=20 + d)
        same_dim = [p for p, e in zip(parts, envs) if e.dim == d]
        if same_dim:
            ne = same_dim[0].info()["e"]
            edges = np.arange((ne // 256) * 256, dtype=np.int64)
            models[d].train(same_dim[0], edges, epochs=2, batch=256, lr=2e-3)
    ms = [models[e.dim] for e in envs]
    for p, m in zip(parts, ms):
        m.score(p)
    union = mpap.mpap_graph_concat(parts)
    params = [mpap.search_params(e.beta, e.n_obj, e.radius, e.lam, heuristic=1) for e in envs]
    eager = mpap.mpap_search_batch(union, params)
    plan = mpap.Plan(union, params, parts=parts, models=ms)
    for _ in range(2):
        res = plan.run()
        same_result(res, eager, len(envs))
        res.close()
    eager.close()
    # change one model: the next launch scores with the new weights
    m0 = ms[0]
    w = m0.get_params()
    w[-1] += 0.05  # output bias: every predicted drift grows
    m0.set_params(w)
    for p, m in zip(parts, ms):
        m.score(p)
    union2 = mpap.mpap_graph_concat(parts)
    eager2 = mpap.mpap_search_batch(union2, params)
    res = plan.run()
    same_result(res, eager2, len(envs))
    res.close()
    eager2.close()
    union2.close()
    plan.close()
    union.close()
    for p in parts:
        p.close()
    for m in models.values():
        m.close()
