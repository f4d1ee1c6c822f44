"""Online updates (Sec. 3, online implementation) through the C ABI:

* mpap_graph_add_boxes checks the roadmap's edges against newly found boxes
  only; the result is, bit for bit, the roadmap the library and the oracle
  build for the same samples with the boxes in the map;
* mpap_search_update continues an earlier search on the changed roadmap; every
  node front and the goal front equal a fresh search of the changed roadmap
  and the oracle's -- after obstacles are added (2D, 3D with three
  objectives, the 20,000-sample 3D workload), and on small graphs whose edges
  get dearer, cheaper, removed or added and whose relocalisation flags flip.
"""
import numpy as np
import pytest

from oracle import graph as ograph, search as osearch
from paper_1705_02408_amd import synth
from tests.graphs import from_edges, front_digest

pytestmark = pytest.mark.gpu
mpap = pytest.importorskip("paper_1705_02408_amd.mpap")


def bits(a):
    return np.ascontiguousarray(a, dtype=np.float32).view(np.uint32)


def assert_same_graph(got, want, what):
    for k in ("row_ptr", "col", "reset", "goal"):
        assert np.array_equal(got[k], want[k]), (what, k)
    for k in ("cost", "drift"):
        assert np.array_equal(bits(got[k]), bits(want[k])), (what, k)


def assert_same_fronts(a, b, n, what):
    bad = [v for v in range(n) if front_digest(a.node_front(v)) != front_digest(b.node_front(v))]
    assert not bad, (what, len(bad), bad[:8])
    assert np.array_equal(bits(a.goal_front().vecs), bits(b.goal_front().vecs)), what


CASES = [("2d", lambda: synth.plain2d(0), 5), ("3d", lambda: synth.plain3d(3, n=1500), 4)]


@pytest.mark.parametrize("name,make,nbox", CASES)
def test_added_boxes_give_the_rebuilt_roadmap(name, make, nbox):
    env = make()
    lo, hi = synth.discovered_boxes(env, 1, nbox)
    env2 = synth.with_boxes(env, lo, hi)
    g0 = mpap.mpap_build_graph(env)
    g1 = mpap.mpap_graph_add_boxes(g0, lo, hi)
    fresh = mpap.mpap_build_graph(env2)
    got = g1.export()
    assert_same_graph(got, fresh.export(), (name, "library build"))
    assert_same_graph(got, ograph.build_graph(env2), (name, "oracle build"))
    assert g1.info()["e"] < g0.info()["e"]
    for g in (g0, g1, fresh):
        g.close()


@pytest.mark.parametrize("name,make,nbox", CASES)
def test_update_after_obstacles_equals_a_fresh_search(name, make, nbox):
    env = make()
    lo, hi = synth.discovered_boxes(env, 2, nbox)
    env2 = synth.with_boxes(env, lo, hi)
    g0 = mpap.mpap_build_graph(env)
    r0 = mpap.mpap_search(g0, env.beta, env.n_obj, env.radius, env.lam)
    g1 = mpap.mpap_graph_add_boxes(g0, lo, hi)
    upd = mpap.mpap_search_update(r0, g1, env.beta, env.n_obj, env.radius, env.lam)
    fresh = mpap.mpap_search(g1, env.beta, env.n_obj, env.radius, env.lam)
    n = g1.info()["n"]
    assert_same_fronts(upd, fresh, n, name)
    su, sf = upd.stats(), fresh.stats()
    assert su["front_labels"] == sf["front_labels"] and su["relaxations"] == sf["relaxations"]
    print(f"{name}: update expanded {su['labels_expanded']} labels in {su['gpu_ms']:.2f} ms, "
          f"a fresh search {sf['labels_expanded']} in {sf['gpu_ms']:.2f} ms", flush=True)
    # the oracle on its own build of the changed map
    og = ograph.build_graph(env2)
    ref = osearch.search(og, env.beta, env.n_obj)
    rv, _, _ = osearch.goal_front(ref, og["goal"])
    assert np.array_equal(bits(upd.goal_front().vecs), bits(rv))
    bad = [v for v in range(n) if front_digest(upd.node_front(v)) != front_digest(ref.node_front(v))]
    assert not bad, (name, len(bad), bad[:8])
    # witnesses re-walk on the changed map
    fr = upd.goal_front()
    for k in range(min(5, fr.vecs.shape[0])):
        c, d, m, ok = osearch.rewalk(og, upd.path(int(fr.label[k])), env.beta, env.n_obj)
        assert ok and bits([c, d, m]).tolist() == bits(fr.vecs[k]).tolist()
    # a second update on top of the first
    lo2, hi2 = synth.discovered_boxes(env, 3, 2)
    g2 = mpap.mpap_graph_add_boxes(g1, lo2, hi2)
    upd2 = mpap.mpap_search_update(upd, g2, env.beta, env.n_obj, env.radius, env.lam)
    fresh2 = mpap.mpap_search(g2, env.beta, env.n_obj, env.radius, env.lam)
    assert_same_fronts(upd2, fresh2, n, (name, "second update"))
    for r in (upd2, fresh2, upd, fresh, r0):
        r.close()
    for g in (g2, g1, g0):
        g.close()


def changed_copy(g, seed):
    """g with some edges dearer, some cheaper, some drifts changed, some edges
    removed, some added, and some relocalisation flags flipped."""
    rng = np.random.default_rng(seed)
    n = g["row_ptr"].shape[0] - 1
    edges = []
    for u in range(n):
        for e in range(g["row_ptr"][u], g["row_ptr"][u + 1]):
            edges.append([u, int(g["col"][e]), float(g["cost"][e]), float(g["drift"][e])])
    keep = []
    for u, v, c, d in edges:
        x = rng.random()
        if x < 0.08:
            continue                                  # removed
        if x < 0.16:
            c = float(np.float32(c * 1.5))            # dearer
        elif x < 0.24:
            c = float(np.float32(max(c * 0.6, 0.01)))  # cheaper
        elif x < 0.30:
            d = float(np.float32(d * 0.5))            # less drift
        keep.append((u, v, c, d))
    have = {(u, v) for u, v, _, _ in keep}
    for _ in range(n // 3):                           # added
        u, v = (int(t) for t in rng.integers(0, n, 2))
        if u != v and (u, v) not in have:
            have.add((u, v))
            keep.append((u, v, float(np.float32(0.2 + rng.random())),
                         float(np.float32(0.2 * rng.random()))))
    reset = g["reset"].copy()
    flip = rng.integers(1, n, 2)
    reset[flip] ^= 1
    return from_edges(n, keep, reset, g["goal"])


def upload(g):
    return mpap.mpap_graph_from_csr(g["row_ptr"], g["col"], g["cost"], g["drift"], g["reset"],
                                    g["goal"])


@pytest.mark.parametrize("seed,n_obj,ints,lam", [(0, 2, False, 0.5), (1, 3, False, 0.25),
                                                 (2, 2, True, 1.0), (3, 3, True, 2.0),
                                                 (4, 2, False, 0.1), (5, 3, False, 0.5)])
def test_update_after_edge_changes_equals_the_oracle(seed, n_obj, ints, lam):
    g0 = synth.tiny_random_graph(seed, n=40, p_reset=0.2, mean_degree=3.0, integer_costs=ints)
    d0 = upload(g0)
    r0 = mpap.mpap_search(d0, 0.9, n_obj, 1.0, lam)
    cur_r, cur_d = r0, d0
    for step in range(3):
        g1 = changed_copy(g0 if step == 0 else g1, 100 * seed + step)
        d1 = upload(g1)
        upd = mpap.mpap_search_update(cur_r, d1, 0.9, n_obj, 1.0, lam)
        ref = osearch.search(g1, 0.9, n_obj)
        for v in range(40):
            assert front_digest(upd.node_front(v)) == front_digest(ref.node_front(v)), (step, v)
        rv, _, _ = osearch.goal_front(ref, g1["goal"])
        assert np.array_equal(bits(upd.goal_front().vecs), bits(rv)), step
        if cur_r is not r0:
            cur_r.close()
        cur_r, cur_d = upd, d1
    cur_r.close()
    r0.close()


def test_update_full_size_3d():
    """The 20,000-sample 3D workload (three objectives) after five obstacles
    are found: the update equals a fresh search."""
    env = synth.plain3d(0)
    lo, hi = synth.discovered_boxes(env, 4, 5)
    g0 = mpap.mpap_build_graph(env)
    r0 = mpap.mpap_search(g0, env.beta, 3, env.radius, env.lam)
    g1 = mpap.mpap_graph_add_boxes(g0, lo, hi)
    upd = mpap.mpap_search_update(r0, g1, env.beta, 3, env.radius, env.lam)
    fresh = mpap.mpap_search(g1, env.beta, 3, env.radius, env.lam)
    su, sf = upd.stats(), fresh.stats()
    print(f"3D full size: {g0.info()['e'] - g1.info()['e']} edges removed; update "
          f"{su['labels_expanded']} labels, {su['gpu_ms']:.2f} ms; fresh "
          f"{sf['labels_expanded']} labels, {sf['gpu_ms']:.2f} ms", flush=True)
    assert su["front_labels"] == sf["front_labels"]
    assert np.array_equal(bits(upd.goal_front().vecs), bits(fresh.goal_front().vecs))
    n = g1.info()["n"]
    for v in range(0, n, 37):
        assert front_digest(upd.node_front(v)) == front_digest(fresh.node_front(v)), v
    for r in (upd, fresh, r0):
        r.close()
    g1.close()
    g0.close()


def test_update_refuses_a_different_search():
    env = synth.plain2d(0, n=400)
    g0 = mpap.mpap_build_graph(env)
    r0 = mpap.mpap_search(g0, env.beta, env.n_obj, env.radius, env.lam)
    with pytest.raises(mpap.MpapError) as ei:
        mpap.mpap_search_update(r0, g0, env.beta * 0.5, env.n_obj, env.radius, env.lam)
    assert ei.value.status == mpap.MPAP_ERR_INVAL
    early = mpap.mpap_search(g0, env.beta, env.n_obj, env.radius, env.lam, early_stop=1)
    with pytest.raises(mpap.MpapError):
        mpap.mpap_search_update(early, g0, env.beta, env.n_obj, env.radius, env.lam)
    # an update on the unchanged roadmap keeps everything and expands nothing
    same = mpap.mpap_search_update(r0, g0, env.beta, env.n_obj, env.radius, env.lam)
    assert same.stats()["labels_expanded"] == 0
    assert_same_fronts(same, r0, g0.info()["n"], "unchanged")
    for r in (same, early, r0):
        r.close()
    g0.close()
