"""Pins for the plain Alg. 3 oracle (oracle/explore.py), each against
something other than itself:

* run to an empty P_open, its per-node fronts equal those of the label-setting
  oracle (mosearch.c, itself pinned by walk enumeration) for every group cost
  factor lambda -- the group loop and the label-setting order reach the same
  fronts;
* the early stop of the loop condition (Sec. 3) on a hand-worked instance in
  tests/golden/early_stop_spread.json: where it ends and what it returns,
  for a coarse and a fine group step;
* with a group step at most half the least edge cost, the early-stopped
  minimum-cost plan P_soln is the exact least goal cost (a plan cheaper than
  the first goal plan in a group has all its prefixes expanded in earlier
  groups);
* every plan the early-stopped loop holds is a feasible plan: weakly dominated
  by (or equal to) a member of the exact front at its node, and its parent
  chain re-walks to its own bits;
* a root inside the goal set ends the loop before any expansion.
"""
import numpy as np
import pytest

from oracle import explore, search
from paper_1705_02408_amd import synth
from tests.graphs import as_vecs, load_golden

F32 = np.float32


def bits(a):
    return np.ascontiguousarray(a, dtype=np.float32).view(np.uint32)


def rewalk(g, path, beta, n_obj):
    c = d = m = F32(0.0)
    for u, v in zip(path[:-1], path[1:]):
        e = [k for k in range(g["row_ptr"][u], g["row_ptr"][u + 1]) if g["col"][k] == v][0]
        c = F32(c + g["cost"][e])
        dpre = F32(d + g["drift"][e])
        assert dpre <= F32(beta)
        d = F32(0.0) if g["reset"][v] else dpre
        if n_obj == 3:
            m = F32(max(m, dpre))
    return c, d, m


CASES = [  # (seed, n, p_reset, n_obj, integer costs, beta)
    (0, 30, 0.0, 2, False, 0.9),
    (1, 30, 0.2, 3, False, 0.9),
    (2, 30, 0.0, 2, True, 1.0),
    (3, 24, 0.3, 3, True, 0.75),
    (4, 20, 0.5, 2, False, 0.5),
]


@pytest.mark.parametrize("seed,n,p_reset,n_obj,ints,beta", CASES)
@pytest.mark.parametrize("lam", [0.05, 0.5, 4.0])
def test_exact_mode_equals_label_setting(seed, n, p_reset, n_obj, ints, beta, lam):
    g = synth.tiny_random_graph(seed, n=n, p_reset=p_reset, mean_degree=3.0,
                                integer_costs=ints)
    ref = search.search(g, beta, n_obj)
    ex = explore.explore(g, beta, n_obj, lam, 1.0)
    assert not ex.stopped
    for v in range(n):
        assert np.array_equal(bits(ex.node_front(v)), bits(ref.node_front(v))), v


def test_exact_mode_on_a_small_roadmap():
    env = synth.plain2d(0, n=120)
    from oracle import graph as ograph
    g = ograph.build_graph(env)
    ref = search.search(g, env.beta, env.n_obj)
    ex = explore.explore(g, env.beta, env.n_obj, env.lam, env.radius)
    n = g["row_ptr"].shape[0] - 1
    for v in range(n):
        assert np.array_equal(bits(ex.node_front(v)), bits(ref.node_front(v))), v


def test_early_stop_golden():
    spec, g = load_golden("early_stop_spread.json")
    full = explore.explore(g, spec["beta"], spec["n_obj"], 1.0, 10.0)
    assert np.array_equal(bits(full.goal_front(g["goal"])), bits(as_vecs(spec["exact_goal_front"])))
    for case in spec["cases"]:
        ex = explore.explore(g, spec["beta"], spec["n_obj"], case["lam"], case["radius"],
                             early_stop=True)
        assert ex.stopped and ex.groups == case["groups"], case
        assert np.array_equal(bits(ex.goal_front(g["goal"])), bits(as_vecs(case["goal_front"])))
        for v, rows in case["node_fronts"].items():
            assert np.array_equal(bits(ex.node_front(int(v))), bits(as_vecs(rows))), (case, v)


@pytest.mark.parametrize("seed,n,p_reset,n_obj,ints,beta", CASES)
def test_fine_groups_stop_at_the_least_goal_cost(seed, n, p_reset, n_obj, ints, beta):
    g = synth.tiny_random_graph(seed, n=n, p_reset=p_reset, mean_degree=3.0,
                                integer_costs=ints)
    ref = search.search(g, beta, n_obj)
    exact, _, _ = search.goal_front(ref, g["goal"])
    step = float(np.min(g["cost"])) / 2
    ex = explore.explore(g, beta, n_obj, step, 1.0, early_stop=True)
    got = ex.goal_front(g["goal"])
    if exact.shape[0] == 0:
        assert got.shape[0] == 0 and not ex.stopped
    else:
        assert ex.stopped
        assert bits(got[0, 0]) == bits(exact[0, 0])


@pytest.mark.parametrize("seed,n,p_reset,n_obj,ints,beta", CASES)
@pytest.mark.parametrize("lam", [0.5, 2.0, 8.0])
def test_early_stopped_plans_are_feasible(seed, n, p_reset, n_obj, ints, beta, lam):
    g = synth.tiny_random_graph(seed, n=n, p_reset=p_reset, mean_degree=3.0,
                                integer_costs=ints)
    ref = search.search(g, beta, n_obj)
    ex = explore.explore(g, beta, n_obj, lam, 1.0, early_stop=True)
    for v in range(n):
        exact = ref.node_front(v)
        for p in ex.fronts[v]:
            vec = np.array(ex.vec[p], np.float32)
            assert np.any(np.all(exact <= vec, axis=1)), (v, vec)
            path = []
            a = p
            while a >= 0:
                path.append(ex.node[a])
                a = ex.parent[a]
            c, d, m = rewalk(g, path[::-1], beta, n_obj)
            assert bits([c, d, m]).tolist() == bits(vec).tolist()
    exact_goal, _, _ = search.goal_front(ref, g["goal"])
    got = ex.goal_front(g["goal"])
    if got.shape[0]:
        assert got[0, 0] >= exact_goal[0, 0]


def test_root_in_goal_stops_before_expanding():
    g = synth.tiny_random_graph(3, n=20)
    g = dict(g)
    g["goal"] = g["goal"].copy()
    g["goal"][0] = 1
    ex = explore.explore(g, 1.0, 2, 0.5, 1.0, early_stop=True)
    assert ex.stopped and ex.groups == 0
    assert bits(ex.goal_front(g["goal"])).tolist() == [[0, 0, 0]]
