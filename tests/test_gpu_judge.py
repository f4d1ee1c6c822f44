"""The learned heuristic's judge and analytic fallback inside the library
(mpap_judge), the per-query skip flag of batched searches, and saved network
weights.

A trained network must pass the judge (every goal-front plan, re-walked with
the analytic drift, within 1e-2 relative drift error and within the bound);
a corrupted one must fail it, and the fallback must then answer every query
with exactly the oracle's front on the analytic drift (the oracle's own
roadmaps, which the library's roadmaps equal bit for bit)."""
import numpy as np
import pytest

from oracle import graph as ograph, mlp, search as osearch
from paper_1705_02408_amd import synth

pytestmark = pytest.mark.gpu
mpap = pytest.importorskip("paper_1705_02408_amd.mpap")


def bits(a):
    return np.ascontiguousarray(a, dtype=np.float32).view(np.uint32)


def train_net(dim, seed):
    """A surrogate trained on a roadmap that is not part of the judged batch."""
    env = (synth.make_env(500 + seed, 2, 8000, 20, 30, 20.0, 0.3, 2, blob_amp=0.3) if dim == 2
           else synth.make_env(600 + seed, 3, 8000, 100, 80, 40.0, 0.25, 2, blob_amp=0.4))
    g = mpap.mpap_build_graph(env)
    e = g.info()["e"]
    edges = np.random.default_rng(seed).permutation(e)[: (e // 4096) * 4096]
    s = mpap.Surrogate(seed=seed)
    s.train(g, edges, epochs=8, batch=4096, lr=2e-3)
    g.close()
    return s


@pytest.fixture(scope="module")
def judged_batch():
    envs = []
    q = 0
    while len(envs) < 6:
        e = synth.batch_query(21, q, nmin=1500, nmax=4000)
        q += 1
        if ograph.goal_mask(e.pos, e.goal, e.goal_radius).sum() > 0:
            envs.append(e)
    parts = [mpap.mpap_build_graph(e) for e in envs]
    refs = []
    for e, p in zip(envs, parts):
        g = ograph.build_graph(e)
        got = p.export()
        assert np.array_equal(bits(got["drift"]), bits(g["drift"]))
        assert np.array_equal(got["col"], g["col"]) and np.array_equal(got["reset"], g["reset"])
        ref = osearch.search(g, e.beta, e.n_obj)
        refs.append((g, ref, osearch.goal_front(ref, g["goal"])[0]))
    nets = {2: train_net(2, 1), 3: train_net(3, 2)}
    yield envs, parts, refs, nets
    for s in nets.values():
        s.close()
    for p in parts:
        p.close()


def union_of(parts, envs, nets, corrupt=()):
    for k, (p, e) in enumerate(zip(parts, envs)):
        nets[e.dim].score(p)
    if corrupt:
        bad = mpap.Surrogate()
        p0 = mlp.flat(mlp.init_params(1))
        p0[-1] = -500.0  # output bias: every predicted drift clamps to zero
        bad.set_params(p0)
        for k in corrupt:
            bad.score(parts[k])
        bad.close()
    return mpap.mpap_graph_concat(parts)


def params(envs, heuristic=1, skip=()):
    return [mpap.search_params(e.beta, e.n_obj, e.radius, e.lam, heuristic=heuristic,
                               skip=int(k in skip)) for k, e in enumerate(envs)]


def test_trained_networks_pass_the_judge(judged_batch):
    envs, parts, refs, nets = judged_batch
    union = union_of(parts, envs, nets)
    res = mpap.mpap_search_batch(union, params(envs))
    failed = res.judge(1e-2, fallback=False)
    print(f"judge rejected {int(failed.sum())} of {len(envs)} queries", flush=True)
    assert not failed.any()
    assert res.stats()["judged_failed"] == 0
    # every passed front re-walks within the tolerance (the judge's own rule)
    for q, e in enumerate(envs):
        fr = res.goal_front(q)
        rs = mpap.mpap_rescore_front(res, q)
        assert rs["feasible"].all()
        floor = 1e-3 * e.beta
        for col, key in ((1, "drift"), (2, "maxdrift")):
            a = rs[key].astype(np.float64)
            assert np.all(np.abs(fr.vecs[:, col] - a) / np.maximum(a, floor) <= 1e-2)
    with pytest.raises(mpap.MpapError):
        res.judge()  # a result is judged once
    res.close()
    union.close()


def test_corrupted_network_is_rejected_and_the_fallback_is_exact(judged_batch):
    envs, parts, refs, nets = judged_batch
    corrupt = (0, 2, 3)
    union = union_of(parts, envs, nets, corrupt=corrupt)
    res = mpap.mpap_search_batch(union, params(envs))
    failed = res.judge(1e-2, fallback=True)
    st = res.stats()
    print(f"rejected {np.nonzero(failed)[0].tolist()}, fallback {st['fallback_ms']:.2f} ms",
          flush=True)
    for k in corrupt:
        if refs[k][2].shape[0]:
            assert failed[k], k
    assert st["judged_failed"] == int(failed.sum()) and st["fallback_ms"] > 0
    off = mpap.mpap_graph_queries(union)
    for q, (e, (g, ref, rv)) in enumerate(zip(envs, refs)):
        fr = res.goal_front(q)
        if failed[q]:
            # answered by the analytic re-search: the oracle's front, bit for bit
            assert np.array_equal(bits(fr.vecs), bits(rv)), q
            for v in range(0, g["reset"].shape[0], 37):
                a = res.node_front(int(off[q]) + v)
                a = a[np.lexsort((a[:, 2], a[:, 1], a[:, 0]))] if a.shape[0] else a
                assert np.array_equal(bits(a), bits(ref.node_front(v))), (q, v)
        # every witness re-walks on the analytic drift (ids unique across the
        # two searches), and the cost is exact
        for k in range(fr.vecs.shape[0]):
            path = res.path(int(fr.label[k]))
            local = [u - int(off[q]) for u in path]
            assert local[0] == 0 and g["goal"][local[-1]]
            c, d, m, ok = osearch.rewalk(g, local, e.beta, e.n_obj)
            assert c == fr.vecs[k, 0]
            if failed[q]:
                assert ok and d == fr.vecs[k, 1]
        rs = mpap.mpap_rescore_front(res, q)
        assert np.array_equal(bits(rs["cost"]), bits(fr.vecs[:, 0])), q
    res.close()
    union.close()


def test_skipped_queries_are_left_out(judged_batch):
    envs, parts, refs, nets = judged_batch
    union = mpap.mpap_graph_concat(parts)
    full = mpap.mpap_search_batch(union, params(envs, heuristic=0))
    part = mpap.mpap_search_batch(union, params(envs, heuristic=0, skip=(1, 4)))
    off = mpap.mpap_graph_queries(union)
    for q in range(len(envs)):
        if q in (1, 4):
            assert part.goal_front(q).vecs.shape[0] == 0
            assert part.node_front(int(off[q])).shape[0] == 0
        else:
            assert np.array_equal(bits(part.goal_front(q).vecs), bits(refs[q][2])), q
            assert np.array_equal(bits(full.goal_front(q).vecs), bits(refs[q][2])), q
    assert part.stats()["front_labels"] < full.stats()["front_labels"]
    full.close()
    part.close()
    union.close()


def test_surrogate_weights_round_trip(tmp_path):
    s = mpap.Surrogate(seed=3)
    p = s.get_params()
    p[-1] = 0.125
    s.set_params(p)
    path = str(tmp_path / "net.bin")
    s.save(path)
    t = mpap.Surrogate()
    t.load(path)
    assert np.array_equal(t.get_params().view(np.uint32), p.view(np.uint32))
    raw = bytearray(open(path, "rb").read())
    assert raw[:8] == b"MPAPSUR1" and len(raw) == 8 + 4 + 4 * 5313 + 4
    raw[100] ^= 1  # one flipped bit: the hash no longer matches
    bad = tmp_path / "bad.bin"
    bad.write_bytes(bytes(raw))
    with pytest.raises(mpap.MpapError):
        t.load(str(bad))
    with pytest.raises(mpap.MpapError):
        t.load(str(tmp_path / "missing.bin"))
    s.close()
    t.close()
