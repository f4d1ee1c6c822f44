"""Host logic of the autotuner: coordinate descent over the settings that
never change a result, the cached choice, and applying it to parameters
(timings replaced by a synthetic cost function; no GPU)."""
import pytest

from paper_1705_02408_amd import autotune, mpap


class FakeGraph:
    def info(self):
        return {"n": 5000, "e": 100000, "n_goal": 3}


def cost(params):
    p = params[0]
    # a separable cost whose minimum is lambda 1.0, near_scan 32, 512 threads,
    # wave threshold -1, stage cap 0, merges by halves always
    return ((p.lambda_ - 1.0) ** 2 + abs(p.near_scan - 32) / 8 +
            (0 if p.block_threads == 512 else 1) + (0 if p.wave_min_targets == -1 else 0.5) +
            (0 if p.stage_cap == 0 else 0.25) + (0 if p.merge_halves == 8192 else 0.125) + 10.0)


def test_descent_finds_the_separable_minimum(tmp_path, monkeypatch):
    calls = []

    def fake_time(graph, params, repeats):
        calls.append(params)
        return cost(params)
    monkeypatch.setattr(autotune, "_time", fake_time)
    monkeypatch.setattr(autotune, "_device_name", lambda: "gfx950")
    base = [mpap.search_params(0.3, 2, 0.05, 0.5, heuristic=1) for _ in range(3)]
    cache = str(tmp_path / "cache.json")
    ch = autotune.tune(FakeGraph(), base, [2, 3], 2, cache_path=cache, repeats=1)
    assert (ch.lam, ch.near_scan, ch.block_threads, ch.wave_min_targets, ch.stage_cap,
            ch.merge_halves) == (1.0, 32, 512, -1, 0, 8192)
    assert ch.kernel_ms == pytest.approx(10.0)
    # every timed setting keeps the caller's other fields
    for ps in calls:
        assert all(p.heuristic == 1 and p.beta == pytest.approx(0.3) for p in ps)
    n_calls = len(calls)
    # a second call is answered from the cache
    ch2 = autotune.tune(FakeGraph(), base, [2, 3], 2, cache_path=cache, repeats=1)
    assert len(calls) == n_calls and ch2.fields() == ch.fields()
    out = autotune.apply(base, ch)
    assert [p.block_threads for p in out] == [512] * 3 and out[0].heuristic == 1
    assert out[0].lambda_ == 1.0 and out[0].near_scan == 32 and out[0].wave_min_targets == -1
    assert out[0].merge_halves == 8192
