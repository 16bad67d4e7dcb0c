"""Host logic of the autotuner (no GPU): candidate choice, skipping, caching."""
from paper_1404_2303_amd import autotune


def test_picks_the_fastest_and_caches(tmp_path):
    path = str(tmp_path / "c.json")
    calls = []

    def timer(p):
        calls.append(p)
        if p["cell_target"] == 24:
            raise autotune.CandidateUnusable("too small for this workload")
        return abs(p["cell_target"] - 48) + (0.5 if p["h_margin"] != 0.1 else 0.0)

    best = autotune.tune(timer, "k", "gfx950", cache_path=path)
    assert best["cell_target"] == 48 and best["h_margin"] == 0.1 and best["cached"] is False
    n = len(calls)
    again = autotune.tune(timer, "k", "gfx950", cache_path=path)
    assert again["cell_target"] == 48 and again["cached"] is True and len(calls) == n
    other = autotune.tune(lambda p: p["cell_target"], "k2", "gfx950", cache_path=path)
    assert other["cell_target"] == 24


def test_workload_class_buckets():
    a = autotune.workload_class(2 ** 20, 1, "fp32")
    b = autotune.workload_class(2 ** 20 + 5, 1, "fp32")
    c = autotune.workload_class(4_690_000, 256, "fp32")
    assert a == b and a != c and "fp32" in c


def test_failures_other_than_unusable_candidates_propagate(tmp_path):
    import pytest

    def timer(p):
        if p["cell_target"] == 48:
            raise RuntimeError("a broken candidate")
        return 1.0

    with pytest.raises(RuntimeError, match="broken"):
        autotune.tune(timer, "k", "gfx950", cache_path=str(tmp_path / "c.json"))


def test_staged_search_keeps_each_stage_best(tmp_path):
    path = str(tmp_path / "c.json")
    seen = []

    def timer(p):
        seen.append(dict(p))
        t = abs(p["cell_target"] - 64) + (0.5 if p["h_margin"] != 0.1 else 0.0)
        t += {2: 0.0, 1: 0.3}.get(p.get("sweep", 2), 0.0) + (0.2 if p.get("staging", 0) else 0.0)
        t += 0.1 * abs(p.get("shared_min", 128) - 64) / 64
        if p.get("shared_min") == 256:
            raise autotune.CandidateUnusable("not for this workload")
        return t

    best = autotune.tune_staged(timer, "k", "gfx950", cache_path=path)
    assert best["cell_target"] == 64 and best["h_margin"] == 0.1
    assert best["sweep"] == 2 and best["staging"] == 0 and best["shared_min"] == 64
    # later stages were timed on top of the earlier best
    assert all(p["cell_target"] == 64 for p in seen if "sweep" in p)
    n = len(seen)
    again = autotune.tune_staged(timer, "k", "gfx950", cache_path=path)
    assert again["cached"] and len(seen) == n and again["shared_min"] == 64
