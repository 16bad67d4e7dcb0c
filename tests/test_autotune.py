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
