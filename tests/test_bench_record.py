"""Host-side checks of the bench line's roofline record: the measured HBM
traffic and the executed FP32 arithmetic are read from rocprofv3 summaries
only while the kernel sources hash to the value a summary records, and the
committed instruction-mix summary's executed figure follows from its own
counts."""
import hashlib
import os
import re

import bench


def _sources_hash():
    h = hashlib.sha256()
    for f in bench.KERNEL_SOURCES:
        with open(os.path.join(bench.ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def test_committed_counter_summary_is_consistent():
    text = open(os.path.join(bench.ROOT, bench.COUNTERS_PROFILE)).read()

    def count(name):
        return float(re.search(r"\| " + name + r" \| ([0-9.e+-]+) \|", text).group(1))

    recorded = int(re.search(r"density_executed_fp32_flop: (\d+)", text).group(1))
    expect = (2 * count("SQ_INSTS_VALU_FMA_F32") + count("SQ_INSTS_VALU_MUL_F32") + count("SQ_INSTS_VALU_ADD_F32")
              + count("SQ_INSTS_VALU_TRANS_F32")) * 64
    assert abs(recorded - expect) <= 1e-3 * expect


def test_profile_values_follow_the_sources(tmp_path, monkeypatch):
    cur = _sources_hash()
    traffic = tmp_path / "traffic.md"
    counters = tmp_path / "counters.md"
    traffic.write_text(f"# summary\n\ndensity_traffic_bytes: 123456789\nsource_sha256: {cur}\n")
    counters.write_text(f"# summary\n\ndensity_executed_fp32_flop: 987654321\nsource_sha256: {cur}\n")
    monkeypatch.setattr(bench, "TRAFFIC_PROFILE", str(traffic))
    monkeypatch.setattr(bench, "COUNTERS_PROFILE", str(counters))
    assert bench.measured_traffic() == 123456789
    assert bench.measured_executed_flop() == 987654321
    res = {"P": 4.9e7, "S": 4.74e7, "precision": "fp32", "kernel_ms": {"density_ms": 0.7, "force_ms": 0.6}}
    rl = bench.roofline(res)
    assert rl["kernel"] == "density" and rl["bound"] == "alu" and rl["peak"] == 157.3
    assert abs(rl["frac"] - rl["achieved"] / rl["peak"]) < 1e-15
    assert rl["traffic"] == 123456789
    assert abs(rl["executed"]["TFLOP/s"] - 987654321 / 0.7e-3 / 1e12) < 1e-9
    # a changed kernel source invalidates both
    src = tmp_path / "changed.h"
    src.write_text("// not the kernel that was profiled\n")
    monkeypatch.setattr(bench, "KERNEL_SOURCES", bench.KERNEL_SOURCES + [str(src)])
    assert bench.measured_traffic() is None and bench.measured_executed_flop() is None
    rl = bench.roofline(res)
    assert rl["traffic"] is None and rl["executed"] is None
