"""Host-side checks of the bench line's roofline record: the measured HBM
traffic and the executed FP32 arithmetic are read from the committed
rocprofv3 summaries only while the kernel sources hash to the value the
summary records, and the executed figure follows from the summary's own
instruction counts."""
import re

import bench


def test_profile_values_follow_the_sources(tmp_path, monkeypatch):
    assert bench.measured_traffic() is not None
    flop = bench.measured_executed_flop()
    assert flop is not None
    # the recorded figure is (2 FMA + MUL + ADD + TRANS) x 64 of the summary's table
    text = open(bench.os.path.join(bench.ROOT, bench.COUNTERS_PROFILE)).read()

    def count(name):
        return float(re.search(r"\| " + name + r" \| ([0-9.e+-]+) \|", text).group(1))

    expect = (2 * count("SQ_INSTS_VALU_FMA_F32") + count("SQ_INSTS_VALU_MUL_F32") + count("SQ_INSTS_VALU_ADD_F32")
              + count("SQ_INSTS_VALU_TRANS_F32")) * 64
    assert abs(flop - expect) <= 1e-3 * expect
    # a changed kernel source invalidates both
    src = tmp_path / "changed.h"
    src.write_text("// not the kernel that was profiled\n")
    monkeypatch.setattr(bench, "KERNEL_SOURCES", bench.KERNEL_SOURCES + [str(src)])
    assert bench.measured_traffic() is None
    assert bench.measured_executed_flop() is None


def test_roofline_record():
    res = {"P": 4.9e7, "S": 4.74e7, "precision": "fp32",
           "kernel_ms": {"density_ms": 0.7, "force_ms": 0.6}}
    rl = bench.roofline(res)
    assert rl["kernel"] == "density" and rl["bound"] == "alu" and rl["peak"] == 157.3
    assert abs(rl["frac"] - rl["achieved"] / rl["peak"]) < 1e-15
    ex = rl["executed"]
    assert ex is not None and ex["over_algorithmic"] > 1.0
    assert abs(ex["TFLOP/s"] - bench.measured_executed_flop() / 0.7e-3 / 1e12) < 1e-9
