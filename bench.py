#!/usr/bin/env python3
"""Benchmark: SPH pair interactions per second (density + force) on one MI355X.

Workload: 2^20 particles on a 128 x 128 x 64 cubic lattice of spacing 1/128
(periodic 1 x 1 x 1/2 box), every site jittered by U(-0.1, 0.1) spacings,
velocities N(0, 0.1), u = 1, equal masses; seeded.

One step = the whole hot path over that input, starting from the initial
smoothing lengths: cell build (keys, radix sort, cells, neighbour lists,
cell-ordered copies) -> 13-direction orderings -> density with the Newton
iteration on h (and the per-particle quantities between the stages) ->
force with viscosity.  The initial h is restored (one device copy) at the
start of every step, inside the timed region.

Unit of work: one unordered pair {i, j} with r_ij < max(h_i, h_j) at the solved
h, counted once per stage, so a step credits P = P_density + P_force =
sum_i n_pairs_i pair interactions.  Extra Newton rounds are timed but not
credited.

Roofline: the interaction kernels are bound by plain FP32/FP64 vector ALU
work.  Algorithmic FLOPs per launch (FMA = 2, add/mul = 1, sqrt/rsqrt/div = 1,
compare/select = 0, counted term by term from Eqs. (2)-(5) and the Sec. 4.1
viscosity once per unordered pair, as a symmetric evaluation would do them):
    density: 26 per pair (separation 3, r^2 5, r 1, velocity difference 3,
               dv.dx 5, dv x dx 9: shared by both sides)
             + 26 per side with r < h_side (q 1, w 5, w' 3, q w' 1, w'/q 1,
               the four sums of rho, N, dN/dh, drho/dh 6, m g 1, divergence 2,
               curl 6)
    force:   68 per pair (separation 3, r^2 5, 1/r 1, r 1, dv 3, dv.dx 5,
               w_ij 1, q_i, q_j 2, both gradients 6, signal speed 3,
               Pi_ij 5, f_i + f_j 1, the viscous factor 3, the pressure
               scalar 3, the two scalings by the masses 4, both sides'
               accelerations 12 and du/dt 10)
The line also gives the fraction at round per-pair constants of 70 (density)
and 120 (force) FLOP, an earlier estimate of the same work.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

FLOPS_DENSITY_PAIR = 26
FLOPS_DENSITY_SIDE = 26
FLOPS_FORCE_PAIR = 68
FLOPS_ROUND = {"density": 70, "force": 120}   # round per-pair estimate, reported beside the count
PEAK = {"fp32": 157.3, "fp64": 78.6}   # MI355X vector TFLOP/s (published)

METRIC = "pair interactions/sec (density+force) at 1M particles; plain vs batched/FP32 form"


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def ensure_built():
    from paper_1404_2303_amd import sph
    if not os.path.exists(sph.LIB_PATH):
        import __graft_entry__
        __graft_entry__.build()


def run_form(ps, precision, steps, warmup, **params):
    import torch
    from paper_1404_2303_amd import sph
    parts = sph.Particles.from_numpy(ps, "cuda:0")
    h0 = parts.h.clone()
    ctx = sph.Context(ps.box, precision=precision, **params)
    ctx.enable_timing(True)
    n = parts.n
    fout = {k: torch.empty(n, dtype=torch.float64, device="cuda:0") for k in ("ax", "ay", "az", "dudt")}
    fout["n_pairs"] = torch.empty(n, dtype=torch.int32, device="cuda:0")

    def step():
        parts.h.copy_(h0)
        ctx.build_cells(parts)
        ctx.sort()
        ctx.density(parts, want=("rho", "n_dens", "n_iter"))
        ctx.force(parts, out=fout)

    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    kt = {"build_ms": [], "sort_ms": [], "density_ms": [], "force_ms": []}
    step_ms = []
    start = torch.cuda.Event(enable_timing=True)
    end = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        start.record()
        step()
        end.record()
        end.synchronize()
        step_ms.append(start.elapsed_time(end))
        times = ctx.kernel_times()
        for k in kt:
            kt[k].append(times[k])
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    # counts from one more pass over the same input
    parts.h.copy_(h0)
    ctx.build_cells(parts)
    ctx.sort()
    dd = ctx.density(parts, want=("n_dens", "n_iter"))
    ff = ctx.force(parts, out=fout)
    torch.cuda.synchronize()
    P = int(ff["n_pairs"].sum().item())          # ordered -> 2 stages x unordered
    S = int(dd["n_dens"].sum().item())           # density sides with r < h_side
    iters = dd["n_iter"].cpu().numpy()
    stats = ctx.stats()
    ctx.close()
    med = lambda v: float(np.median(v))
    return {
        "precision": precision,
        "P": P,
        "S": S,
        "ms_per_step": float(np.mean(step_ms)),
        "ms_median": med(step_ms),
        "wall_s": wall,
        "kernel_ms": {k: med(v) for k, v in kt.items()},
        "newton_mean": float(np.mean(iters)),
        "newton_max": int(np.max(iters)),
        "cells": int(stats["n_cells"]),
        "grid": list(stats["grid"]),
    }


def run_graph(ps, precision, steps, warmup, batch=None, params=None):
    """The pass captured once as a HIP graph (h restored from the initial guess
    inside the graph) and replayed; no host synchronisation inside a step."""
    import torch
    from paper_1404_2303_amd import sph
    parts = sph.Particles.from_numpy(ps, "cuda:0")
    h0 = parts.h.clone()
    ctx = sph.Context(ps.box, precision=precision, **(params or {}))
    b = sph.Batch(*batch) if batch is not None else None
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        _, fout = ctx.graph_capture(parts, b, h_init=h0)
        ctx.check()
        for _ in range(warmup):
            ctx.graph_launch()
        torch.cuda.synchronize()
        ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(steps)]
        torch.cuda.synchronize()
        for a, e in ev:
            a.record()
            ctx.graph_launch()
            e.record()
        torch.cuda.synchronize()
        ms = [a.elapsed_time(e) for a, e in ev]
        ctx.check()
        P = int(fout["n_pairs"].sum().item())
    ctx.close()
    return {"P": P, "ms_per_step": float(np.mean(ms)), "ms_median": float(np.median(ms))}


def run_per_box_loop(ps, precision, offsets, lens, params=None):
    """Baseline for the batched form: every box through its own plain calls."""
    import torch
    from paper_1404_2303_amd import sph, workloads
    ctxs, parts = [], []
    for b in range(len(offsets) - 1):
        sl = slice(offsets[b], offsets[b + 1])
        sub = workloads.ParticleSet(pos=ps.pos[sl], vel=ps.vel[sl], m=ps.m[sl], u=ps.u[sl], h0=ps.h0[sl],
                                    box=lens[b])
        parts.append((sph.Particles.from_numpy(sub, "cuda:0"), None))
        ctxs.append(sph.Context(lens[b], precision=precision, **(params or {})))
    h0s = [p.h.clone() for p, _ in parts]

    def one_step():
        P = 0
        outs = []
        for ctx, (p, _), h0 in zip(ctxs, parts, h0s):
            p.h.copy_(h0)
            d, f = ctx.run(p)
            outs.append(f["n_pairs"])
        return outs

    one_step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    outs = one_step()
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    P = int(sum(int(o.sum().item()) for o in outs))
    for c in ctxs:
        c.close()
    return {"P": P, "ms_per_step": dt * 1e3}


def batched_section(steps, warmup, tune=True):
    """256 independent boxes, log-uniform counts in [2048, 65536]: one captured
    pass over all boxes vs a loop of per-box plain calls."""
    import torch
    from paper_1404_2303_amd import autotune, workloads
    ps, offsets, lens = workloads.batch()
    arch = torch.cuda.get_device_properties(0).gcnArchName.split(":")[0]
    params, tuned = {}, None
    if tune:
        key = autotune.workload_class(ps.n, len(offsets) - 1, "fp32")
        tuned = autotune.tune_staged(autotune.gpu_timer(ps, "fp32", batch=_BatchArgs(offsets, lens)), key, arch)
        params = {k: v for k, v in tuned.items() if k != "cached"}
    g = run_graph(ps, "fp32", steps, warmup, batch=(offsets, lens), params=params)
    loop = run_per_box_loop(ps, "fp32", offsets, lens, params=params)
    return {"workload": f"{len(offsets) - 1} periodic unit boxes, log-uniform counts in [2048, 65536], "
                        f"{ps.n} particles, uniform-random positions seeded per box, v=0, u=1",
            "n": ps.n, "pairs_per_step": g["P"], "value": g["P"] / (g["ms_per_step"] * 1e-3),
            "ms_per_step": g["ms_per_step"], "per_box_loop_value": loop["P"] / (loop["ms_per_step"] * 1e-3),
            "per_box_loop_ms": loop["ms_per_step"], "speedup_vs_loop": loop["ms_per_step"] / g["ms_per_step"],
            "tuned": tuned}


def adjoint_section(steps, warmup):
    """Reverse mode on the 64^3 jittered lattice (262,144 particles, FP32 pair
    arithmetic): loss sum (rho - rho_t)^2 + sum |a|^2; the forward pass once,
    then sph_backward with the implicit h derivative timed alone and a full
    forward + backward step timed together."""
    import torch
    from paper_1404_2303_amd import sph, workloads
    ps = workloads.config4()
    rt = torch.as_tensor(workloads.density_target(ps.pos, float(np.sum(ps.m))), device="cuda:0")
    parts = sph.Particles.from_numpy(ps, "cuda:0")
    h0 = parts.h.clone()
    ctx = sph.Context(ps.box, precision="fp32", keep_adjoint=1)
    ctx.enable_timing(True)

    def forward():
        parts.h.copy_(h0)
        d, f = ctx.run(parts)
        return d, f

    def backward(d, f):
        a = torch.stack([f["ax"], f["ay"], f["az"]], 1)
        return ctx.backward(parts, 2 * (d["rho"] - rt), 2 * a, None, implicit_h=True)

    d, f = forward()
    for _ in range(warmup):
        backward(d, f)
    torch.cuda.synchronize()
    bw = []
    for _ in range(steps):
        backward(d, f)
        bw.append(ctx.kernel_times()["backward_ms"])
    P = int(f["n_pairs"].sum().item())
    start, end = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    fb = []
    for _ in range(max(3, steps // 2)):
        start.record()
        d, f = forward()
        backward(d, f)
        end.record()
        end.synchronize()
        fb.append(start.elapsed_time(end))
    ctx.close()
    bms = float(np.median(bw))
    return {"workload": "jittered cubic lattice 64^3 (262,144 particles), spacing 1/64, unit box, v~N(0,0.1); "
                        "loss sum (rho-rho_t)^2 + sum |a|^2, gradient in x through the solved h",
            "n": ps.n, "pairs": P, "backward_ms": bms, "backward_pairs_per_s": P / (bms * 1e-3),
            "forward_backward_ms": float(np.median(fb))}


def multires_section(steps, warmup, tune=True):
    """The 2,097,152-particle Plummer mixture (32 spheres, scale radii log-uniform
    in [0.005, 0.05], 20% uniform background; h spans ~100x) on the hierarchical
    decomposition, FP32 pair arithmetic, leaf size autotuned.  First h from
    sph_estimate_h, solved once outside the timed region; a timed step restores
    h to that solution (the state a simulation step starts from) and runs build,
    sort, density and force.  A cold pass from the estimate is timed once as
    well."""
    import torch
    from paper_1404_2303_amd import autotune, sph, workloads
    ps = workloads.config2()
    parts = sph.Particles.from_numpy(ps, "cuda:0")
    # the leaf size is tuned on the graph-captured pass from the solved h
    probe = sph.Context(ps.box, precision="fp32", max_depth=10, split_count=256)
    probe.estimate_h(parts)
    probe.run(parts)
    h_solved = parts.h.clone()
    probe.close()
    split_count, tuned = 256, None
    if tune:
        arch = torch.cuda.get_device_properties(0).gcnArchName.split(":")[0]
        key = "tree|" + autotune.workload_class(ps.n, 1, "fp32")
        tuned = autotune.tune(autotune.gpu_timer(ps, "fp32", h_init=h_solved, fixed={"max_depth": 10}), key, arch,
                              candidates=autotune.TREE_CANDIDATES)
        split_count = int(tuned["split_count"])
    parts.h.copy_(torch.as_tensor(ps.h0, device="cuda:0"))
    ctx = sph.Context(ps.box, precision="fp32", max_depth=10, split_count=split_count)
    ctx.enable_timing(True)
    n = parts.n
    fout = {k: torch.empty(n, dtype=torch.float64, device="cuda:0") for k in ("ax", "ay", "az", "dudt")}
    fout["n_pairs"] = torch.empty(n, dtype=torch.int32, device="cuda:0")
    ctx.estimate_h(parts)
    h_est = parts.h.clone()
    start, end = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    start.record()
    ctx.build_cells(parts)
    ctx.sort()
    ctx.density(parts, want=("n_dens",))
    ctx.force(parts, out=fout)
    end.record()
    end.synchronize()
    cold_ms = start.elapsed_time(end)
    cold_rebuilds = ctx.stats()["rebuilds"]
    h_sol = parts.h.clone()
    del h_est

    def step():
        parts.h.copy_(h_sol)
        ctx.build_cells(parts)
        ctx.sort()
        ctx.density(parts, want=("n_dens",))
        ctx.force(parts, out=fout)

    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    ms, kt = [], {"build_ms": [], "sort_ms": [], "density_ms": [], "force_ms": []}
    for _ in range(steps):
        start.record()
        step()
        end.record()
        end.synchronize()
        ms.append(start.elapsed_time(end))
        t = ctx.kernel_times()
        for k in kt:
            kt[k].append(t[k])
    P = int(fout["n_pairs"].sum().item())
    st = ctx.stats()
    ctx.close()
    step_ms = float(np.median(ms))
    return {"workload": "Plummer mixture: 32 spheres x 52,428 + 419,456 uniform background (2,097,152 particles), "
                        "scale radii log-uniform [0.005, 0.05], periodic unit cube, v~N(0,0.1), u=1",
            "n": n, "pairs_per_step": P, "value": P / (step_ms * 1e-3), "ms_per_step": step_ms,
            "kernel_ms": {k: float(np.median(v)) for k, v in kt.items()},
            "leaves": int(st["n_cells"]), "depth": int(st["depth"]), "top_grid": list(st["grid"]),
            "split_count": split_count, "tuned": tuned, "cold_pass_ms": cold_ms,
            "cold_rebuilds": int(cold_rebuilds)}


class _BatchArgs:
    """Adapter: a Batch built lazily inside the timer (keeps host arrays alive)."""

    def __init__(self, offsets, lens):
        from paper_1404_2303_amd import sph
        self.b = sph.Batch(offsets, lens)
        self.c = self.b.c


KERNEL_SOURCES = ["paper_1404_2303_amd/csrc/passes.hip", "paper_1404_2303_amd/csrc/sweep.h",
                  "paper_1404_2303_amd/csrc/pairs.h",
                  "paper_1404_2303_amd/csrc/kernels.h", "paper_1404_2303_amd/csrc/sph_internal.h"]
TRAFFIC_PROFILE = "profiles/traffic_lattice2p20_fp32.md"
COUNTERS_PROFILE = "profiles/counters_lattice2p20_fp32.md"


def _profile_value(path, key):
    """An integer a committed rocprofv3 summary records for the density kernel,
    or None when the kernel sources changed since the counters were taken."""
    import hashlib
    try:
        h = hashlib.sha256()
        for f in KERNEL_SOURCES:
            with open(os.path.join(ROOT, f), "rb") as fh:
                h.update(fh.read())
        fields = {}
        with open(os.path.join(ROOT, path)) as fh:
            for line in fh:
                if ":" in line and line.split(":")[0] in (key, "source_sha256"):
                    k, v = line.split(":", 1)
                    fields[k.strip()] = v.strip()
        if fields.get("source_sha256") != h.hexdigest():
            return None
        return int(fields[key])
    except (OSError, KeyError, ValueError):
        return None


def measured_traffic():
    """HBM bytes per launch of the density kernel (FETCH_SIZE + WRITE_SIZE, calibrated)."""
    return _profile_value(TRAFFIC_PROFILE, "density_traffic_bytes")


def measured_executed_flop():
    """FP32 arithmetic the density launch issues, from the instruction-mix counters:
    (2 FMA + MUL + ADD + TRANS) wave64 instructions x 64 lanes."""
    return _profile_value(COUNTERS_PROFILE, "density_executed_fp32_flop")


def roofline(res):
    """Dominant interaction kernel's algorithmic FLOP rate against the vector peak."""
    P_unordered = res["P"] / 2.0
    dens_flops = FLOPS_DENSITY_PAIR * P_unordered + FLOPS_DENSITY_SIDE * res["S"]
    force_flops = FLOPS_FORCE_PAIR * P_unordered
    km = res["kernel_ms"]
    cand = [("density", dens_flops, km["density_ms"]), ("force", force_flops, km["force_ms"])]
    name, flops, ms = max(cand, key=lambda c: c[2])
    achieved = flops / (ms * 1e-3) / 1e12
    peak = PEAK["fp64" if res["precision"] == "fp64" else "fp32"]
    traffic = measured_traffic() if (name == "density" and res["precision"] == "fp32") else None
    executed = measured_executed_flop() if (name == "density" and res["precision"] == "fp32") else None
    round_flops = FLOPS_ROUND[name] * P_unordered
    return {"bound": "alu", "kernel": name, "achieved": achieved, "peak": peak, "unit": "TFLOP/s",
            "frac": achieved / peak, "traffic": traffic,
            # the counters' issued FP32 arithmetic at this run's kernel time (None once the
            # kernel has changed since the counters were taken)
            "executed": None if executed is None else {
                "TFLOP/s": executed / (ms * 1e-3) / 1e12, "frac": executed / (ms * 1e-3) / 1e12 / peak,
                "over_algorithmic": executed / flops},
            "flop_per_unit": {"density_pair": FLOPS_DENSITY_PAIR, "density_side": FLOPS_DENSITY_SIDE,
                              "force_pair": FLOPS_FORCE_PAIR, "units": {"pairs": P_unordered, "sides": res["S"]}},
            "frac_at_round_constants": round_flops / (ms * 1e-3) / 1e12 / peak,
            "other": {c[0]: {"TFLOP/s": c[1] / (c[2] * 1e-3) / 1e12, "ms": c[2]} for c in cand}}


def _cpu_model():
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(seed=0):
    """The FP64 oracle on a bounded sample: the same lattice law on 128 x 64 x 32
    sites, timed with every thread OpenMP offers (the value) and on one core."""
    import oracle
    from paper_1404_2303_amd import workloads
    ps = workloads.lattice((128, 64, 32), 1.0 / 128, 0.1, 0.1, seed)

    def timed():
        t0 = time.perf_counter()
        out = oracle.full_pass(ps.pos, ps.vel, ps.m, ps.u, ps.h0, ps.box, tol=1e-10)
        return time.perf_counter() - t0, int(np.sum(out["force"]["count"]))

    threads = oracle.num_threads()
    dt, P = timed()
    oracle.set_num_threads(1)
    dt1, P1 = timed()
    oracle.set_num_threads(threads)
    return {"value": P / dt, "unit": "pair interactions/s", "cores": threads, "kind": "oracle",
            "sample": f"FP64 oracle, full density(h-iteration)+force pass on a 128x64x32 jittered lattice "
                      f"({ps.n} particles, same spacing/jitter/velocity law), {dt:.2f} s, P={P}",
            "one_core": {"value": P1 / dt1, "cores": 1, "seconds": dt1},
            "nproc": os.cpu_count(), "cpu": _cpu_model()}


def integrate_section(steps, warmup):
    """Time integration of the Sod shock tube of Sec. 4.2 at the paper's size
    (8 x 1 x 1 periodic box, 810,448 + 202,612 particles on FCC | simple cubic
    lattices, density 4 | 1, pressure 1 | 0.1795), FP32 pair arithmetic,
    Balsara switch of the |div v| form: kick-drift-kick steps of the length
    Eq. (6) allows, each step a full rebuild, 13 orderings, density with the
    Newton iteration, force with the time-step criterion, and the kicks.  The
    dense side's cells hold ~110 particles (cells are sized by the light
    side's h): wide staging of the density stage."""
    import torch
    from paper_1404_2303_amd import sph, workloads
    ps = workloads.sod(37)

    def run(reuse):
        parts = sph.Particles.from_numpy(ps, "cuda:0")
        ctx = sph.Context(ps.box, precision="fp32", balsara_form=sph.SPH_BALSARA_DIV, reuse=reuse,
                          staging=sph.SPH_STAGING_WIDE)
        ctx.enable_timing(True)
        d, acc = ctx.run(parts)
        t_box = torch.zeros(1, dtype=torch.float64, device="cuda:0")
        dt_box = torch.zeros(1, dtype=torch.float64, device="cuda:0")
        for _ in range(warmup):
            ctx.step_adaptive(parts, acc, t_box, 1e30, 1.0, dt_box=dt_box)
        torch.cuda.synchronize()
        start, end = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        t0 = float(t_box[0])
        refreshed = 0
        ms = 0.0
        kt = {"density_ms": [], "force_ms": []}
        for _ in range(steps):
            start.record()
            ctx.step_adaptive(parts, acc, t_box, 1e30, 1.0, dt_box=dt_box)
            end.record()
            end.synchronize()
            ms += start.elapsed_time(end)
            st = ctx.stats()
            reused = st["refreshes"] > 0 and st["rebuilds"] == 0
            refreshed += 1 if reused else 0
            times = ctx.kernel_times()
            for k in kt:
                kt[k].append((reused, times[k]))
        ms /= steps
        kernel = {}
        for k, v in kt.items():
            a = [t for r, t in v if r]
            b = [t for r, t in v if not r]
            kernel[k] = {"reused_steps": float(np.mean(a)) if a else None,
                         "rebuilt_steps": float(np.mean(b)) if b else None}
        P = int(acc["n_pairs"].sum().item())
        t1 = float(t_box[0])
        ctx_drift = ctx.stats()["drift"]
        ctx.close()
        return {"ms_per_step": ms, "pairs_per_step": P, "pairs_per_s": P / (ms * 1e-3),
                "mean_dt": (t1 - t0) / steps, "steps_reusing_cells": refreshed, "kernel_ms": kernel,
                "drift_last": ctx_drift}

    return {"workload": "Sod shock tube, 8x1x1 periodic box, FCC|simple-cubic lattices of cell 1/37 "
                        f"({ps.n} particles), adaptive steps by Eq. (6), C_CFL 1/4",
            "n": ps.n, "steps": steps, "rebuild_every_step": run(sph.SPH_REUSE_OFF),
            "reuse_cells_and_orderings": run(sph.SPH_REUSE_ORDERINGS),
            "reuse_cells_resort": run(sph.SPH_REUSE_CELLS)}


def mts_section(base_steps):
    """Multiple time-stepping on the blast wave of Sec. 4.2 at about the
    paper's size (face-centred cubic lattice of 1,000,188 particles, energy 1
    on the 28 central particles, background pressure 1e-6, Balsara switch of
    the |div v| form): the same simulated interval, base_steps times the
    smallest initial time step of Eq. (6), advanced (a) with every particle
    stepping at the smallest current time step (sph_step_adaptive) and (b) with
    power-of-two time bins on that base step, up to 2^10 (sph_mts_step), with
    and without reuse of the cells."""
    import torch
    from paper_1404_2303_amd import sph, workloads
    ps = workloads.sedov(63)
    ev = lambda: (torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))

    def global_steps(t_end):
        parts = sph.Particles.from_numpy(ps, "cuda:0")
        ctx = sph.Context(ps.box, precision="fp32", balsara_form=sph.SPH_BALSARA_DIV)
        d, acc = ctx.run(parts)
        t_box = torch.zeros(1, dtype=torch.float64, device="cuda:0")
        a, b = ev()
        torch.cuda.synchronize()
        a.record()
        nst = 0
        while float(t_box[0]) < t_end and nst < 100000:
            ctx.step_adaptive(parts, acc, t_box, t_end, 1.0)
            nst += 1
        b.record()
        b.synchronize()
        ctx.close()
        return {"ms": a.elapsed_time(b), "steps": nst}

    def mts(dtb, reuse):
        parts = sph.Particles.from_numpy(ps, "cuda:0")
        ctx = sph.Context(ps.box, precision="fp32", balsara_form=sph.SPH_BALSARA_DIV, reuse=reuse)
        acc, bins = ctx.mts_init(parts, dtb, 10)
        a, b = ev()
        torch.cuda.synchronize()
        a.record()
        for _ in range(base_steps):
            ctx.mts_step(parts, acc, bins)
        b.record()
        b.synchronize()
        ms = a.elapsed_time(b)
        # the active fractions of one more cycle of base steps, counted (untimed)
        counts = [ctx.mts_step(parts, acc, bins, count=True) for _ in range(16)]
        ctx.close()
        return {"ms": ms, "base_steps": base_steps, "active_fraction_next_16": float(np.mean(counts)) / ps.n}

    parts = sph.Particles.from_numpy(ps, "cuda:0")
    ctx = sph.Context(ps.box, precision="fp32", balsara_form=sph.SPH_BALSARA_DIV)
    d, f = ctx.run(parts)
    dtb = float(f["dt"].min().item())
    ctx.close()
    t_end = base_steps * dtb
    g = global_steps(t_end)
    m0 = mts(dtb, sph.SPH_REUSE_OFF)
    m1 = mts(dtb, sph.SPH_REUSE_ORDERINGS)
    return {"workload": f"Sedov blast, FCC lattice of {ps.n} particles, E = 1 on 28 central particles, "
                        "background P = 1e-6, unit periodic box",
            "t_end": t_end, "dt_base": dtb, "global_smallest_step": g, "mts": m0, "mts_reuse": m1,
            "speedup_mts": g["ms"] / m0["ms"], "speedup_mts_reuse": g["ms"] / m1["ms"]}


def orderings_section(reps=5):
    """Time of the 13 orderings (sph_sort) where cells exceed one wavefront's
    sort (256 particles): a uniform-random 2^20 set on grids of ~300, ~1000
    and ~2000 particles per cell, whose orderings are made from those of
    their sub-cells shifted and merged (Sec. 3.3)."""
    import torch
    from paper_1404_2303_amd import sph, workloads
    ps = workloads.uniform(1 << 20, seed=1, sigma_v=0.1)
    parts = sph.Particles.from_numpy(ps, "cuda:0")
    out = {"workload": "uniform-random 2^20 particles, unit periodic box, FP32 positions in the cell frame"}
    for ct in (300, 1000, 2000):
        ctx = sph.Context(ps.box, precision="fp32", cell_target=ct)
        ctx.enable_timing(True)
        ts = []
        for r in range(reps + 1):
            ctx.build_cells(parts)
            ctx.sort()
            torch.cuda.synchronize()
            if r:
                ts.append(ctx.kernel_times()["sort_ms"])
        ctx.check()   # reads the cell count back
        nc = int(ctx.stats()["n_cells"])
        ctx.close()
        out[f"cell_target_{ct}"] = {"sort_ms": float(np.median(ts)), "cells": nc, "mean_per_cell": ps.n / nc}
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-plain", action="store_true", help="skip the FP64 (plain) form")
    ap.add_argument("--no-batched", action="store_true", help="skip the 256-box batched workload")
    ap.add_argument("--no-adjoint", action="store_true", help="skip the reverse-mode timing")
    ap.add_argument("--no-multires", action="store_true", help="skip the 2M-particle Plummer mixture")
    ap.add_argument("--no-integrate", action="store_true", help="skip the Sod time-integration timing")
    ap.add_argument("--no-mts", action="store_true", help="skip the multiple time-stepping timing")
    ap.add_argument("--no-layouts", action="store_true", help="skip the timing of the shared sweep layout")
    ap.add_argument("--no-orderings", action="store_true", help="skip the timing of big-cell orderings")
    ap.add_argument("--no-tune", action="store_true", help="default parameters for the headline pass (no autotuning)")
    ap.add_argument("--params", default="",
                    help="JSON object of sph_params fields for the headline pass in place of autotuning "
                         "(e.g. the 'tuned' values of an earlier line, so that a profiler sees no tuning)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: this build runs on one GPU; --gpus {args.gpus} is not supported", file=sys.stderr)
        sys.exit(2)
    import torch
    if not torch.cuda.is_available():
        print("bench.py: no GPU visible", file=sys.stderr)
        sys.exit(2)
    torch.cuda.set_device(0)
    ensure_built()
    from paper_1404_2303_amd import workloads
    ps = workloads.config1()
    log(f"workload: {ps.n} particles, box {ps.box.tolist()}")
    # the FP32 pass's decomposition and tiles, tuned on this workload (cached per class)
    params, tuned = {}, None
    if args.params:
        tuned = {k: v for k, v in json.loads(args.params).items() if k != "cached"}
        params = dict(tuned)
        tuned["given"] = True
        log("given:", json.dumps(params))
    elif not args.no_tune:
        from paper_1404_2303_amd import autotune
        arch = torch.cuda.get_device_properties(0).gcnArchName.split(":")[0]
        key = "grid|" + autotune.workload_class(ps.n, 1, "fp32")
        tuned = autotune.tune_staged(autotune.gpu_timer(ps, "fp32"), key, arch)
        params = {k: v for k, v in tuned.items() if k != "cached"}
        log("tuned:", json.dumps(tuned))
    fast = run_form(ps, "fp32", args.steps, args.warmup, **params)
    log("fp32_acc64:", json.dumps(fast))
    plain = None
    if not args.no_plain:
        plain = run_form(ps, "fp64", args.steps, args.warmup)
        log("fp64:", json.dumps(plain))
    graph = run_graph(ps, "fp32", args.steps, args.warmup, params=params)
    log("fp32 graph:", json.dumps(graph))
    rl = roofline(fast)
    # the chosen form: the captured FP32 pass when it is the faster one
    use_graph = graph["ms_per_step"] < fast["ms_per_step"] and graph["P"] == fast["P"]
    step_ms = graph["ms_per_step"] if use_graph else fast["ms_per_step"]
    value = fast["P"] / (step_ms * 1e-3)
    line = {
        "metric": METRIC,
        "value": value,
        "unit": "pair interactions/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": step_ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "jittered cubic lattice 128x128x64 (2^20 particles), spacing 1/128, "
                               "periodic 1x1x0.5 box, v~N(0,0.1), u=1; build+sort+density(h-Newton)+force",
                   "n": ps.n, "form": ("graph-captured pass, " if use_graph else "eager calls, ") +
                                       "fp32 pair arithmetic and per-list partial sums, fp64 totals and Newton step",
                   "eager_ms_per_step": fast["ms_per_step"], "graph_ms_per_step": graph["ms_per_step"],
                   "pairs_per_step": fast["P"], "kernel_ms": fast["kernel_ms"],
                   "newton_mean": fast["newton_mean"], "newton_max": fast["newton_max"],
                   "cells": fast["cells"], "grid": fast["grid"], "tuned": tuned,
                   "pair_kernel_rate": fast["P"] / ((fast["kernel_ms"]["density_ms"] + fast["kernel_ms"]["force_ms"]) * 1e-3)},
        "roofline": rl,
    }
    if plain is not None:
        line["plain_fp64"] = {"value": plain["P"] / (plain["ms_per_step"] * 1e-3), "ms_per_step": plain["ms_per_step"],
                              "kernel_ms": plain["kernel_ms"], "roofline": roofline(plain)}
    if not args.no_layouts:
        # the other sweep layout (sph_params.sweep) on the same workload, for the record
        from paper_1404_2303_amd import sph
        lay = {}
        for prec in ("fp32", "fp64"):
            r = run_form(ps, prec, max(3, args.steps // 4), 2, sweep=sph.SPH_SWEEP_SHARED)
            lay[prec] = {"ms_per_step": r["ms_per_step"], "kernel_ms": r["kernel_ms"], "P": r["P"]}
        line["sweep_shared"] = lay
        log("sweep_shared:", json.dumps(lay))
    if not args.no_orderings:
        line["orderings"] = orderings_section()
        log("orderings:", json.dumps(line["orderings"]))
    if not args.no_batched:
        line["batched"] = batched_section(max(3, args.steps // 4), 2)
        log("batched:", json.dumps(line["batched"]))
    if not args.no_multires:
        line["multires"] = multires_section(max(3, args.steps // 2), 1)
        log("multires:", json.dumps(line["multires"]))
    if not args.no_integrate:
        line["integrate"] = integrate_section(max(5, args.steps // 2), 2)
        log("integrate:", json.dumps(line["integrate"]))
    if not args.no_mts:
        line["mts"] = mts_section(64)
        log("mts:", json.dumps(line["mts"]))
    if not args.no_adjoint:
        line["adjoint"] = adjoint_section(args.steps, args.warmup)
        log("adjoint:", json.dumps(line["adjoint"]))
    if not args.no_cpu:
        line["cpu_baseline"] = cpu_baseline()
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
