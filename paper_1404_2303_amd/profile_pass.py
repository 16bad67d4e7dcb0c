"""Runs whole passes (build, sort, density, force) of a named workload, for
profilers (rocprofv3 --kernel-trace / --pmc) to record.

    python -m paper_1404_2303_amd.profile_pass --workload lattice --passes 2 --copy-mib 512
    python -m paper_1404_2303_amd.profile_pass --workload lattice --params '{"h_margin": 0.05}'
    python -m paper_1404_2303_amd.profile_pass --workload sod --steps 20 --reuse 1
    python -m paper_1404_2303_amd.profile_pass --workload sedov --steps 64 --reuse 1

--copy-mib adds device-to-device copies of that size after the passes, a
kernel of known traffic that calibrates the memory counters.  The sod
workload (the shock tube at 1,013,060 particles) runs --steps adaptive
kick-drift-kick steps instead, with the decomposition reuse mode --reuse;
the sedov workload (the blast wave at 1,000,188 particles) runs --steps base
steps of multiple time-stepping (bins up to 2^10 of the smallest initial
time step).
"""
from __future__ import annotations

import argparse
import json


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--workload", choices=("lattice", "mixture", "lattice64", "sod", "sedov"), default="lattice")
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--reuse", type=int, default=0)
    ap.add_argument("--precision", choices=("fp32", "fp64"), default="fp32")
    ap.add_argument("--passes", type=int, default=2)
    ap.add_argument("--copy-mib", type=int, default=0)
    ap.add_argument("--shared-min", type=int, default=128,
                    help="cells of more particles than this are swept shared (sph_params.shared_min)")
    ap.add_argument("--staging", choices=("compact", "wide"), default="compact",
                    help="density staging of the lattice and mixture workloads (sph_params.staging)")
    ap.add_argument("--walk-counts", action="store_true",
                    help="lattice or mixture: run the counting build (build_lib --count) and print the candidates "
                         "the density and force walks test and the list entries they keep, per pass")
    ap.add_argument("--params", default="",
                    help="JSON object of further sph_params fields for the lattice and mixture workloads, "
                         "e.g. the tuned values a bench line reports; they override the options above")
    args = ap.parse_args()
    import time

    import torch
    from . import sph, workloads
    if args.walk_counts:
        from . import build_lib
        sph.LIB_PATH = build_lib.COUNT_LIB
    if args.workload == "sod":
        ps = workloads.sod(37)
        parts = sph.Particles.from_numpy(ps, "cuda:0")
        ctx = sph.Context(ps.box, precision=args.precision, balsara_form=sph.SPH_BALSARA_DIV, reuse=args.reuse,
                          staging=sph.SPH_STAGING_WIDE)
        d, acc = ctx.run(parts)
        t_box = torch.zeros(1, dtype=torch.float64, device="cuda:0")
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            ctx.step_adaptive(parts, acc, t_box, 1e30, 1.0)
        torch.cuda.synchronize()
        print(f"{args.steps} steps, {1e3 * (time.perf_counter() - t0) / args.steps:.3f} ms per step", flush=True)
        ctx.close()
        print("passes done", flush=True)
        return
    if args.workload == "sedov":
        ps = workloads.sedov(63)
        parts = sph.Particles.from_numpy(ps, "cuda:0")
        ctx = sph.Context(ps.box, precision=args.precision, balsara_form=sph.SPH_BALSARA_DIV, reuse=args.reuse)
        d, f = ctx.run(parts)
        dtb = float(f["dt"].min().item())
        acc, bins = ctx.mts_init(parts, dtb, 10)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            ctx.mts_step(parts, acc, bins)
        torch.cuda.synchronize()
        print(f"{args.steps} base steps, {1e3 * (time.perf_counter() - t0) / args.steps:.3f} ms per base step",
              flush=True)
        ctx.close()
        print("passes done", flush=True)
        return
    if args.workload == "lattice":
        ps, params = workloads.config1(), {}
    elif args.workload == "lattice64":
        ps, params = workloads.config4(), {}
    else:
        ps, params = workloads.config2(), {"max_depth": 10, "split_count": 256}
    parts = sph.Particles.from_numpy(ps, "cuda:0")
    staging = sph.SPH_STAGING_WIDE if args.staging == "wide" else sph.SPH_STAGING_COMPACT
    params = dict(params, shared_min=args.shared_min, staging=staging)
    if args.params:
        params.update({k: v for k, v in json.loads(args.params).items() if k != "cached"})
    print("params:", json.dumps(params), flush=True)
    ctx = sph.Context(ps.box, precision=args.precision, **params)
    if args.workload == "mixture":
        ctx.estimate_h(parts)
        ctx.run(parts)
    h0 = parts.h.clone()
    if args.walk_counts:
        import ctypes
        lib = sph.load_library()
        lib.sph_walk_tally.restype = ctypes.c_int
        lib.sph_walk_tally.argtypes = [ctypes.c_void_p, ctypes.c_int]
        tally = (ctypes.c_ulonglong * 4)()
        ctx.run(parts)   # the same start as the passes below
        torch.cuda.synchronize()
        parts.h.copy_(h0)
        lib.sph_walk_tally(tally, 1)
        d, f = ctx.run(parts)
        torch.cuda.synchronize()
        if lib.sph_walk_tally(tally, 1) != 0:
            raise RuntimeError("sph_walk_tally failed")
        sides = int(d["n_dens"].sum().item())      # pairs with r < h_i, one per target side
        pairs = int(f["n_pairs"].sum().item())      # pairs with r < max(h_i, h_j), counted from both sides
        out = {"density_tests": tally[0], "density_list_entries": tally[1], "force_tests": tally[2],
               "force_list_entries": tally[3], "density_sides": sides, "force_pairs_both_sides": pairs,
               "density_tests_per_side": tally[0] / max(sides, 1),
               "force_tests_per_pair_side": tally[2] / max(pairs, 1)}
        print(json.dumps(out), flush=True)
        ctx.close()
        print("passes done", flush=True)
        return
    for _ in range(args.passes):
        parts.h.copy_(h0)
        ctx.run(parts)
    torch.cuda.synchronize()
    if args.copy_mib > 0:
        x = torch.ones(args.copy_mib * 1024 * 1024 // 4, dtype=torch.float32, device="cuda:0")
        y = torch.empty_like(x)
        for _ in range(2):
            y.copy_(x)
        torch.cuda.synchronize()
    ctx.close()
    print("passes done", flush=True)


if __name__ == "__main__":
    main()
