"""Runs whole passes (build, sort, density, force) of a named workload, for
profilers (rocprofv3 --kernel-trace / --pmc) to record.

    python -m paper_1404_2303_amd.profile_pass --workload lattice --passes 2 --copy-mib 512

--copy-mib adds device-to-device copies of that size after the passes, a
kernel of known traffic that calibrates the memory counters.
"""
from __future__ import annotations

import argparse


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--workload", choices=("lattice", "mixture", "lattice64"), default="lattice")
    ap.add_argument("--precision", choices=("fp32", "fp64"), default="fp32")
    ap.add_argument("--passes", type=int, default=2)
    ap.add_argument("--copy-mib", type=int, default=0)
    args = ap.parse_args()
    import torch
    from . import sph, workloads
    if args.workload == "lattice":
        ps, params = workloads.config1(), {}
    elif args.workload == "lattice64":
        ps, params = workloads.config4(), {}
    else:
        ps, params = workloads.config2(), {"max_depth": 10, "split_count": 256}
    parts = sph.Particles.from_numpy(ps, "cuda:0")
    ctx = sph.Context(ps.box, precision=args.precision, **params)
    if args.workload == "mixture":
        ctx.estimate_h(parts)
        ctx.run(parts)
    h0 = parts.h.clone()
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
