"""Writes config1_sample.txt: FP64 oracle values at 64 sampled particles of the
2^20-particle jittered lattice of the bench line (workloads.config1(), seed 0).

Calls only the oracle (h solved for every particle, then density for all and
the force stage on the sample).  Takes a few minutes on the CPU.
Run from the repository root: python tests/golden/make_config1_sample.py
"""
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_1404_2303_amd import workloads  # noqa: E402

COLUMNS = ["index", "h", "rho", "omega", "div", "curl_x", "curl_y", "curl_z", "f", "P", "c",
           "ax", "ay", "az", "dudt", "kappa_a", "kappa_u", "count", "band", "n_dens", "dndh"]


def sample_indices(n, k=64, seed=3):
    rng = np.random.default_rng(seed)
    return np.unique(rng.choice(n, k, replace=False))


def main():
    ps = workloads.config1()
    sel = sample_indices(ps.n)
    out = oracle.full_pass(ps.pos, ps.vel, ps.m, ps.u, ps.h0, ps.box, tol=1e-12, force_sel=sel)
    d, g, f = out["dens"], out["ghost"], out["force"]
    rows = np.column_stack([sel, out["h"][sel], d["rho"][sel], g["omega"][sel], d["div"][sel], d["curl"][sel],
                            g["f"][sel], g["P"][sel], g["c"][sel], f["a"][sel], f["dudt"][sel], f["kappa_a"][sel],
                            f["kappa_u"][sel], f["count"][sel], f["band"][sel], d["count"][sel], d["dndh"][sel]])
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "config1_sample.txt")
    np.savetxt(path, rows, fmt="%.17g", header=" ".join(COLUMNS))
    print("wrote", path, rows.shape)


if __name__ == "__main__":
    main()
