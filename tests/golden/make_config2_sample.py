"""Writes config2_sample.txt: FP64 oracle values at 64 sampled particles of the
2,097,152-particle Plummer mixture (workloads.config2(), seed 0).

Calls only the oracle (h solved for every particle, then density for all and
the force stage on the sample).  Takes several minutes on the CPU.
Run from the repository root: python tests/golden/make_config2_sample.py
"""
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)
sys.path.insert(0, os.path.dirname(os.path.abspath(__file__)))

import oracle  # noqa: E402
import sample_columns  # noqa: E402
from paper_1404_2303_amd import workloads  # noqa: E402

def sample_indices(n, k=64, seed=2):
    """Half uniformly over all particles, half over the cluster particles (index < n_spheres * n_per)."""
    rng = np.random.default_rng(seed)
    a = rng.choice(n, k // 2, replace=False)
    b = rng.choice(32 * 52428, k // 2, replace=False)
    return np.unique(np.concatenate([a, b]))


def main():
    ps = workloads.config2()
    sel = sample_indices(ps.n)
    out = oracle.full_pass(ps.pos, ps.vel, ps.m, ps.u, ps.h0, ps.box, tol=1e-12, force_sel=sel)
    cols, data = sample_columns.rows(ps, out, sel, signal=False)
    sample_columns.write(os.path.join(os.path.dirname(os.path.abspath(__file__)), "config2_sample.txt"), cols, data)


if __name__ == "__main__":
    main()
