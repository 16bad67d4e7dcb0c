"""Writes sedov_sample.txt: FP64 oracle values at 64 sampled particles of the
Sedov blast of the bench (workloads.sedov(63): 1,000,188 particles on a
face-centred cubic lattice, energy on the 28 central particles, Balsara switch
of the |div v| form), half uniformly over the box and half within 0.05 of its
centre.

Calls only the oracle (h solved for every particle, then density for all and
the force stage and the time step of Eq. (6) on the sample).
Run from the repository root: python tests/golden/make_sedov_sample.py
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

def sample_indices(ps, k=64, seed=4):
    rng = np.random.default_rng(seed)
    near = np.where(np.linalg.norm(ps.pos - 0.5 * ps.box, axis=1) < 0.05)[0]
    a = rng.choice(ps.n, k // 2, replace=False)
    b = rng.choice(near, k // 2, replace=False)
    return np.unique(np.concatenate([a, b]))


def main():
    ps = workloads.sedov(63)
    sel = sample_indices(ps)
    out = oracle.full_pass(ps.pos, ps.vel, ps.m, ps.u, ps.h0, ps.box, tol=1e-12, force_sel=sel, balsara_form=1,
                           gamma=ps.meta["gamma"])
    cols, data = sample_columns.rows(ps, out, sel, signal=True)
    sample_columns.write(os.path.join(os.path.dirname(os.path.abspath(__file__)), "sedov_sample.txt"), cols, data)


if __name__ == "__main__":
    main()
