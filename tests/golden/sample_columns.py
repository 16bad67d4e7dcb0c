"""Columns of the sampled oracle values (config1/config2/Sod/Sedov samples).

Used only by the make_*_sample.py scripts, which call the oracle alone.  Per
sampled particle: the oracle's h, the density-stage quantities, the force
stage (a, du/dt, their pair-term magnitude sums kappa and h sensitivities
sens), the neighbour counts of both stages, and the count bands of each
precision form: the pairs whose r/h lies within the precision to which that
form solves h (oracle.h_precision), which may fall on either side of the
support (Eq. (2)'s strict r < h).
"""
import numpy as np

import oracle

# precision of h of each form: (relative h tolerance, tolerance on N)
H_PRECISION = {"fp32": (2e-6, 2e-4), "fp64": (1e-9, 1e-8)}

BASE = ["index", "h", "rho", "omega", "div", "curl_x", "curl_y", "curl_z", "f", "P", "c",
        "ax", "ay", "az", "dudt", "kappa_a", "kappa_u", "sens_a", "sens_u", "count", "n_dens", "dndh",
        "dband_fp32", "fband_fp32", "dband_fp64", "fband_fp64"]
SIGNAL = ["dt", "vsig_lo", "vsig_hi"]


def rows(ps, out, sel, signal=False):
    """(column names, rows) of the sample sel from an oracle.full_pass output."""
    d, g, f = out["dens"], out["ghost"], out["force"]
    cols = list(BASE)
    data = [sel, out["h"][sel], d["rho"][sel], g["omega"][sel], d["div"][sel], d["curl"][sel],
            g["f"][sel], g["P"][sel], g["c"][sel], f["a"][sel], f["dudt"][sel], f["kappa_a"][sel],
            f["kappa_u"][sel], f["sens_a"][sel], f["sens_u"][sel], f["count"][sel], d["count"][sel],
            d["dndh"][sel]]
    for prec in ("fp32", "fp64"):
        h_rel, ngb = H_PRECISION[prec]
        width = oracle.h_precision(out["h"], d["dndh"], h_rel, ngb)
        b = oracle.bands(ps.pos, out["h"], ps.box, width, sel=sel)
        data += [b["dband"][sel], b["fband"][sel]]
    if signal:
        s = out["signal"]
        cols += SIGNAL
        data += [s["dt"][sel], s["vsig_lo"][sel], s["vsig_hi"][sel]]
    return cols, np.column_stack(data)


def write(path, cols, data):
    np.savetxt(path, data, fmt="%.17g", header=" ".join(cols))
    print("wrote", path, data.shape)


def load(path):
    """Column name -> array of a sample file."""
    ref = np.loadtxt(path, ndmin=2)
    cols = open(path).readline().lstrip("# ").split()
    return {c: ref[:, k] for k, c in enumerate(cols)}
