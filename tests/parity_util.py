"""Helpers of the GPU parity tests: run the HIP path through the C ABI and
compare it with the FP64 oracle under the tolerances stated here.

Tolerances (derived from the arithmetic of each form):

FP64 form -- both sides solve N_i(h_i) = 48 to 1e-10 and differ only in
summation order: h, rho, P, c relative 1e-9; Omega, f absolute 1e-9;
div, curl 1e-9 of their RMS; a, du/dt 1e-9 of kappa (the sum of the
magnitudes of the pair contributions, the natural scale of a cancelling sum).

FP32 form -- pair terms in FP32 (unit roundoff 6e-8, ~10 roundings per term,
so about 1e-6 per term), sums in FP64 (each reached through FP32 partial sums
over one neighbour list, of at most 48 pairs in the density stage and 32 in
the force stage: at most 48 x 6e-8 ~ 3e-6 of the summed magnitudes, the size
of the per-term error already allowed; the Newton decision sees at most
~3e-5 in N, inside its 1e-4 stopping band and the 2e-4 band below), and the
Newton iteration stops at
|N - 48| <= 1e-4, which moves h by at most ~1e-4/(h dN/dh) ~ 1e-4/144 ~ 7e-7
relative (more where h dN/dh is small, so h is also allowed the band
ngb/(h |dN/dh|) of each particle, ngb the tolerance on N).  Hence: h relative 2e-6;
rho, P, c relative 1e-5 (rho ~ h^-3 moves by 3 x 2e-6); Omega, f absolute
1e-5; a, du/dt 1e-5 of kappa.  The divergence and curl carry the prefactor
8/(pi h^5) and a sum whose terms move with h again, so their relative
sensitivity to h is up to ~8 and the h band alone moves them by up to
8 x 2e-6 = 1.6e-5: div, curl 3e-5 of (RMS + |value|).

The Balsara switch f = |curl| / (|div| + |curl| + eps c/h) moves by at most
(|d curl| + |d div|) / den, den its denominator, so besides its absolute
tolerance it is allowed the div and curl tolerance scaled that way:
vec (rms_div + rms_curl + |div| + |curl|) / den.

The h tolerance also reaches a and du/dt through the kernel gradients, most
where a pair sits near the edge of a support: w' vanishes there like (1-q)^2,
so the pair term moves by up to 2q/(1-q) times the relative change of h (a
particle whose force comes from one neighbour at q = 0.994 has a sensitivity
of ~300).  a and du/dt are therefore measured against kappa + (h tolerance /
a tolerance) sens, sens the oracle's sum of the magnitudes of the derivatives
of the pair terms with respect to ln h_i and ln h_j.

Neighbour counts (pairs with r < max(h_i, h_j)) must match exactly except
for pairs within 1e-6 relative of the support radius, which the oracle counts
per particle ("band").
"""
import numpy as np
import torch

import oracle
from paper_1404_2303_amd import sph

BALSARA_EPS = 1e-4

TOL = {
    "fp64": dict(h=1e-9, rho=1e-9, omega=1e-9, vec=1e-9, f=1e-9, a=1e-9, ngb=1e-8),
    "fp32": dict(h=2e-6, rho=1e-5, omega=1e-5, vec=3e-5, f=1e-5, a=1e-5, ngb=2e-4),
}


def log(msg):
    print(msg, flush=True)


def gpu_run(ps, precision, batch=None, estimate=False, **params):
    """One build -> sort -> density -> force pass through the C ABI; with
    estimate=True the initial h comes from sph_estimate_h (hierarchy only)."""
    parts = sph.Particles.from_numpy(ps, "cuda:0")
    box = ps.box if batch is None else (1.0, 1.0, 1.0)
    ctx = sph.Context(box, precision=precision, **params)
    b = None if batch is None else sph.Batch(*batch)
    if estimate:
        ctx.estimate_h(parts, b)
    d, f = ctx.run(parts, b)
    torch.cuda.synchronize()
    out = {k: v.cpu().numpy() for k, v in d.items()}
    out.update({k: v.cpu().numpy() for k, v in f.items()})
    out["h"] = parts.h.cpu().numpy()
    out["a"] = np.stack([out["ax"], out["ay"], out["az"]], axis=1)
    out["stats"] = ctx.stats()
    ctx.close()
    return out


def oracle_run(ps, tol=1e-10, force_sel=None):
    return oracle.full_pass(ps.pos, ps.vel, ps.m, ps.u, ps.h0, ps.box, tol=tol, force_sel=force_sel)


def compare(g, ref, precision, sel=None, force_sel=None, label=""):
    """Element-wise comparison; returns a dict of the worst normalised errors."""
    t = TOL[precision]
    n = len(g["h"])
    sel = np.arange(n) if sel is None else np.asarray(sel)
    fsel = sel if force_sel is None else np.asarray(force_sel)
    dens, gh, frc = ref["dens"], ref["ghost"], ref["force"]
    err = {}

    def rel(a, b):
        return np.max(np.abs(a / b - 1.0)) if len(a) else 0.0

    # h: the solves stop at |N - n_ngb| <= tol, so h is fixed to tol / |dN/dh|
    h_band = np.maximum(t["h"], t["ngb"] / (ref["h"][sel] * np.abs(dens["dndh"][sel])))
    err["h"] = np.max(np.abs(g["h"][sel] / ref["h"][sel] - 1.0) / h_band) * t["h"] if len(sel) else 0.0
    err["rho"] = rel(g["rho"][sel], dens["rho"][sel])
    err["P"] = rel(g["pressure"][sel], gh["P"][sel])
    err["c"] = rel(g["sound"][sel], gh["c"][sel])
    err["omega"] = np.max(np.abs(g["omega"][sel] - gh["omega"][sel]))
    rms_d = np.sqrt(np.mean(dens["div"][sel] ** 2))
    rms_c = np.sqrt(np.mean(np.sum(dens["curl"][sel] ** 2, axis=1)))
    cm = np.linalg.norm(dens["curl"][sel], axis=1)
    den = np.abs(dens["div"][sel]) + cm + BALSARA_EPS * gh["c"][sel] / ref["h"][sel]
    f_bound = np.maximum(t["f"], t["vec"] * (rms_d + rms_c + np.abs(dens["div"][sel]) + cm) / den)
    err["f"] = np.max(np.abs(g["balsara"][sel] - gh["f"][sel]) / f_bound) * t["f"]
    err["ngb"] = np.max(np.abs(g["n_ngb"][sel] - 48.0))
    rms_div = np.sqrt(np.mean(dens["div"][sel] ** 2)) + 1e-300
    rms_curl = np.sqrt(np.mean(np.sum(dens["curl"][sel] ** 2, axis=1))) + 1e-300
    err["div"] = np.max(np.abs(g["div_v"][sel] - dens["div"][sel]) / (rms_div + np.abs(dens["div"][sel])))
    err["curl"] = np.max(np.linalg.norm(g["curl_v"][sel] - dens["curl"][sel], axis=1) /
                         (rms_curl + np.linalg.norm(dens["curl"][sel], axis=1)))
    ka = frc["kappa_a"][fsel] + t["h"] / t["a"] * frc["sens_a"][fsel] + 1e-300
    ku = frc["kappa_u"][fsel] + t["h"] / t["a"] * frc["sens_u"][fsel] + 1e-300
    err["a"] = np.max(np.linalg.norm(g["a"][fsel] - frc["a"][fsel], axis=1) / ka)
    err["dudt"] = np.max(np.abs(g["dudt"][fsel] - frc["dudt"][fsel]) / ku)
    dc = np.abs(g["n_pairs"][fsel].astype(np.int64) - frc["count"][fsel])
    err["count_excess"] = int(np.max(dc - frc["band"][fsel])) if len(fsel) else 0
    log(f"[{label} {precision}] " + " ".join(f"{k}={v:.2e}" if isinstance(v, float) else f"{k}={v}"
                                            for k, v in err.items()))
    assert err["h"] <= t["h"], err
    assert err["rho"] <= t["rho"] and err["P"] <= t["rho"] and err["c"] <= t["rho"], err
    assert err["omega"] <= t["omega"] and err["f"] <= t["f"], err
    assert err["ngb"] <= t["ngb"], err
    assert err["div"] <= t["vec"] and err["curl"] <= t["vec"], err
    assert err["a"] <= t["a"] and err["dudt"] <= t["a"], err
    assert err["count_excess"] <= 0, err
    return err
