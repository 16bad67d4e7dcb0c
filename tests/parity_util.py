"""Helpers of the GPU parity tests: run the HIP path through the C ABI and
compare it with the FP64 oracle under the tolerances stated here.

Tolerances (derived from the arithmetic of each form):

FP64 form -- both sides solve N_i(h_i) = 48 to 1e-10 and differ only in
summation order: h, rho, P, c relative 1e-9; Omega, f absolute 1e-9;
div, curl 1e-9 of their RMS; a, du/dt 1e-9 of the quantity (below).

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
1e-5; a, du/dt 1e-5 of the quantity (below).  The divergence and curl carry the prefactor
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
of ~300).  a and du/dt are therefore measured against

    |a_gpu - a_ora| <= tol_a * max(|a_ora,i|, RMS a_ora) + dh * sens_i,

tol_a the tolerance of the arithmetic (1e-5 in FP32, 1e-9 in FP64) relative to
the quantity itself (the RMS over the compared particles stands in where |a_i|
is small), dh the largest relative difference between the GPU's and the
oracle's h over the compared particles (each within its own tolerance above),
and sens_i the oracle's sum of the magnitudes of the derivatives of i's pair
terms with respect to ln h_i and ln h_j: the reach of the h difference into
a.  The error relative to kappa (the sum of the magnitudes of the pair terms,
the scale of a cancelling sum) is logged as a diagnostic.

Neighbour counts of both stages (density: r < h_i; force: r < max(h_i, h_j))
must match exactly except for pairs whose r/h lies within the precision to
which the form solves h (at least 1e-6), which the oracle counts per
particle ("bands"): a pair that close to the support may fall either way.
"""
import numpy as np
import torch

import os
import sys

import oracle
from paper_1404_2303_amd import sph

sys.path.insert(0, os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden"))
import sample_columns  # noqa: E402

load_sample = sample_columns.load

BALSARA_EPS = 1e-4

TOL = {
    "fp64": dict(h=1e-9, rho=1e-9, omega=1e-9, vec=1e-9, f=1e-9, a=1e-9, ngb=1e-8),
    "fp32": dict(h=2e-6, rho=1e-5, omega=1e-5, vec=3e-5, f=1e-5, a=1e-5, ngb=2e-4),
}
# the sample files carry the count bands of these h precisions
assert all(sample_columns.H_PRECISION[k] == (v["h"], v["ngb"]) for k, v in TOL.items())


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


def oracle_run(ps, tol=1e-10, force_sel=None, target=48.0, h0=None, **kw):
    """The oracle's full pass (initial h: ps.h0 unless h0 is given; keyword
    arguments go to oracle.full_pass), and the count bands of both precision
    forms."""
    ref = oracle.full_pass(ps.pos, ps.vel, ps.m, ps.u, ps.h0 if h0 is None else h0, ps.box, tol=tol,
                           force_sel=force_sel, target=target, **kw)
    ref["target"] = target
    ref["bands"] = {}
    for prec, t in TOL.items():
        width = oracle.h_precision(ref["h"], ref["dens"]["dndh"], t["h"], t["ngb"])
        ref["bands"][prec] = oracle.bands(ps.pos, ref["h"], ps.box, width,
                                          sel=force_sel if force_sel is not None else None)
    return ref


def force_errors(a_gpu, du_gpu, a_ref, du_ref, kappa_a, kappa_u, sens_a, sens_u, dh, t_a):
    """Errors of a and du/dt in units of their bounds (<= 1 passes), and the
    same errors relative to kappa (diagnostic)."""
    na = np.linalg.norm(a_ref, axis=1)
    rms_a = np.sqrt(np.mean(na ** 2))
    rms_u = np.sqrt(np.mean(du_ref ** 2))
    ba = t_a * np.maximum(na, rms_a) + dh * sens_a + 1e-300
    bu = t_a * np.maximum(np.abs(du_ref), rms_u) + dh * sens_u + 1e-300
    ea = np.linalg.norm(a_gpu - a_ref, axis=1)
    eu = np.abs(du_gpu - du_ref)
    return {"a": float(np.max(ea / ba)), "dudt": float(np.max(eu / bu)),
            "a_rel": float(np.max(ea / np.maximum(na, rms_a + 1e-300))),
            "a/kappa": float(np.max(ea / (kappa_a + 1e-300))),
            "dudt/kappa": float(np.max(eu / (kappa_u + 1e-300)))}


def _log_errors(label, precision, err):
    log(f"[{label} {precision}] " + " ".join(f"{k}={v:.2e}" if isinstance(v, float) else f"{k}={v}"
                                            for k, v in err.items()))


def compare(g, ref, precision, sel=None, force_sel=None, label=""):
    """Element-wise comparison; returns a dict of the worst normalised errors."""
    t = TOL[precision]
    n = len(g["h"])
    sel = np.arange(n) if sel is None else np.asarray(sel)
    fsel = sel if force_sel is None else np.asarray(force_sel)
    dens, gh, frc = ref["dens"], ref["ghost"], ref["force"]
    bands = ref["bands"][precision]
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
    err["ngb"] = np.max(np.abs(g["n_ngb"][sel] - ref.get("target", 48.0)))
    rms_div = np.sqrt(np.mean(dens["div"][sel] ** 2)) + 1e-300
    rms_curl = np.sqrt(np.mean(np.sum(dens["curl"][sel] ** 2, axis=1))) + 1e-300
    err["div"] = np.max(np.abs(g["div_v"][sel] - dens["div"][sel]) / (rms_div + np.abs(dens["div"][sel])))
    err["curl"] = np.max(np.linalg.norm(g["curl_v"][sel] - dens["curl"][sel], axis=1) /
                         (rms_curl + np.linalg.norm(dens["curl"][sel], axis=1)))
    dh = float(np.max(np.abs(g["h"][fsel] / ref["h"][fsel] - 1.0))) if len(fsel) else 0.0
    err["dh"] = dh
    err.update(force_errors(g["a"][fsel], g["dudt"][fsel], frc["a"][fsel], frc["dudt"][fsel], frc["kappa_a"][fsel],
                            frc["kappa_u"][fsel], frc["sens_a"][fsel], frc["sens_u"][fsel], dh, t["a"]))
    dc = np.abs(g["n_pairs"][fsel].astype(np.int64) - frc["count"][fsel])
    err["count_excess"] = int(np.max(dc - bands["fband"][fsel])) if len(fsel) else 0
    if "n_dens" in g:
        dd = np.abs(g["n_dens"][sel].astype(np.int64) - dens["count"][sel])
        err["dcount_excess"] = int(np.max(dd - bands["dband"][sel])) if len(sel) else 0
    _log_errors(label, precision, err)
    assert err["h"] <= t["h"], err
    assert err["rho"] <= t["rho"] and err["P"] <= t["rho"] and err["c"] <= t["rho"], err
    assert err["omega"] <= t["omega"] and err["f"] <= t["f"], err
    assert err["ngb"] <= t["ngb"], err
    assert err["div"] <= t["vec"] and err["curl"] <= t["vec"], err
    assert err["a"] <= 1.0 and err["dudt"] <= 1.0, err
    assert err["count_excess"] <= 0, err
    assert err.get("dcount_excess", 0) <= 0, err
    return err


def compare_sample(g, R, precision, label="", idx=None):
    """The GPU outputs at the oracle's sampled particles (a sample file read by
    sample_columns.load) under the same tolerances as compare()."""
    t = TOL[precision]
    idx = R["index"].astype(np.int64) if idx is None else idx
    e = {}
    h_band = np.maximum(t["h"], t["ngb"] / (R["h"] * np.abs(R["dndh"])))
    e["h"] = float(np.max(np.abs(g["h"][idx] / R["h"] - 1) / h_band) * t["h"])
    e["rho"] = float(np.max(np.abs(g["rho"][idx] / R["rho"] - 1)))
    if "pressure" in g:
        e["P"] = float(np.max(np.abs(g["pressure"][idx] / R["P"] - 1)))
        e["c"] = float(np.max(np.abs(g["sound"][idx] / R["c"] - 1)))
    e["omega"] = float(np.max(np.abs(g["omega"][idx] - R["omega"])))
    e["f"] = float(np.max(np.abs(g["balsara"][idx] - R["f"])))
    rd = np.sqrt(np.mean(R["div"] ** 2)) + 1e-300
    e["div"] = float(np.max(np.abs(g["div_v"][idx] - R["div"]) / (rd + np.abs(R["div"]))))
    if "curl_v" in g:
        curl = np.stack([R["curl_x"], R["curl_y"], R["curl_z"]], 1)
        rc = np.sqrt(np.mean(np.sum(curl ** 2, 1))) + 1e-300
        e["curl"] = float(np.max(np.linalg.norm(g["curl_v"][idx] - curl, axis=1) / (rc + np.linalg.norm(curl, axis=1))))
    dh = float(np.max(np.abs(g["h"][idx] / R["h"] - 1)))
    e["dh"] = dh
    a = np.stack([R["ax"], R["ay"], R["az"]], 1)
    e.update(force_errors(g["a"][idx], g["dudt"][idx], a, R["dudt"], R["kappa_a"], R["kappa_u"], R["sens_a"],
                          R["sens_u"], dh, t["a"]))
    e["count"] = int(np.max(np.abs(g["n_pairs"][idx] - R["count"]) - R[f"fband_{precision}"]))
    if "n_dens" in g:
        e["dcount"] = int(np.max(np.abs(g["n_dens"][idx] - R["n_dens"]) - R[f"dband_{precision}"]))
    _log_errors(label, precision, e)
    assert e["h"] <= t["h"] and e["rho"] <= t["rho"] and e["omega"] <= t["omega"] and e["f"] <= t["f"], e
    assert e.get("P", 0.0) <= t["rho"] and e.get("c", 0.0) <= t["rho"], e
    assert e["div"] <= t["vec"] and e.get("curl", 0.0) <= t["vec"], e
    assert e["a"] <= 1.0 and e["dudt"] <= 1.0, e
    assert e["count"] <= 0 and e.get("dcount", 0) <= 0, e
    return e
