"""GPU parity of sph_step (kick-drift-kick, Sec. 4.1) against the oracle's
kdk_step, and the step's invariants on the GPU.

Tolerances.  A step moves v by dt/2 (a_old + a_new) and u likewise, so the
velocity error of a step is dt times the error of a (a fraction of kappa, the
sum of the magnitudes of a's pair terms: 1e-9 in FP64, 1e-5 in FP32) plus the
carried error; errors are measured against rms|v| + dt rms(kappa) per step
taken.  Positions move by dt v: their error is dt times the velocity error.
"""
import numpy as np
import pytest
import torch

import oracle
from paper_1404_2303_amd import sph, workloads
from parity_util import log

pytestmark = pytest.mark.gpu

TOL = {"fp64": 1e-8, "fp32": 1e-4}


def _state(n=2000, seed=41):
    rng = np.random.default_rng(seed)
    ps = workloads.uniform(n, seed=seed, sigma_v=0.4)
    ps.m[:] *= rng.uniform(0.6, 1.4, n)
    ps.u[:] = rng.uniform(0.5, 1.5, n)
    return ps


def _gpu_steps(ps, precision, dt, nsteps, batch=None):
    parts = sph.Particles.from_numpy(ps, "cuda:0")
    box = ps.box if batch is None else (1.0, 1.0, 1.0)
    ctx = sph.Context(box, precision=precision)
    b = None if batch is None else sph.Batch(*batch)
    d, f = ctx.run(parts, b)
    acc = {k: f[k] for k in ("ax", "ay", "az", "dudt")}
    out = []
    for _ in range(nsteps):
        ctx.step(parts, acc, dt, b)
        torch.cuda.synchronize()
        out.append({"pos": np.stack([parts.x.cpu().numpy(), parts.y.cpu().numpy(), parts.z.cpu().numpy()], 1),
                    "vel": np.stack([parts.vx.cpu().numpy(), parts.vy.cpu().numpy(), parts.vz.cpu().numpy()], 1),
                    "u": parts.u.cpu().numpy(), "h": parts.h.cpu().numpy()})
    ctx.close()
    return out


def _oracle_steps(ps, dt, nsteps):
    f = oracle.full_pass(ps.pos, ps.vel, ps.m, ps.u, ps.h0, ps.box)
    pos, vel, u, h, a, du = ps.pos, ps.vel, ps.u, f["h"], f["force"]["a"], f["force"]["dudt"]
    kap = f["force"]["kappa_a"]
    out = []
    for _ in range(nsteps):
        s = oracle.kdk_step(pos, vel, ps.m, u, h, ps.box, a, du, dt)
        pos, vel, u, h, a, du = s["pos"], s["vel"], s["u"], s["h"], s["a"], s["dudt"]
        out.append(s)
    return out, kap


def _compare(g, r, box, dt, k, kap, precision, label):
    vs = np.sqrt(np.mean(np.sum(r["vel"] ** 2, 1))) + k * dt * np.sqrt(np.mean(kap ** 2))
    ev = np.max(np.abs(g["vel"] - r["vel"])) / vs
    d = g["pos"] - r["pos"]
    d -= box * np.rint(d / box)
    ex = np.max(np.abs(d)) / (dt * vs)
    eu = np.max(np.abs(g["u"] - r["u"])) / (np.sqrt(np.mean(r["u"] ** 2)) + k * dt * np.sqrt(np.mean(kap ** 2)))
    eh = np.max(np.abs(g["h"] / r["h"] - 1.0))
    log(f"  [{label} step {k}] v {ev:.2e} x {ex:.2e} u {eu:.2e} h {eh:.2e}")
    t = TOL[precision]
    assert ev <= t and ex <= t and eu <= t, (ev, ex, eu)
    assert eh <= (1e-9 if precision == "fp64" else 2e-6)
    assert np.all(g["pos"] >= 0.0) and np.all(g["pos"] < box)


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_three_steps_match_oracle(precision):
    ps = _state()
    dt = 0.004
    log(f"case kdk 3 steps 2000 {precision}")
    g = _gpu_steps(ps, precision, dt, 3)
    r, kap = _oracle_steps(ps, dt, 3)
    for k in range(3):
        _compare(g[k], r[k], ps.box, dt, k + 1, kap, precision, "kdk")


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_lattice_at_rest_stays_at_rest(precision):
    ps = workloads.lattice((12, 12, 12), 1.0 / 12, jitter=0.0, sigma_v=0.0)
    log(f"case lattice at rest {precision}")
    ref = oracle.full_pass(ps.pos, ps.vel, ps.m, ps.u, ps.h0, ps.box)
    kap = np.max(ref["force"]["kappa_a"])
    dt = 0.01
    g = _gpu_steps(ps, precision, dt, 3)
    tol = 1e-12 if precision == "fp64" else 1e-5
    for k, s in enumerate(g, start=1):
        vmax = np.max(np.abs(s["vel"]))
        d = s["pos"] - ps.pos
        d -= ps.box * np.rint(d / ps.box)
        log(f"  step {k}: max|v| {vmax:.2e} max|dx| {np.max(np.abs(d)):.2e} (dt kappa {dt * kap:.2e})")
        assert vmax <= tol * k * dt * kap
        assert np.max(np.abs(d)) <= tol * k * k * dt * dt * kap


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_momentum_is_conserved(precision):
    ps = _state(3000, 43)
    log(f"case momentum 3000 {precision}")
    ref = oracle.full_pass(ps.pos, ps.vel, ps.m, ps.u, ps.h0, ps.box)
    skap = np.sum(ps.m * ref["force"]["kappa_a"])
    p0 = np.sum(ps.m[:, None] * ps.vel, 0)
    dt = 0.004
    g = _gpu_steps(ps, precision, dt, 4)
    tol = 1e-12 if precision == "fp64" else 1e-6
    for k, s in enumerate(g, start=1):
        dp = np.max(np.abs(np.sum(ps.m[:, None] * s["vel"], 0) - p0))
        log(f"  step {k}: |dp| {dp:.2e} (dt sum m kappa {dt * skap:.2e})")
        assert dp <= tol * k * dt * skap


def test_batched_step_matches_per_box_oracle():
    # three boxes of different shapes and counts, with velocities, stepped together
    boxes = [(1.0, 1.0, 1.0), (0.8, 1.0, 0.9), (1.2, 0.9, 1.0)]
    sets = [workloads.uniform(n, seed=60 + b, box=bx, sigma_v=0.3) for b, (n, bx) in
            enumerate(zip((1500, 2600, 4000), boxes))]
    offsets = np.concatenate([[0], np.cumsum([s_.n for s_ in sets])]).astype(np.int64)
    lens = np.asarray(boxes, dtype=np.float64)
    cat = workloads.ParticleSet(pos=np.concatenate([s_.pos for s_ in sets]),
                                vel=np.concatenate([s_.vel for s_ in sets]),
                                m=np.concatenate([s_.m for s_ in sets]), u=np.concatenate([s_.u for s_ in sets]),
                                h0=np.concatenate([s_.h0 for s_ in sets]), box=np.ones(3))
    log(f"case batched kdk step {cat.n} in 3 boxes")
    dt = 0.004
    g = _gpu_steps(cat, "fp64", dt, 2, batch=(offsets, lens))
    for b, sub in enumerate(sets):
        s, e = offsets[b], offsets[b + 1]
        r, kap = _oracle_steps(sub, dt, 2)
        for k in range(2):
            gb = {key: v[s:e] for key, v in g[k].items()}
            _compare(gb, r[k], sub.box, dt, k + 1, kap, "fp64", f"box{b}")
