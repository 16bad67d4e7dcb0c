"""Pins of the oracle's kick-drift-kick step (Sec. 4.1: velocity Verlet with
a fixed time step): symmetric states that must not move, exact translation,
momentum conservation, and second-order convergence of the energy error."""
import numpy as np
import pytest

import oracle
from paper_1404_2303_amd import workloads


def _lattice(k=8, v0=(0.0, 0.0, 0.0)):
    ps = workloads.lattice((k, k, k), 1.0 / k, jitter=0.0, sigma_v=0.0)
    ps.vel[:] = np.asarray(v0)
    return ps


def _run(ps, dt, nsteps, alpha=oracle.ALPHA):
    pos, vel, u, h = ps.pos.copy(), ps.vel.copy(), ps.u.copy(), ps.h0.copy()
    f = oracle.full_pass(pos, vel, ps.m, u, h, ps.box, alpha=alpha)
    a, du, h = f["force"]["a"], f["force"]["dudt"], f["h"]
    states = []
    for _ in range(nsteps):
        s = oracle.kdk_step(pos, vel, ps.m, u, h, ps.box, a, du, dt, alpha=alpha)
        pos, vel, u, h, a, du = s["pos"], s["vel"], s["u"], s["h"], s["a"], s["dudt"]
        states.append(s)
    return states


def test_lattice_at_rest_stays_at_rest():
    ps = _lattice()
    x0 = ps.pos.copy()
    for s in _run(ps, 0.01, 3):
        assert np.max(np.abs(s["vel"])) < 1e-12
        d = s["pos"] - x0
        d -= ps.box * np.rint(d / ps.box)
        assert np.max(np.abs(d)) < 1e-14
        assert np.max(np.abs(s["u"] - 1.0)) < 1e-12


def test_uniform_translation_moves_rigidly():
    # every pair has v_ij = 0, so no force, no heating: x(t) = x0 + v0 t
    v0 = np.array([0.3, -0.7, 0.45])
    ps = _lattice(v0=v0)
    dt = 0.01
    for k, s in enumerate(_run(ps, dt, 4), start=1):
        d = s["pos"] - (ps.pos + v0 * dt * k)
        d -= ps.box * np.rint(d / ps.box)
        assert np.max(np.abs(d)) < 1e-13
        assert np.max(np.abs(s["vel"] - v0)) < 1e-12
        assert np.all(s["pos"] >= 0.0) and np.all(s["pos"] < 1.0)


def test_momentum_is_conserved():
    rng = np.random.default_rng(3)
    ps = workloads.uniform(1500, seed=3, sigma_v=0.5)
    ps.m[:] *= rng.uniform(0.5, 1.5, ps.n)
    p0 = np.sum(ps.m[:, None] * ps.vel, axis=0)
    scale = np.sum(ps.m * np.linalg.norm(ps.vel, axis=1))
    for s in _run(ps, 0.005, 5):
        p = np.sum(ps.m[:, None] * s["vel"], axis=0)
        assert np.max(np.abs(p - p0)) < 1e-12 * scale


def test_energy_error_is_second_order():
    # without viscosity the total energy sum m (v^2/2 + u) is conserved by the
    # equations of motion; KDK leaves an O(dt^2) error at a fixed end time
    ps = workloads.lattice((8, 8, 8), 1.0 / 8, jitter=0.2, sigma_v=0.3, seed=5)
    E = lambda vel, u: np.sum(ps.m * (0.5 * np.sum(vel * vel, axis=1) + u))
    E0 = E(ps.vel, ps.u)
    T = 0.08
    errs = []
    for nsteps in (8, 16):
        s = _run(ps, T / nsteps, nsteps, alpha=0.0)[-1]
        errs.append(abs(E(s["vel"], s["u"]) - E0))
    ratio = errs[0] / errs[1]
    assert errs[0] > 0 and 3.0 < ratio < 5.5, (errs, ratio)
