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


# ---------------------------------------------------------------- multiple time-stepping
def test_time_bins():
    dtb = 0.01
    dt = np.array([0.005, 0.01, 0.0199, 0.02, 0.05, 1.0, np.inf])
    np.testing.assert_array_equal(oracle.time_bin(dt, dtb, 4, 0), [0, 0, 0, 1, 2, 4, 4])
    # a step must start on a multiple of its length: at base step 6, bin 2 (4 steps) is not allowed
    np.testing.assert_array_equal(oracle.time_bin(np.array([0.05, 0.02]), dtb, 4, 6), [1, 1])
    np.testing.assert_array_equal(oracle.time_bin(np.array([0.05]), dtb, 4, 8), [2])


def test_mts_with_one_bin_is_the_fixed_step():
    ps = workloads.uniform(700, seed=21, sigma_v=0.3)
    ps.u[:] = np.random.default_rng(21).uniform(0.5, 1.5, ps.n)
    dtb = 0.002
    r = oracle.mts_integrate(ps.pos, ps.vel, ps.m, ps.u, ps.h0, ps.box, dtb, 0, 3)
    assert list(r["active"]) == [ps.n] * 3
    f = oracle.full_pass(ps.pos, ps.vel, ps.m, ps.u, ps.h0, ps.box)
    pos, vel, u, h, a, du = ps.pos, ps.vel, ps.u, f["h"], f["force"]["a"], f["force"]["dudt"]
    for _ in range(3):
        s = oracle.kdk_step(pos, vel, ps.m, u, h, ps.box, a, du, dtb)
        pos, vel, u, h, a, du = s["pos"], s["vel"], s["u"], s["h"], s["a"], s["dudt"]
    np.testing.assert_allclose(r["vel"], vel, rtol=0, atol=1e-12)
    np.testing.assert_allclose(r["u"], u, rtol=1e-12)
    np.testing.assert_allclose(r["h"], h, rtol=1e-12)


def test_mts_with_every_particle_in_bin_one_is_the_double_step():
    # every time step of Eq. (6) is far above 2 dt_base: with at most one bin all
    # particles take steps of 2 dt_base, which is one kick-drift-kick step of that length
    ps = workloads.uniform(700, seed=22, sigma_v=0.1)
    dtb = 1e-4
    r = oracle.mts_integrate(ps.pos, ps.vel, ps.m, ps.u, ps.h0, ps.box, dtb, 1, 2)
    assert list(r["active"]) == [0, ps.n]
    f = oracle.full_pass(ps.pos, ps.vel, ps.m, ps.u, ps.h0, ps.box)
    s = oracle.kdk_step(ps.pos, ps.vel, ps.m, ps.u, f["h"], ps.box, f["force"]["a"], f["force"]["dudt"], 2 * dtb)
    d = r["pos"] - s["pos"]
    d -= ps.box * np.rint(d / ps.box)
    assert np.max(np.abs(d)) < 1e-15
    np.testing.assert_allclose(r["vel"], s["vel"], rtol=0, atol=1e-13)
    np.testing.assert_allclose(r["h"], s["h"], rtol=1e-12)


def test_mts_inactive_particles_only_drift():
    # two regions: hot particles (small steps) in a slab, cold ones (large steps) elsewhere
    ps = workloads.uniform(900, seed=23, sigma_v=0.05)
    ps.u[:] = np.where(ps.pos[:, 0] < 0.3, 20.0, 0.05)
    f = oracle.full_pass(ps.pos, ps.vel, ps.m, ps.u, ps.h0, ps.box)
    dtb = float(np.min(f["signal"]["dt"]))
    r1 = oracle.mts_integrate(ps.pos, ps.vel, ps.m, ps.u, ps.h0, ps.box, dtb, 3, 1)
    bins0 = oracle.time_bin(f["signal"]["dt"], dtb, 3, 0)
    assert bins0.max() >= 2 and bins0.min() == 0
    idle = bins0 >= 1   # not at the end of a step after one base step
    # their velocities carry only the opening half kick, their energies too
    span = 2.0 ** bins0[idle] * dtb
    np.testing.assert_allclose(r1["vel"][idle], ps.vel[idle] + 0.5 * span[:, None] * f["force"]["a"][idle],
                               rtol=1e-13, atol=1e-15)
    np.testing.assert_allclose(r1["h"][idle], f["h"][idle], rtol=0, atol=0)
    assert r1["active"][0] == np.sum(bins0 == 0)
