"""Pins of the FP64 oracle against facts fixed by the paper and by mathematics.

Nothing here compares the oracle with itself: each test checks it against a
closed form, a high-precision lattice evaluation, a brute-force count, an
exact conservation law or a symmetry of the equations in Gonnet (2014),
Sec. 2.1 and Sec. 4.1.
"""
import math
import os

import numpy as np
import pytest
from scipy import integrate

import oracle
from paper_1404_2303_amd import workloads

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _golden(name):
    vals = {}
    with open(os.path.join(GOLDEN, name)) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            k, v = line.split()
            vals[k] = float(v)
    return vals


# ---------------------------------------------------------------- kernel W, Sec. 2.1
@pytest.mark.parametrize("h", [1.0, 0.37, 2e-3])
def test_kernel_normalisation(h):
    # int W dV = 4 pi int_0^h r^2 W(r,h) dr = 1 for a normalised kernel
    f = lambda r: 4.0 * math.pi * r * r * oracle.kernel_W(r, h)
    val = integrate.quad(f, 0.0, 0.5 * h, epsabs=0, epsrel=1e-13)[0]
    val += integrate.quad(f, 0.5 * h, h, epsabs=0, epsrel=1e-13)[0]
    assert abs(val - 1.0) < 1e-12


def test_kernel_values_and_continuity():
    w, dw = oracle.kernel_w, oracle.kernel_dw
    assert w(0.0)[0] == 1.0
    eps = 1e-12
    # both branches meet at q = 1/2 with value 1/4 and slope -3/2
    for q in (0.5 - eps, 0.5, 0.5 + eps):
        assert abs(w(q)[0] - 0.25) < 1e-10
        assert abs(dw(q)[0] + 1.5) < 1e-10
    # compact support: value and slope vanish at q = 1 and beyond
    for q in (1.0, 1.0 + 1e-9, 1.5, 7.0):
        assert abs(w(q)[0]) < 1e-20 and abs(dw(q)[0]) < 1e-15
    # central value of W
    for h in (1.0, 0.1):
        assert oracle.kernel_W(0.0, h) == pytest.approx(8.0 / (math.pi * h ** 3), rel=1e-15)
    # curvature of both branches at q = 1/2: 6 from either side
    d = 1e-5
    left = (dw(0.5 - d)[0] - dw(0.5 - 2 * d)[0]) / d
    right = (dw(0.5 + 2 * d)[0] - dw(0.5 + d)[0]) / d
    assert abs(left - 6.0) < 1e-3 and abs(right - 6.0) < 1e-3


@pytest.mark.parametrize("q", [0.1, 0.3, 0.49, 0.6, 0.8, 0.97])
def test_kernel_derivatives_match_finite_differences(q):
    d = 1e-6
    fd = (oracle.kernel_w(q + d)[0] - oracle.kernel_w(q - d)[0]) / (2 * d)
    assert oracle.kernel_dw(q)[0] == pytest.approx(fd, rel=1e-8, abs=1e-10)
    h, r = 0.7, 0.7 * q
    fdr = (oracle.kernel_W(r + d, h) - oracle.kernel_W(r - d, h)) / (2 * d)
    assert oracle.kernel_dWdr(r, h) == pytest.approx(fdr, rel=1e-7)
    fdh = (oracle.kernel_W(r, h + d) - oracle.kernel_W(r, h - d)) / (2 * d)
    assert oracle.kernel_dWdh(r, h) == pytest.approx(fdh, rel=1e-7)
    fd2 = (oracle.kernel_dw(q + d)[0] - oracle.kernel_dw(q - d)[0]) / (2 * d)
    assert oracle.kernel_d2w(q)[0] == pytest.approx(fd2, rel=1e-7, abs=1e-8)


# ---------------------------------------------------------------- perfect lattice
def _perfect_lattice(k=12, mass=3.7, u=1.0):
    ps = workloads.lattice((k, k, k), 1.0 / k, jitter=0.0, sigma_v=0.0)
    ps.m[:] = mass
    ps.u[:] = u
    return ps


def test_lattice_density_against_high_precision_values():
    g = _golden("lattice_sc.txt")
    k = 12
    ps = _perfect_lattice(k)
    dx = 1.0 / k
    h, it = oracle.solve_h(ps.pos, ps.h0, ps.box, tol=1e-12)
    assert np.all(it > 0)
    assert np.allclose(h / dx, g["h_over_dx"], rtol=1e-10, atol=0)
    d = oracle.density(ps.pos, ps.vel, ps.m, h, ps.box)
    mn = ps.m[0] * k ** 3
    assert np.allclose(d["rho"] / mn, g["rho_over_mn"], rtol=1e-10, atol=0)
    assert np.all(d["count"] == int(g["neighbours"]))
    assert np.allclose(d["nngb"], 48.0, atol=1e-10)
    gh = oracle.ghost(d, ps.u, h)
    assert np.allclose(gh["omega"], g["omega"], rtol=1e-10, atol=0)


def test_lattice_at_rest_has_no_force():
    k = 12
    ps = _perfect_lattice(k)
    out = oracle.full_pass(ps.pos, ps.vel, ps.m, ps.u, ps.h0, ps.box)
    f = out["force"]
    scale = np.max(f["kappa_a"])
    assert scale > 0
    assert np.max(np.abs(f["a"])) < 1e-12 * scale
    assert np.max(np.abs(f["dudt"])) < 1e-12 * np.max(f["kappa_u"] + 1e-300)
    assert np.max(np.abs(out["dens"]["div"])) == 0.0
    assert np.all(out["force"]["count"] == out["force"]["count"][0])


# ---------------------------------------------------------------- neighbour sets vs brute force
def _brute_counts(pos, R, box, exclude_self=True):
    n = len(pos)
    cnt = np.zeros(n, dtype=np.int64)
    for s in range(0, n, 512):
        d = pos[s:s + 512, None, :] - pos[None, :, :]
        d -= box * np.rint(d / box)
        r = np.sqrt(np.sum(d * d, axis=2))
        cnt[s:s + 512] = np.sum(r < R[s:s + 512, None], axis=1)
    return cnt - (1 if exclude_self else 0)


def test_neighbour_counts_match_brute_force():
    ps = workloads.config0()
    h, _ = oracle.solve_h(ps.pos, ps.h0, ps.box)
    d = oracle.density(ps.pos, ps.vel, ps.m, h, ps.box)
    assert np.array_equal(d["count"], _brute_counts(ps.pos, h, ps.box))
    gh = oracle.ghost(d, ps.u, h)
    f = oracle.force(ps.pos, ps.vel, ps.m, h, d["rho"], gh["A"], gh["c"], gh["f"], ps.box)
    # force range r < max(h_i, h_j): brute force over all pairs
    pos, box = ps.pos, ps.box
    cnt = np.zeros(ps.n, dtype=np.int64)
    for s in range(0, ps.n, 512):
        dd = pos[s:s + 512, None, :] - pos[None, :, :]
        dd -= box * np.rint(dd / box)
        r = np.sqrt(np.sum(dd * dd, axis=2))
        hij = np.maximum(h[s:s + 512, None], h[None, :])
        ok = r < hij
        ok[np.arange(min(512, ps.n - s)), np.arange(s, min(s + 512, ps.n))] = False
        cnt[s:s + 512] = ok.sum(axis=1)
    assert np.array_equal(f["count"], cnt)


def test_solved_h_is_the_unique_root():
    ps = workloads.uniform(1500, seed=3)
    h1, _ = oracle.solve_h(ps.pos, ps.h0, ps.box, tol=1e-11)
    h2, _ = oracle.solve_h(ps.pos, 0.3 * ps.h0, ps.box, tol=1e-11)
    h3, _ = oracle.solve_h(ps.pos, 2.5 * ps.h0, ps.box, tol=1e-11)
    assert np.allclose(h1, h2, rtol=1e-9) and np.allclose(h1, h3, rtol=1e-9)
    d = oracle.density(ps.pos, None, ps.m, h1, ps.box)
    assert np.max(np.abs(d["nngb"] - 48.0)) <= 1e-11
    # equal masses: rho (4 pi/3) h^3 / m is the same sum as N
    assert np.allclose(d["rho"] * 4 * math.pi / 3 * h1 ** 3 / ps.m, d["nngb"], rtol=1e-12)


def test_h_derivatives_match_finite_differences():
    ps = workloads.uniform(800, seed=5, sigma_v=0.3)
    h, _ = oracle.solve_h(ps.pos, ps.h0, ps.box)
    sel = np.arange(0, 800, 7)
    eps = 1e-7
    d0 = oracle.density(ps.pos, ps.vel, ps.m, h, ps.box, sel=sel)
    dp = oracle.density(ps.pos, ps.vel, ps.m, h * (1 + eps), ps.box, sel=sel)
    dm = oracle.density(ps.pos, ps.vel, ps.m, h * (1 - eps), ps.box, sel=sel)
    dh = 2 * eps * h[sel]
    fd_rho = (dp["rho"][sel] - dm["rho"][sel]) / dh
    fd_n = (dp["nngb"][sel] - dm["nngb"][sel]) / dh
    assert np.allclose(d0["drhodh"][sel], fd_rho, rtol=1e-5)
    assert np.allclose(d0["dndh"][sel], fd_n, rtol=1e-5)


# ---------------------------------------------------------------- force: exact invariants
def _random_state(n=2000, seed=11):
    rng = np.random.default_rng(seed)
    ps = workloads.uniform(n, seed=seed, sigma_v=0.4)
    ps.m[:] = ps.m * rng.uniform(0.5, 1.5, n)
    ps.u[:] = rng.uniform(0.3, 2.0, n)
    return ps


def test_momentum_and_energy_conservation():
    ps = _random_state()
    out = oracle.full_pass(ps.pos, ps.vel, ps.m, ps.u, ps.h0, ps.box)
    f = out["force"]
    m = ps.m
    # sum_i m_i a_i = 0: every pair term enters i and j with opposite signs
    mom = np.sum(m[:, None] * f["a"], axis=0)
    scale = np.sum(m * f["kappa_a"])
    assert np.max(np.abs(mom)) < 1e-13 * scale
    # sum_i m_i (du_i/dt + v_i . a_i) = 0: total energy is conserved by Eqs. (4)-(5)
    e = np.sum(m * (f["dudt"] + np.sum(ps.vel * f["a"], axis=1)))
    escale = np.sum(m * (f["kappa_u"] + np.linalg.norm(ps.vel, axis=1) * f["kappa_a"]))
    assert abs(e) < 1e-13 * escale
    assert np.all(out["ghost"]["f"] >= 0) and np.all(out["ghost"]["f"] <= 1)


def test_galilean_invariance():
    ps = _random_state(1200, seed=2)
    a = oracle.full_pass(ps.pos, ps.vel, ps.m, ps.u, ps.h0, ps.box)
    b = oracle.full_pass(ps.pos, ps.vel + np.array([0.7, -1.3, 2.1]), ps.m, ps.u, ps.h0, ps.box)
    sa = a["force"]["kappa_a"]
    assert np.all(np.abs(a["force"]["a"] - b["force"]["a"]) <= 1e-10 * sa[:, None])
    assert np.allclose(a["dens"]["div"], b["dens"]["div"], rtol=1e-9, atol=1e-9)
    assert np.allclose(a["dens"]["curl"], b["dens"]["curl"], rtol=1e-9, atol=1e-9)


def test_periodic_translation_invariance():
    ps = _random_state(1200, seed=4)
    a = oracle.full_pass(ps.pos, ps.vel, ps.m, ps.u, ps.h0, ps.box)
    shifted = np.mod(ps.pos + np.array([0.313, 0.5, 0.871]), 1.0)
    b = oracle.full_pass(shifted, ps.vel, ps.m, ps.u, ps.h0, ps.box)
    assert np.allclose(a["h"], b["h"], rtol=1e-9)
    assert np.all(np.abs(a["force"]["a"] - b["force"]["a"]) <= 1e-9 * a["force"]["kappa_a"][:, None])


def test_viscous_heating_is_non_negative_and_vanishes_for_receding_pairs():
    ps = _random_state(1500, seed=8)
    h, _ = oracle.solve_h(ps.pos, ps.h0, ps.box)
    d = oracle.density(ps.pos, ps.vel, ps.m, h, ps.box)
    gh = oracle.ghost(d, ps.u, h)
    args = (ps.pos, ps.vel, ps.m, h, d["rho"], gh["A"], gh["c"], gh["f"], ps.box)
    f0 = oracle.force(*args, alpha=0.0)
    f1 = oracle.force(*args, alpha=0.8)
    visc = f1["dudt"] - f0["dudt"]
    assert np.all(visc >= -1e-12 * f1["kappa_u"])
    assert np.sum(visc) > 0
    # a cluster expanding homologously: every pair recedes, so Pi = 0 and the
    # result does not depend on alpha
    rng = np.random.default_rng(1)
    n = 600
    c = np.array([0.5, 0.5, 0.5])
    pos = c + (rng.random((n, 3)) - 0.5) * 0.25
    vel = 0.9 * (pos - c)
    m = np.full(n, 1.0 / n)
    h0 = np.full(n, 0.05)
    box = np.ones(3)
    h, _ = oracle.solve_h(pos, h0, box)
    d = oracle.density(pos, vel, m, h, box)
    gh = oracle.ghost(d, np.ones(n), h)
    a0 = oracle.force(pos, vel, m, h, d["rho"], gh["A"], gh["c"], gh["f"], box, alpha=0.0)
    a1 = oracle.force(pos, vel, m, h, d["rho"], gh["A"], gh["c"], gh["f"], box, alpha=2.0)
    assert np.array_equal(a0["a"], a1["a"]) and np.array_equal(a0["dudt"], a1["dudt"])


def test_pressure_force_is_repulsive_for_two_particles():
    # two particles at rest, isolated in a large box: a_1 points away from particle 2
    pos = np.array([[0.5, 0.5, 0.5], [0.53, 0.51, 0.49]])
    vel = np.zeros((2, 3))
    m = np.array([1.0, 2.0])
    h = np.array([0.1, 0.07])
    box = np.ones(3)
    d = oracle.density(pos, vel, m, h, box)
    gh = oracle.ghost(d, np.array([1.0, 0.5]), h)
    f = oracle.force(pos, vel, m, h, d["rho"], gh["A"], gh["c"], gh["f"], box)
    r12 = pos[0] - pos[1]
    assert np.dot(f["a"][0], r12) > 0 and np.dot(f["a"][1], r12) < 0
    assert np.allclose(np.cross(f["a"][0], r12), 0, atol=1e-12 * np.linalg.norm(f["a"][0]))
    assert np.allclose(m[0] * f["a"][0], -m[1] * f["a"][1], rtol=1e-13)


@pytest.mark.parametrize("sep, A, f", [(0.05, (1.0, 0.5), (0.0, 0.0)), (0.097, (1.0, 0.5), (0.3, 0.9)),
                                       (0.066, (1e-6, 1e-6), (1.0, 1.0)), (0.0695, (2.0, 1e-3), (0.5, 0.2))])
def test_h_sensitivity_of_the_force_matches_finite_differences(sep, A, f):
    # one approaching pair isolated in a large box, h_1 = 0.1, h_2 = 0.07 (the
    # pair inside one or both supports, near the edge of one in the second and
    # fourth cases, viscosity dominant in the third): sens_a and sens_u of
    # particle 1 must equal the magnitudes of the central differences of its a
    # and du/dt over ln h_1 plus those over ln h_2, rho, A, c and f held fixed.
    e = np.array([0.6, 0.64, -0.48])
    pos = np.array([[0.5, 0.5, 0.5], 0.5 + sep * e])
    vel = np.array([[0.3, -0.1, 0.2], [-0.4, 0.3, -0.5]])
    m = np.array([1.0, 2.0])
    h = np.array([0.1, 0.07])
    rho, A, c, f = np.array([3.0, 2.5]), np.array(A), np.array([1.0, 1.3]), np.array(f)
    box = np.ones(3)
    run = lambda hh: oracle.force(pos, vel, m, hh, rho, A, c, f, box, alpha=1.5, sel=[0])
    ref = run(h)
    assert ref["count"][0] == 1
    eps = 1e-6
    fd_a, fd_u = 0.0, 0.0
    for k in range(2):
        up, dn = h.copy(), h.copy()
        up[k] *= math.exp(eps)
        dn[k] *= math.exp(-eps)
        p, q = run(up), run(dn)
        fd_a += np.linalg.norm(p["a"][0] - q["a"][0]) / (2 * eps)
        fd_u += abs(p["dudt"][0] - q["dudt"][0]) / (2 * eps)
    assert ref["sens_a"][0] == pytest.approx(fd_a, rel=1e-6)
    assert ref["sens_u"][0] == pytest.approx(fd_u, rel=1e-6)
    # near the edge of a support the sensitivity far exceeds the term itself
    if abs(sep / 0.1 - 1) < 0.05:
        assert ref["sens_a"][0] > 10 * ref["kappa_a"][0]


# ---------------------------------------------------------------- div / curl, Sec. 4.1
def _interior_lattice(k=20, mass=3.7):
    ps = workloads.lattice((k, k, k), 1.0 / k, jitter=0.0, sigma_v=0.0)
    ps.m[:] = mass
    c = np.full(3, 0.5)
    inner = np.where(np.all(np.abs(ps.pos - c) < 0.2, axis=1))[0]
    return ps, c, inner


def test_divergence_of_a_compression_field():
    ps, c, inner = _interior_lattice()
    kappa = 0.37
    vel = -kappa * (ps.pos - c)
    h, _ = oracle.solve_h(ps.pos, ps.h0, ps.box, sel=inner)
    h = np.where(np.isin(np.arange(ps.n), inner), h, ps.h0)
    d = oracle.density(ps.pos, vel, ps.m, h, ps.box, sel=inner)
    # continuum limit: div v = -3 kappa, curl v = 0
    assert np.allclose(d["div"][inner], -3 * kappa, rtol=2e-2)
    assert np.max(np.abs(d["curl"][inner])) < 1e-10


def test_curl_of_a_rigid_rotation():
    ps, c, inner = _interior_lattice()
    omega = np.array([0.2, -0.5, 0.9])
    vel = np.cross(omega, ps.pos - c)
    h, _ = oracle.solve_h(ps.pos, ps.h0, ps.box, sel=inner)
    h = np.where(np.isin(np.arange(ps.n), inner), h, ps.h0)
    d = oracle.density(ps.pos, vel, ps.m, h, ps.box, sel=inner)
    # continuum limit: curl v = 2 omega, div v = 0
    assert np.allclose(d["curl"][inner], 2 * omega, rtol=2e-2, atol=1e-3)
    assert np.max(np.abs(d["div"][inner])) < 1e-10
    gh = oracle.ghost(d, np.ones(ps.n), h)
    assert np.all(gh["f"][inner] > 0.99)


# ---------------------------------------------------------------- force magnitude, Eqs. (4)-(5) and Sec. 4.1
GAMMA = 5.0 / 3.0


def test_pressure_gradient_on_a_perfect_lattice_is_exact():
    """u linear in x (u = u0 + g x, so P = (gamma-1) rho u is linear) on a
    perfect simple-cubic lattice at rest: at interior particles Eq. (4) gives
    exactly a = -grad P / rho = -(gamma-1) g x-hat.  On the lattice the
    kernel-gradient sum that Eq. (4) forms is sum_j m r_x^2 W'/r = -Omega rho
    (cubic symmetry; the same sum gives Omega through d rho/dh), and the
    1/Omega inside A = P/(Omega rho^2) cancels it.  A dropped Omega (1% here),
    a doubled or misplaced pressure term or a wrong sign all break it."""
    ps, c, inner = _interior_lattice()
    g = 0.8
    u = 2.0 + g * (ps.pos[:, 0] - 0.5)
    out = oracle.full_pass(ps.pos, ps.vel, ps.m, u, ps.h0, ps.box)
    a = out["force"]["a"][inner]
    assert abs(out["ghost"]["omega"][inner[0]] - 1.0) > 5e-3   # Omega matters here
    np.testing.assert_allclose(a[:, 0], -(GAMMA - 1.0) * g, rtol=1e-10)
    assert np.max(np.abs(a[:, 1:])) < 1e-10 * (GAMMA - 1.0) * g
    assert np.max(np.abs(out["force"]["dudt"][inner])) == 0.0


def _ints():
    w = lambda q: np.where(q <= 0.5, 1 - 6 * q * q + 6 * q ** 3, 2 * (1 - q) ** 3)
    dw = lambda q: np.where(q <= 0.5, 18 * q * q - 12 * q, -6 * (1 - q) ** 2)
    j4 = integrate.quad(lambda q: q ** 4 * dw(q), 0, 1, points=[0.5])[0]
    j5 = integrate.quad(lambda q: q ** 5 * dw(q), 0, 1, points=[0.5])[0]
    return j4, j5


def test_compression_heating_on_a_perfect_lattice():
    """Uniform compression v = -beta (x - c) of a perfect lattice, |div v| form
    of the Balsara switch.

    Pressure part of Eq. (5) (alpha = 0): the first law, du/dt = (P/rho^2)
    d rho/dt = 3 beta P / rho, holds exactly on the lattice (the same lattice
    sum -Omega rho as above).

    Viscous part (the difference to alpha = 0.8): every pair approaches at
    w_ij = -beta r, so Pi_ij = alpha beta r (2c + 3 beta r) / (2 rho) and the
    viscous du/dt is -(f alpha beta^2 / (4 rho)) sum_j m (2c + 3 beta r) r^2 W'(r).
    Its continuum limit (sum_j m -> rho int d^3r) is
    -8 f alpha beta^2 (2 c h J4 + 3 beta h^2 J5), J_k = int_0^1 q^k w'(q) dq,
    with f = 3 beta / (3 beta + 1e-4 c / h); the lattice differs from it by
    its discretisation (~1%).  A doubled or halved viscosity, the 1/4 and 1/8
    of Sec. 4.1 exchanged, or Pi over the mean instead of the sum of the
    densities all miss it by a factor of two or more."""
    ps, c, inner = _interior_lattice()
    beta = 0.37
    vel = -beta * (ps.pos - c)
    u = np.full(ps.n, 1.3)
    p0 = oracle.full_pass(ps.pos, vel, ps.m, u, ps.h0, ps.box, alpha=0.0, balsara_form=1)
    rho, P = p0["dens"]["rho"][inner], p0["ghost"]["P"][inner]
    np.testing.assert_allclose(p0["force"]["dudt"][inner], 3.0 * beta * P / rho, rtol=1e-12)
    assert np.max(np.abs(p0["force"]["a"][inner])) < 1e-12 * np.max(p0["force"]["kappa_a"][inner])
    p1 = oracle.full_pass(ps.pos, vel, ps.m, u, ps.h0, ps.box, alpha=0.8, balsara_form=1)
    visc = p1["force"]["dudt"][inner] - p0["force"]["dudt"][inner]
    h, cs = p1["h"][inner], p1["ghost"]["c"][inner]
    j4, j5 = _ints()
    f = 3 * beta / (3 * beta + 1e-4 * cs / h)
    pred = -8.0 * f * 0.8 * beta ** 2 * (2.0 * cs * h * j4 + 3.0 * beta * h * h * j5)
    assert np.all(pred > 0)
    np.testing.assert_allclose(visc, pred, rtol=0.02)


def test_sod_tube_plateau_matches_the_riemann_solution():
    """The Sec. 4.2 shock tube on 8 lattice cells per unit length (10,240
    particles), integrated by the oracle to t = 1.5 with steps from Eq. (6),
    |div v| Balsara form: on the plateau between the contact and the shock
    (0.25 in from both) the pressure, velocity and density are the exact
    Riemann star state (oracle/riemann.py, pinned to textbook values) to 3%.
    The star state moves with the pressure force's magnitude (a doubled
    pressure term acts like a stiffer gas), so this pins the scale of
    Eq. (4)-(5) that the conservation tests leave free."""
    from oracle import riemann
    ps = workloads.sod(8)
    g = ps.meta["gamma"]
    t_end = 1.5
    st = oracle.integrate(ps.pos, ps.vel, ps.m, ps.u, ps.h0, ps.box, t_end, 1.0, gamma=g, balsara_form=1)
    out = oracle.full_pass(st["pos"], st["vel"], ps.m, st["u"], st["h"], ps.box, gamma=g, balsara_form=1)
    rho, P = out["dens"]["rho"], out["ghost"]["P"]
    L, R = workloads.SOD_LEFT, workloads.SOD_RIGHT
    p_star, u_star, _, rho_star = riemann.star_state(L, R, g)
    s_shock = riemann.shock_speed_right(L, R, g)
    for x0, sgn in ((4.0, 1.0), (8.0, -1.0)):
        x = st["pos"][:, 0].copy()
        if x0 == 8.0:
            x = np.where(x < 4.0, x + 8.0, x)   # unwrap the periodic interface
        d = sgn * (x - x0)
        m = (d > u_star * t_end + 0.25) & (d < s_shock * t_end - 0.25)
        assert m.sum() >= 100
        assert abs(np.mean(P[m]) / p_star - 1) < 0.03
        assert abs(sgn * np.mean(st["vel"][m, 0]) / u_star - 1) < 0.03
        assert abs(np.mean(rho[m]) / rho_star - 1) < 0.03
