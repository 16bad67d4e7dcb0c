"""Pins of the oracle's time-step criterion (Eq. (6)), of the two forms of the
Balsara switch (Sec. 4.1), and of the exact Riemann solver the Sod shock tube
of Sec. 4.2 is compared with."""
import math

import numpy as np
import pytest

import oracle
from oracle import riemann
from paper_1404_2303_amd import workloads

CFL = 0.25


def _pair(d, v, h=(0.2, 0.2), c=(1.0, 1.0), box=(1.0, 1.0, 1.0)):
    """Two particles at 0.5 -+ d/2 on the x axis with velocities (+-v, 0, 0)."""
    pos = np.array([[0.5 - d / 2, 0.5, 0.5], [0.5 + d / 2, 0.5, 0.5]])
    vel = np.array([[v, 0.0, 0.0], [-v, 0.0, 0.0]])
    return oracle.signal_dt(pos, vel, np.array(h, float), np.array(c, float), np.array(box, float), cfl=CFL)


def test_isolated_particle_uses_its_own_sound_speed():
    # no neighbour within max(h_i, h_j): only j = i, whose term is 2 c_i
    s = _pair(0.3, 0.7, h=(0.2, 0.25), c=(1.5, 4.0))
    np.testing.assert_allclose(s["vsig"], [3.0, 8.0], rtol=0, atol=0)
    np.testing.assert_allclose(s["dt"], [CFL * 0.2 / 1.5, CFL * 0.25 / 4.0], rtol=1e-15)


def test_head_on_pair_closed_form():
    # r_ij = x_i - x_j = (-d, 0, 0), v_ij = (2v, 0, 0): v_ij . r_ij / r_ij = -2v,
    # vsig = c_i + c_j + 6 v
    v, c1, c2 = 0.3, 1.0, 2.0
    s = _pair(0.1, v, c=(c1, c2))
    vs = c1 + c2 + 6 * v
    np.testing.assert_allclose(s["vsig"], [max(vs, 2 * c1), max(vs, 2 * c2)], rtol=1e-15)
    np.testing.assert_allclose(s["dt"], CFL * 2 * 0.2 / s["vsig"], rtol=1e-15)


def test_receding_pair_has_no_approach_term():
    s = _pair(0.1, -0.3, c=(1.0, 2.0))
    np.testing.assert_allclose(s["vsig"], [3.0, 4.0], rtol=1e-15)


def test_range_is_the_force_range_max_h():
    # r = 0.15 is outside h_0 = 0.1 but inside h_1 = 0.2: the pair interacts
    # in the force stage (r < max(h_i, h_j)) and so enters both maxima
    s = _pair(0.15, 0.0, h=(0.1, 0.2), c=(1.0, 3.0))
    np.testing.assert_allclose(s["vsig"], [4.0, 6.0], rtol=1e-15)
    s = _pair(0.25, 0.0, h=(0.1, 0.2), c=(1.0, 3.0))
    np.testing.assert_allclose(s["vsig"], [2.0, 6.0], rtol=1e-15)


def test_galilean_invariance_and_uniform_state():
    ps = workloads.uniform(600, seed=5, sigma_v=0.4)
    h = np.full(ps.n, 0.12)
    c = np.random.default_rng(5).uniform(0.5, 1.5, ps.n)
    a = oracle.signal_dt(ps.pos, ps.vel, h, c, ps.box, cfl=CFL)
    b = oracle.signal_dt(ps.pos, ps.vel + np.array([3.0, -1.0, 0.5]), h, c, ps.box, cfl=CFL)
    np.testing.assert_allclose(a["dt"], b["dt"], rtol=1e-12)
    # at rest with one sound speed every term is 2c: dt = C_CFL h / c
    u = oracle.signal_dt(ps.pos, np.zeros_like(ps.vel), h, np.full(ps.n, 0.8), ps.box, cfl=CFL)
    np.testing.assert_allclose(u["dt"], CFL * h / 0.8, rtol=1e-15)
    # the band values bracket the exact one
    assert np.all(a["vsig_lo"] <= a["vsig"]) and np.all(a["vsig"] <= a["vsig_hi"])


def test_full_pass_reports_the_time_step():
    ps = workloads.uniform(800, seed=2, sigma_v=0.2)
    out = oracle.full_pass(ps.pos, ps.vel, ps.m, ps.u, ps.h0, ps.box)
    c = out["ghost"]["c"]
    dt = out["signal"]["dt"]
    # dt <= C_CFL h / c (the self term), with equality only for particles no neighbour approaches faster
    assert np.all(dt <= CFL * out["h"] / c * (1 + 1e-15))
    assert np.any(dt < 0.9 * CFL * out["h"] / c)


def test_balsara_forms():
    ps = workloads.uniform(700, seed=4, sigma_v=0.3)
    out = oracle.full_pass(ps.pos, ps.vel, ps.m, ps.u, ps.h0, ps.box)
    d, h = out["dens"], out["h"]
    g0 = oracle.ghost(d, ps.u, h, balsara_form=0)
    g1 = oracle.ghost(d, ps.u, h, balsara_form=1)
    cm = np.linalg.norm(d["curl"], axis=1)
    eps = 1e-4 * g0["c"] / h
    # the two numerators share the denominator: f0 + f1 + eps/den = 1
    np.testing.assert_allclose(g0["f"] + g1["f"] + eps / (np.abs(d["div"]) + cm + eps), 1.0, rtol=1e-13)
    # pure compression (curl = 0): form 1 switches the viscosity on, form 0 off
    pos = np.array([[0.5, 0.5, 0.5]])
    dens = {"rho": np.ones(1), "drhodh": np.zeros(1), "div": np.array([-2.0]), "curl": np.zeros((1, 3))}
    f0 = oracle.ghost(dens, np.ones(1), np.array([0.1]), balsara_form=0)["f"]
    f1 = oracle.ghost(dens, np.ones(1), np.array([0.1]), balsara_form=1)["f"]
    assert f0[0] == 0.0 and 0.999 < f1[0] < 1.0


# ---------------------------------------------------------------- exact Riemann solver
# Star states of the classic shock-tube tests, gamma = 1.4, as tabulated by
# Toro, "Riemann Solvers and Numerical Methods for Fluid Dynamics", Table 4.3.
TORO = [
    # (rho, u, p) left, (rho, u, p) right, p*, u*, rho*_L, rho*_R
    ((1.0, 0.0, 1.0), (0.125, 0.0, 0.1), 0.30313, 0.92745, 0.42632, 0.26557),
    ((1.0, -2.0, 0.4), (1.0, 2.0, 0.4), 0.00189, 0.00000, 0.02185, 0.02185),
    ((1.0, 0.0, 1000.0), (1.0, 0.0, 0.01), 460.894, 19.5975, 0.57506, 5.99924),
]


@pytest.mark.parametrize("case", TORO)
def test_riemann_star_state_matches_textbook(case):
    left, right, ps, us, rl, rr = case
    p, u, rsl, rsr = riemann.star_state(left, right, 1.4)
    for got, want in ((p, ps), (u, us), (rsl, rl), (rsr, rr)):
        assert abs(got - want) <= 5e-5 * max(abs(want), 1.0), (got, want)


SOD = ((4.0, 0.0, 1.0), (1.0, 0.0, 0.1795))   # Sec. 4.2 (rho, u, P); gamma 5/3
G = 5.0 / 3.0


def test_sod_shock_satisfies_rankine_hugoniot():
    left, right = SOD
    ps, us, rsl, rsr = riemann.star_state(left, right, G)
    S = riemann.shock_speed_right(left, right, G)
    rr, ur, pr = right
    # fluxes through the moving shock: mass, momentum, energy
    m1, m2 = rr * (ur - S), rsr * (us - S)
    assert abs(m1 - m2) < 1e-10 * abs(m1)
    mom1 = rr * (ur - S) ** 2 + pr
    mom2 = rsr * (us - S) ** 2 + ps
    assert abs(mom1 - mom2) < 1e-10 * mom1
    E = lambda rho, u, p: p / (G - 1) + 0.5 * rho * u * u
    en1 = (E(rr, ur, pr) + pr) * (ur - S) / rr / (ur - S)   # specific enthalpy flux per mass flux
    h1 = (G / (G - 1)) * pr / rr + 0.5 * (ur - S) ** 2
    h2 = (G / (G - 1)) * ps / rsr + 0.5 * (us - S) ** 2
    assert abs(h1 - h2) < 1e-10 * h1
    assert en1 > 0


def test_sod_rarefaction_is_isentropic_with_constant_invariant():
    left, right = SOD
    rl, ul, pl = left
    cl = math.sqrt(G * pl / rl)
    ps, us, rsl, _ = riemann.star_state(left, right, G)
    csl = math.sqrt(G * ps / rsl)
    S = np.linspace(ul - cl, us - csl, 41)[1:-1]   # inside the fan
    rho, u, p = riemann.solution(S, left, right, G)
    np.testing.assert_allclose(p / rho ** G, pl / rl ** G, rtol=1e-12)
    c = np.sqrt(G * p / rho)
    np.testing.assert_allclose(u + 2 * c / (G - 1), ul + 2 * cl / (G - 1), rtol=1e-12)
    # the fan is a C- characteristic family: S = u - c
    np.testing.assert_allclose(u - c, S, rtol=1e-12, atol=1e-12)
    # contact: pressure and velocity continuous, density jumps
    r2, u2, p2 = riemann.solution(np.array([us - 1e-9, us + 1e-9]), left, right, G)
    assert abs(p2[0] - p2[1]) < 1e-12 and abs(u2[0] - u2[1]) < 1e-12 and abs(r2[0] - r2[1]) > 0.1


def test_riemann_mirror_symmetry_and_trivial_case():
    left, right = SOD
    S = np.linspace(-2, 2, 81)
    r1, u1, p1 = riemann.solution(S, left, right, G)
    mir = lambda s: (s[0], -s[1], s[2])
    r2, u2, p2 = riemann.solution(-S, mir(right), mir(left), G)
    np.testing.assert_allclose(r1, r2, rtol=1e-12)
    np.testing.assert_allclose(u1, -u2, rtol=1e-12, atol=1e-14)
    np.testing.assert_allclose(p1, p2, rtol=1e-12)
    r, u, p = riemann.solution(S, (2.0, 0.3, 1.5), (2.0, 0.3, 1.5), G)
    np.testing.assert_allclose(r, 2.0, rtol=1e-12)
    np.testing.assert_allclose(u, 0.3, rtol=1e-10)
    np.testing.assert_allclose(p, 1.5, rtol=1e-12)


# ---------------------------------------------------------------- Sedov-Taylor blast
def test_sedov_constant_matches_textbook():
    from oracle import sedov
    # R = xi0 (E t^2/rho0)^(1/5): xi0 = 1.033 for gamma = 1.4 (Taylor 1950;
    # Landau & Lifshitz, Fluid Mechanics, Sec. 106) and 1.1517 for gamma = 5/3
    assert abs(sedov.xi0(1.4) - 1.033) < 1e-3
    assert abs(sedov.xi0(5.0 / 3.0) - 1.1517) < 1e-3


def test_sedov_profile_is_a_solution_with_rankine_hugoniot_front():
    from oracle import sedov
    g = 5.0 / 3.0
    xs, psi, phi, pi = sedov.profile(g, xi_min=0.05, n=401)
    # the front carries the strong-shock jump
    assert abs(psi[0] - (g + 1) / (g - 1)) < 1e-12 and abs(phi[0] - 2 / (g + 1)) < 1e-12
    # entropy p rho^-gamma of each shell grows inward (earlier, stronger shocks)
    Q = pi * psi ** (-g)
    assert np.all(np.diff(Q) > 0)
    # mass conservation: the swept-up mass 4/3 pi R^3 rho0 sits inside the front
    mass = -np.trapezoid(psi * xs * xs, xs) * 4 * np.pi
    assert abs(mass - 4 * np.pi / 3) < 2e-3 * 4 * np.pi / 3 + 4 * np.pi * 0.05 ** 3
    # the residual of the momentum equation along the solution is small
    dphi = np.gradient(phi, xs)
    dpi = np.gradient(pi, xs)
    res = (phi - xs) * dphi - 1.5 * phi + dpi / psi
    assert np.max(np.abs(res[5:-5])) < 1e-3


def test_sedov_generator_energy():
    ps = workloads.sedov(12)
    e = np.sum(ps.m * ps.u)
    assert abs(e - 1.0 - ps.m[0] * ps.u.min() * (ps.n - 28)) < 1e-12
    r = np.linalg.norm(ps.pos - 0.5, axis=1)
    hot = np.sort(r[ps.meta["hot"]])
    # complete shells: the next particle lies strictly farther out
    assert np.sort(r)[28] > hot[-1] + 1e-9
