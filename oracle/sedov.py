"""Self-similar point blast in a uniform cold gas (Sedov-Taylor), for the blast
wave test of Sec. 4.2 (TEST INFRASTRUCTURE).

An energy E released at the origin of a gas of density rho0 and negligible
pressure drives a strong spherical shock of radius R(t) = xi0 (E t^2 / rho0)^(1/5).
Behind it the flow is self-similar in xi = r / R:

    v = dR/dt phi(xi),   rho = rho0 psi(xi),   p = rho0 (dR/dt)^2 pi(xi).

Substituting into the spherical Euler equations (mass, momentum, and entropy
p rho^-gamma conserved along particle paths), with R ~ t^(2/5) so that
(d^2R/dt^2) R / (dR/dt)^2 = -3/2, gives three ordinary differential
equations in xi, with D = phi - xi:

    D psi' + psi phi'                 = -2 psi phi / xi
    D phi' + pi' / psi                =  3/2 phi
    D (pi'/pi - gamma psi'/psi)       =  3

solved here for (psi', phi', pi') and integrated inward from the strong-shock
(Rankine-Hugoniot) values at xi = 1:

    phi = 2/(gamma+1),  psi = (gamma+1)/(gamma-1),  pi = 2/(gamma+1).

Energy conservation fixes xi0: E = 4 pi rho0 (dR/dt)^2 R^3 I with
I = int_0^1 (psi phi^2 / 2 + pi/(gamma-1)) xi^2 dxi, and (dR/dt)^2 R^3 =
(4/25) xi0^5 E / rho0, so xi0 = (25 / (16 pi I))^(1/5).
"""
from __future__ import annotations

import math

import numpy as np
from scipy.integrate import solve_ivp


def _rhs(xi, y, g):
    psi, phi, pi = y
    D = phi - xi
    b = (1.5 * phi - pi * (3.0 - 2.0 * g * phi / xi) / (psi * D)) / (D - g * pi / (psi * D))
    a = (-2.0 * psi * phi / xi - psi * b) / D
    c = pi / D * (3.0 - 2.0 * g * phi / xi - g * b)
    return [a, b, c]


def profile(gamma, xi_min=1e-4, n=2001):
    """(xi, psi, phi, pi) on a grid from 1 down to xi_min."""
    g = float(gamma)
    y0 = [(g + 1.0) / (g - 1.0), 2.0 / (g + 1.0), 2.0 / (g + 1.0)]
    xs = np.linspace(1.0, xi_min, n)
    sol = solve_ivp(_rhs, (1.0, xi_min), y0, args=(g,), t_eval=xs, rtol=1e-11, atol=1e-13, method="DOP853")
    if not sol.success:
        raise RuntimeError(sol.message)
    return sol.t, sol.y[0], sol.y[1], sol.y[2]


def xi0(gamma):
    """The constant of R = xi0 (E t^2 / rho0)^(1/5)."""
    xs, psi, phi, pi = profile(gamma)
    f = (0.5 * psi * phi * phi + pi / (gamma - 1.0)) * xs * xs
    I = -np.trapezoid(f, xs)   # xs runs from 1 down
    return (25.0 / (16.0 * math.pi * I)) ** 0.2


def shock_radius(t, E, rho0, gamma):
    return xi0(gamma) * (E * t * t / rho0) ** 0.2
