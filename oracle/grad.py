"""Gradient oracle for the SPH density and force stages (TEST INFRASTRUCTURE).

A dense FP64 evaluation of the forward model in plain PyTorch (CPU), written
independently of sph_oracle.c, differentiated by torch.autograd:

  Sec. 2.1  W, Eq. (2) rho, Eq. (3) N and its h-derivative, Omega, P, Eqs. (4)-(5);
  Sec. 4.1  velocity divergence and curl, Balsara switch, Monaghan-Balsara viscosity.

All pairs are formed explicitly (minimum image), so it is meant for a few
thousand particles.  The smoothing lengths are either given (fixed-h
derivative) or the solved roots of N_i(h_i) = N_ngb.  In the solved case the
value of h comes from the root found by the C oracle, and its dependence on
the positions is attached through one Newton step evaluated at that root,
h = h* - (N(h*, x) - N_ngb) / (dN/dh)(h*) with the denominator held
constant: at the root this has the value h* and the derivative
dh/dx = -(dN/dx)/(dN/dh) of the implicit function theorem.

Losses: loss_of (density misfit plus squared accelerations) and
linear_loss_of (constant weights on rho, a and du/dt, whose gradient is the
vector-Jacobian product an adjoint computes); gradients() and vjp() return
their gradients.

Also here: finite differences of a loss through the C oracle, in a position
(h re-solved at every evaluation: loss_fd) or in one h (loss_fd_h),
optionally restricted to the particles near the perturbed one, which is what
a large particle set needs.
"""
from __future__ import annotations

import math

import numpy as np
import torch

from . import ALPHA, GAMMA, N_NGB, density, force, ghost, solve_h

BALSARA_EPS = 1e-4


def _w(q):
    inner = 1.0 - 6.0 * q * q + 6.0 * q * q * q
    t = 1.0 - q
    outer = 2.0 * t * t * t
    return torch.where(q <= 0.5, inner, outer) * (q < 1.0)


def _dw(q):
    inner = -12.0 * q + 18.0 * q * q
    t = 1.0 - q
    outer = -6.0 * t * t
    return torch.where(q <= 0.5, inner, outer) * (q < 1.0)


def model(x, v, m, u, h, box, gamma=GAMMA, alpha=ALPHA, beps=BALSARA_EPS, balsara_form=0):
    """Dense forward pass: returns dict with rho, N, dNdh, omega, div, curl, f, A, c, a, dudt.

    balsara_form 0: f = |curl v| / (|div v| + |curl v| + eps c/h) as Sec. 4.1
    prints it; 1: |div v| in the numerator (Balsara 1995)."""
    n = x.shape[0]
    box_t = torch.as_tensor(box, dtype=x.dtype)
    d = x[:, None, :] - x[None, :, :]                     # r_ij = x_i - x_j
    d = d - box_t * torch.round(d / box_t)                  # minimum image
    eye = torch.eye(n, dtype=x.dtype)
    off = 1.0 - eye
    r = torch.sqrt((d * d).sum(-1) + eye)                  # diagonal set to 1, masked below
    hi = h[:, None]
    q = r / hi                                              # row i uses h_i
    w = _w(q) * off
    dw = _dw(q) * off
    mj = m[None, :]
    S_w = w.sum(1)
    S_mw = (mj * w).sum(1) + m                              # self term w(0) = 1
    S_mqdw = (mj * q * dw).sum(1)
    k3 = 8.0 / (math.pi * h ** 3)
    rho = k3 * S_mw
    N = 32.0 / 3.0 * (1.0 + S_w)
    dNdh = -32.0 / 3.0 / h * (q * dw).sum(1)
    drho = -8.0 / (math.pi * h ** 4) * (3.0 * S_mw + S_mqdw)
    omega = 1.0 + h / (3.0 * rho) * drho
    # grad W(r_ij, h_i) = 8/(pi h_i^5) g(q) r_ij,  g = w'/q
    g = torch.where(q > 0, dw / torch.where(q > 0, q, torch.ones_like(q)), torch.zeros_like(q))
    Gi = 8.0 / (math.pi * hi ** 5) * g                     # row i: h_i
    dv = v[None, :, :] - v[:, None, :]                      # v_j - v_i
    div = (mj * Gi * (dv * d).sum(-1)).sum(1) / rho
    cross = torch.cross(dv, d, dim=-1)
    curl = -(mj[..., None] * Gi[..., None] * cross).sum(1) / rho[:, None]
    P = (gamma - 1.0) * rho * u
    c = torch.sqrt(gamma * P / rho)
    A = P / (omega * rho * rho)
    c2 = (curl * curl).sum(1)
    # |curl|, with derivative 0 at curl = 0 (where the norm has none)
    cm = torch.where(c2 > 0, torch.sqrt(torch.where(c2 > 0, c2, torch.ones_like(c2))), torch.zeros_like(c2))
    den = div.abs() + cm + beps * c / h
    num = div.abs() if balsara_form == 1 else cm
    f = torch.where(den > 0, num / torch.where(den > 0, den, torch.ones_like(den)), torch.zeros_like(den))
    # force stage
    Gj = Gi.transpose(0, 1)                                 # grad W(r_ij, h_j) uses row j
    rng = (r < torch.maximum(hi, h[None, :])) * off
    vij = -dv                                               # v_i - v_j
    vr = (vij * d).sum(-1)
    wij = torch.clamp(vr / r, max=0.0) * rng
    Pi = -alpha * (c[:, None] + c[None, :] - 3.0 * wij) * wij / (rho[:, None] + rho[None, :])
    F = f[:, None] + f[None, :]
    Gs = Gi + Gj
    phi = (-mj * (A[:, None] * Gi + A[None, :] * Gj) - 0.25 * mj * Pi * Gs * F) * rng
    a = (phi[..., None] * d).sum(1)
    dudt = ((A[:, None] * mj * vr * Gi + 0.125 * mj * Pi * vr * Gs * F) * rng).sum(1)
    return {"rho": rho, "N": N, "dNdh": dNdh, "omega": omega, "div": div, "curl": curl, "f": f, "A": A,
            "c": c, "a": a, "dudt": dudt}


def loss_of(out, rho_target):
    """L = sum_i (rho_i - rho_t,i)^2 + sum_i |a_i|^2."""
    return ((out["rho"] - rho_target) ** 2).sum() + (out["a"] ** 2).sum()


def linear_loss_of(out, g_rho, g_a, g_dudt):
    """L = sum_i g_rho,i rho_i + g_a,i . a_i + g_u,i (du/dt)_i with constant weights
    (its gradient is the vector-Jacobian product with those weights)."""
    L = (out["rho"] * g_rho).sum() + (out["a"] * g_a).sum() + (out["dudt"] * g_dudt).sum()
    return L


def _tensors(pos, vel, m, u):
    x = torch.tensor(np.asarray(pos), dtype=torch.float64, requires_grad=True)
    v = torch.tensor(np.asarray(vel), dtype=torch.float64)
    mt = torch.tensor(np.broadcast_to(np.asarray(m, dtype=np.float64), (len(pos),)).copy())
    ut = torch.tensor(np.broadcast_to(np.asarray(u, dtype=np.float64), (len(pos),)).copy())
    return x, v, mt, ut


def _grad(pos, vel, m, u, h, box, loss, solve, target, tol, balsara_form=0):
    x, v, mt, ut = _tensors(pos, vel, m, u)
    if solve:
        hstar, _ = solve_h(pos, h, box, target=target, tol=tol)
        hs = torch.tensor(hstar)
        nd = model(x, v, mt, ut, hs, box, balsara_form=balsara_form)
        ht = hs - (nd["N"] - target) / nd["dNdh"].detach()
        L = loss(model(x, v, mt, ut, ht, box, balsara_form=balsara_form))
        L.backward()
        return x.grad.numpy().copy(), None, float(L.detach()), hstar
    ht = torch.tensor(np.asarray(h, dtype=np.float64), requires_grad=True)
    L = loss(model(x, v, mt, ut, ht, box, balsara_form=balsara_form))
    L.backward()
    return x.grad.numpy().copy(), ht.grad.numpy().copy(), float(L.detach()), np.asarray(h)


def gradients(pos, vel, m, u, h, box, rho_target, solve=True, target=N_NGB, tol=1e-13):
    """dL/dx (N,3) and, for fixed h, dL/dh (N,), of loss_of, from the dense model.

    solve=True: h is the solved root (h given is the initial guess) and the
    returned position gradient includes dh/dx; the h gradient is None.
    Returns (dL/dx, dL/dh or None, L, h used).
    """
    rt = torch.tensor(np.asarray(rho_target, dtype=np.float64))
    return _grad(pos, vel, m, u, h, box, lambda out: loss_of(out, rt), solve, target, tol)


def vjp(pos, vel, m, u, h, box, g_rho, g_a, g_dudt, solve=True, target=N_NGB, tol=1e-13, balsara_form=0):
    """dL/dx and (fixed h) dL/dh of linear_loss_of with weights g_rho (N,), g_a (N,3),
    g_dudt (N,): the vector-Jacobian product of (rho, a, du/dt) with respect to the
    positions (and h).  Same conventions as gradients()."""
    t = lambda a: torch.tensor(np.asarray(a, dtype=np.float64))
    gr, ga, gu = t(g_rho), t(g_a), t(g_dudt)
    return _grad(pos, vel, m, u, h, box, lambda out: linear_loss_of(out, gr, ga, gu), solve, target, tol,
                 balsara_form)


# ---------------------------------------------------------------- finite differences through the C oracle
def _oracle_outputs(pos, vel, m, u, h, box, sel_dens, sel_force):
    d = density(pos, vel, m, h, box, sel=sel_dens)
    gh = ghost(d, u, h)
    fr = force(pos, vel, m, h, d["rho"], gh["A"], gh["c"], gh["f"], box, sel=sel_force)
    return d["rho"], fr["a"], fr["dudt"]


def _local(pos, k, box, local):
    """Indices of the particles within 2R of x_k (every input that the outputs
    within R can see) and, in that subset, the particles within 1.5R (to be
    re-evaluated), within R (whose outputs enter the loss) and k itself."""
    dd = pos - pos[k]
    dd -= box * np.rint(dd / box)
    r = np.sqrt((dd * dd).sum(1))
    idx = np.where(r < 2.0 * local)[0]
    rs = r[idx]
    return idx, np.where(rs < 1.5 * local)[0], np.where(rs < local)[0], int(np.searchsorted(idx, k))


def _loss(rho, a, dudt, near2, rho_target, weights):
    if weights is None:
        return np.sum((rho[near2] - rho_target[near2]) ** 2) + np.sum(a[near2] ** 2)
    g_rho, g_a, g_dudt = weights
    return (np.sum(g_rho[near2] * rho[near2]) + np.sum(g_a[near2] * a[near2]) +
            np.sum(g_dudt[near2] * dudt[near2]))


def _subset(idx, *arrays):
    return [None if a is None else (tuple(x[idx] for x in a) if isinstance(a, tuple) else np.asarray(a)[idx])
            for a in arrays]


def loss_fd(pos, vel, m, u, h0, box, rho_target, k, axis, eps, solve=True, h_fixed=None, local=None, tol=1e-13,
            weights=None):
    """Central difference of L in x_k[axis] through the C oracle.

    L is loss_of(rho_target), or, when weights = (g_rho, g_a, g_dudt) is
    given, linear_loss_of with those weights (rho_target is then unused).
    local: None for the whole set, or a radius R >= 2 h_max: the loss
    difference only involves the particles within R of x_k (their outputs see
    h and positions within 1.5R, whose h see positions within 2R), so only
    those are evaluated, on the subset of particles within 2R.  With
    solve=False the smoothing lengths h_fixed are kept; with solve=True,
    h_fixed (if given) must be the solved h of the unperturbed set and saves
    solving it again.
    """
    pos = np.array(pos, dtype=np.float64)
    n = len(pos)
    m = np.broadcast_to(np.asarray(m, dtype=np.float64), (n,))
    u = np.broadcast_to(np.asarray(u, dtype=np.float64), (n,))
    vel = np.asarray(vel, dtype=np.float64)
    base_h = h_fixed
    if solve and base_h is None:
        base_h, _ = solve_h(pos, h0, box, tol=tol)
    near3 = near2 = None
    if local is not None:
        idx, near3, near2, k = _local(pos, k, box, local)
        pos, vel, m, u, base_h, rho_target, weights = _subset(idx, pos, vel, m, u, base_h, rho_target, weights)
    else:
        near2 = np.arange(n)
    vals = []
    for sgn in (+1, -1):
        p = pos.copy()
        p[k, axis] += sgn * eps
        h = base_h.copy()
        if solve:
            h, _ = solve_h(p, h, box, tol=tol, sel=near3)
        rho, a, dudt = _oracle_outputs(p, vel, m, u, h, box, near3, near2 if local is not None else None)
        vals.append(_loss(rho, a, dudt, near2, rho_target, weights))
    return (vals[0] - vals[1]) / (2 * eps)


def loss_fd_h(pos, vel, m, u, h, box, rho_target, k, eps, local=None, weights=None):
    """Central difference of L in h_k with the positions and every other h held
    fixed (the fixed-h derivative), through the C oracle.  local as in loss_fd."""
    pos = np.asarray(pos, dtype=np.float64)
    n = len(pos)
    m = np.broadcast_to(np.asarray(m, dtype=np.float64), (n,))
    u = np.broadcast_to(np.asarray(u, dtype=np.float64), (n,))
    vel = np.asarray(vel, dtype=np.float64)
    h = np.asarray(h, dtype=np.float64)
    near3 = None
    if local is not None:
        idx, near3, near2, k = _local(pos, k, box, local)
        pos, vel, m, u, h, rho_target, weights = _subset(idx, pos, vel, m, u, h, rho_target, weights)
    else:
        near2 = np.arange(n)
    vals = []
    for sgn in (+1, -1):
        hh = h.copy()
        hh[k] += sgn * eps
        rho, a, dudt = _oracle_outputs(pos, vel, m, u, hh, box, near3, near2 if local is not None else None)
        vals.append(_loss(rho, a, dudt, near2, rho_target, weights))
    return (vals[0] - vals[1]) / (2 * eps)
