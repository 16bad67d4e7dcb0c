"""Seeded synthetic particle sets (inputs only: no SPH arithmetic here).

The paper's own workloads (Sod shock, Sedov blast, a cosmological volume,
Sec. 4.2) are not reproduced; these generators stand in for them with the
shapes, counts and structures listed below.  Every array is FP64 NumPy, all
boxes are periodic, masses are equal within a box, and ``h0`` is an initial
guess for the smoothing length taken from the mean inter-particle spacing:
the radius of a sphere that holds ``n_ngb`` particles at the mean number
density.  The solved smoothing lengths do not depend on it.

Sets
----
``uniform``    N uniform-random positions in a box (default: 4096 in the unit cube).
``lattice``    a cubic lattice of spacing ``dx`` filling the box, every site
               displaced by U(-jitter, jitter)*dx per component; velocities
               N(0, sigma_v) per component.
``plummer``    ``n_sph`` Plummer spheres plus a uniform background: centres
               U[0,1)^3, scale radii log-uniform in [a_min, a_max], radii
               r = a (X^(-2/3) - 1)^(-1/2) with X ~ U(0,1), redrawn while
               r >= r_cut, isotropic directions, wrapped into the box.
``batch``      independent uniform boxes with log-uniform counts, seeded per box.
``sod``        the shock tube of Sec. 4.2: a periodic 8 x 1 x 1 box, density 4
               and pressure 1 on x < 4 (face-centred cubic lattice, 4 sites
               per lattice cell), density 1 and pressure 0.1795 on x >= 4
               (simple cubic lattice of the same cell), equal masses, at rest.
``sedov``      the blast wave of Sec. 4.2: a face-centred cubic lattice at rest
               with density 1 and a small pressure in the periodic unit cube,
               and the energy E on the particles nearest the centre.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

N_NGB = 48.0


@dataclass
class ParticleSet:
    pos: np.ndarray            # (N, 3)
    vel: np.ndarray            # (N, 3)
    m: np.ndarray              # (N,)
    u: np.ndarray              # (N,)
    h0: np.ndarray             # (N,)
    box: np.ndarray            # (3,)
    name: str = ""
    meta: dict = field(default_factory=dict)

    @property
    def n(self) -> int:
        return int(self.pos.shape[0])


def mean_spacing_h(n_per_volume: float, n_ngb: float = N_NGB) -> float:
    """Radius of a sphere holding n_ngb particles at number density n_per_volume."""
    return (3.0 * n_ngb / (4.0 * math.pi * n_per_volume)) ** (1.0 / 3.0)


def _finish(pos, vel, box, name, u=1.0, meta=None):
    n = pos.shape[0]
    vol = float(np.prod(box))
    m = np.full(n, vol / max(n, 1))
    h0 = np.full(n, mean_spacing_h(max(n, 1) / vol))
    return ParticleSet(pos=np.ascontiguousarray(pos, dtype=np.float64),
                       vel=np.ascontiguousarray(vel, dtype=np.float64),
                       m=m, u=np.full(n, float(u)), h0=h0,
                       box=np.asarray(box, dtype=np.float64), name=name, meta=meta or {})


def uniform(n: int = 4096, seed: int = 0, box=(1.0, 1.0, 1.0), sigma_v: float = 0.0) -> ParticleSet:
    """Uniform-random positions; v = 0 unless sigma_v > 0; u = 1."""
    rng = np.random.default_rng(seed)
    box = np.asarray(box, dtype=np.float64)
    pos = rng.random((n, 3)) * box
    vel = rng.normal(0.0, sigma_v, (n, 3)) if sigma_v > 0 else np.zeros((n, 3))
    return _finish(pos, vel, box, f"uniform{n}")


def lattice(sites=(128, 128, 64), dx: float = 1.0 / 128, jitter: float = 0.1,
            sigma_v: float = 0.1, seed: int = 0) -> ParticleSet:
    """Jittered cubic lattice with sites[0]*sites[1]*sites[2] particles.

    The default (128 x 128 x 64 sites of spacing 1/128 in a 1 x 1 x 1/2 box)
    has 2^20 particles at the number density of a 128^3 lattice in the unit
    cube.
    """
    rng = np.random.default_rng(seed)
    sx, sy, sz = sites
    box = np.array([sx * dx, sy * dx, sz * dx])
    ii, jj, kk = np.meshgrid(np.arange(sx), np.arange(sy), np.arange(sz), indexing="ij")
    base = np.stack([ii.ravel(), jj.ravel(), kk.ravel()], axis=1).astype(np.float64)
    off = rng.uniform(-jitter, jitter, base.shape) if jitter > 0 else 0.0
    pos = (base + 0.5 + off) * dx
    pos = np.mod(pos, box)
    vel = rng.normal(0.0, sigma_v, base.shape) if sigma_v > 0 else np.zeros(base.shape)
    return _finish(pos, vel, box, f"lattice{sx}x{sy}x{sz}")


def plummer_mixture(n_spheres: int = 32, n_per_sphere: int = 52428, n_background: int = 419456,
                    a_min: float = 0.005, a_max: float = 0.05, r_cut: float = 0.5,
                    sigma_v: float = 0.1, seed: int = 0) -> ParticleSet:
    """Plummer spheres plus a uniform background in the periodic unit cube."""
    rng = np.random.default_rng(seed)
    centres = rng.random((n_spheres, 3))
    radii = np.exp(rng.uniform(math.log(a_min), math.log(a_max), n_spheres))
    parts = []
    for c, a in zip(centres, radii):
        r = np.empty(n_per_sphere)
        todo = np.arange(n_per_sphere)
        while todo.size:
            X = rng.random(todo.size)
            X = np.where(X <= 0.0, 1e-300, X)
            rr = a / np.sqrt(X ** (-2.0 / 3.0) - 1.0)
            ok = rr < r_cut
            r[todo[ok]] = rr[ok]
            todo = todo[~ok]
        d = rng.normal(size=(n_per_sphere, 3))
        d /= np.linalg.norm(d, axis=1, keepdims=True)
        parts.append(c + r[:, None] * d)
    parts.append(rng.random((n_background, 3)))
    pos = np.mod(np.concatenate(parts, axis=0), 1.0)
    vel = rng.normal(0.0, sigma_v, pos.shape) if sigma_v > 0 else np.zeros(pos.shape)
    ps = _finish(pos, vel, np.ones(3), "plummer_mixture",
                 meta={"centres": centres, "scale_radii": radii})
    return ps


def batch_counts(n_boxes: int = 256, n_min: int = 2048, n_max: int = 65536, seed: int = 0):
    """Log-uniform particle counts, one per box."""
    rng = np.random.default_rng(seed)
    return np.rint(np.exp(rng.uniform(math.log(n_min), math.log(n_max), n_boxes))).astype(np.int64)


def batch(n_boxes: int = 256, n_min: int = 2048, n_max: int = 65536, seed: int = 0):
    """Independent periodic unit boxes, uniform-random positions seeded by box id.

    Returns (concatenated ParticleSet with per-box masses and h0, offsets (nbox+1,),
    box lengths (nbox, 3)).
    """
    counts = batch_counts(n_boxes, n_min, n_max, seed)
    sets = [uniform(int(c), seed=b) for b, c in enumerate(counts)]
    offsets = np.concatenate([[0], np.cumsum(counts)]).astype(np.int64)
    cat = ParticleSet(pos=np.concatenate([s.pos for s in sets]),
                      vel=np.concatenate([s.vel for s in sets]),
                      m=np.concatenate([s.m for s in sets]),
                      u=np.concatenate([s.u for s in sets]),
                      h0=np.concatenate([s.h0 for s in sets]),
                      box=np.ones(3), name=f"batch{n_boxes}")
    lens = np.ones((n_boxes, 3))
    return cat, offsets, lens


SOD_LEFT = (4.0, 0.0, 1.0)       # (rho, v, P) on x < L/2
SOD_RIGHT = (1.0, 0.0, 0.1795)   # (rho, v, P) on x >= L/2


def sod(k: int = 16, length: float = 8.0, gamma: float = 5.0 / 3.0) -> ParticleSet:
    """Sod shock tube of Sec. 4.2 in a periodic length x 1 x 1 box.

    Lattice cells of edge 1/k: the dense half holds a face-centred cubic
    lattice (4 sites per cell), the light half a simple cubic one (1 site per
    cell), so that equal masses m = 1/k^3 give densities 4 and 1.  The
    internal energy per unit mass is set from the pressure of each side,
    u = P / ((gamma - 1) rho).  With k = 37 there are 810,448 + 202,612
    particles (the paper uses 800,000 + 200,000).  The interfaces are at
    x = length/2 and at x = 0 (periodic).
    """
    a = 1.0 / k
    nx = int(round(length * k))
    half = nx // 2
    ii, jj, kk = np.meshgrid(np.arange(half), np.arange(k), np.arange(k), indexing="ij")
    cell = np.stack([ii.ravel(), jj.ravel(), kk.ravel()], axis=1).astype(np.float64)
    fcc = np.array([[0.0, 0.0, 0.0], [0.5, 0.5, 0.0], [0.5, 0.0, 0.5], [0.0, 0.5, 0.5]]) + 0.25
    dense = ((cell[:, None, :] + fcc[None, :, :]) * a).reshape(-1, 3)
    light = (cell + np.array([half, 0.0, 0.0]) + 0.5) * a
    pos = np.concatenate([dense, light])
    n_d = dense.shape[0]
    n = pos.shape[0]
    box = np.array([nx * a, 1.0, 1.0])
    rl, _, pl = SOD_LEFT
    rr, _, pr = SOD_RIGHT
    u = np.empty(n)
    u[:n_d] = pl / ((gamma - 1.0) * rl)
    u[n_d:] = pr / ((gamma - 1.0) * rr)
    h0 = np.empty(n)
    h0[:n_d] = mean_spacing_h(4.0 * k ** 3)
    h0[n_d:] = mean_spacing_h(1.0 * k ** 3)
    return ParticleSet(pos=np.ascontiguousarray(pos), vel=np.zeros((n, 3)), m=np.full(n, a ** 3), u=u, h0=h0,
                       box=box, name=f"sod{n}", meta={"n_dense": n_d, "x0": box[0] / 2, "gamma": gamma})


def sedov(k: int = 24, E: float = 1.0, p_background: float = 1e-6, n_inject: int = 28,
          gamma: float = 5.0 / 3.0) -> ParticleSet:
    """Blast wave of Sec. 4.2: 4 k^3 particles on a face-centred cubic lattice
    (cells of edge 1/k) in the periodic unit cube, density 1, at rest, with
    pressure p_background everywhere except the n_inject particles nearest the
    box centre, which share the energy E equally (u_i = E / (n_inject m)).
    The centre is a tetrahedral site of the lattice, ringed by complete
    shells of 4, 12 and 12 particles: n_inject = 28 takes the three (the
    paper heats 26 particles of its lattice).  The paper uses about 101^3
    particles (k = 63 here gives 1,000,188).
    """
    a = 1.0 / k
    ii, jj, kk = np.meshgrid(np.arange(k), np.arange(k), np.arange(k), indexing="ij")
    cell = np.stack([ii.ravel(), jj.ravel(), kk.ravel()], axis=1).astype(np.float64)
    fcc = np.array([[0.0, 0.0, 0.0], [0.5, 0.5, 0.0], [0.5, 0.0, 0.5], [0.0, 0.5, 0.5]]) + 0.25
    pos = ((cell[:, None, :] + fcc[None, :, :]) * a).reshape(-1, 3)
    n = pos.shape[0]
    m = 1.0 / n
    r = np.linalg.norm(pos - 0.5, axis=1)
    hot = np.argsort(r, kind="stable")[:n_inject]
    u = np.full(n, p_background / (gamma - 1.0))
    u[hot] = E / (n_inject * m)
    return ParticleSet(pos=np.ascontiguousarray(pos), vel=np.zeros((n, 3)), m=np.full(n, m), u=u,
                       h0=np.full(n, mean_spacing_h(float(n))), box=np.ones(3), name=f"sedov{n}",
                       meta={"E": E, "rho0": 1.0, "centre": np.full(3, 0.5), "hot": hot, "gamma": gamma})


def density_target(pos: np.ndarray, mean_density: float, amp: float = 0.1) -> np.ndarray:
    """Sinusoidal target field rho_t(x) = mean * (1 + amp sin(2 pi x))."""
    return mean_density * (1.0 + amp * np.sin(2.0 * math.pi * pos[:, 0]))


# Named configurations
def config0() -> ParticleSet:
    """4096 uniform-random particles, unit cube, seed 0, v = 0, u = 1."""
    return uniform(4096, seed=0)


def config1(seed: int = 0) -> ParticleSet:
    """2^20 particles: 128 x 128 x 64 jittered lattice, spacing 1/128, v ~ N(0, 0.1)."""
    return lattice((128, 128, 64), 1.0 / 128, 0.1, 0.1, seed)


def config2(seed: int = 0) -> ParticleSet:
    """2^21 particles: 32 Plummer spheres + 20% uniform background."""
    return plummer_mixture(seed=seed)


def config4(seed: int = 0) -> ParticleSet:
    """64^3 jittered lattice in the unit cube, v ~ N(0, 0.1)."""
    return lattice((64, 64, 64), 1.0 / 64, 0.1, 0.1, seed)


def small_lattice(k: int = 16, jitter: float = 0.1, sigma_v: float = 0.1, seed: int = 0) -> ParticleSet:
    """k^3 jittered lattice in the unit cube (small parity case)."""
    return lattice((k, k, k), 1.0 / k, jitter, sigma_v, seed)
