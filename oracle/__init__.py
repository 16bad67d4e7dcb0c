"""FP64 CPU oracle for the SPH density and force stages (TEST INFRASTRUCTURE).

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  The GPU library never calls it and
shares no code with it.

The arithmetic lives in ``sph_oracle.c`` (plain C, FP64, one-sided gathers
over a periodic cell list); this module only marshals numpy arrays.  Each
function names the part of Gonnet (2014) it evaluates:

* :func:`kernel_w`, :func:`kernel_dw`, :func:`kernel_d2w` -- cubic spline w(q) and
  its first two derivatives, Sec. 2.1.
* :func:`solve_h` -- Newton iteration of Eq. (3) for N_i(h_i) = N_ngb.
* :func:`density` -- Eq. (2), Eq. (3) and dN/dh, drho/dh (for Omega), and the
  velocity divergence and curl of Sec. 4.1.
* :func:`ghost` -- Omega, P, sound speed, A = P/(Omega rho^2), Balsara f.
* :func:`force` -- Eqs. (4)-(5) plus the Monaghan-Balsara viscosity, Sec. 4.1.
* :func:`full_pass` -- the two stages in the paper's order (Sec. 2.1:
  density for all particles first, then force).
* :func:`signal_dt` -- the signal speed and time step of Eq. (6).
* :func:`kdk_step` -- one kick-drift-kick velocity-Verlet step with a fixed
  time step (the integrator of Sec. 4.1).
* :func:`integrate` -- kick-drift-kick steps to a final time, each step
  limited by the smallest time step of Eq. (6).
* :func:`time_bin`, :func:`mts_integrate` -- multiple time-stepping: power-of-two
  time bins, only the particles at the end of their own step active.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "sph_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

GAMMA = 5.0 / 3.0   # Sec. 4.2 constants
ALPHA = 0.8
N_NGB = 48.0
CFL = 0.25

ORA_OK, ORA_E_ARG, ORA_E_H_TOO_LARGE, ORA_E_NOT_CONVERGED, ORA_E_OOM = 0, 1, 2, 3, 4


class OracleError(RuntimeError):
    pass


def build(force: bool = True) -> str:
    """Compile sph_oracle.c into liboracle.so (gcc, -O2, OpenMP, no fast-math)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        cmd = ["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-o", tmp, _SRC, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=True)
        lib = ctypes.CDLL(_LIB)
        d, i64, i32 = ctypes.c_double, ctypes.c_int64, ctypes.c_int
        P = ctypes.c_void_p
        lib.ora_w.restype = d
        lib.ora_w.argtypes = [d]
        lib.ora_dw.restype = d
        lib.ora_dw.argtypes = [d]
        lib.ora_W.restype = d
        lib.ora_W.argtypes = [d, d]
        lib.ora_dWdr.restype = d
        lib.ora_dWdr.argtypes = [d, d]
        lib.ora_d2w.restype = d
        lib.ora_d2w.argtypes = [d]
        lib.ora_dWdr_dlnh.restype = d
        lib.ora_dWdr_dlnh.argtypes = [d, d]
        lib.ora_dWdh.restype = d
        lib.ora_dWdh.argtypes = [d, d]
        lib.ora_solve_h.restype = i32
        lib.ora_solve_h.argtypes = [i64, P, P, P, P, d, d, i32, i64, P, P, P]
        lib.ora_density.restype = i32
        lib.ora_density.argtypes = [i64, P, P, P, P, P, P, P, P, P, i64, P] + [P] * 8
        lib.ora_ghost.restype = None
        lib.ora_ghost.argtypes = [i64, P, P, P, P, P, P, d, i32, P, P, P, P, P]
        lib.ora_signal.restype = i32
        lib.ora_signal.argtypes = [i64, P, P, P, P, P, P, P, P, P, d, i64, P, P, P, P, P]
        lib.ora_force.restype = i32
        lib.ora_force.argtypes = [i64, P, P, P, P, P, P, P, P, P, P, P, P, P, d, i64, P] + [P] * 10
        lib.ora_bands.restype = i32
        lib.ora_bands.argtypes = [i64, P, P, P, P, P, P, i64, P, P, P]
        lib.ora_num_threads.restype = i32
        lib.ora_num_threads.argtypes = []
        lib.ora_set_num_threads.restype = None
        lib.ora_set_num_threads.argtypes = [i32]
        _lib = lib
    return _lib


def _c(a, dtype=np.float64):
    return np.ascontiguousarray(a, dtype=dtype)


def _p(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def _check(st, what):
    if st != ORA_OK:
        names = {1: "invalid argument", 2: "h too large for the periodic box",
                 3: "not converged", 4: "out of memory"}
        raise OracleError(f"{what}: {names.get(st, st)}")


def num_threads() -> int:
    return int(_load().ora_num_threads())


def set_num_threads(n: int) -> None:
    """Threads of the OpenMP loops of the calls that follow."""
    _load().ora_set_num_threads(int(n))


def kernel_w(q):
    lib = _load()
    return np.array([lib.ora_w(float(v)) for v in np.atleast_1d(q)])


def kernel_dw(q):
    lib = _load()
    return np.array([lib.ora_dw(float(v)) for v in np.atleast_1d(q)])


def kernel_d2w(q):
    lib = _load()
    return np.array([lib.ora_d2w(float(v)) for v in np.atleast_1d(q)])


def kernel_W(r, h):
    return _load().ora_W(float(r), float(h))


def kernel_dWdr(r, h):
    return _load().ora_dWdr(float(r), float(h))


def kernel_dWdh(r, h):
    return _load().ora_dWdh(float(r), float(h))


def _split(pos):
    pos = np.asarray(pos, dtype=np.float64)
    return _c(pos[:, 0]), _c(pos[:, 1]), _c(pos[:, 2])


def _sel(sel, n):
    if sel is None:
        return n, None
    s = _c(sel, np.int64)
    return len(s), s


def solve_h(pos, h0, box, target=N_NGB, tol=1e-10, maxit=100, sel=None, raise_on_fail=True):
    """Smoothing lengths with N_i(h_i) = target (Eq. (3)); returns (h, iters)."""
    lib = _load()
    x, y, z = _split(pos)
    n = len(x)
    h = _c(np.broadcast_to(np.asarray(h0, dtype=np.float64), (n,))).copy()
    it = np.zeros(n, dtype=np.int32)
    L = _c(box)
    ns, s = _sel(sel, n)
    st = lib.ora_solve_h(n, _p(x), _p(y), _p(z), _p(L), float(target), float(tol), int(maxit),
                         ns, _p(s), _p(h), _p(it))
    if raise_on_fail:
        _check(st, "solve_h")
    return h, it


def density(pos, vel, m, h, box, sel=None):
    """Density-stage sums at fixed h (Eq. (2), Eq. (3), Sec. 4.1 div/curl)."""
    lib = _load()
    x, y, z = _split(pos)
    n = len(x)
    vel = np.zeros((n, 3)) if vel is None else np.asarray(vel, dtype=np.float64)
    vx, vy, vz = _c(vel[:, 0]), _c(vel[:, 1]), _c(vel[:, 2])
    m = _c(np.broadcast_to(np.asarray(m, dtype=np.float64), (n,)))
    h = _c(h)
    L = _c(box)
    ns, s = _sel(sel, n)
    out = {k: np.full(n, np.nan) for k in ("rho", "nngb", "dndh", "drhodh", "div")}
    out["curl"] = np.full((n, 3), np.nan)
    out["count"] = np.full(n, -1, dtype=np.int32)
    out["band"] = np.full(n, -1, dtype=np.int32)
    st = lib.ora_density(n, _p(x), _p(y), _p(z), _p(vx), _p(vy), _p(vz), _p(m), _p(h), _p(L),
                         ns, _p(s), _p(out["rho"]), _p(out["nngb"]), _p(out["dndh"]),
                         _p(out["drhodh"]), _p(out["div"]), _p(out["curl"]), _p(out["count"]),
                         _p(out["band"]))
    _check(st, "density")
    return out


def ghost(dens, u, h, gamma=GAMMA, balsara_form=0):
    """Omega, P, c, A, Balsara f from the density-stage sums (Sec. 2.1, Sec. 4.1).

    balsara_form 0 puts |curl v| over the denominator, as Sec. 4.1 prints the
    switch; 1 puts |div v| there, the switch of Balsara (1995) that it cites.
    """
    lib = _load()
    rho = _c(dens["rho"])
    n = len(rho)
    u = _c(np.broadcast_to(np.asarray(u, dtype=np.float64), (n,)))
    out = {k: np.empty(n) for k in ("omega", "P", "c", "A", "f")}
    lib.ora_ghost(n, _p(rho), _p(_c(dens["drhodh"])), _p(_c(h)), _p(u), _p(_c(dens["div"])),
                  _p(_c(dens["curl"])), float(gamma), int(balsara_form), _p(out["omega"]), _p(out["P"]),
                  _p(out["c"]), _p(out["A"]), _p(out["f"]))
    return out


def force(pos, vel, m, h, rho, A, c, f, box, alpha=ALPHA, sel=None):
    """Eqs. (4)-(5) with Monaghan-Balsara viscosity (Sec. 4.1).  Besides a and
    du/dt: kappa_a, kappa_u (sums of the magnitudes of the pair terms) and
    sens_a, sens_u (sums of the magnitudes of each pair term's derivatives with
    respect to ln h_i and ln h_j, the other inputs held fixed): the scales of
    the rounding and of the h tolerance in a and du/dt."""
    lib = _load()
    x, y, z = _split(pos)
    n = len(x)
    vel = np.zeros((n, 3)) if vel is None else np.asarray(vel, dtype=np.float64)
    vx, vy, vz = _c(vel[:, 0]), _c(vel[:, 1]), _c(vel[:, 2])
    m = _c(np.broadcast_to(np.asarray(m, dtype=np.float64), (n,)))
    L = _c(box)
    ns, s = _sel(sel, n)
    out = {k: np.full(n, np.nan) for k in ("ax", "ay", "az", "dudt", "kappa_a", "kappa_u", "sens_a", "sens_u")}
    out["count"] = np.full(n, -1, dtype=np.int32)
    out["band"] = np.full(n, -1, dtype=np.int32)
    st = lib.ora_force(n, _p(x), _p(y), _p(z), _p(vx), _p(vy), _p(vz), _p(m), _p(_c(h)),
                       _p(_c(rho)), _p(_c(A)), _p(_c(c)), _p(_c(f)), _p(L), float(alpha), ns, _p(s),
                       _p(out["ax"]), _p(out["ay"]), _p(out["az"]), _p(out["dudt"]),
                       _p(out["kappa_a"]), _p(out["kappa_u"]), _p(out["count"]), _p(out["band"]),
                       _p(out["sens_a"]), _p(out["sens_u"]))
    _check(st, "force")
    out["a"] = np.stack([out["ax"], out["ay"], out["az"]], axis=1)
    return out


def signal_dt(pos, vel, h, c, box, cfl=CFL, sel=None):
    """Signal speed and time step of Eq. (6) (vsig, vsig_lo, vsig_hi, dt)."""
    lib = _load()
    x, y, z = _split(pos)
    n = len(x)
    vel = np.zeros((n, 3)) if vel is None else np.asarray(vel, dtype=np.float64)
    vx, vy, vz = _c(vel[:, 0]), _c(vel[:, 1]), _c(vel[:, 2])
    ns, s = _sel(sel, n)
    out = {k: np.full(n, np.nan) for k in ("vsig", "vsig_lo", "vsig_hi", "dt")}
    st = lib.ora_signal(n, _p(x), _p(y), _p(z), _p(vx), _p(vy), _p(vz), _p(_c(h)), _p(_c(c)),
                        _p(_c(box)), float(cfl), ns, _p(s), _p(out["vsig"]), _p(out["vsig_lo"]),
                        _p(out["vsig_hi"]), _p(out["dt"]))
    _check(st, "signal_dt")
    return out


def bands(pos, h, box, width, sel=None):
    """Pairs that a smoothing length known to relative precision ``width``
    (scalar or one value per particle) may classify either way: per particle,
    the pairs within that relative distance of the density range r < h_i
    ("dband") and of the force range r < max(h_i, h_j) ("fband", with the
    width of whichever particle has the larger h).  Counting only."""
    lib = _load()
    x, y, z = _split(pos)
    n = len(x)
    bw = _c(np.broadcast_to(np.asarray(width, dtype=np.float64), (n,)))
    ns, s = _sel(sel, n)
    out = {"dband": np.full(n, -1, dtype=np.int32), "fband": np.full(n, -1, dtype=np.int32)}
    st = lib.ora_bands(n, _p(x), _p(y), _p(z), _p(_c(h)), _p(bw), _p(_c(box)), ns, _p(s),
                       _p(out["dband"]), _p(out["fband"]))
    _check(st, "bands")
    return out


def h_precision(h, dndh, h_rel, ngb_tol):
    """Relative precision of a smoothing length solved to |N - n_ngb| <= ngb_tol
    with h itself compared to h_rel: max(h_rel, ngb_tol / (h |dN/dh|)), and no
    finer than the 1e-6 rounding band of the support."""
    return np.maximum(np.maximum(h_rel, 1e-6), ngb_tol / (np.asarray(h) * np.abs(np.asarray(dndh))))


def full_pass(pos, vel, m, u, h0, box, target=N_NGB, tol=1e-10, maxit=100,
              gamma=GAMMA, alpha=ALPHA, force_sel=None, balsara_form=0, cfl=CFL):
    """Density stage for every particle (h solved), then the force stage.

    The two stages run in the order of Sec. 2.1: all densities (and the
    per-particle ghost quantities) before any force.  ``force_sel`` restricts
    the force stage and the time step of Eq. (6) to a subset of particles
    (their neighbours' ghost quantities are still computed for all particles).
    """
    h, iters = solve_h(pos, h0, box, target=target, tol=tol, maxit=maxit)
    dens = density(pos, vel, m, h, box)
    gh = ghost(dens, u, h, gamma=gamma, balsara_form=balsara_form)
    frc = force(pos, vel, m, h, dens["rho"], gh["A"], gh["c"], gh["f"], box, alpha=alpha,
                sel=force_sel)
    sig = signal_dt(pos, vel, h, gh["c"], box, cfl=cfl, sel=force_sel)
    return {"h": h, "iters": iters, "dens": dens, "ghost": gh, "force": frc, "signal": sig}


def kdk_step(pos, vel, m, u, h, box, a_old, dudt_old, dt, target=N_NGB, tol=1e-10, gamma=GAMMA, alpha=ALPHA,
             balsara_form=0, cfl=CFL):
    """One kick-drift-kick step (Sec. 4.1 names velocity Verlet with a fixed
    step).  The forces at the new positions need velocities and energies at
    the new time, which the kick has not produced yet; they are predicted
    with the old accelerations (v_half + dt/2 a_old, u_half + dt/2 dudt_old).

    Returns a dict with the new pos (wrapped into the box), vel, u, the solved
    h (h is the initial guess), and the new a and du/dt.
    """
    box = np.asarray(box, dtype=np.float64)
    hdt = 0.5 * dt
    v_half = np.asarray(vel, dtype=np.float64) + hdt * np.asarray(a_old, dtype=np.float64)
    u_half = np.asarray(u, dtype=np.float64) + hdt * np.asarray(dudt_old, dtype=np.float64)
    x_new = np.mod(np.asarray(pos, dtype=np.float64) + dt * v_half, box)
    x_new = np.where(x_new >= box, x_new - box, x_new)
    v_pred = v_half + hdt * np.asarray(a_old, dtype=np.float64)
    u_pred = u_half + hdt * np.asarray(dudt_old, dtype=np.float64)
    out = full_pass(x_new, v_pred, m, u_pred, h, box, target=target, tol=tol, gamma=gamma, alpha=alpha,
                    balsara_form=balsara_form, cfl=cfl)
    a_new = out["force"]["a"]
    du_new = out["force"]["dudt"]
    return {"pos": x_new, "vel": v_half + hdt * a_new, "u": u_half + hdt * du_new, "h": out["h"],
            "a": a_new, "dudt": du_new, "dt": out["signal"]["dt"]}


def integrate(pos, vel, m, u, h, box, t_end, dt_max, max_steps=100000, **kw):
    """Kick-drift-kick steps from t = 0 to t_end, each step as long as the
    smallest time step of Eq. (6) of the previous force evaluation allows
    (Sec. 4.2 runs its blast wave this way), capped by dt_max and clipped so
    that the last step ends at t_end.  Starts with a full pass for the
    initial accelerations.  Returns the final state and the steps taken.
    """
    box = np.asarray(box, dtype=np.float64)
    f0 = full_pass(pos, vel, m, u, h, box, **kw)
    st = {"pos": np.asarray(pos, dtype=np.float64), "vel": np.asarray(vel, dtype=np.float64),
          "u": np.asarray(u, dtype=np.float64), "h": f0["h"], "a": f0["force"]["a"],
          "dudt": f0["force"]["dudt"], "dt": f0["signal"]["dt"]}
    t, steps = 0.0, []
    while t < t_end and len(steps) < max_steps:
        dt = min(float(np.min(st["dt"])), dt_max)
        last = t + dt >= t_end
        if last:
            dt = t_end - t
        st = kdk_step(st["pos"], st["vel"], m, st["u"], st["h"], box, st["a"], st["dudt"], dt, **kw)
        t = t_end if last else t + dt
        steps.append(dt)
    st["t"] = t
    st["steps"] = np.array(steps)
    return st


def time_bin(dt, dt_base, max_bin, n_next):
    """Time bin of each particle for multiple time-stepping (Sec. 4.1): the
    largest k with 2^k dt_base <= dt (k >= 0; the bin whose step does not
    exceed the particle's own step of Eq. (6)), at most max_bin, and lowered
    until the particle's next step starts on a multiple of its length:
    n_next % 2^k == 0, n_next the index of the next base step."""
    dt = np.asarray(dt, dtype=np.float64)
    # floor(log2(dt / dt_base)) exactly: dt / dt_base = mant 2^e with mant in [1/2, 1)
    _, e = np.frexp(np.where(np.isfinite(dt) & (dt > 0), dt / dt_base, 1.0))
    k = np.clip(e.astype(np.int64) - 1, 0, max_bin)
    k = np.where(np.isinf(dt), max_bin, k)
    while True:
        bad = (k > 0) & ((n_next % (1 << k)) != 0)
        if not bad.any():
            return k
        k = np.where(bad, k - 1, k)


def mts_integrate(pos, vel, m, u, h, box, dt_base, max_bin, nsteps, target=N_NGB, tol=1e-10, gamma=GAMMA,
                  alpha=ALPHA, balsara_form=0, cfl=CFL):
    """Multiple time-stepping (Sec. 4.1): particle i sits in time bin k_i
    (time_bin) and takes kick-drift-kick steps of 2^k_i dt_base; it is active,
    i.e. included in the density and force calculations as a target, only at
    the ends of its own steps.  One base step n:

      1. particles starting a step (n % 2^k == 0) take the opening half kick
         v += T/2 a, u += T/2 du/dt with their own T = 2^k dt_base;
      2. every particle drifts, x += dt_base v;
      3. particles ending a step ((n+1) % 2^k == 0) are active: their h is
         solved and their density-stage quantities (rho, A, c, f) recomputed at
         the new positions; the other particles keep the values of their last
         active step.  Velocities and energies enter at the end of the base
         step, predicted from each particle's last kick with its stored
         acceleration;
      4. the active particles' forces (every particle a source), the closing
         half kick with the new accelerations, their new time step of Eq. (6)
         and their new bin.

    The initial state is one full pass with every particle active.  Returns
    the final state (pos, vel, u, h, a, dudt, dt, bins) and the number of
    active particles of each base step.
    """
    box = np.asarray(box, dtype=np.float64)
    kw = dict(target=target, tol=tol, gamma=gamma, alpha=alpha, balsara_form=balsara_form, cfl=cfl)
    f0 = full_pass(pos, vel, m, u, h, box, **kw)
    x = np.asarray(pos, dtype=np.float64).copy()
    v = np.asarray(vel, dtype=np.float64).copy()
    uu = np.broadcast_to(np.asarray(u, dtype=np.float64), (len(x),)).copy()
    h = f0["h"].copy()
    rho, A, c, f = f0["dens"]["rho"].copy(), f0["ghost"]["A"].copy(), f0["ghost"]["c"].copy(), f0["ghost"]["f"].copy()
    a, du, dt = f0["force"]["a"].copy(), f0["force"]["dudt"].copy(), f0["signal"]["dt"].copy()
    bins = time_bin(dt, dt_base, max_bin, 0)
    counts = []
    for n in range(nsteps):
        span = np.left_shift(1, bins)
        T = span * dt_base
        start = (n % span) == 0
        v += (start * 0.5 * T)[:, None] * a
        uu += start * 0.5 * T * du
        x = np.mod(x + dt_base * v, box)
        x = np.where(x >= box, x - box, x)
        tau = ((n % span) + 1) * dt_base - 0.5 * T
        pv = v + tau[:, None] * a
        pu = uu + tau * du
        sel = np.where(((n + 1) % span) == 0)[0]
        counts.append(len(sel))
        if len(sel) == 0:
            continue
        h, _ = solve_h(x, h, box, target=target, tol=tol, sel=sel)
        d = density(x, pv, m, h, box, sel=sel)
        g = ghost(d, pu, h, gamma=gamma, balsara_form=balsara_form)
        rho[sel], A[sel], c[sel], f[sel] = d["rho"][sel], g["A"][sel], g["c"][sel], g["f"][sel]
        fr = force(x, pv, m, h, rho, A, c, f, box, alpha=alpha, sel=sel)
        sig = signal_dt(x, pv, h, c, box, cfl=cfl, sel=sel)
        a[sel], du[sel], dt[sel] = fr["a"][sel], fr["dudt"][sel], sig["dt"][sel]
        v[sel] += (0.5 * T[sel])[:, None] * a[sel]
        uu[sel] += 0.5 * T[sel] * du[sel]
        bins[sel] = time_bin(dt[sel], dt_base, max_bin, n + 1)
    return {"pos": x, "vel": v, "u": uu, "h": h, "a": a, "dudt": du, "dt": dt, "bins": bins,
            "active": np.array(counts), "rho": rho, "A": A, "c": c, "f": f}
