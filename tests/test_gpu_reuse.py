"""GPU parity of pseudo-Verlet reuse (sph_refresh; params.reuse in the step):
density and force on a decomposition built before the particles moved,
against the oracle at the moved positions, under the tolerances of
parity_util (the result of a sweep does not depend on which cell pair finds a
pair, so reuse may only change the summation order).  Covers a drift inside
the slack (no rebuild), a drift beyond it (sph_density rebuilds), particles
that cross the periodic box face, the hierarchy, several boxes, and steps of
the integrator with reuse against the oracle's steps."""
import numpy as np
import pytest
import torch

import oracle
from paper_1404_2303_amd import sph, workloads
from parity_util import compare, log, oracle_run

pytestmark = pytest.mark.gpu


def _state(n=3000, seed=91, sigma_v=0.3):
    rng = np.random.default_rng(seed)
    ps = workloads.uniform(n, seed=seed, sigma_v=sigma_v)
    ps.m[:] *= rng.uniform(0.6, 1.4, n)
    ps.u[:] = rng.uniform(0.5, 1.5, n)
    return ps


def _moved(ps, shift):
    q = workloads.ParticleSet(pos=np.mod(ps.pos + shift, ps.box), vel=ps.vel.copy(), m=ps.m.copy(), u=ps.u.copy(),
                              h0=ps.h0.copy(), box=ps.box.copy())
    return q


def _to_dev(parts, q):
    for d, k in enumerate("xyz"):
        getattr(parts, k).copy_(torch.as_tensor(q.pos[:, d]))


def _collect(ctx, parts, d, f):
    torch.cuda.synchronize()
    out = {k: v.cpu().numpy() for k, v in d.items()}
    out.update({k: v.cpu().numpy() for k, v in f.items()})
    out["h"] = parts.h.cpu().numpy()
    out["a"] = np.stack([out["ax"], out["ay"], out["az"]], axis=1)
    out["stats"] = ctx.stats()
    return out


def _refresh_run(ps, q, precision, **params):
    """Build and sort on ps (h solved there), then move to q, refresh, density, force."""
    parts = sph.Particles.from_numpy(ps, "cuda:0")
    ctx = sph.Context(ps.box, precision=precision, **params)
    ctx.run(parts)
    _to_dev(parts, q)
    ctx.refresh(parts)
    d = ctx.density(parts)
    f = ctx.force(parts)
    out = _collect(ctx, parts, d, f)
    ctx.close()
    return out


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_refresh_within_the_slack(precision):
    ps = _state()
    rng = np.random.default_rng(1)
    shift = rng.normal(0.0, 0.002, ps.pos.shape)
    q = _moved(ps, shift)
    log(f"case refresh small drift {ps.n} {precision}")
    g = _refresh_run(ps, q, precision)
    st = g["stats"]
    log(f"  stats {st}")
    assert st["refreshes"] == 1 and st["rebuilds"] == 0 and st["drift"] > 0
    ref = oracle_run(q, h0=ps.h0)
    compare(g, ref, precision, label="refresh")


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_refresh_beyond_the_slack_rebuilds(precision):
    ps = _state(seed=92)
    rng = np.random.default_rng(2)
    q = _moved(ps, rng.normal(0.0, 0.03, ps.pos.shape))
    log(f"case refresh large drift {ps.n} {precision}")
    g = _refresh_run(ps, q, precision)
    log(f"  stats {g['stats']}")
    assert g["stats"]["rebuilds"] >= 1
    ref = oracle_run(q, h0=ps.h0)
    compare(g, ref, precision, label="refresh-rebuild")


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_refresh_across_the_periodic_face(precision):
    # every particle moves by +0.004 in x: those within 0.004 of x = 1 wrap to x ~ 0
    # while their cell stays at the upper face
    ps = _state(seed=93)
    q = _moved(ps, np.array([0.004, -0.003, 0.002]))
    crossing = np.sum(ps.pos[:, 0] > 1.0 - 0.004)
    log(f"case refresh periodic crossing {ps.n} {precision} ({crossing} particles cross x = 1)")
    assert crossing > 0
    g = _refresh_run(ps, q, precision)
    assert g["stats"]["rebuilds"] == 0
    ref = oracle_run(q, h0=ps.h0)
    compare(g, ref, precision, label="refresh-periodic")


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
@pytest.mark.parametrize("resort", [False, True])
def test_refresh_moving_next_to_resting(precision, resort):
    # the half x > 0.5 is scrambled by random displacements (its stored orderings
    # go stale), the other half is at rest: sweeps of resting targets over moving
    # sources need the full allowance of the sources' stale orderings
    ps = _state(6000, 95)
    rng = np.random.default_rng(5)
    shift = rng.normal(0.0, 0.006, ps.pos.shape) * (ps.pos[:, :1] > 0.5)
    q = _moved(ps, shift)
    log(f"case refresh moving|resting {ps.n} {precision} resort={resort}")
    parts = sph.Particles.from_numpy(ps, "cuda:0")
    ctx = sph.Context(ps.box, precision=precision)
    ctx.run(parts)
    _to_dev(parts, q)
    ctx.refresh(parts)
    if resort:
        ctx.sort()
    d = ctx.density(parts)
    f = ctx.force(parts)
    g = _collect(ctx, parts, d, f)
    ctx.close()
    log(f"  stats {g['stats']}")
    assert g["stats"]["refreshes"] == 1 and g["stats"]["rebuilds"] == 0
    ref = oracle_run(q, h0=ps.h0)
    compare(g, ref, precision, label="refresh-half")


def test_refresh_on_the_hierarchy():
    rng = np.random.default_rng(7)
    clump = 0.5 + 0.04 * rng.normal(size=(3000, 3))
    pos = np.mod(np.concatenate([clump, rng.random((3000, 3))]), 1.0)
    ps = workloads._finish(pos, rng.normal(0, 0.3, pos.shape), np.ones(3), "clump")
    log("case refresh hierarchy fp32")
    parts = sph.Particles.from_numpy(ps, "cuda:0")
    ctx = sph.Context(ps.box, precision="fp32", max_depth=6, split_count=64, split_frac=0.5)
    ctx.estimate_h(parts)
    ctx.run(parts)
    h_built = parts.h.cpu().numpy()
    # the leaves deep in the clump have h ~ 0.005 and a slack of ~10% of it:
    # a drift of ~1e-4 stays inside
    q = _moved(ps, rng.normal(0.0, 1e-5, ps.pos.shape))
    _to_dev(parts, q)
    ctx.refresh(parts)
    d = ctx.density(parts)
    f = ctx.force(parts)
    g = _collect(ctx, parts, d, f)
    ctx.close()
    log(f"  stats {g['stats']}")
    assert g["stats"]["depth"] > 0 and g["stats"]["refreshes"] == 1 and g["stats"]["rebuilds"] == 0
    ref = oracle_run(q, h0=h_built)
    compare(g, ref, "fp32", label="refresh-tree")


def _steps(ps, precision, dt, nsteps, reuse, batch=None):
    parts = sph.Particles.from_numpy(ps, "cuda:0")
    box = ps.box if batch is None else (1.0, 1.0, 1.0)
    ctx = sph.Context(box, precision=precision, reuse=int(reuse))
    b = None if batch is None else sph.Batch(*batch)
    d, f = ctx.run(parts, b)
    acc = {k: f[k] for k in ("ax", "ay", "az", "dudt")}
    out, refreshes = [], 0
    for _ in range(nsteps):
        ctx.step(parts, acc, dt, b)
        torch.cuda.synchronize()
        st = ctx.stats()
        refreshes += 1 if st["refreshes"] > 0 and st["rebuilds"] == 0 else 0
        out.append({"pos": np.stack([parts.x.cpu().numpy(), parts.y.cpu().numpy(), parts.z.cpu().numpy()], 1),
                    "vel": np.stack([parts.vx.cpu().numpy(), parts.vy.cpu().numpy(), parts.vz.cpu().numpy()], 1),
                    "u": parts.u.cpu().numpy(), "h": parts.h.cpu().numpy()})
    ctx.close()
    return out, refreshes


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
@pytest.mark.parametrize("mode", [sph.SPH_REUSE_ORDERINGS, sph.SPH_REUSE_CELLS])
def test_steps_with_reuse_match_oracle(precision, mode):
    ps = _state(2000, 94, sigma_v=0.4)
    dt, nsteps = 0.002, 4
    log(f"case kdk with reuse mode {mode} {ps.n} {precision}")
    g, reused = _steps(ps, precision, dt, nsteps, mode)
    f = oracle.full_pass(ps.pos, ps.vel, ps.m, ps.u, ps.h0, ps.box)
    pos, vel, u, h, a, du = ps.pos, ps.vel, ps.u, f["h"], f["force"]["a"], f["force"]["dudt"]
    kap = f["force"]["kappa_a"]
    tol = {"fp64": 1e-8, "fp32": 1e-4}[precision]
    for k in range(nsteps):
        r = oracle.kdk_step(pos, vel, ps.m, u, h, ps.box, a, du, dt)
        pos, vel, u, h, a, du = r["pos"], r["vel"], r["u"], r["h"], r["a"], r["dudt"]
        vs = np.sqrt(np.mean(np.sum(r["vel"] ** 2, 1))) + (k + 1) * dt * np.sqrt(np.mean(kap ** 2))
        ev = np.max(np.abs(g[k]["vel"] - r["vel"])) / vs
        eu = np.max(np.abs(g[k]["u"] - r["u"])) / (1.0 + (k + 1) * dt * np.sqrt(np.mean(kap ** 2)))
        log(f"  step {k + 1}: v {ev:.2e} u {eu:.2e}")
        assert ev <= tol and eu <= tol
    log(f"  steps that reused the decomposition: {reused} of {nsteps}")
    assert reused >= nsteps - 1


def test_batched_steps_with_reuse_match_plain_steps():
    boxes = [(1.0, 1.0, 1.0), (0.8, 1.0, 0.9), (1.2, 0.9, 1.0)]
    sets = [workloads.uniform(n, seed=160 + b, box=bx, sigma_v=0.3) for b, (n, bx) in
            enumerate(zip((1500, 2600, 4000), boxes))]
    offsets = np.concatenate([[0], np.cumsum([s_.n for s_ in sets])]).astype(np.int64)
    cat = workloads.ParticleSet(pos=np.concatenate([s_.pos for s_ in sets]),
                                vel=np.concatenate([s_.vel for s_ in sets]),
                                m=np.concatenate([s_.m for s_ in sets]), u=np.concatenate([s_.u for s_ in sets]),
                                h0=np.concatenate([s_.h0 for s_ in sets]), box=np.ones(3))
    lens = np.asarray(boxes, dtype=np.float64)
    log(f"case batched kdk with reuse {cat.n} in 3 boxes")
    a, reused = _steps(cat, "fp64", 0.003, 3, sph.SPH_REUSE_ORDERINGS, batch=(offsets, lens))
    b, _ = _steps(cat, "fp64", 0.003, 3, sph.SPH_REUSE_OFF, batch=(offsets, lens))
    assert reused >= 2
    for k in range(3):
        for key in ("vel", "u", "h"):
            scale = np.max(np.abs(b[k][key])) + 1e-300
            e = np.max(np.abs(a[k][key] - b[k][key])) / scale
            log(f"  step {k + 1} {key}: {e:.2e}")
            assert e <= 1e-10
