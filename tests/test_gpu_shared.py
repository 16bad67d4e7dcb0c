"""GPU parity of the shared sweep layout (sph_params.sweep = SPH_SWEEP_SHARED):
the sources of a target cell staged once per work-group, four lanes per
target, cells that need several staging batches left to the split kernels.

The oracle and the tolerances are those of test_gpu_parity (tests/parity_util.py);
the layouts differ only in the order of summation.  Cases: a uniform set
whose dense cells exceed the shared staging (deferred cells next to swept
ones), the jittered lattice (no deferral), a particle whose lists overflow,
coincident pairs, cells of more than 64 particles (several rounds of 64
targets), the 2^20 lattice sample of the bench line, the multiple
time-stepping masks, and the adjoint fed by a shared forward pass.
"""
import os

import numpy as np
import pytest
import torch

import oracle
from oracle import grad as og
from paper_1404_2303_amd import sph, workloads
from parity_util import compare, compare_sample, gpu_run, load_sample, log, oracle_run

pytestmark = pytest.mark.gpu
HERE = os.path.dirname(os.path.abspath(__file__))
SHARED = {"sweep": sph.SPH_SWEEP_SHARED}


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_shared_config0_with_deferred_cells(precision):
    ps = workloads.config0()
    log(f"case shared config0 {precision}")
    ref = oracle_run(ps)
    g = gpu_run(ps, precision, **SHARED)
    compare(g, ref, precision, label="shared config0")


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_shared_lattice(precision):
    ps = workloads.small_lattice(16)
    log(f"case shared lattice 16^3 {precision}")
    ref = oracle_run(ps)
    g = gpu_run(ps, precision, **SHARED)
    compare(g, ref, precision, label="shared lattice16")


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_shared_same_as_split(precision):
    # both layouts on one input: the same h and counts; sums equal up to order
    ps = workloads.uniform(3001, seed=21, box=(1.0, 0.7, 0.55), sigma_v=0.3)
    log(f"case shared vs split ragged 3001 {precision}")
    a = gpu_run(ps, precision, sweep=sph.SPH_SWEEP_SPLIT)
    b = gpu_run(ps, precision, **SHARED)
    np.testing.assert_array_equal(a["n_dens"], b["n_dens"])
    np.testing.assert_array_equal(a["n_pairs"], b["n_pairs"])
    rel = 1e-12 if precision == "fp64" else 1e-5
    assert np.max(np.abs(a["h"] / b["h"] - 1.0)) <= rel
    assert np.max(np.abs(a["rho"] / b["rho"] - 1.0)) <= 10 * rel


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_shared_list_overflow(precision):
    # one particle at the centre of an empty sphere: ~100 neighbours, more
    # than a list holds, so its lists are evaluated as they fill
    ps = workloads.uniform(3000, seed=31, sigma_v=0.3)
    c = np.array([0.5, 0.5, 0.5])
    keep = np.linalg.norm(ps.pos - c, axis=1) > 0.12
    n = int(keep.sum()) + 1
    ps = workloads.ParticleSet(pos=np.concatenate([ps.pos[keep], c[None]]),
                               vel=np.concatenate([ps.vel[keep], np.zeros((1, 3))]),
                               m=np.full(n, 1.0 / n), u=np.ones(n), h0=np.full(n, ps.h0[0]), box=ps.box,
                               name="void")
    log(f"case shared void {n} {precision}")
    ref = oracle_run(ps)
    assert ref["force"]["count"][-1] > 100
    g = gpu_run(ps, precision, **SHARED)
    compare(g, ref, precision, label="shared void")


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_shared_coincident_particles(precision):
    ps = workloads.uniform(3000, seed=43, sigma_v=0.3)
    ps.pos[2000:2060] = ps.pos[:60]
    log(f"case shared coincident pairs 3000 {precision}")
    ref = oracle_run(ps)
    g = gpu_run(ps, precision, **SHARED)
    for k in ("rho", "h", "a", "dudt", "div_v", "curl_v", "balsara"):
        assert np.all(np.isfinite(g[k])), k
    compare(g, ref, precision, label="shared coincident")


@pytest.mark.parametrize("cell_target", [100, 200])
def test_shared_cells_of_several_rounds(cell_target):
    # cells of about 100 and 200 particles: two and more rounds of 64 targets
    # over one staging (or deferred when their sources do not fit)
    ps = workloads.uniform(20000, seed=7, sigma_v=0.2)
    log(f"case shared cells of ~{cell_target} fp64")
    ref = oracle_run(ps)
    g = gpu_run(ps, "fp64", cell_target=cell_target, **SHARED)
    compare(g, ref, "fp64", label=f"shared ct{cell_target}")


def test_shared_config1_sampled():
    """The 2^20 lattice of the bench line with the shared layout, at the
    oracle's sample (tests/golden/config1_sample.txt)."""
    R = load_sample(os.path.join(HERE, "golden", "config1_sample.txt"))
    ps = workloads.config1()
    log(f"case shared config1 {ps.n} fp32")
    g = gpu_run(ps, "fp32", **SHARED)
    compare_sample(g, R, "fp32", label="shared config1")


def test_shared_mts_matches_split():
    # multiple time-stepping: cells without active particles pass their stored
    # quantities on; both layouts give the same bins, active counts and state
    ps = workloads.uniform(1500, seed=31, sigma_v=0.05)
    ps.u[:] = np.where(ps.pos[:, 0] < 0.3, 20.0, 0.05)
    f0 = oracle.full_pass(ps.pos, ps.vel, ps.m, ps.u, ps.h0, ps.box)
    dtb = float(np.min(f0["signal"]["dt"])) * 0.9
    log(f"case shared mts 1500 fp64 dt_base {dtb:.4g}")
    out = {}
    for lab, sw in (("split", sph.SPH_SWEEP_SPLIT), ("shared", sph.SPH_SWEEP_SHARED)):
        parts = sph.Particles.from_numpy(ps, "cuda:0")
        ctx = sph.Context(ps.box, precision="fp64", sweep=sw)
        acc, bins = ctx.mts_init(parts, dtb, 3)
        counts = [ctx.mts_step(parts, acc, bins, count=True) for _ in range(8)]
        torch.cuda.synchronize()
        out[lab] = (np.array(counts), bins.cpu().numpy(), parts.x.cpu().numpy(), parts.vx.cpu().numpy(),
                    parts.u.cpu().numpy())
        ctx.close()
    np.testing.assert_array_equal(out["split"][0], out["shared"][0])
    np.testing.assert_array_equal(out["split"][1], out["shared"][1])
    assert len(set(out["shared"][0])) > 2
    for i in (2, 3, 4):
        s, t = out["split"][i], out["shared"][i]
        assert np.max(np.abs(s - t)) <= 1e-9 * (np.max(np.abs(s)) + 1.0)


def test_shared_forward_feeds_the_adjoint():
    # the reverse pass reads the per-particle sums the shared density keeps
    rng = np.random.default_rng(17)
    ps = workloads.uniform(1200, seed=17, sigma_v=0.4)
    ps.m[:] *= rng.uniform(0.6, 1.4, ps.n)
    ps.u[:] = rng.uniform(0.5, 1.5, ps.n)
    w = (rng.normal(size=ps.n), rng.normal(size=(ps.n, 3)), rng.normal(size=ps.n))
    log("case shared forward + adjoint dense 1200 fp64")
    dev = lambda a: torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda:0")
    parts = sph.Particles.from_numpy(ps, "cuda:0")
    ctx = sph.Context(ps.box, precision="fp64", keep_adjoint=1, **SHARED)
    ctx.run(parts)
    gx, gh = ctx.backward(parts, dev(w[0]), dev(w[1]), dev(w[2]), implicit_h=False, want_h=True)
    torch.cuda.synchronize()
    gx, gh = gx.cpu().numpy(), gh.cpu().numpy()
    ctx.close()
    hs, _ = oracle.solve_h(ps.pos, ps.h0, ps.box, tol=1e-13)
    rx, rh, _, _ = og.vjp(ps.pos, ps.vel, ps.m, ps.u, hs, ps.box, *w, solve=False)
    err = lambda g, r: np.max(np.abs(g - r) / (np.abs(r) + np.sqrt(np.mean(r ** 2)) + 1e-300))
    ex, eh = err(gx, rx), err(gh, rh)
    log(f"  dL/dx err {ex:.2e} dL/dh err {eh:.2e}")
    assert ex <= 1e-8 and eh <= 1e-8
