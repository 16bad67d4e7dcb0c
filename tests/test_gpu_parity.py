"""GPU parity: the HIP path (through the C ABI) against the FP64 oracle.

Every input is a seeded synthetic set from paper_1404_2303_amd.workloads;
tolerances are derived in tests/parity_util.py.
"""
import os

import numpy as np
import pytest
import torch

import oracle
from paper_1404_2303_amd import sph, workloads
from parity_util import TOL, compare, compare_sample, gpu_run, load_sample, log, oracle_run

pytestmark = pytest.mark.gpu
HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.fixture(scope="module")
def config0_ref():
    ps = workloads.config0()
    return ps, oracle_run(ps)


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_config0_uniform_4096(config0_ref, precision):
    ps, ref = config0_ref
    log(f"case config0 uniform 4096 {precision}")
    g = gpu_run(ps, precision)
    compare(g, ref, precision, label="config0")
    assert np.all(g["n_iter"] > 0)


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_ragged_box_varied_masses(precision):
    # non-cubic box, N not a multiple of anything, masses and energies varied
    rng = np.random.default_rng(21)
    ps = workloads.uniform(3001, seed=21, box=(1.0, 0.7, 0.55), sigma_v=0.3)
    ps.m[:] *= rng.uniform(0.6, 1.4, ps.n)
    ps.u[:] = rng.uniform(0.5, 2.0, ps.n)
    log(f"case ragged box 3001 {precision}")
    ref = oracle_run(ps)
    g = gpu_run(ps, precision)
    compare(g, ref, precision, label="ragged")


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_jittered_lattice(precision):
    ps = workloads.small_lattice(16)
    log(f"case lattice 16^3 {precision}")
    ref = oracle_run(ps)
    g = gpu_run(ps, precision)
    compare(g, ref, precision, label="lattice16")


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_particle_in_a_void(precision):
    # one particle at the centre of an empty sphere: its h is the largest and its
    # ~100 pairs overflow the per-lane neighbour lists several times, across
    # segment boundaries
    ps = workloads.uniform(3000, seed=31, sigma_v=0.3)
    c = np.array([0.5, 0.5, 0.5])
    keep = np.linalg.norm(ps.pos - c, axis=1) > 0.12
    n = int(keep.sum()) + 1
    ps = workloads.ParticleSet(pos=np.concatenate([ps.pos[keep], c[None]]),
                               vel=np.concatenate([ps.vel[keep], np.zeros((1, 3))]),
                               m=np.full(n, 1.0 / n), u=np.ones(n), h0=np.full(n, ps.h0[0]), box=ps.box,
                               name="void")
    log(f"case void {n} {precision}")
    ref = oracle_run(ps)
    assert ref["force"]["count"][-1] > 100
    g = gpu_run(ps, precision)
    compare(g, ref, precision, label="void")


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_isolated_particle_many_pairs(precision):
    # uniform set whose sparsest particle has h = 2x the smallest and 74 pairs
    ps = workloads.uniform(1200, seed=17, sigma_v=0.4)
    log(f"case uniform 1200 seed 17 {precision}")
    ref = oracle_run(ps)
    g = gpu_run(ps, precision)
    compare(g, ref, precision, label="u1200")


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_coincident_particles(precision):
    """Pairs at r = 0 with i != j (60 particles placed on top of others, with
    their own velocities): W(0) enters the density, the kernel gradient and the
    approach speed of such a pair are zero (the reading of the undefined r = 0
    case), and no 0/0 reaches any output."""
    ps = workloads.uniform(3000, seed=43, sigma_v=0.3)
    ps.pos[2000:2060] = ps.pos[:60]
    log(f"case coincident pairs 3000 {precision}")
    ref = oracle_run(ps)
    g = gpu_run(ps, precision)
    for k in ("rho", "h", "a", "dudt", "div_v", "curl_v", "balsara"):
        assert np.all(np.isfinite(g[k])), k
    compare(g, ref, precision, label="coincident")


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_pairs_exactly_at_the_support(precision):
    """A perfect simple cubic lattice with the neighbour target set to N(h) at
    h = sqrt(5) spacings: the solved h is that distance, so the 24 lattice
    neighbours of the fifth shell of every particle sit on the edge of its
    support (q = 1 up to the precision of h).  W and grad W vanish there; the
    counts of such pairs are exempt through the bands."""
    k = 16
    ps = workloads.lattice((k, k, k), 1.0 / k, 0.0, 0.2, seed=5)
    shells = [(1, 6), (2, 12), (3, 8), (4, 6)]   # |n|^2 and multiplicity of the lattice shells inside sqrt(5)
    target = 32.0 / 3.0 * (1.0 + sum(c * oracle.kernel_w(np.sqrt(s / 5.0))[0] for s, c in shells))
    log(f"case support edge lattice {k}^3 {precision}: n_ngb {target:.12f}")
    ref = oracle_run(ps, target=target)
    assert np.allclose(ref["h"], np.sqrt(5.0) / k, rtol=1e-9)
    assert np.all(ref["bands"][precision]["dband"] == 24)
    g = gpu_run(ps, precision, n_ngb=target)
    compare(g, ref, precision, label="support edge")


def test_tiny_three_cells_per_dimension():
    ps = workloads.uniform(800, seed=3, sigma_v=0.2)
    log("case tiny 800 fp64")
    ref = oracle_run(ps)
    g = gpu_run(ps, "fp64")
    assert tuple(g["stats"]["grid"]) == (3, 3, 3)
    compare(g, ref, "fp64", label="tiny")


@pytest.mark.parametrize("cell_target", [16, 100, 200, 1000])
def test_decomposition_invariance(cell_target):
    """Cell size changes which loop finds a pair, never the result."""
    ps = workloads.uniform(6000, seed=9, sigma_v=0.3)
    log(f"case decomposition cell_target={cell_target}")
    base = gpu_run(ps, "fp64")
    other = gpu_run(ps, "fp64", cell_target=cell_target)
    assert np.array_equal(base["n_pairs"], other["n_pairs"])
    assert np.allclose(base["h"], other["h"], rtol=1e-11, atol=0)
    assert np.allclose(base["rho"], other["rho"], rtol=1e-11, atol=0)
    ka = np.max(np.abs(base["a"]))
    assert np.max(np.abs(base["a"] - other["a"])) <= 1e-9 * ka


@pytest.mark.parametrize("staging", [sph.SPH_STAGING_COMPACT, sph.SPH_STAGING_WIDE])
@pytest.mark.parametrize("n,cell_target,lo,hi", [(40000, 100, 64, 128), (6000, 200, 128, 256)])
def test_large_cells_fp32(n, cell_target, lo, hi, staging):
    """Cells of 65..128 and 129..256 particles on average: the orderings of two
    and four words per lane of the wavefront sort (keys rounded down below
    their index bits), under both stagings of the density stage (sources that
    overflow the compact one take several batches)."""
    ps = workloads.uniform(n, seed=10, sigma_v=0.3)
    g = gpu_run(ps, "fp32", cell_target=cell_target, staging=staging)
    mean = ps.n / g["stats"]["n_cells"]
    log(f"case large cells fp32 n={n} cell_target={cell_target}: {g['stats']['n_cells']} cells, mean {mean:.0f}")
    assert lo < mean <= hi
    compare(g, oracle_run(ps), "fp32", label=f"cells {cell_target}")


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
@pytest.mark.parametrize("n,cell_target,lo,hi", [(30000, 1000, 256, 1500), (100000, 3000, 2048, 4096)])
def test_cells_ordered_by_merging(n, cell_target, lo, hi, precision):
    """Cells of more than 256 particles: their orderings are made by one
    work-group from those of their sub-cells of depth 1 to 3, shifted into
    the parent's frame and merged (Sec. 3.3); any misplaced particle would cut
    the sorted sweeps short and lose pairs."""
    ps = workloads.uniform(n, seed=11, sigma_v=0.3)
    g = gpu_run(ps, precision, cell_target=cell_target)
    mean = ps.n / g["stats"]["n_cells"]
    log(f"case merged orderings {precision} n={n} cell_target={cell_target}: {g['stats']['n_cells']} cells, mean {mean:.0f}")
    assert lo < mean <= hi
    compare(g, oracle_run(ps), precision, label=f"merged cells {cell_target}")


def test_crowded_cell_ordering():
    """A clump of 400 particles inside a cube of 1/64 of a big cell's edge:
    more than 256 in one depth-3 sub-cell, so that cell's orderings come from
    runs of 256 consecutive particles instead; the other big cells take the
    sub-cell construction.  FP64 only: the clump's spacing is 3e-3 of the
    cell's edge, so FP32 positions in the cell's frame resolve its pair
    separations to ~3e-5 only, above the FP32 parity bound."""
    precision = "fp64"
    ps = workloads.uniform(12000, seed=13, sigma_v=0.2)
    rng = np.random.default_rng(13)
    ps.pos[:400] = 0.52 + 0.004 * rng.random((400, 3))
    ps.h0[:400] = 0.005
    g = gpu_run(ps, precision, cell_target=1000)
    log(f"case crowded cell {precision}: {g['stats']['n_cells']} cells")
    compare(g, oracle_run(ps), precision, label="crowded cell")


def test_momentum_and_energy_conservation_gpu():
    ps = workloads.uniform(8000, seed=5, sigma_v=0.5)
    log("case conservation 8000 fp64")
    g = gpu_run(ps, "fp64")
    mom = np.sum(ps.m[:, None] * g["a"], axis=0)
    scale = np.sum(ps.m * np.linalg.norm(g["a"], axis=1))
    assert np.max(np.abs(mom)) < 1e-9 * scale
    e = np.sum(ps.m * (g["dudt"] + np.sum(ps.vel * g["a"], axis=1)))
    escale = np.sum(ps.m * (np.abs(g["dudt"]) + np.linalg.norm(ps.vel, axis=1) * np.linalg.norm(g["a"], axis=1)))
    assert abs(e) < 1e-9 * escale


# ---------------------------------------------------------------- edge cases and errors
def _ctx_and_parts(ps, **kw):
    return sph.Context(ps.box, precision=kw.pop("precision", "fp64"), **kw), sph.Particles.from_numpy(ps, "cuda:0")


def test_empty_input():
    log("case empty")
    ps = workloads.uniform(0, seed=0)
    ctx, parts = _ctx_and_parts(ps)
    d, f = ctx.run(parts)
    torch.cuda.synchronize()
    assert d["rho"].numel() == 0 and f["ax"].numel() == 0
    ctx.close()


def test_nonfinite_input_is_reported():
    log("case nonfinite")
    ps = workloads.uniform(1000, seed=1)
    ps.pos[17, 1] = np.nan
    ctx, parts = _ctx_and_parts(ps)
    ctx.build_cells(parts)
    ctx.sort()
    with pytest.raises(sph.SPHError) as e:
        ctx.density(parts)
    assert e.value.status == sph.SPH_E_NONFINITE
    ctx.close()


def test_h_too_large_is_reported():
    log("case h too large")
    ps = workloads.uniform(1000, seed=1)
    ps.h0[:] = 0.4   # more than a third of the box
    ctx, parts = _ctx_and_parts(ps)
    ctx.build_cells(parts)
    ctx.sort()
    with pytest.raises(sph.SPHError) as e:
        ctx.density(parts)
    assert e.value.status == sph.SPH_E_H_TOO_LARGE
    ctx.close()


def test_not_converged_is_reported():
    log("case max_iter=1")
    ps = workloads.uniform(1000, seed=2)
    ctx, parts = _ctx_and_parts(ps, max_iter=1)
    ctx.build_cells(parts)
    ctx.sort()
    d = ctx.density(parts, allow_unconverged=True)
    torch.cuda.synchronize()
    assert ctx.last_density_status == sph.SPH_E_NOT_CONVERGED
    it = d["n_iter"].cpu().numpy()
    assert np.all(it == -1)
    ctx.close()


def test_calls_out_of_order():
    log("case state")
    ps = workloads.uniform(500, seed=2)
    ctx, parts = _ctx_and_parts(ps)
    with pytest.raises(sph.SPHError) as e:
        ctx.sort()
    assert e.value.status == sph.SPH_E_STATE
    with pytest.raises(sph.SPHError) as e:
        ctx.force(parts)
    assert e.value.status == sph.SPH_E_STATE
    ctx.build_cells(parts)
    with pytest.raises(sph.SPHError) as e:
        ctx.density(parts)
    assert e.value.status == sph.SPH_E_STATE
    ctx.close()


def test_rebuild_when_h_outgrows_the_cells():
    """Initial h far too small: cells are built for it, the iteration outgrows
    them, and the library rebuilds until the solution fits."""
    ps = workloads.uniform(4000, seed=4, sigma_v=0.1)
    ps.h0[:] *= 0.2
    log("case rebuild")
    ref = oracle_run(ps)
    g = gpu_run(ps, "fp64", cell_target=8, h_margin=0.0)
    assert g["stats"]["rebuilds"] >= 1
    compare(g, ref, "fp64", label="rebuild")


def test_kernel_times_before_any_force_leave_no_error():
    # timing enabled, density only: the force events were never recorded; asking for
    # the times must not leave a HIP error behind for the next launch to report
    ps = workloads.uniform(3000, seed=12)
    log("case kernel times without a force call")
    parts = sph.Particles.from_numpy(ps, "cuda:0")
    ctx = sph.Context(ps.box, precision="fp32")
    ctx.enable_timing(True)
    ctx.build_cells(parts)
    ctx.sort()
    ctx.density(parts, want=("rho",))
    t = ctx.kernel_times()
    assert t["force_ms"] == 0.0 and t["density_ms"] > 0.0 and t["build_ms"] > 0.0
    parts.h.add_(0.0)   # a torch launch after the query
    torch.cuda.synchronize()
    ctx.close()


def _config1_graph(ps):
    """The pass as the bench line times it: captured once with h restored from the
    initial guess inside the graph, then replayed (twice here)."""
    parts = sph.Particles.from_numpy(ps, "cuda:0")
    h0 = parts.h.clone()
    n = ps.n
    dout = {k: torch.empty(n, dtype=torch.float64, device="cuda:0")
            for k in ("rho", "omega", "div_v", "balsara", "pressure", "sound")}
    dout["curl_v"] = torch.empty((n, 3), dtype=torch.float64, device="cuda:0")
    dout["n_dens"] = torch.empty(n, dtype=torch.int32, device="cuda:0")
    ctx = sph.Context(ps.box, precision="fp32")
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        _, fout = ctx.graph_capture(parts, None, h_init=h0, dout=dout)
        ctx.check()
        ctx.graph_launch()
        ctx.graph_launch()
        torch.cuda.synchronize()
        ctx.check()
    out = {k: v.cpu().numpy() for k, v in dout.items()}
    out.update({k: v.cpu().numpy() for k, v in fout.items()})
    out["h"] = parts.h.cpu().numpy()
    out["a"] = np.stack([out["ax"], out["ay"], out["az"]], axis=1)
    out["stats"] = ctx.stats()
    ctx.close()
    return out


@pytest.mark.parametrize("precision,mode", [("fp32", "eager"), ("fp32", "graph"), ("fp64", "eager")])
def test_config1_sampled(precision, mode):
    """The 2^20-particle jittered lattice of the bench line, in its launch
    configuration (default parameters; eager calls, or the captured FP32 pass
    replayed as the bench times it) and in the plain FP64 form the bench
    reports beside it, checked at the oracle's sample
    (tests/golden/config1_sample.txt, written by make_config1_sample.py from the
    oracle alone)."""
    R = load_sample(os.path.join(HERE, "golden", "config1_sample.txt"))
    ps = workloads.config1()
    log(f"case config1 {ps.n} {precision} {mode}")
    g = gpu_run(ps, precision) if mode == "eager" else _config1_graph(ps)
    log(f"  cells {g['stats']['n_cells']} grid {g['stats']['grid']}")
    compare_sample(g, R, precision, label=f"config1 {mode}")
