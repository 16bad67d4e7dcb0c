"""GPU parity of the hierarchical decomposition (Sec. 3.2: cells split while
crowded, leaves at many levels, interaction lists from a tree walk) against
the FP64 oracle, on multi-resolution sets.  Tolerances as in parity_util.
"""
import os

import numpy as np
import pytest
import torch

import oracle
from oracle import grad as og
from paper_1404_2303_amd import sph, workloads
from parity_util import TOL, compare, compare_sample, gpu_run, load_sample, log, oracle_run

pytestmark = pytest.mark.gpu

TREE = dict(max_depth=8, split_count=32)
HERE = os.path.dirname(os.path.abspath(__file__))


def small_mixture(seed=3):
    """4 Plummer spheres of 6000 + 6000 background particles (h spans ~100x)."""
    return workloads.plummer_mixture(n_spheres=4, n_per_sphere=6000, n_background=6000, seed=seed)


@pytest.fixture(scope="module")
def mixture():
    ps = small_mixture()
    return ps, oracle_run(ps)


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_mixture_30000(mixture, precision):
    ps, ref = mixture
    log(f"case tree mixture 30000 {precision}")
    g = gpu_run(ps, precision, estimate=True, **TREE)
    st = g["stats"]
    log(f"  leaves {st['n_cells']} depth {st['depth']} top grid {st['grid']} rebuilds {st['rebuilds']}")
    assert st["depth"] >= 6 and st["n_cells"] > np.prod(st["grid"])
    compare(g, ref, precision, label="mixture")


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
@pytest.mark.parametrize("shared_min", [64, 1 << 30])
def test_mixture_large_leaves_shared_force(mixture, precision, shared_min):
    """Leaves of up to 256 particles (split count 256): the force stage swept
    shared (each wavefront its own 64 targets over all four staged regions)
    for every leaf of more than 64 particles, and never; both against the
    oracle."""
    ps, ref = mixture
    log(f"case tree mixture 30000 {precision}, split count 256, force shared above {shared_min}")
    g = gpu_run(ps, precision, estimate=True, max_depth=8, split_count=256, shared_min=shared_min)
    compare(g, ref, precision, label=f"mixture-shared{shared_min}")


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_uniform_split_once(precision):
    # top cells of about 1100 particles (3 per dimension) whose h is below half
    # their edge split once: the uniform set runs on leaves of level 1
    ps = workloads.uniform(30000, seed=5, sigma_v=0.3)
    log(f"case tree uniform 30000 split once {precision}")
    ref = oracle_run(ps)
    g = gpu_run(ps, precision, max_depth=3, split_count=64, split_frac=0.5, cell_target=30000 // 27)
    st = g["stats"]
    log(f"  leaves {st['n_cells']} depth {st['depth']} top grid {st['grid']}")
    assert st["n_cells"] > np.prod(st["grid"])
    compare(g, ref, precision, label="split-once")


def test_void_particle_tree():
    ps = workloads.uniform(3000, seed=31, sigma_v=0.3)
    c = np.array([0.5, 0.5, 0.5])
    keep = np.linalg.norm(ps.pos - c, axis=1) > 0.12
    n = int(keep.sum()) + 1
    ps = workloads.ParticleSet(pos=np.concatenate([ps.pos[keep], c[None]]),
                               vel=np.concatenate([ps.vel[keep], np.zeros((1, 3))]),
                               m=np.full(n, 1.0 / n), u=np.ones(n), h0=np.full(n, ps.h0[0]), box=ps.box)
    log(f"case tree void {n}")
    ref = oracle_run(ps)
    g = gpu_run(ps, "fp64", max_depth=5, split_count=8, split_frac=0.5)
    compare(g, ref, "fp64", label="void-tree")


def test_batched_boxes_tree():
    boxes = [(1.0, 1.0, 1.0), (0.8, 1.0, 0.9), (1.0, 1.0, 1.0)]
    sets = [workloads.uniform(2500, seed=70, box=boxes[0], sigma_v=0.2),
            workloads.uniform(4000, seed=71, box=boxes[1], sigma_v=0.2),
            workloads.plummer_mixture(n_spheres=2, n_per_sphere=3000, n_background=2000, seed=72)]
    offsets = np.concatenate([[0], np.cumsum([s.n for s in sets])]).astype(np.int64)
    cat = workloads.ParticleSet(pos=np.concatenate([s.pos for s in sets]), vel=np.concatenate([s.vel for s in sets]),
                                m=np.concatenate([s.m for s in sets]), u=np.concatenate([s.u for s in sets]),
                                h0=np.concatenate([s.h0 for s in sets]), box=np.ones(3))
    log(f"case tree batched {cat.n} in 3 boxes")
    g = gpu_run(cat, "fp32", batch=(offsets, np.asarray(boxes)), estimate=True, **TREE)
    for b, s in enumerate(sets):
        ref = oracle_run(s)
        lo, hi = offsets[b], offsets[b + 1]
        gb = {k: (v[lo:hi] if isinstance(v, np.ndarray) and len(v) == cat.n else v) for k, v in g.items()}
        compare(gb, ref, "fp32", label=f"tree-box{b}")


def test_estimated_h_is_close_to_the_solution(mixture):
    ps, ref = mixture
    parts = sph.Particles.from_numpy(ps, "cuda:0")
    ctx = sph.Context(ps.box, precision="fp64", **TREE)
    ctx.estimate_h(parts)
    torch.cuda.synchronize()
    he = parts.h.cpu().numpy()
    ctx.close()
    lr = np.abs(np.log(he / ref["h"]))
    p99 = np.percentile(lr, 99)
    log(f"case tree estimate_h: median |log ratio| {np.median(lr):.3f}, 99th percentile {p99:.3f}, max {lr.max():.3f}")
    assert np.median(lr) < 0.3 and p99 < np.log(3.0)


def test_adjoint_on_the_hierarchy():
    # a small clustered set through the hierarchy: gradients against the dense oracle
    rng = np.random.default_rng(8)
    ps = workloads.plummer_mixture(n_spheres=1, n_per_sphere=1000, n_background=1000, a_min=0.05, a_max=0.05,
                                   sigma_v=0.3, seed=8)
    w = (rng.normal(size=ps.n), rng.normal(size=(ps.n, 3)), rng.normal(size=ps.n))
    log(f"case tree adjoint {ps.n}")
    parts = sph.Particles.from_numpy(ps, "cuda:0")
    ctx = sph.Context(ps.box, precision="fp64", max_depth=6, split_count=16, split_frac=0.5, keep_adjoint=1)
    ctx.estimate_h(parts)
    ctx.run(parts)
    dev = lambda a: torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda:0")
    gx = ctx.backward(parts, dev(w[0]), dev(w[1]), dev(w[2]), implicit_h=True).cpu().numpy()
    st = ctx.stats()
    ctx.close()
    rx, _, _, _ = og.vjp(ps.pos, ps.vel, ps.m, ps.u, ps.h0, ps.box, *w, solve=True)
    e = np.max(np.abs(gx - rx) / (np.abs(rx) + np.sqrt(np.mean(rx ** 2))))
    log(f"  leaves {st['n_cells']} depth {st['depth']} err {e:.2e}")
    assert st["n_cells"] > np.prod(st["grid"])
    assert e <= 1e-8


@pytest.mark.parametrize("split_count", [64, 256])
def test_config2_sampled_fp32(split_count):
    """The 2,097,152-particle Plummer mixture through the hierarchy, checked at
    the oracle's sample (tests/golden/config2_sample.txt, written by
    make_config2_sample.py from the oracle alone); split count 256 is the
    bench's autotuned launch configuration."""
    R = load_sample(os.path.join(HERE, "golden", "config2_sample.txt"))
    ps = workloads.config2()
    log(f"case tree config2 {ps.n} fp32 split_count {split_count}")
    g = gpu_run(ps, "fp32", estimate=True, max_depth=10, split_count=split_count)
    st = g["stats"]
    log(f"  leaves {st['n_cells']} depth {st['depth']} top grid {st['grid']} rebuilds {st['rebuilds']}")
    compare_sample(g, R, "fp32", label=f"config2 split {split_count}")


def test_graph_replay_on_the_hierarchy(mixture):
    # the whole tree build and pass captured once and replayed from the solved h:
    # equal to the eager pass from the same h (up to the order of the cross-wave sums)
    ps, ref = mixture
    log("case tree graph replay 30000 fp32")
    parts = sph.Particles.from_numpy(ps, "cuda:0")
    ctx = sph.Context(ps.box, precision="fp32", **TREE)
    ctx.estimate_h(parts)
    ctx.run(parts)
    h_sol = parts.h.clone()
    parts.h.copy_(h_sol)
    d, f = ctx.run(parts)
    eager = {k: v.clone() for k, v in f.items()}
    eager_h = parts.h.clone()
    scale = float(torch.max(torch.abs(eager["ax"])))
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        _, fout = ctx.graph_capture(parts, None, h_init=h_sol)
        for rep in range(3):
            for v in fout.values():
                v.zero_()
            ctx.graph_launch()
            ctx.check()
            stream.synchronize()
            assert torch.equal(fout["n_pairs"], eager["n_pairs"]), rep
            assert torch.allclose(parts.h, eager_h, rtol=1e-12, atol=0), rep
            for k in ("ax", "ay", "az"):
                assert float(torch.max(torch.abs(fout[k] - eager[k]))) <= 1e-12 * scale, (rep, k)
    ctx.close()
