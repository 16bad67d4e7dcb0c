"""Batched form: many independent periodic boxes in one set of launches, and
the whole pass captured in a HIP graph.

The batched calls must reproduce per-box calls (each box alone in its own
context); graph replays must reproduce the eager pass."""
import numpy as np
import pytest
import torch

import oracle
from paper_1404_2303_amd import sph, workloads
from parity_util import compare, log, oracle_run

pytestmark = pytest.mark.gpu


def _small_batch(nbox=12, n_min=2000, n_max=6000, seed=3):
    counts = workloads.batch_counts(nbox, n_min, n_max, seed)
    sets, lens = [], []
    rng = np.random.default_rng(seed)
    for b, c in enumerate(counts):
        L = rng.uniform(0.85, 1.2, 3)
        sets.append(workloads.uniform(int(c), seed=100 + b, box=L, sigma_v=0.2))
        lens.append(L)
    offsets = np.concatenate([[0], np.cumsum(counts)]).astype(np.int64)
    cat = workloads.ParticleSet(pos=np.concatenate([s.pos for s in sets]), vel=np.concatenate([s.vel for s in sets]),
                                m=np.concatenate([s.m for s in sets]), u=np.concatenate([s.u for s in sets]),
                                h0=np.concatenate([s.h0 for s in sets]), box=np.ones(3))
    return sets, cat, offsets, np.array(lens)


def _run(ps, precision, batch=None, box=None):
    parts = sph.Particles.from_numpy(ps, "cuda:0")
    ctx = sph.Context(box if box is not None else ps.box, precision=precision)
    d, f = ctx.run(parts, sph.Batch(*batch) if batch is not None else None)
    torch.cuda.synchronize()
    out = {"h": parts.h.cpu().numpy(), "rho": d["rho"].cpu().numpy(),
           "a": torch.stack([f["ax"], f["ay"], f["az"]], 1).cpu().numpy(), "dudt": f["dudt"].cpu().numpy(),
           "n_pairs": f["n_pairs"].cpu().numpy()}
    ctx.close()
    return out


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_batched_equals_per_box_calls(precision):
    sets, cat, offsets, lens = _small_batch()
    log(f"case batched vs per-box {precision}: {len(sets)} boxes, {cat.n} particles")
    g = _run(cat, precision, batch=(offsets, lens))
    for b, ps in enumerate(sets):
        one = _run(ps, precision)
        sl = slice(offsets[b], offsets[b + 1])
        assert np.array_equal(g["n_pairs"][sl], one["n_pairs"]), b
        assert np.allclose(g["h"][sl], one["h"], rtol=1e-12, atol=0), b
        assert np.allclose(g["rho"][sl], one["rho"], rtol=1e-12, atol=0), b
        scale = np.max(np.abs(one["a"]))
        assert np.max(np.abs(g["a"][sl] - one["a"])) <= 1e-12 * scale, b


def test_batched_parity_against_oracle():
    sets, cat, offsets, lens = _small_batch(nbox=6, seed=8)
    log(f"case batched parity: {cat.n} particles")
    parts = sph.Particles.from_numpy(cat, "cuda:0")
    ctx = sph.Context((1, 1, 1), precision="fp32")
    d, f = ctx.run(parts, sph.Batch(offsets, lens))
    torch.cuda.synchronize()
    for b, ps in enumerate(sets):
        sl = slice(offsets[b], offsets[b + 1])
        ref = oracle_run(ps)
        g = {k: v[sl].cpu().numpy() for k, v in d.items()}
        g.update({k: v[sl].cpu().numpy() for k, v in f.items()})
        g["h"] = parts.h[sl].cpu().numpy()
        g["a"] = np.stack([g["ax"], g["ay"], g["az"]], 1)
        compare(g, ref, "fp32", label=f"box{b}")
    ctx.close()


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_graph_replays_match_the_eager_pass(precision):
    sets, cat, offsets, lens = _small_batch(nbox=8, seed=5)
    log(f"case graph replay {precision}: {cat.n} particles")
    eager = _run(cat, precision, batch=(offsets, lens))
    parts = sph.Particles.from_numpy(cat, "cuda:0")
    h_init = parts.h.clone()
    ctx = sph.Context((1, 1, 1), precision=precision)
    batch = sph.Batch(offsets, lens)
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        _, fout = ctx.graph_capture(parts, batch, h_init=h_init)
        for rep in range(3):
            parts.h.fill_(0.123)            # eager work between replays
            fout["ax"].zero_()
            ctx.graph_launch()
            ctx.check()
            torch.cuda.synchronize()
            a = torch.stack([fout["ax"], fout["ay"], fout["az"]], 1).cpu().numpy()
            assert np.array_equal(fout["n_pairs"].cpu().numpy(), eager["n_pairs"]), rep
            assert np.allclose(parts.h.cpu().numpy(), eager["h"], rtol=1e-12, atol=0), rep
            scale = np.max(np.abs(eager["a"]))
            assert np.max(np.abs(a - eager["a"])) <= 1e-12 * scale, rep
    ctx.close()


def test_density_async_and_check():
    ps = workloads.uniform(3000, seed=4, sigma_v=0.2)
    log("case density_async")
    parts = sph.Particles.from_numpy(ps, "cuda:0")
    ctx = sph.Context(ps.box, precision="fp64")
    ctx.build_cells(parts)
    ctx.sort()
    n = parts.n
    d = {"rho": torch.empty(n, dtype=torch.float64, device="cuda:0")}
    c = sph.sph_density_out(*[sph._ptr(d.get(k)) for k in sph.DENSITY_FIELDS])
    assert sph.sph_density_async(ctx.ctx, parts.c_struct(), c, sph._stream()) == sph.SPH_OK
    assert ctx.check() == sph.SPH_OK
    ref = oracle_run(ps)
    assert np.allclose(d["rho"].cpu().numpy(), ref["dens"]["rho"], rtol=1e-9)
    ctx.close()


@pytest.mark.parametrize("cell_target", [32, 64])
def test_full_batch_as_the_bench_runs_it(cell_target):
    """The 256-box set of the bench (5.36M particles, log-uniform counts in
    [2048, 65536]) as one captured pass, replayed; the smallest and largest box
    and two others checked whole against the oracle.  Cell size 32 is the one
    the autotuner picks on this set, 64 the default."""
    cat, offsets, lens = workloads.batch()
    counts = np.diff(offsets)
    rng = np.random.default_rng(4)
    boxes = sorted({int(np.argmin(counts)), int(np.argmax(counts))} | set(int(b) for b in rng.choice(256, 2)))
    log(f"case full batch {cat.n} particles, cell_target {cell_target}, boxes {boxes}")
    parts = sph.Particles.from_numpy(cat, "cuda:0")
    h0 = parts.h.clone()
    n = cat.n
    dout = {k: torch.empty(n, dtype=torch.float64, device="cuda:0") for k in ("rho", "omega", "div_v", "balsara",
                                                                            "pressure", "sound", "n_ngb")}
    dout["curl_v"] = torch.empty((n, 3), dtype=torch.float64, device="cuda:0")
    ctx = sph.Context((1, 1, 1), precision="fp32", cell_target=cell_target)
    batch = sph.Batch(offsets, lens)
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        _, fout = ctx.graph_capture(parts, batch, h_init=h0, dout=dout)
        ctx.check()
        ctx.graph_launch()
        ctx.graph_launch()
        torch.cuda.synchronize()
        ctx.check()
    for b in boxes:
        sl = slice(offsets[b], offsets[b + 1])
        ps = workloads.uniform(int(counts[b]), seed=b)
        ref = oracle_run(ps)
        g = {k: v[sl].cpu().numpy() for k, v in dout.items()}
        g.update({k: v[sl].cpu().numpy() for k, v in fout.items()})
        g["h"] = parts.h[sl].cpu().numpy()
        g["a"] = np.stack([g["ax"], g["ay"], g["az"]], 1)
        compare(g, ref, "fp32", label=f"box{b} n={counts[b]}")
    ctx.close()
