"""sph_pass_noalloc, the allocation-free entry point: the same pass as the
context calls (sph_build_cells, sph_sort, sph_density, sph_force) with the
library's fixed per-GPU array as the workspace.  Two calls in a row, the
second on a smaller input, each checked against the context pass on the same
input and against the FP64 oracle (tolerances of tests/parity_util.py)."""
import numpy as np
import pytest
import torch

from paper_1404_2303_amd import sph, workloads
from parity_util import TOL, compare, gpu_run, log, oracle_run

pytestmark = pytest.mark.gpu


def _noalloc(ps, precision, **kw):
    parts = sph.Particles.from_numpy(ps, "cuda:0")
    n = ps.n
    dout = {k: torch.empty(n, dtype=torch.float64, device="cuda:0")
            for k in ("rho", "omega", "n_ngb", "div_v", "balsara", "pressure", "sound")}
    dout["curl_v"] = torch.empty((n, 3), dtype=torch.float64, device="cuda:0")
    for k in ("n_iter", "n_dens"):
        dout[k] = torch.empty(n, dtype=torch.int32, device="cuda:0")
    _, fout = sph.pass_noalloc(parts, ps.box, precision, dout=dout, **kw)
    torch.cuda.synchronize()
    out = {k: v.cpu().numpy() for k, v in dout.items()}
    out.update({k: v.cpu().numpy() for k, v in fout.items()})
    out["h"] = parts.h.cpu().numpy()
    out["a"] = np.stack([out["ax"], out["ay"], out["az"]], axis=1)
    return out


def _same_pass(g, c, precision):
    """The two passes run the same kernels on the same input: they agree to
    the summation order of the sums (FP64 additions in LDS in the order the
    wavefronts arrive), far inside the oracle tolerances."""
    t = TOL[precision]
    e_h = np.max(np.abs(g["h"] / c["h"] - 1))
    e_rho = np.max(np.abs(g["rho"] / c["rho"] - 1))
    na = np.linalg.norm(c["a"], axis=1)
    e_a = np.max(np.linalg.norm(g["a"] - c["a"], axis=1) / np.maximum(na, np.sqrt(np.mean(na ** 2))))
    d_pairs = int(np.max(np.abs(g["n_pairs"] - c["n_pairs"])))
    log(f"  vs context pass: h {e_h:.2e} rho {e_rho:.2e} a {e_a:.2e} pair-count diff {d_pairs}")
    assert e_h <= t["h"] and e_rho <= t["rho"] and e_a <= t["a"]
    assert d_pairs <= 1


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_noalloc_pass_twice_matches_the_context_pass(precision):
    for n, seed in ((20000, 51), (7000, 52)):   # the second call smaller than the first
        ps = workloads.uniform(n, seed=seed, sigma_v=0.3)
        log(f"case noalloc {precision} n={n} seed={seed}")
        g = _noalloc(ps, precision)
        c = gpu_run(ps, precision)
        _same_pass(g, c, precision)
        compare(g, oracle_run(ps), precision, label=f"noalloc n={n}")


def test_noalloc_at_the_maximum_size():
    """SPH_NOALLOC_MAX_PARTICLES particles in the FP64 form (the largest
    workspace) fit the array."""
    n = sph.SPH_NOALLOC_MAX_PARTICLES
    ps = workloads.lattice((32, 32, 32), 1.0 / 32, 0.1, 0.2, seed=9)
    assert ps.n == n
    log(f"case noalloc fp64 at the maximum n={n}")
    g = _noalloc(ps, "fp64")
    c = gpu_run(ps, "fp64")
    _same_pass(g, c, "fp64")


def test_noalloc_refuses_what_it_cannot_hold():
    log("case noalloc refusals")
    ps = workloads.uniform(sph.SPH_NOALLOC_MAX_PARTICLES + 1, seed=3)
    parts = sph.Particles.from_numpy(ps, "cuda:0")
    with pytest.raises(sph.SPHError) as e:
        sph.pass_noalloc(parts, ps.box, "fp32")
    assert e.value.status == sph.SPH_E_CAPACITY
    small = workloads.uniform(2000, seed=3)
    parts = sph.Particles.from_numpy(small, "cuda:0")
    for kw in ({"max_depth": 4}, {"keep_adjoint": 1}, {"reuse": sph.SPH_REUSE_CELLS}):
        with pytest.raises(sph.SPHError) as e:
            sph.pass_noalloc(parts, small.box, "fp32", **kw)
        assert e.value.status == sph.SPH_E_INVALID_ARG, kw
