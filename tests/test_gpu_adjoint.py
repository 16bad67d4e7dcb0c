"""GPU parity of the hand-written adjoint (sph_backward) against the gradient
oracle (dense FP64 autograd model, and central differences through the C
oracle at the 262,144-particle size).

Tolerances.  Errors are measured per component against |ref| + RMS(ref) (the
RMS over the compared components is the natural scale of a cancelling sum).

FP64 form, dense oracle: both sides evaluate the same terms in FP64 and
differ in summation order and in the solved h (1e-10 vs 1e-13 in N):
1e-8.

FP32 form, dense oracle: the pair terms are FP32 (about 1e-6 relative each),
the upstream weights are exact inputs, and h carries the 2e-6 relative band
of the FP32 Newton tolerance; the gradient of a sum of kernel derivatives
moves with h at up to ~10x its relative change, so 2e-5 from h plus the
cancellation of ~100 pair terms of 1e-6: 1e-4.

Central differences at 262,144 particles (FP64 loss sum of ~500 local terms
of magnitude ~60, eps = 1e-6 against a spacing of 1/64): the difference
itself is good to ~1e-8 relative.  FP64 form: 1e-6.  FP32 form: the loss
is dominated by sum |a|^2 and the forward a enters the upstream gradient
2a; the FP32 a is within ~1e-6 of kappa (the sum of the magnitudes of its
pair terms) of the FP64 oracle (the parity tests bound it by 1e-5), and
kappa/|a| is ~30 on this lattice (median), so the upstream is good to ~3e-5,
and the adjoint's own FP32 pair sums, cancelling in the same way, to a
similar amount: 1e-4.
"""
import numpy as np
import pytest
import torch

import oracle
from oracle import grad as og
from paper_1404_2303_amd import sph, workloads
from parity_util import log

pytestmark = pytest.mark.gpu

TOL_DENSE = {"fp64": 1e-8, "fp32": 1e-4}
TOL_FD = {"fp64": 1e-6, "fp32": 1e-4}


def _dev(a):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda:0")


def _err(g, ref):
    scale = np.sqrt(np.mean(ref ** 2)) + 1e-300
    return np.max(np.abs(g - ref) / (np.abs(ref) + scale))


def _dense_state(n=1200, seed=17):
    rng = np.random.default_rng(seed)
    ps = workloads.uniform(n, seed=seed, sigma_v=0.4)
    ps.m[:] *= rng.uniform(0.6, 1.4, n)
    ps.u[:] = rng.uniform(0.5, 1.5, n)
    w = (rng.normal(size=n), rng.normal(size=(n, 3)), rng.normal(size=n))
    return ps, w


def _gpu_vjp(ps, precision, w, implicit):
    parts = sph.Particles.from_numpy(ps, "cuda:0")
    ctx = sph.Context(ps.box, precision=precision, keep_adjoint=1)
    ctx.run(parts)
    gx, gh = ctx.backward(parts, _dev(w[0]), _dev(w[1]), _dev(w[2]), implicit_h=implicit, want_h=True)
    torch.cuda.synchronize()
    out = gx.cpu().numpy(), gh.cpu().numpy(), parts.h.cpu().numpy()
    ctx.close()
    return out


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
@pytest.mark.parametrize("implicit", [False, True])
def test_adjoint_matches_dense_oracle(precision, implicit):
    ps, w = _dense_state()
    log(f"case adjoint dense 1200 {precision} implicit={implicit}")
    gx, gh, h = _gpu_vjp(ps, precision, w, implicit)
    hs, _ = oracle.solve_h(ps.pos, ps.h0, ps.box, tol=1e-13)
    rx, rh, _, _ = og.vjp(ps.pos, ps.vel, ps.m, ps.u, ps.h0 if implicit else hs, ps.box, *w, solve=implicit)
    ex = _err(gx, rx)
    log(f"  dL/dx err {ex:.2e}")
    assert ex <= TOL_DENSE[precision]
    if implicit:
        assert np.all(gh == 0.0)
    else:
        eh = _err(gh, rh)
        log(f"  dL/dh err {eh:.2e}")
        assert eh <= TOL_DENSE[precision]


@pytest.mark.parametrize("which", ["rho", "a", "dudt"])
def test_adjoint_each_upstream_alone(which):
    # each output's reverse path on its own (the others' weights zero / NULL)
    ps, w = _dense_state(900, 23)
    log(f"case adjoint upstream {which} alone fp64")
    parts = sph.Particles.from_numpy(ps, "cuda:0")
    ctx = sph.Context(ps.box, precision="fp64", keep_adjoint=1)
    ctx.run(parts)
    kw = {"rho": (w[0], None, None), "a": (None, w[1], None), "dudt": (None, None, w[2])}[which]
    gx, gh = ctx.backward(parts, *[None if a is None else _dev(a) for a in kw], implicit_h=False, want_h=True)
    torch.cuda.synchronize()
    hs, _ = oracle.solve_h(ps.pos, ps.h0, ps.box, tol=1e-13)
    zw = [np.zeros_like(a) if b is None else a for a, b in zip(w, kw)]
    rx, rh, _, _ = og.vjp(ps.pos, ps.vel, ps.m, ps.u, hs, ps.box, *zw, solve=False)
    ex, eh = _err(gx.cpu().numpy(), rx), _err(gh.cpu().numpy(), rh)
    log(f"  err x {ex:.2e} h {eh:.2e}")
    assert ex <= TOL_DENSE["fp64"] and eh <= TOL_DENSE["fp64"]
    ctx.close()


def test_autograd_function_matches_dense_oracle():
    ps, _ = _dense_state(1000, 29)
    rt = workloads.density_target(ps.pos, float(np.sum(ps.m)))
    log("case SPHPass autograd 1000 fp64")
    ctx = sph.Context(ps.box, precision="fp64", keep_adjoint=1)
    pos = _dev(ps.pos).requires_grad_(True)
    rho, a, dudt = sph.SPHPass.apply(pos, _dev(ps.vel), _dev(ps.m), _dev(ps.u), _dev(ps.h0), ctx)
    L = ((rho - _dev(rt)) ** 2).sum() + (a ** 2).sum()
    (g,) = torch.autograd.grad(L, pos)
    rx, _, Lref, _ = og.gradients(ps.pos, ps.vel, ps.m, ps.u, ps.h0, ps.box, rt, solve=True)
    ex = _err(g.cpu().numpy(), rx)
    log(f"  L {float(L):.12e} ref {Lref:.12e} err {ex:.2e}")
    assert abs(float(L) / Lref - 1.0) <= 1e-9
    assert ex <= TOL_DENSE["fp64"]
    ctx.close()


def test_fixed_h_autograd_function_matches_dense_oracle():
    """SPHPassFixedH: the sums at a given h (not the root of Eq. (3)) and their
    gradients in the positions and in h, against the dense model at that h."""
    ps, _ = _dense_state(1000, 37)
    rng = np.random.default_rng(37)
    hs, _ = oracle.solve_h(ps.pos, ps.h0, ps.box, tol=1e-13)
    h = hs * rng.uniform(0.97, 1.03, ps.n)
    rt = workloads.density_target(ps.pos, float(np.sum(ps.m)))
    log("case SPHPassFixedH autograd 1000 fp64")
    ctx = sph.Context(ps.box, precision="fp64", keep_adjoint=1, fixed_h=1)
    pos = _dev(ps.pos).requires_grad_(True)
    ht = _dev(h).requires_grad_(True)
    rho, a, dudt = sph.SPHPassFixedH.apply(pos, ht, _dev(ps.vel), _dev(ps.m), _dev(ps.u), ctx)
    ref_d = oracle.density(ps.pos, ps.vel, ps.m, h, ps.box)
    e_rho = np.max(np.abs(rho.detach().cpu().numpy() / ref_d["rho"] - 1))
    L = ((rho - _dev(rt)) ** 2).sum() + (a ** 2).sum()
    gx, gh = torch.autograd.grad(L, (pos, ht))
    rx, rh, Lref, _ = og.gradients(ps.pos, ps.vel, ps.m, ps.u, h, ps.box, rt, solve=False)
    ex, eh = _err(gx.cpu().numpy(), rx), _err(gh.cpu().numpy(), rh)
    log(f"  rho err {e_rho:.2e} L {float(L):.12e} ref {Lref:.12e} err x {ex:.2e} h {eh:.2e}")
    assert e_rho <= 1e-10
    assert abs(float(L) / Lref - 1.0) <= 1e-9
    assert ex <= TOL_DENSE["fp64"] and eh <= TOL_DENSE["fp64"]
    ctx.close()


def test_backward_of_a_replaced_state_is_refused():
    """A second forward pass on the same context replaces the state the first
    one's backward would differentiate: that backward fails (SPH_E_STATE)
    instead of returning the gradients of the other state.  A context
    without keep_adjoint has nothing to differentiate."""
    ps, _ = _dense_state(800, 41)
    log("case stale backward 800 fp64")
    ctx = sph.Context(ps.box, precision="fp64", keep_adjoint=1)
    pos1 = _dev(ps.pos).requires_grad_(True)
    out1 = sph.SPHPass.apply(pos1, _dev(ps.vel), _dev(ps.m), _dev(ps.u), _dev(ps.h0), ctx)
    pos2 = _dev(ps.pos + 1e-3).requires_grad_(True)
    out2 = sph.SPHPass.apply(pos2, _dev(ps.vel), _dev(ps.m), _dev(ps.u), _dev(ps.h0), ctx)
    with pytest.raises(sph.SPHError) as e:
        torch.autograd.grad(out1[0].sum(), pos1)
    assert e.value.status == sph.SPH_E_STATE
    (g2,) = torch.autograd.grad(out2[0].sum(), pos2)   # the current state still differentiates
    assert torch.isfinite(g2).all()
    ctx.close()
    plain = sph.Context(ps.box, precision="fp64")
    parts = sph.Particles.from_numpy(ps, "cuda:0")
    plain.run(parts)
    with pytest.raises(sph.SPHError) as e:
        plain.backward(parts, _dev(np.ones(ps.n)), None, None, implicit_h=True)
    assert e.value.status == sph.SPH_E_STATE
    plain.close()


def test_adjoint_translation_invariance_fp32():
    # with h solved, the loss of a frozen per-particle target is invariant under
    # a rigid shift of all particles, so sum_k dL/dx_k = 0
    ps = workloads.config4()
    rt = workloads.density_target(ps.pos, float(np.sum(ps.m)))
    log("case adjoint translation invariance 262144 fp32")
    parts = sph.Particles.from_numpy(ps, "cuda:0")
    ctx = sph.Context(ps.box, precision="fp32", keep_adjoint=1)
    d, f = ctx.run(parts)
    a = torch.stack([f["ax"], f["ay"], f["az"]], 1)
    gx = ctx.backward(parts, 2 * (d["rho"] - _dev(rt)), 2 * a, None, implicit_h=True)
    tot = gx.sum(0).abs().max().item()
    mag = gx.abs().sum().item()
    log(f"  |sum| {tot:.3e} sum|g| {mag:.3e}")
    assert tot <= 1e-6 * mag
    ctx.close()


# ---------------------------------------------------------------- 262,144 particles vs central differences
@pytest.fixture(scope="module")
def fd_case():
    ps = workloads.config4()
    rt = workloads.density_target(ps.pos, float(np.sum(ps.m)))
    hs, _ = oracle.solve_h(ps.pos, ps.h0, ps.box, tol=1e-13)
    R = 2.2 * hs.max()
    rng = np.random.default_rng(404)
    ks = rng.choice(ps.n, 64, replace=False)
    axes = rng.integers(0, 3, 64)
    log("fd reference: 64 coordinates of the 262144 lattice (oracle, local)")
    fd = np.array([og.loss_fd(ps.pos, ps.vel, ps.m, ps.u, ps.h0, ps.box, rt, int(k), int(ax), 1e-6,
                              solve=True, h_fixed=hs, local=R) for k, ax in zip(ks, axes)])
    kh = ks[:16]
    fdh = np.array([og.loss_fd_h(ps.pos, ps.vel, ps.m, ps.u, hs, ps.box, rt, int(k), 1e-7, local=R) for k in kh])
    return dict(ps=ps, rt=rt, ks=ks, axes=axes, fd=fd, kh=kh, fdh=fdh)


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
def test_adjoint_matches_central_differences_262144(fd_case, precision):
    ps, rt = fd_case["ps"], fd_case["rt"]
    log(f"case adjoint FD 262144 {precision}")
    parts = sph.Particles.from_numpy(ps, "cuda:0")
    ctx = sph.Context(ps.box, precision=precision, keep_adjoint=1)
    d, f = ctx.run(parts)
    a = torch.stack([f["ax"], f["ay"], f["az"]], 1)
    g_rho, g_a = 2 * (d["rho"] - _dev(rt)), 2 * a
    gx = ctx.backward(parts, g_rho, g_a, None, implicit_h=True).cpu().numpy()
    gs = gx[fd_case["ks"], fd_case["axes"]]
    e = _err(gs, fd_case["fd"])
    log(f"  implicit-h dL/dx vs FD: err {e:.2e}")
    assert e <= TOL_FD[precision]
    # fixed-h derivative in h at the solved h
    _, gh = ctx.backward(parts, g_rho, g_a, None, implicit_h=False, want_h=True)
    ghs = gh.cpu().numpy()[fd_case["kh"]]
    eh = _err(ghs, fd_case["fdh"])
    log(f"  fixed-h dL/dh vs FD: err {eh:.2e}")
    assert eh <= TOL_FD[precision]
    ctx.close()
