"""Host check of the in-range test of the sorted walk (the neighbour search of
Sec. 3.3, FP32 form): r^2/2 is taken as K_i + a_j - x_i . x_j with the
halved squared norms K_i, a_j reduced by 32 units of rounding, by three fused
multiply-adds, against the range rad^2/2 rounded up by 8 units (density), or
the larger of that and h_j^2/2 (force).  The reductions are meant to make the
test conservative: no pair with r below the range may be dropped, whatever the
positions' magnitude relative to the range.  Emulated in numpy float32 with
each FMA as an exact product plus one rounding (float32 products are exact in
float64)."""
import numpy as np

F = np.float32
EPS = float(np.finfo(np.float32).eps)


def fma(a, b, c):
    return (a.astype(np.float64) * b.astype(np.float64) + c.astype(np.float64)).astype(np.float32)


def half_sq_lo(v):
    lo = F(0.5 * (1 - 32 * EPS / 2))
    x, y, z = v[:, 0], v[:, 1], v[:, 2]
    return ((x * x + y * y) + z * z) * lo


def walk_test_density(xi, xj, rad):
    ki, aj = half_sq_lo(xi), half_sq_lo(xj)
    c_half = F(0.5) * rad * rad * F(1 + 8 * EPS)
    t = fma(-xi[:, 2], xj[:, 2], fma(-xi[:, 1], xj[:, 1], fma(-xi[:, 0], xj[:, 0], aj)))
    return t < (c_half - ki)


def walk_test_force(xi, xj, rad, hj):
    ki, aj = half_sq_lo(xi), half_sq_lo(xj)
    c_half = F(0.5) * rad * rad * F(1 + 8 * EPS)
    sh = F(0.5) * hj * hj
    t = fma(-xi[:, 2], xj[:, 2], fma(-xi[:, 1], xj[:, 1], fma(-xi[:, 0], xj[:, 0], aj + ki)))
    return t < np.maximum(c_half, sh)


def _pairs(rng, n, inside):
    scale = 10.0 ** rng.uniform(-1, 2, n)                 # |x| / rad from 0.1 to 100
    rad = (10.0 ** rng.uniform(-3, 0, n)).astype(np.float32)
    xi = ((rng.uniform(-1, 1, (n, 3)) * (scale * rad)[:, None])).astype(np.float32)
    d = rng.normal(size=(n, 3))
    d /= np.linalg.norm(d, axis=1)[:, None]
    rel = 10.0 ** rng.uniform(-8, -3, n)
    r = rad * (1 - rel) if inside else rad * (1 + rel)
    xj = (xi.astype(np.float64) + d * r[:, None]).astype(np.float32)
    r_true = np.linalg.norm(xi.astype(np.float64) - xj.astype(np.float64), axis=1)
    return xi, xj, rad, r_true


def test_no_pair_in_range_is_dropped():
    rng = np.random.default_rng(0)
    xi, xj, rad, r_true = _pairs(rng, 400000, inside=True)
    sel = r_true < rad
    assert sel.sum() > 300000
    assert np.all(walk_test_density(xi[sel], xj[sel], rad[sel]))
    # force: the pair is in range of j's support (h_j > r), i's range smaller
    hj = (r_true[sel] * (1 + 1e-7)).astype(np.float32)
    hj = np.where(hj > r_true[sel], hj, np.nextafter(hj, np.float32(np.inf)))
    assert np.all(walk_test_force(xi[sel], xj[sel], (0.5 * rad[sel]).astype(np.float32), hj))


def test_few_pairs_outside_are_listed():
    # the pair arithmetic discards what the walk lists beyond the range; the
    # allowance is a thin shell (relative width ~1e-6 of |x|^2 / rad^2)
    rng = np.random.default_rng(1)
    xi, xj, rad, r_true = _pairs(rng, 200000, inside=False)
    listed = walk_test_density(xi, xj, rad)
    excess = (r_true[listed] / rad[listed]) ** 2 - 1
    xmag = (np.linalg.norm(xi[listed], axis=1) / rad[listed]) ** 2
    assert np.all(excess <= 1e-5 * (1 + xmag))
