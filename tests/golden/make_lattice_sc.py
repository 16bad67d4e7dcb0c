"""Writes lattice_sc.txt: density-stage values on a perfect simple-cubic lattice.

Independent of the oracle and of the GPU library: the sums of Eq. (2) and
Eq. (3) (Gonnet 2014, Sec. 2.1) over the lattice points around one site are
evaluated exactly in 40-digit decimal arithmetic, and N(h) = 48 is solved by
bisection.  Lattice spacing 1, particle mass 1 (so m n = 1).
"""
import itertools
import os
from decimal import Decimal as D, getcontext

getcontext().prec = 40
PI = D("3.141592653589793238462643383279502884197")


def w(q):
    if q <= D(1) / 2:
        return 1 - 6 * q * q + 6 * q * q * q
    if q <= 1:
        t = 1 - q
        return 2 * t * t * t
    return D(0)


def dw(q):
    if q <= D(1) / 2:
        return -12 * q + 18 * q * q
    if q <= 1:
        t = 1 - q
        return -6 * t * t
    return D(0)


def main():
    dist = [D(i * i + j * j + k * k).sqrt() for i, j, k in itertools.product(range(-4, 5), repeat=3)]

    def count(H):
        return D(32) / 3 * sum(w(r / H) for r in dist if r < H)

    lo, hi = D(2), D("2.5")
    for _ in range(130):
        mid = (lo + hi) / 2
        if count(mid) < 48:
            lo = mid
        else:
            hi = mid
    H = (lo + hi) / 2
    rho = sum(D(8) / (PI * H ** 3) * w(r / H) for r in dist if r < H)
    drho = sum(-D(8) / (PI * H ** 4) * (3 * w(r / H) + (r / H) * dw(r / H)) for r in dist if r < H)
    omega = 1 + H / (3 * rho) * drho
    nn = sum(1 for r in dist if 0 < r < H)
    out = os.path.join(os.path.dirname(os.path.abspath(__file__)), "lattice_sc.txt")
    with open(out, "w") as f:
        f.write("# Simple-cubic lattice, spacing 1, m = 1: Eq. (2)/(3) of Gonnet (2014) Sec. 2.1\n")
        f.write("# at the smoothing length where N_ngb = 48 (40-digit decimal evaluation,\n")
        f.write("# tests/golden/make_lattice_sc.py)\n")
        f.write(f"h_over_dx {H:.20f}\n")
        f.write(f"rho_over_mn {rho:.20f}\n")
        f.write(f"omega {omega:.20f}\n")
        f.write(f"neighbours {nn}\n")


if __name__ == "__main__":
    main()
