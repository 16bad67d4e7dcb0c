// pairs.h -- the pair terms of the two interaction stages of Gonnet (2014),
// Sec. 2.1 (density, Eqs. (2)-(3), with the divergence and curl of Sec. 4.1)
// and Eqs. (4)-(5) with the viscosity of Sec. 4.1 (force), shared by the
// sweep layouts of the interaction kernels.
#pragma once

#include "sweep.h"

namespace sph {
// ---------------------------------------------------------------- density
struct DensAcc {
    double w, qdw;
    int n;
};
// the sums of one pass over a list, in the pair precision: added to the FP64
// totals once per list (at most LISTW pairs)
template <typename R>
struct DensPart {
    R w, qdw, mw, mqdw, div, cx, cy, cz;
    int n;
};

// w(q) and q w'(q) of the kernel of Sec. 2.1 without branches, t = 1 - q and
// u = max(1 - 2q, 0): w = 2 t^3 - u^3 and q w' = 6 q (u^2 - t^2), which are
// 1 - 6q^2 + 6q^3 and q (18q^2 - 12q) for q <= 1/2 (callers mask q >= 1)
template <typename R>
__device__ __forceinline__ void kern_w_qdw(R q, R& w, R& qdw)
{
    const R t = (R)1 - q, u = fmax(fma((R)-2, q, (R)1), (R)0);
    const R t2 = t * t, u2 = u * u;
    w = fma((R)2 * t2, t, -(u2 * u));
    qdw = (R)6 * q * (u2 - t2);
}

// Newton evaluation: the two sums of Eq. (3) (N and dN/dh need w and q w'),
// into partial sums of one list in the pair precision
template <typename R>
__device__ __forceinline__ void count_pair(R& sw, R& sq, bool ok, R xi, R yi, R zi, R hinv, R h2,
                                           typename Vec4T<R>::T e)
{
    const R dx = xi - e.x, dy = yi - e.y, dz = zi - e.z;
    const R r2 = dx * dx + dy * dy + dz * dz;
    ok = ok && r2 < h2;
    const R q = fast_sqrt(r2) * hinv;
    R w, qdw;
    kern_w_qdw(q, w, qdw);
    sw += ok ? w : (R)0;
    sq += ok ? qdw : (R)0;
}

// All density-stage terms of one pair: Eq. (2), Eq. (3), d rho/dh and the
// velocity divergence and curl of Sec. 4.1 (gradient prefactor applied later)
template <typename R>
__device__ __forceinline__ void density_pair(DensPart<R>& b, bool ok, R xi, R yi, R zi, R vxi, R vyi, R vzi, R h,
                                             R hinv, R h2, typename Vec4T<R>::T e, typename Vec4T<R>::T vm)
{
    const R dx = xi - e.x, dy = yi - e.y, dz = zi - e.z;
    const R r2 = dx * dx + dy * dy + dz * dz;
    ok = ok && r2 < h2;
    const R rinv = r2 > (R)0 ? fast_rsqrt(r2) : (R)0;
    const R q = r2 * rinv * hinv;
    // the kernel without branches, t = 1 - q, u = max(1 - 2q, 0): w = 2 t^3 - u^3,
    // g = w'/q = -6 (u + t) min(1, t/q), which is 18q - 12 for q <= 1/2 and
    // -6 t^2 / q above (zero at r = 0, where the pair adds nothing anyway)
    const R t = (R)1 - q, u = fmax(fma((R)-2, q, (R)1), (R)0);
    const R w = fma((R)2 * t * t, t, -(u * u * u));
    const R gq = (R)-6 * (u + t) * fmin((R)1, t * (h * rinv));
    const R qdw = gq * q * q;
    const R mj = ok ? vm.w : (R)0;  // masked pairs contribute nothing
    const R dvx = vm.x - vxi, dvy = vm.y - vyi, dvz = vm.z - vzi;
    const R mg = mj * gq;
    b.w += ok ? w : (R)0;
    b.qdw += ok ? qdw : (R)0;
    b.mw += mj * w;
    b.mqdw += mj * qdw;
    b.div += mg * (dvx * dx + dvy * dy + dvz * dz);
    b.cx += mg * (dvy * dz - dvz * dy);
    b.cy += mg * (dvz * dx - dvx * dz);
    b.cz += mg * (dvx * dy - dvy * dx);
    b.n += ok ? 1 : 0;
}

// ---------------------------------------------------------------- force
template <typename R>
struct ForceAcc {
    double ax, ay, az, du;
    R vsig;   // largest c_i + c_j - 3 w_ij over the pairs in range (Eq. (6))
    int n;
};
// the sums of one pass over a list (at most LISTW pairs) in the pair precision
template <typename R>
struct ForcePart {
    R ax, ay, az, du;
};

template <typename R>
struct ForceTarget {
    R x, y, z, vx, vy, vz, h, hinv, gk, A, rho, c, f;
};

// Eqs. (4)-(5) and the Monaghan-Balsara viscosity of Sec. 4.1 for one pair
// (one-sided: the contribution of j to particle i).  Pairs outside both
// supports contribute exactly zero (both kernel gradients vanish there).
template <typename R>
__device__ __forceinline__ void force_pair(ForceAcc<R>& a, ForcePart<R>& b, bool ok, const ForceTarget<R>& ti, R alpha,
                                           typename Vec4T<R>::T e, typename Vec4T<R>::T vm,
                                           typename Vec4T<R>::T g0, typename Vec4T<R>::T g1)
{
    const R dx = ti.x - e.x, dy = ti.y - e.y, dz = ti.z - e.z;
    const R r2 = dx * dx + dy * dy + dz * dz;
    const R rinv = r2 > (R)0 ? fast_rsqrt(r2) : (R)0;
    const R r = r2 * rinv;
    const R qi = r * ti.hinv, qj = r * g0.x;
    // grad W(r, h) = 8/(pi h^5) g(q) r_vec with g = w'/q = -6 (u + t) min(1, t/q),
    // t = max(1 - q, 0), u = max(1 - 2q, 0): 18q - 12 for q <= 1/2, -6 t^2/q
    // up to q = 1, zero beyond and (rinv = 0) at r = 0, without branches
    auto grad = [&](R q, R h, R gk) {
        const R t = fmax((R)1 - q, (R)0), u = fmax(fma((R)-2, q, (R)1), (R)0);
        return gk * (R)-6 * (u + t) * fmin((R)1, t * (h * rinv));
    };
    const R gwi = grad(qi, ti.h, ti.gk);
    const R gwj = grad(qj, g1.z, g0.y);
    const R mj = ok ? vm.w : (R)0;  // masked pairs contribute nothing
    const R vr = (ti.vx - vm.x) * dx + (ti.vy - vm.y) * dy + (ti.vz - vm.z) * dz;
    const R wij = fmin(vr * rinv, (R)0);
    const R vsig = ti.c + g1.x - (R)3 * wij;   // signal speed of Eq. (6), >= 0
    const R Pi = -alpha * vsig * wij * fast_rcp(ti.rho + g0.w);
    const R T = Pi * (gwi + gwj) * (ti.f + g1.y);
    const R agi = ti.A * gwi;
    const R sc = -mj * (agi + g0.z * gwj + (R)0.25 * T);
    const R pdu = mj * vr * (agi + (R)0.125 * T);
    b.ax += sc * dx;
    b.ay += sc * dy;
    b.az += sc * dz;
    b.du += pdu;
    // lists may hold a few pairs just outside both supports: they add nothing
    // above (zero gradients) and are neither counted nor signal pairs
    const bool in = ok && (qi < (R)1 || qj < (R)1);
    a.vsig = in ? fmax(a.vsig, vsig) : a.vsig;
    a.n += in ? 1 : 0;
}

}  // namespace sph
