// adjoint.hip -- hand-written reverse mode of the density and force stages
// (Gonnet 2014, Sec. 2.1 Eqs. (2)-(5) and the Sec. 4.1 viscosity) with
// respect to the positions and smoothing lengths, for gfx950.
//
// Given dL/drho, dL/da and dL/d(du/dt) (caller order), the adjoint runs:
//   1. force sweep     every pair term of Eqs. (4)-(5) + viscosity is
//                      differentiated for both of its orderings; each target
//                      particle gathers dL/dx, dL/dh and the adjoints of its
//                      A, rho and Balsara f;
//   2. ghost step      elementwise reverse of Omega, P, A, the divergence, the
//                      curl and the Balsara switch: adjoints of the density
//                      sums (sum m w, sum m q w', the divergence and curl sums)
//                      and the explicit h terms;
//   3. density sweep   reverse of the density sums, both orderings of a pair;
//   4. implicit h      when h is the solved root of N_i(h_i) = N_ngb
//                      (Eq. (3)), dh_i/dx = -(dN_i/dx)/(dN_i/dh_i) depends on
//                      particle i alone, so lambda_i = (dL/dh_i)/(dN_i/dh_i)
//                      and one more sweep adds -sum_i lambda_i dN_i/dx.
// The sweeps reuse the staging and sorted walk of the force stage (pairs
// with r < max(h_i, h_j)); every target particle is written by one workgroup.
#include "sweep.h"

namespace sph {

enum { ADJ_FORCE = 0, ADJ_DENSITY = 1, ADJ_IMPLICIT = 2 };
constexpr int NACC_ADJ = 7;

// w''(q) of the cubic spline
template <typename R> __device__ __forceinline__ R kern_ddw(R q)
{
    return q <= (R)0.5 ? (R)36 * q - (R)12 : (R)12 * ((R)1 - q);
}

// g'(q) for g = w'/q: 18 on the inner branch, 6 (1 - q^2) / q^2 on the outer
template <typename R> __device__ __forceinline__ R kern_dg(R q, R qinv)
{
    return q <= (R)0.5 ? (R)18 : (R)6 * ((R)1 - q * q) * qinv * qinv;
}

// Kernel-gradient factor G(r, h) = 8/(pi h^5) g(r/h) (grad W = G r_vec) and
// its derivatives in r and h; zero outside the support and at r = 0.
template <typename R>
struct KGrad {
    R G, dGdr, dGdh;
};

template <typename R>
__device__ __forceinline__ KGrad<R> kgrad(R r, R rinv, R h, R hinv, R K)
{
    const R q = r * hinv;
    const bool in = (q < (R)1) & (r > (R)0);
    const R qinv = h * rinv;
    const R g = kern_g(q, qinv);
    const R gp = kern_dg(q, qinv);
    KGrad<R> o;
    o.G = in ? K * g : (R)0;
    o.dGdr = in ? K * gp * hinv : (R)0;
    o.dGdh = in ? -K * hinv * ((R)5 * g + q * gp) : (R)0;
    return o;
}

// Reverse of one ordered pair term of the force stage: particle a gets
//   a_a  += phi r_ab,  phi = -m_b (A_a G_a + A_b G_b) - 1/4 m_b Pi (G_a + G_b) F,
//   du_a += psi,       psi = A_a m_b vr G_a + 1/8 m_b Pi vr (G_a + G_b) F,
// with T = (dL/da_a) . (phi r_ab) + (dL/ddu_a) psi.  Returns dT/dr_ab (vector)
// and dT/dG_a, dT/dG_b, dT/dA_a, dT/dA_b, dT/drho (either), dT/df (either).
template <typename R>
struct FPair {
    R gx, gy, gz, tGa, tGb, tAa, tAb, trho, tF;
};

template <typename R>
__device__ __forceinline__ FPair<R> force_pair_adj(R rx, R ry, R rz, R rinv, R vx, R vy, R vz, const KGrad<R>& Ga,
                                                   const KGrad<R>& Gb, R Aa, R Ab, R ca, R cb, R rhoa, R rhob, R fa,
                                                   R fb, R mb, typename Vec4T<R>::T ab, R alpha)
{
    const R s = ab.x * rx + ab.y * ry + ab.z * rz;
    const R u = ab.w;
    const R vr = vx * rx + vy * ry + vz * rz;
    const bool neg = vr < (R)0;
    const R w = neg ? vr * rinv : (R)0;
    const R irs = fast_rcp(rhoa + rhob);
    const R Pi = -alpha * (ca + cb - (R)3 * w) * w * irs;
    const R F = fa + fb;
    const R Gs = Ga.G + Gb.G;
    const R phi = -mb * (Aa * Ga.G + Ab * Gb.G) - (R)0.25 * mb * Pi * Gs * F;
    FPair<R> o;
    o.tGa = s * (-mb * Aa - (R)0.25 * mb * Pi * F) + u * (Aa * mb * vr + (R)0.125 * mb * Pi * vr * F);
    o.tGb = s * (-mb * Ab - (R)0.25 * mb * Pi * F) + u * ((R)0.125 * mb * Pi * vr * F);
    const R tPi = s * (-(R)0.25 * mb * Gs * F) + u * ((R)0.125 * mb * vr * Gs * F);
    o.tF = s * (-(R)0.25 * mb * Pi * Gs) + u * ((R)0.125 * mb * Pi * vr * Gs);
    R tvr = u * (Aa * mb * Ga.G + (R)0.125 * mb * Pi * Gs * F);
    o.tAa = s * (-mb * Ga.G) + u * (mb * vr * Ga.G);
    o.tAb = s * (-mb * Gb.G);
    const R tw = tPi * (-alpha * (ca + cb - (R)6 * w) * irs);
    R tr = o.tGa * Ga.dGdr + o.tGb * Gb.dGdr;
    if (neg) {
        tvr += tw * rinv;
        tr += tw * (-w * rinv);
    }
    o.trho = tPi * (-Pi * irs);
    o.gx = phi * ab.x + tr * rx * rinv + tvr * vx;
    o.gy = phi * ab.y + tr * ry * rinv + tvr * vy;
    o.gz = phi * ab.z + tr * rz * rinv + tvr * vz;
    return o;
}

// Reverse of one ordered pair of the density sums of particle a (r < h_a):
//   Phi = Sw_bar m_b w + Sq_bar m_b q w' + D_bar m_b g (dv . r) + C_bar . (m_b g dv x r),
// q = r/h_a, r = x_a - x_b, dv = v_b - v_a.  Returns dPhi/dr (vector) and dPhi/dh_a.
template <typename R>
__device__ __forceinline__ void density_pair_adj(R rx, R ry, R rz, R r, R rinv, R h, R hinv, R dvx, R dvy, R dvz,
                                                 R mb, typename Vec4T<R>::T sb0, typename Vec4T<R>::T sb1, R& gx,
                                                 R& gy, R& gz, R& gh)
{
    const R q = r * hinv;
    const R qinv = h * rinv;
    const R w1 = kern_dw(q), w2 = kern_ddw(q);
    const R g = kern_g(q, qinv), gp = kern_dg(q, qinv);
    const R cx = dvy * rz - dvz * ry, cy = dvz * rx - dvx * rz, cz = dvx * ry - dvy * rx;  // dv x r
    const R E = sb0.z * (dvx * rx + dvy * ry + dvz * rz) + sb1.x * cx + sb1.y * cy + sb1.z * cz;
    const R dq = mb * (sb0.x * w1 + sb0.y * (w1 + q * w2) + (r > (R)0 ? gp * E : (R)0));
    const R rad = dq * hinv * rinv;
    const R mg = mb * g;
    // d/dr of (dv . r) is dv; of C_bar . (dv x r) = r . (C_bar x dv) is C_bar x dv
    gx = rad * rx + mg * (sb0.z * dvx + (sb1.y * dvz - sb1.z * dvy));
    gy = rad * ry + mg * (sb0.z * dvy + (sb1.z * dvx - sb1.x * dvz));
    gz = rad * rz + mg * (sb0.z * dvz + (sb1.x * dvy - sb1.y * dvx));
    gh = dq * (-q * hinv);
}

template <typename R, int MODE>
__global__ __launch_bounds__(WGS) void k_adj_sweep(Decomp dc, CellData<R> cd, Sorted<R> so, GhostData<R> gd,
                                                   AdjData<R> ad, PassConsts pc)
{
    using R4 = typename Vec4T<R>::T;
    using SM = Smem<R, NACC_ADJ, true>;
    __shared__ SM s;
    const int tid = threadIdx.x;
    const int w = __builtin_amdgcn_readfirstlane(tid >> 6);  // uniform: the wavefront index
    const int lane = tid & (kWave - 1);
    const int ncells = *dc.ncells;
    const R alpha = (R)pc.alpha;
    const R k323 = (R)(32.0 / 3.0);
    if (*dc.status & (ST_NONFINITE | ST_H_TOO_LARGE | ST_CAPACITY)) return;
    while (true) {
        if (tid == 0) s.unit = atomicAdd(dc.qhead, 1);
        __syncthreads();
        const int unit = s.unit;
        __syncthreads();
        if (unit >= ncells) break;
        const CellInfo T = dc.cells[unit];
        const BoxInfo B = dc.boxes[T.box];
        const int nsrc = dc.src_count[unit];
        const float margin = 1e-5f * (float)fmax(B.e[0], fmax(B.e[1], B.e[2]));
        const float mstage = margin + cell_dr(dc, unit);   // targets may have left the cell by this
        const float Hst = gd.cell_hmax[unit];
        int k = 0, p = 0;
        stage_wave<R, true>(s, w, dc, cd, so, gd, B, unit, T.level, nsrc, k, p, Hst, mstage);
        const bool single = k >= nsrc;
        for (int c0 = 0; c0 < T.count; c0 += kWave) {
            const int ti = c0 + lane;
            const bool valid = ti < T.count;
            const uint32_t gi = (uint32_t)(T.start + (valid ? ti : 0));
            const R4 ri = cd.rp[gi];
            const R xi = ri.x, yi = ri.y, zi = ri.z;
            const R4 vmi = cd.vm[gi], g0i = gd.g0[gi], g1i = gd.g1[gi];
            const R hi = g1i.z, hinvi = g0i.x;
            R4 abi = {}, sb0i = {}, sb1i = {};
            if (MODE == ADJ_FORCE) abi = ad.ab[gi];
            if (MODE != ADJ_FORCE) sb0i = ad.sb0[gi];
            if (MODE == ADJ_DENSITY) sb1i = ad.sb1[gi];
            const float fxi = (float)xi, fyi = (float)yi, fzi = (float)zi, fh = (float)hi;
            for (int a = w; a < NACC_ADJ; a += NW) s.red[a][lane] = 0.0;
            __syncthreads();
            double acc[NACC_ADJ] = {0, 0, 0, 0, 0, 0, 0};
            auto pair = [&](bool ok, int j) {
                const R4 e = s.st[w][j];
                const uint32_t g = s.sg[w][j];
                const R4 vmj = cd.vm[g], g0j = gd.g0[g], g1j = gd.g1[g];
                const R rx = xi - e.x, ry = yi - e.y, rz = zi - e.z;
                const R r2 = rx * rx + ry * ry + rz * rz;
                const R r = fast_sqrt(r2);
                const R rinv = r > (R)0 ? fast_rcp(r) : (R)0;
                const R hj = g1j.z, hinvj = g0j.x;
                R gx = 0, gy = 0, gz = 0, gh = 0;
                if (MODE == ADJ_FORCE) {
                    const R4 abj = ad.ab[g];
                    const KGrad<R> Gi = kgrad(r, rinv, hi, hinvi, g0i.y);
                    const KGrad<R> Gj = kgrad(r, rinv, hj, hinvj, g0j.y);
                    const R vx = vmi.x - vmj.x, vy = vmi.y - vmj.y, vz = vmi.z - vmj.z;
                    // ordering (i, j): the target is the first particle
                    const FPair<R> d = force_pair_adj(rx, ry, rz, rinv, vx, vy, vz, Gi, Gj, g0i.z, g0j.z, g1i.x, g1j.x,
                                                      g0i.w, g0j.w, g1i.y, g1j.y, vmj.w, abi, alpha);
                    // ordering (j, i): the target is the second particle (r and v flip sign)
                    const FPair<R> b = force_pair_adj(-rx, -ry, -rz, rinv, -vx, -vy, -vz, Gj, Gi, g0j.z, g0i.z, g1j.x,
                                                      g1i.x, g0j.w, g0i.w, g1j.y, g1i.y, vmi.w, abj, alpha);
                    gx = d.gx - b.gx;
                    gy = d.gy - b.gy;
                    gz = d.gz - b.gz;
                    gh = d.tGa * Gi.dGdh + b.tGb * Gi.dGdh;
                    if (ok) {
                        acc[4] += (double)(d.tAa + b.tAb);
                        acc[5] += (double)(d.trho + b.trho);
                        acc[6] += (double)(d.tF + b.tF);
                    }
                } else if (MODE == ADJ_DENSITY) {
                    const R dvx = vmj.x - vmi.x, dvy = vmj.y - vmi.y, dvz = vmj.z - vmi.z;
                    if (r < hi) {  // the pair enters the target's own sums
                        R ax, ay, az, ah;
                        density_pair_adj(rx, ry, rz, r, rinv, hi, hinvi, dvx, dvy, dvz, vmj.w, sb0i, sb1i, ax, ay,
                                         az, ah);
                        gx += ax; gy += ay; gz += az; gh += ah;
                    }
                    if (r < hj) {  // the pair enters the neighbour's sums (r_ji = -r_ij)
                        const R4 sb0j = ad.sb0[g], sb1j = ad.sb1[g];
                        R bx, by, bz, bh;
                        density_pair_adj(-rx, -ry, -rz, r, rinv, hj, hinvj, -dvx, -dvy, -dvz, vmi.w, sb0j, sb1j, bx,
                                         by, bz, bh);
                        gx -= bx; gy -= by; gz -= bz;
                    }
                } else {  // implicit h: -sum_a lambda_a dN_a/dx_target
                    const R li = sb0i.w, lj = ad.sb0[g].w;
                    const R qi = r * hinvi, qj = r * hinvj;
                    R c = (R)0;
                    if (r < hi) c += li * kern_dw(qi) * hinvi;
                    if (r < hj) c += lj * kern_dw(qj) * hinvj;
                    c = -k323 * c * rinv;
                    gx = c * rx; gy = c * ry; gz = c * rz;
                }
                if (ok) {
                    acc[0] += (double)gx;
                    acc[1] += (double)gy;
                    acc[2] += (double)gz;
                    acc[3] += (double)gh;
                }
            };
            auto process = [&](int n) {
                for (int t = 0;; t++) {
                    const bool v0 = t < n;
                    if (!__any(v0)) break;
                    pair(v0, v0 ? (int)s.list[w][lane][t] : 0);
                }
            };
            int kk = 0, pp = 0;
            do {
                if (!single) stage_wave<R, true>(s, w, dc, cd, so, gd, B, unit, T.level, nsrc, kk, pp, Hst, mstage);
                else kk = nsrc;
                const int selfj = self_index(s, w, ti);
                int seg = 0, jj = s.nseg[w] > 0 ? s.seg_b[w][0] : 0;
                int cnt = 0;
                while (true) {
                    cnt = walk<R, true, NACC_ADJ>(s, w, w, lane, valid, xi, yi, zi, fxi, fyi, fzi, hi, fh, margin, selfj,
                                                  seg, jj, cnt);
                    process(cnt);
                    cnt = 0;
                    if (seg >= s.nseg[w]) break;
                }
            } while (kk < nsrc);
            if (valid)
                for (int a = 0; a < NACC_ADJ; a++) atomicAdd(&s.red[a][lane], acc[a]);
            __syncthreads();
            if (w == 0 && valid) {
                double* xb = ad.xbar + 3 * (int64_t)gi;
                if (MODE == ADJ_FORCE) {
                    xb[0] = s.red[0][lane]; xb[1] = s.red[1][lane]; xb[2] = s.red[2][lane];
                    ad.hbar[gi] = s.red[3][lane];
                    double4 f = ad.fg[gi];
                    f.x = s.red[4][lane]; f.y = s.red[5][lane]; f.z = s.red[6][lane];
                    ad.fg[gi] = f;
                } else {
                    xb[0] += s.red[0][lane]; xb[1] += s.red[1][lane]; xb[2] += s.red[2][lane];
                    if (MODE == ADJ_DENSITY) ad.hbar[gi] += s.red[3][lane];
                }
            }
            __syncthreads();
        }
    }
}

// upstream gradients into cell order
template <typename R>
__global__ void k_adj_prepare(const uint32_t* perm, int64_t n, AdjIO io, AdjData<R> ad)
{
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n) return;
    const uint32_t p = perm[k];
    typename Vec4T<R>::T a;
    a.x = io.g_ax ? (R)io.g_ax[p] : (R)0;
    a.y = io.g_ay ? (R)io.g_ay[p] : (R)0;
    a.z = io.g_az ? (R)io.g_az[p] : (R)0;
    a.w = io.g_dudt ? (R)io.g_dudt[p] : (R)0;
    ad.ab[k] = a;
    ad.fg[k] = make_double4(0.0, 0.0, 0.0, io.g_rho ? io.g_rho[p] : 0.0);
}

// Reverse of the per-particle quantities between the stages (FP64).
template <typename R>
__global__ void k_adj_ghost(const CellData<R> cd, const GhostData<R> gd, AdjData<R> ad, PassConsts pc, int64_t n)
{
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n) return;
    const double kNorm = 8.0 / kPi;
    const double4 s0 = gd.sd0[k], s1 = gd.sd1[k];
    const double h = cd.h[k], u = cd.u[k];
    const double Smw = s0.x, Smq = s0.y, D = s0.w;
    const double k3 = kNorm / (h * h * h), k5 = k3 / (h * h);
    const double rho = k3 * Smw;
    const double omega = -Smq / (3.0 * Smw);
    const double div = k5 * D / rho;
    const double cx = -k5 * s1.x / rho, cy = -k5 * s1.y / rho, cz = -k5 * s1.z / rho;
    const double cm = sqrt(cx * cx + cy * cy + cz * cz);
    const double P = (pc.gamma - 1.0) * rho * u;
    const double c = sqrt(pc.gamma * P / rho);
    const double A = P / (omega * rho * rho);
    const double den = fabs(div) + cm + pc.beps * c / h;
    const double4 fg = ad.fg[k];
    const double Abar = fg.x, fbar = fg.z;
    double rhobar = fg.y + fg.w;
    double hbar = 0.0;
    // Balsara f = X / (|div| + |curl| + eps c / h), X = |curl| or |div|
    double divbar = 0.0, cbx = 0.0, cby = 0.0, cbz = 0.0;
    if (den > 0.0) {
        const double num = pc.balsara_div ? fabs(div) : cm;
        const double denbar = -fbar * num / (den * den);   // through the denominator
        const double numbar = fbar / den;                    // through the numerator
        const double cmbar = denbar + (pc.balsara_div ? 0.0 : numbar);
        const double adbar = denbar + (pc.balsara_div ? numbar : 0.0);
        hbar -= denbar * pc.beps * c / (h * h);
        divbar = div > 0.0 ? adbar : (div < 0.0 ? -adbar : 0.0);
        if (cm > 0.0) { cbx = cmbar * cx / cm; cby = cmbar * cy / cm; cbz = cmbar * cz / cm; }
    }
    // A = (gamma-1) u / (Omega rho)
    const double obar = -Abar * A / omega;
    rhobar += -Abar * A / rho;
    // div = k5 D / rho, curl = -k5 C / rho
    const double Dbar = divbar * k5 / rho;
    rhobar += -divbar * div / rho;
    hbar += divbar * div * (-5.0 / h);
    const double cdot = cbx * cx + cby * cy + cbz * cz;
    rhobar += -cdot / rho;
    hbar += cdot * (-5.0 / h);
    // Omega = -S_mqw' / (3 S_mw), rho = k3 S_mw
    const double Smqbar = -obar / (3.0 * Smw);
    double Smwbar = -obar * omega / Smw + rhobar * k3;
    hbar += rhobar * rho * (-3.0 / h);
    typename Vec4T<R>::T b0, b1;
    b0.x = (R)Smwbar; b0.y = (R)Smqbar; b0.z = (R)Dbar; b0.w = (R)0;
    b1.x = (R)(-cbx * k5 / rho); b1.y = (R)(-cby * k5 / rho); b1.z = (R)(-cbz * k5 / rho); b1.w = (R)0;
    ad.sb0[k] = b0;
    ad.sb1[k] = b1;
    ad.hbar[k] += hbar;
}

// lambda = (dL/dh) / (dN/dh) for the implicit derivative of the solved h
template <typename R>
__global__ void k_adj_lambda(const GhostData<R> gd, AdjData<R> ad, int64_t n)
{
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n) return;
    typename Vec4T<R>::T b0 = ad.sb0[k];
    b0.w = (R)(ad.hbar[k] / gd.sd0[k].z);
    ad.sb0[k] = b0;
}

__global__ void k_adj_output(const uint32_t* perm, int64_t n, const double* xbar, const double* hbar, AdjIO io,
                             int implicit_h)
{
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n) return;
    const uint32_t p = perm[k];
    if (io.gx) io.gx[p] = xbar[3 * k];
    if (io.gy) io.gy[p] = xbar[3 * k + 1];
    if (io.gz) io.gz[p] = xbar[3 * k + 2];
    if (io.gh) io.gh[p] = implicit_h ? 0.0 : hbar[k];
}

static int adj_grid(const void* fn)
{
    int dev = 0, ncu = 0, per = 0;
    (void)hipGetDevice(&dev);
    (void)hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev);
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, fn, WGS, 0) != hipSuccess || per < 1) per = 1;
    return (ncu < 1 ? 1 : ncu) * per;
}

template <typename R>
void launch_adjoint(const Decomp& dc, const CellData<R>& cd, const Sorted<R>& so, const GhostData<R>& gd,
                    const AdjData<R>& ad, const AdjIO& io, const PassConsts& pc, bool implicit_h, int64_t n,
                    hipStream_t st)
{
    const unsigned eg = (unsigned)((n + 255) / 256);
    hipLaunchKernelGGL(k_adj_prepare<R>, dim3(eg), dim3(256), 0, st, dc.perm, n, io, ad);
    launch_reset_counter(dc.qhead, st);
    hipLaunchKernelGGL((k_adj_sweep<R, ADJ_FORCE>), dim3(adj_grid((const void*)k_adj_sweep<R, ADJ_FORCE>)),
                       dim3(WGS), 0, st, dc, cd, so, gd, ad, pc);
    hipLaunchKernelGGL(k_adj_ghost<R>, dim3(eg), dim3(256), 0, st, cd, gd, ad, pc, n);
    launch_reset_counter(dc.qhead, st);
    hipLaunchKernelGGL((k_adj_sweep<R, ADJ_DENSITY>), dim3(adj_grid((const void*)k_adj_sweep<R, ADJ_DENSITY>)),
                       dim3(WGS), 0, st, dc, cd, so, gd, ad, pc);
    if (implicit_h) {
        hipLaunchKernelGGL(k_adj_lambda<R>, dim3(eg), dim3(256), 0, st, gd, ad, n);
        launch_reset_counter(dc.qhead, st);
        hipLaunchKernelGGL((k_adj_sweep<R, ADJ_IMPLICIT>), dim3(adj_grid((const void*)k_adj_sweep<R, ADJ_IMPLICIT>)),
                           dim3(WGS), 0, st, dc, cd, so, gd, ad, pc);
    }
    hipLaunchKernelGGL(k_adj_output, dim3(eg), dim3(256), 0, st, dc.perm, n, ad.xbar, ad.hbar, io,
                       implicit_h ? 1 : 0);
}

template void launch_adjoint<float>(const Decomp&, const CellData<float>&, const Sorted<float>&,
                                    const GhostData<float>&, const AdjData<float>&, const AdjIO&, const PassConsts&,
                                    bool, int64_t, hipStream_t);
template void launch_adjoint<double>(const Decomp&, const CellData<double>&, const Sorted<double>&,
                                     const GhostData<double>&, const AdjData<double>&, const AdjIO&,
                                     const PassConsts&, bool, int64_t, hipStream_t);

}  // namespace sph
