// passes.hip -- the two interaction stages of Gonnet (2014), Sec. 2.1, on
// the cell decomposition of Sec. 3.2 with the sorted pair sweeps of
// Sec. 3.3, for gfx950.
//
// Work unit: one target cell T, processed by one 64-lane wavefront with one
// lane per target particle (cells with more than 64 particles are taken in
// chunks of 64).  The unit gathers from T itself (self interaction) and from
// its 26 neighbours (pair interactions, periodic images included).
//
// Staging.  For each neighbour S in direction d (unit vector u, from T to S)
// the particles of S are read in the stored order along d (reversed for the
// 13 directions that are negatives of stored ones), shifted into T's frame,
// and copied to LDS while their projection u.x stays within reach of T:
// u.x_j <= max_{x in T} u.x + H + margin.  Because the projection never
// exceeds the distance, nothing beyond that prefix can be in range.
//
// Sweep.  Each lane walks the staged segments one after the other; inside a
// segment it stops at the first particle with u.x_j > u.x_i + H_i + margin
// (the early exit of the sorted pair interaction), and otherwise tests the
// true distance.  Particles in range are appended to the lane's neighbour
// list in LDS (the compaction step); when any list is full, or the walk is
// over, every lane evaluates the interaction for its own list.  Lanes thus
// run the expensive arithmetic only on pairs that are in range, each on its
// own particle (a gather: the target particle is written by this wavefront
// alone, so no atomics are needed).
//
// Density (Eqs. (2)-(3)): the Newton iteration on h runs inside the unit,
// re-sweeping the staged neighbourhood for the lanes that have not yet
// converged; the per-particle quantities of the force stage (Omega, P, c,
// A = P/(Omega rho^2), the Balsara switch of Sec. 4.1) are formed at the end.
// Force (Eqs. (4)-(5) + Sec. 4.1 viscosity): one sweep over r < max(h_i, h_j).
//
// Arithmetic: pair terms in R (float or double); every per-particle sum and
// the Newton step in double.
#include "sph_internal.h"
#include "kernels.h"

namespace sph {

constexpr int WG = 64;

template <typename R> struct StageCfg;
template <> struct StageCfg<float> { static constexpr int CAP = 1024; static constexpr int LIST = 64; };
template <> struct StageCfg<double> { static constexpr int CAP = 640; static constexpr int LIST = 64; };

// ---------------------------------------------------------------- kernel W (Sec. 2.1)
// w(q) = 1 - 6q^2 + 6q^3 (q <= 1/2), 2(1-q)^3 (1/2 < q <= 1); callers ensure q < 1.
template <typename R> __device__ __forceinline__ R kern_w(R q)
{
    R a = (R)1 + q * q * ((R)6 * q - (R)6);
    R t = (R)1 - q;
    R b = (R)2 * t * t * t;
    return q <= (R)0.5 ? a : b;
}
// w'(q)
template <typename R> __device__ __forceinline__ R kern_dw(R q)
{
    R a = q * ((R)18 * q - (R)12);
    R t = (R)1 - q;
    R b = (R)-6 * t * t;
    return q <= (R)0.5 ? a : b;
}
// g(q) = w'(q)/q, given qinv = 1/q (only read on the outer branch, q > 1/2)
template <typename R> __device__ __forceinline__ R kern_g(R q, R qinv)
{
    R a = (R)18 * q - (R)12;
    R t = (R)1 - q;
    R b = (R)-6 * t * t * qinv;
    return q <= (R)0.5 ? a : b;
}

template <typename R> __device__ __forceinline__ R rsqrt_t(R v);
template <> __device__ __forceinline__ float rsqrt_t<float>(float v) { return __frsqrt_rn(v); }
template <> __device__ __forceinline__ double rsqrt_t<double>(double v) { return 1.0 / sqrt(v); }

__device__ __forceinline__ double wave_max(double v)
{
    for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
    return v;
}
__device__ __forceinline__ int wave_max_i(int v)
{
    for (int o = 32; o > 0; o >>= 1) v = max(v, __shfl_xor(v, o, 64));
    return v;
}

// ---------------------------------------------------------------- LDS layout
template <typename R, bool FORCE>
struct Smem {
    static constexpr int CAP = StageCfg<R>::CAP;
    static constexpr int LIST = StageCfg<R>::LIST;
    R sx[CAP], sy[CAP], sz[CAP];
    R sh[FORCE ? CAP : 1];
    float sp[CAP];
    uint32_t sg[CAP];
    uint16_t list[LIST][WG];
    int seg_b[kMaxSources], seg_e[kMaxSources];
    float seg_u[kMaxSources][3];
    float seg_bound_extra[kMaxSources];  // force: the source cell's largest h
    int nseg;
};

// Stage sources [k0, ...) starting at traversal position p0 of source k0.
// Returns through (k1, p1) the first source/position not staged.
template <typename R, bool FORCE>
__device__ void stage_batch(Smem<R, FORCE>& s, const Decomp& dc, const CellData<R>& cd,
                            const GhostData<R>& gd, const CellInfo& T, const BoxInfo& B, int tcell,
                            int nsrc, int k0, int p0, float Hst, float margin, int& k1, int& p1)
{
    const int lane = threadIdx.x;
    const int CAP = Smem<R, FORCE>::CAP;
    int fill = 0, nseg = 0;
    int k = k0, p = p0;
    __syncthreads();  // previous readers of the staging buffer are done
    while (k < nsrc) {
        Source src = dc.src[(int64_t)tcell * kMaxSources + k];
        const CellInfo S = dc.cells[src.cell];
        int segb = fill;
        bool complete = true;
        if (src.dir == kSelfDir) {
            int n = S.count - p;
            int take = min(n, CAP - fill);
            for (int t = lane; t < take; t += WG) {
                int g = S.start + p + t;
                s.sx[fill + t] = cd.rx[g];
                s.sy[fill + t] = cd.ry[g];
                s.sz[fill + t] = cd.rz[g];
                if constexpr (FORCE) s.sh[fill + t] = gd.hh[g];
                s.sp[fill + t] = 0.0f;
                s.sg[fill + t] = (uint32_t)g;
            }
            fill += take;
            if (take < n) { complete = false; p += take; }
            if (lane == 0) {
                s.seg_u[nseg][0] = 0.0f; s.seg_u[nseg][1] = 0.0f; s.seg_u[nseg][2] = 0.0f;
                s.seg_bound_extra[nseg] = 0.0f;
            }
        } else {
            int o[3];
            dir_off(src.dir, o);
            float u[3];
            dir_unit(src.dir, u);
            const int sd = dir_sort(src.dir);
            const bool flip = dir_flip(src.dir);
            const R dox = (R)(o[0] * B.e[0]), doy = (R)(o[1] * B.e[1]), doz = (R)(o[2] * B.e[2]);
            const float udo = u[0] * (float)(o[0] * B.e[0]) + u[1] * (float)(o[1] * B.e[1]) +
                              u[2] * (float)(o[2] * B.e[2]);
            float hs = Hst;
            if constexpr (FORCE) hs = fmaxf(Hst, gd.cell_hmax[src.cell]);
            const float reach = fmaxf(u[0], 0.f) * (float)B.e[0] + fmaxf(u[1], 0.f) * (float)B.e[1] +
                                fmaxf(u[2], 0.f) * (float)B.e[2] + hs + margin;
            const int64_t sbase = (int64_t)sd * dc.n + S.start;
            // stage the prefix of the ordering with projection <= reach
            while (p < S.count) {
                int pos = p + lane;
                bool ok = false;
                int l = 0;
                float proj = 0.0f;
                if (pos < S.count) {
                    int idx = flip ? (S.count - 1 - pos) : pos;
                    l = dc.sidx[sbase + idx];
                    float key = dc.skey[sbase + idx];
                    proj = (flip ? -key : key) + udo;
                    ok = proj <= reach;
                }
                uint64_t bal = __ballot(ok);
                int cnt = __popcll(bal);  // valid lanes form a prefix (monotone projections)
                int room = CAP - fill;
                int take = min(cnt, room);
                if (lane < take) {
                    int g = S.start + l;
                    s.sx[fill + lane] = cd.rx[g] + dox;
                    s.sy[fill + lane] = cd.ry[g] + doy;
                    s.sz[fill + lane] = cd.rz[g] + doz;
                    if constexpr (FORCE) s.sh[fill + lane] = gd.hh[g];
                    s.sp[fill + lane] = proj;
                    s.sg[fill + lane] = (uint32_t)g;
                }
                fill += take;
                p += take;
                if (take < cnt) { complete = false; break; }  // out of room
                if (cnt < WG) { p = S.count; break; }          // prefix ended
            }
            if (lane == 0) {
                s.seg_u[nseg][0] = u[0]; s.seg_u[nseg][1] = u[1]; s.seg_u[nseg][2] = u[2];
                s.seg_bound_extra[nseg] = FORCE ? gd.cell_hmax[src.cell] : 0.0f;
            }
        }
        if (lane == 0) { s.seg_b[nseg] = segb; s.seg_e[nseg] = fill; }
        nseg++;
        if (!complete) break;
        k++;
        p = 0;
        if (fill >= CAP) break;
    }
    if (lane == 0) s.nseg = nseg;
    k1 = k;
    p1 = p;
    __syncthreads();
}

// ---------------------------------------------------------------- density
template <typename R>
__global__ __launch_bounds__(WG) void k_density(Decomp dc, CellData<R> cd, GhostData<R> gd,
                                                DensityOut out, PassConsts pc)
{
    __shared__ Smem<R, false> s;
    const int lane = threadIdx.x;
    const int ncells = *dc.ncells;
    const double kNorm = 8.0 / kPi;
    while (true) {
        int unit = 0;
        if (lane == 0) unit = atomicAdd(dc.qhead, 1);
        unit = __shfl(unit, 0, 64);
        if (unit >= ncells) break;
        const CellInfo T = dc.cells[unit];
        const BoxInfo B = dc.boxes[T.box];
        const int nsrc = dc.src_count[unit];
        const double h_lim = fmin(B.e[0], fmin(B.e[1], B.e[2]));
        const float margin = 1e-5f * (float)fmax(B.e[0], fmax(B.e[1], B.e[2]));
        // staging reach: the largest h of the cell, with slack for the iteration
        double hc = 0.0;
        for (int t = lane; t < T.count; t += WG) hc = fmax(hc, cd.h[T.start + t]);
        hc = wave_max(hc);
        float Hst = (float)fmin(hc * (1.0 + pc.h_margin), h_lim);
        int staged_k1 = -1, staged_p1 = 0;  // single-batch staging cache
        bool single = false;
        float cell_hmax = 0.0f;

        for (int c0 = 0; c0 < T.count; c0 += WG) {
            const int ti = c0 + lane;
            const bool valid = ti < T.count;
            const int64_t gi = T.start + (valid ? ti : 0);
            const R xi = cd.rx[gi], yi = cd.ry[gi], zi = cd.rz[gi];
            const R mi = cd.m[gi], vxi = cd.vx[gi], vyi = cd.vy[gi], vzi = cd.vz[gi];
            double h = cd.h[gi];
            double lo = 0.0, hi = INFINITY;
            bool conv = !valid;
            int iters = 0;
            bool failed = false;
            double h_rebuild = 0.0;
            double Sw = 0, Sqdw = 0, Smw = 0, Smqdw = 0, Sdiv = 0, Scx = 0, Scy = 0, Scz = 0;
            while (true) {
                if (!conv) { Sw = Sqdw = Smw = Smqdw = Sdiv = Scx = Scy = Scz = 0.0; iters++; }
                const R hr = (R)h, hinv = (R)(1.0 / h), h2 = hr * hr;
                const float fxi = (float)xi, fyi = (float)yi, fzi = (float)zi;
                const float fh = (float)h + margin;
                int k = 0, p = 0;
                do {
                    int k1, p1;
                    if (!(single && staged_k1 >= 0)) {
                        stage_batch<R, false>(s, dc, cd, gd, T, B, unit, nsrc, k, p, Hst, margin, k1, p1);
                        if (k == 0 && p == 0) { single = (k1 >= nsrc); staged_k1 = k1; staged_p1 = p1; }
                    } else {
                        k1 = staged_k1; p1 = staged_p1;
                    }
                    // ---- sweep with early exit, compaction into per-lane lists
                    const int nseg = s.nseg;
                    bool active = !conv;
                    int seg = 0, jj = 0, je = 0;
                    float bound = 0.0f;
                    bool selfseg = false;
                    auto load_seg = [&](int q) {
                        jj = s.seg_b[q]; je = s.seg_e[q];
                        float ux = s.seg_u[q][0], uy = s.seg_u[q][1], uz = s.seg_u[q][2];
                        selfseg = (ux == 0.0f && uy == 0.0f && uz == 0.0f);
                        bound = selfseg ? INFINITY : (ux * fxi + uy * fyi + uz * fzi + fh);
                    };
                    if (active) { if (nseg > 0) load_seg(0); else active = false; }
                    while (__any(active)) {
                        int cnt = 0;
                        while (true) {
                            if (active) {
                                if (jj < je && s.sp[jj] <= bound) {
                                    R dx = xi - s.sx[jj], dy = yi - s.sy[jj], dz = zi - s.sz[jj];
                                    R r2 = dx * dx + dy * dy + dz * dz;
                                    if (r2 < h2 && s.sg[jj] != (uint32_t)gi) { s.list[cnt][lane] = (uint16_t)jj; cnt++; }
                                    jj++;
                                } else {
                                    seg++;
                                    if (seg < nseg) load_seg(seg); else active = false;
                                }
                            }
                            if (__any(cnt == Smem<R, false>::LIST) || !__any(active)) break;
                        }
                        // ---- interactions of this lane's list (Eq. (2), Eq. (3), Sec. 4.1)
                        for (int t = 0; t < cnt; t++) {
                            const int j = s.list[t][lane];
                            const uint32_t g = s.sg[j];
                            R dx = xi - s.sx[j], dy = yi - s.sy[j], dz = zi - s.sz[j];
                            R r2 = dx * dx + dy * dy + dz * dz;
                            R r = sqrt(r2);
                            R q = r * hinv;
                            R qinv = hr / r;
                            R w = kern_w(q), dw = kern_dw(q), gq = kern_g(q, qinv);
                            R mj = cd.m[g];
                            R dvx = cd.vx[g] - vxi, dvy = cd.vy[g] - vyi, dvz = cd.vz[g] - vzi;
                            R mg = mj * gq;
                            R qdw = q * dw;
                            Sw += (double)w;
                            Sqdw += (double)qdw;
                            Smw += (double)(mj * w);
                            Smqdw += (double)(mj * qdw);
                            Sdiv += (double)(mg * (dvx * dx + dvy * dy + dvz * dz));
                            Scx += (double)(mg * (dvy * dz - dvz * dy));
                            Scy += (double)(mg * (dvz * dx - dvx * dz));
                            Scz += (double)(mg * (dvx * dy - dvy * dx));
                        }
                    }
                    k = k1; p = p1;
                } while (k < nsrc);
                // ---- Newton step on h (Eq. (3)), FP64, safeguarded by a bracket
                bool need_restage = false;
                if (!conv) {
                    const double N = 32.0 / 3.0 * (Sw + 1.0);
                    const double dN = -32.0 / 3.0 / h * Sqdw;
                    const double f = N - pc.n_ngb;
                    if (fabs(f) <= pc.tol) {
                        conv = true;
                    } else if (iters >= pc.max_iter) {
                        conv = true; failed = true;
                    } else {
                        if (f < 0.0) lo = h; else hi = h;
                        double hn = h - f / dN;
                        bool ok = (dN > 0.0) && (hn > lo) && (hn < hi) && (hn >= 0.5 * h) && (hn <= 2.0 * h);
                        if (!ok) hn = isinf(hi) ? 2.0 * h : 0.5 * (lo + hi);
                        if (hn > h_lim) {
                            if (h >= h_lim) {  // root lies beyond what the cells allow
                                atomicOr(dc.status, ST_REBUILD);
                                conv = true; failed = true;
                                h_rebuild = hn;  // handed back as the next guess
                            } else {
                                hn = h_lim;
                            }
                        }
                        if (!conv) {
                            h = hn;
                            if ((float)h > Hst) need_restage = true;
                        }
                    }
                }
                if (__all(conv)) break;
                if (__any(need_restage)) {
                    double hm = wave_max(conv ? 0.0 : h);
                    Hst = (float)fmin(fmax((double)Hst, hm * (1.0 + pc.h_margin)), h_lim);
                    staged_k1 = -1;  // force a fresh staging with the larger reach
                    single = false;
                }
            }
            // ---- per-particle quantities between the stages
            if (valid) {
                const double m = (double)mi;
                const double k3 = kNorm / (h * h * h);
                const double k5 = k3 / (h * h);
                const double rho = k3 * (Smw + m);
                const double drho = -kNorm / (h * h * h * h) * (3.0 * (Smw + m) + Smqdw);
                const double omega = 1.0 + h / (3.0 * rho) * drho;
                const double N = 32.0 / 3.0 * (Sw + 1.0);
                const double div = k5 * Sdiv / rho;
                const double cx = -k5 * Scx / rho, cy = -k5 * Scy / rho, cz = -k5 * Scz / rho;
                const double u = cd.u[gi];
                const double P = (pc.gamma - 1.0) * rho * u;
                const double c = sqrt(pc.gamma * P / rho);
                const double A = P / (omega * rho * rho);
                const double cm = sqrt(cx * cx + cy * cy + cz * cz);
                const double den = fabs(div) + cm + pc.beps * c / h;
                const double bal = den > 0.0 ? cm / den : 0.0;
                cd.h[gi] = h;
                gd.hh[gi] = (R)h; gd.hinv[gi] = (R)(1.0 / h); gd.gk[gi] = (R)k5;
                gd.rho[gi] = (R)rho; gd.A[gi] = (R)A; gd.c[gi] = (R)c; gd.f[gi] = (R)bal;
                const uint32_t pi = dc.perm[gi];
                if (out.h) out.h[pi] = h_rebuild > 0.0 ? h_rebuild : h;
                if (out.rho) out.rho[pi] = rho;
                if (out.omega) out.omega[pi] = omega;
                if (out.nngb) out.nngb[pi] = N;
                if (out.div) out.div[pi] = div;
                if (out.curl) { out.curl[3 * (int64_t)pi] = cx; out.curl[3 * (int64_t)pi + 1] = cy; out.curl[3 * (int64_t)pi + 2] = cz; }
                if (out.balsara) out.balsara[pi] = bal;
                if (out.P) out.P[pi] = P;
                if (out.c) out.c[pi] = c;
                if (out.iters) out.iters[pi] = failed ? -1 : iters;
                if (failed) atomicOr(dc.status, ST_NOT_CONVERGED);
                cell_hmax = fmaxf(cell_hmax, (float)h * (1.0f + 1e-6f));
            }
        }
        cell_hmax = (float)wave_max((double)cell_hmax);
        if (lane == 0) gd.cell_hmax[unit] = cell_hmax;
        __syncthreads();
    }
}

// ---------------------------------------------------------------- force
template <typename R>
__global__ __launch_bounds__(WG) void k_force(Decomp dc, CellData<R> cd, GhostData<R> gd,
                                              ForceOut out, PassConsts pc)
{
    __shared__ Smem<R, true> s;
    const int lane = threadIdx.x;
    const int ncells = *dc.ncells;
    const R alpha = (R)pc.alpha;
    while (true) {
        int unit = 0;
        if (lane == 0) unit = atomicAdd(dc.qhead, 1);
        unit = __shfl(unit, 0, 64);
        if (unit >= ncells) break;
        const CellInfo T = dc.cells[unit];
        const BoxInfo B = dc.boxes[T.box];
        const int nsrc = dc.src_count[unit];
        const float margin = 1e-5f * (float)fmax(B.e[0], fmax(B.e[1], B.e[2]));
        const float Hst = gd.cell_hmax[unit];
        int staged_k1 = -1, staged_p1 = 0;
        bool single = false;
        for (int c0 = 0; c0 < T.count; c0 += WG) {
            const int ti = c0 + lane;
            const bool valid = ti < T.count;
            const int64_t gi = T.start + (valid ? ti : 0);
            const R xi = cd.rx[gi], yi = cd.ry[gi], zi = cd.rz[gi];
            const R vxi = cd.vx[gi], vyi = cd.vy[gi], vzi = cd.vz[gi];
            const R hi = gd.hh[gi], hinvi = gd.hinv[gi], gki = gd.gk[gi];
            const R rhoi = gd.rho[gi], Ai = gd.A[gi], ci = gd.c[gi], fi = gd.f[gi];
            const float fxi = (float)xi, fyi = (float)yi, fzi = (float)zi, fhi = (float)hi;
            double ax = 0, ay = 0, az = 0, du = 0;
            int npairs = 0;
            int k = 0, p = 0;
            do {
                int k1, p1;
                if (!(single && staged_k1 >= 0)) {
                    stage_batch<R, true>(s, dc, cd, gd, T, B, unit, nsrc, k, p, Hst, margin, k1, p1);
                    if (k == 0 && p == 0) { single = (k1 >= nsrc); staged_k1 = k1; staged_p1 = p1; }
                } else {
                    k1 = staged_k1; p1 = staged_p1;
                }
                const int nseg = s.nseg;
                bool active = valid;
                int seg = 0, jj = 0, je = 0;
                float bound = 0.0f;
                auto load_seg = [&](int q) {
                    jj = s.seg_b[q]; je = s.seg_e[q];
                    float ux = s.seg_u[q][0], uy = s.seg_u[q][1], uz = s.seg_u[q][2];
                    bool selfseg = (ux == 0.0f && uy == 0.0f && uz == 0.0f);
                    bound = selfseg ? INFINITY
                                    : (ux * fxi + uy * fyi + uz * fzi + fmaxf(fhi, s.seg_bound_extra[q]) + margin);
                };
                if (active) { if (nseg > 0) load_seg(0); else active = false; }
                while (__any(active)) {
                    int cnt = 0;
                    while (true) {
                        if (active) {
                            if (jj < je && s.sp[jj] <= bound) {
                                R dx = xi - s.sx[jj], dy = yi - s.sy[jj], dz = zi - s.sz[jj];
                                R r2 = dx * dx + dy * dy + dz * dz;
                                R hm = hi > s.sh[jj] ? hi : s.sh[jj];
                                if (r2 < hm * hm && s.sg[jj] != (uint32_t)gi) { s.list[cnt][lane] = (uint16_t)jj; cnt++; }
                                jj++;
                            } else {
                                seg++;
                                if (seg < nseg) load_seg(seg); else active = false;
                            }
                        }
                        if (__any(cnt == Smem<R, true>::LIST) || !__any(active)) break;
                    }
                    npairs += cnt;
                    // ---- Eqs. (4)-(5) and the viscosity of Sec. 4.1 for this lane's list
                    for (int t = 0; t < cnt; t++) {
                        const int j = s.list[t][lane];
                        const uint32_t g = s.sg[j];
                        R dx = xi - s.sx[j], dy = yi - s.sy[j], dz = zi - s.sz[j];
                        R r2 = dx * dx + dy * dy + dz * dz;
                        R r = sqrt(r2);
                        R rinv = r > (R)0 ? (R)1 / r : (R)0;
                        R qi = r * hinvi, qj = r * gd.hinv[g];
                        // grad W(r, h) = 8/(pi h^5) g(q) r_vec, zero outside the support
                        R gwi = qi < (R)1 ? gki * kern_g(qi, hi * rinv) : (R)0;
                        R hj = gd.hh[g];
                        R gwj = qj < (R)1 ? gd.gk[g] * kern_g(qj, hj * rinv) : (R)0;
                        if (r == (R)0) { gwi = (R)0; gwj = (R)0; }
                        R mj = cd.m[g];
                        R vxij = vxi - cd.vx[g], vyij = vyi - cd.vy[g], vzij = vzi - cd.vz[g];
                        R vr = vxij * dx + vyij * dy + vzij * dz;
                        R wij = vr * rinv;
                        wij = wij < (R)0 ? wij : (R)0;
                        R Pi = -alpha * (ci + gd.c[g] - (R)3 * wij) * wij / (rhoi + gd.rho[g]);
                        R fij = fi + gd.f[g];
                        R gsum = gwi + gwj;
                        R sc = -mj * (Ai * gwi + gd.A[g] * gwj) - (R)0.25 * mj * Pi * gsum * fij;
                        R pdu = Ai * mj * vr * gwi + (R)0.125 * mj * Pi * vr * gsum * fij;
                        ax += (double)(sc * dx);
                        ay += (double)(sc * dy);
                        az += (double)(sc * dz);
                        du += (double)pdu;
                    }
                }
                k = k1; p = p1;
            } while (k < nsrc);
            if (valid) {
                const uint32_t pi = dc.perm[gi];
                if (out.ax) out.ax[pi] = ax;
                if (out.ay) out.ay[pi] = ay;
                if (out.az) out.az[pi] = az;
                if (out.dudt) out.dudt[pi] = du;
                if (out.npairs) out.npairs[pi] = npairs;
            }
        }
        __syncthreads();
    }
}

// ---------------------------------------------------------------- launchers
__global__ void k_reset_counter(int32_t* c) { *c = 0; }

void launch_reset_counter(int32_t* c, hipStream_t st)
{
    hipLaunchKernelGGL(k_reset_counter, dim3(1), dim3(1), 0, st, c);
}

template <typename R>
void launch_density(const Decomp& dc, const CellData<R>& cd, const GhostData<R>& gd,
                    const DensityOut& out, const PassConsts& pc, int grid, hipStream_t st)
{
    launch_reset_counter(dc.qhead, st);
    hipLaunchKernelGGL(k_density<R>, dim3(grid), dim3(WG), 0, st, dc, cd, gd, out, pc);
}

template <typename R>
void launch_force(const Decomp& dc, const CellData<R>& cd, const GhostData<R>& gd,
                  const ForceOut& out, const PassConsts& pc, int grid, hipStream_t st)
{
    launch_reset_counter(dc.qhead, st);
    hipLaunchKernelGGL(k_force<R>, dim3(grid), dim3(WG), 0, st, dc, cd, gd, out, pc);
}

template void launch_density<float>(const Decomp&, const CellData<float>&, const GhostData<float>&,
                                    const DensityOut&, const PassConsts&, int, hipStream_t);
template void launch_density<double>(const Decomp&, const CellData<double>&, const GhostData<double>&,
                                     const DensityOut&, const PassConsts&, int, hipStream_t);
template void launch_force<float>(const Decomp&, const CellData<float>&, const GhostData<float>&,
                                  const ForceOut&, const PassConsts&, int, hipStream_t);
template void launch_force<double>(const Decomp&, const CellData<double>&, const GhostData<double>&,
                                   const ForceOut&, const PassConsts&, int, hipStream_t);

static int occupancy_grid(const void* fn)
{
    int dev = 0, ncu = 0, per = 0;
    hipGetDevice(&dev);
    hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev);
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, fn, WG, 0) != hipSuccess || per < 1) per = 1;
    if (ncu < 1) ncu = 1;
    return ncu * per;
}

int density_occupancy_grid(int precision)
{
    return precision == SPH_FP64 ? occupancy_grid((const void*)k_density<double>)
                                 : occupancy_grid((const void*)k_density<float>);
}

int force_occupancy_grid(int precision)
{
    return precision == SPH_FP64 ? occupancy_grid((const void*)k_force<double>)
                                 : occupancy_grid((const void*)k_force<float>);
}

}  // namespace sph
