// passes.hip -- the two interaction stages of Gonnet (2014), Sec. 2.1, on
// the cell decomposition of Sec. 3.2 with the sorted pair sweeps of
// Sec. 3.3, for gfx950.
//
// Work unit: one target cell T and up to 64 of its particles, processed by a
// workgroup of four 64-lane wavefronts.  Every wavefront holds the same 64
// targets (one per lane) and owns a quarter of the interaction sources: a
// quarter of T itself (self interaction) and a fixed share of the 26
// neighbour cells (pair interactions, periodic images included).  The
// partial sums of the four wavefronts are added in LDS.
//
// Staging.  For a neighbour S in direction d (unit vector u, from T to S) a
// wavefront reads the stored ordering of S along d (reversed for the 13
// directions that are negatives of stored ones) and copies the particles,
// shifted into T's frame, to LDS while their projection u.x stays within
// reach of T: u.x_j <= max_{x in T} u.x + H + margin.  Because a projection
// never exceeds the distance, nothing beyond that prefix can be in range.
//
// Sweep.  Each lane walks its wavefront's staged segments one after the
// other; inside a segment it stops at the first particle with
// u.x_j > u.x_i + H_i + margin (the early exit of the sorted pair
// interaction) and otherwise tests the distance.  Particles in range are
// appended to the lane's neighbour list in LDS (the compaction step); when a
// list is full, or the walk is over, every lane evaluates the interaction
// terms for its own list, so the expensive arithmetic only runs on pairs in
// range.  The target particle is written by this workgroup alone (a gather),
// so no global atomics are needed.
//
// Density (Eqs. (2)-(3)): the Newton iteration on h runs inside the unit.
// The first sweep lists the neighbours within a slightly larger radius; later
// Newton evaluations reuse the lists while h stays inside it.  Once every
// wavefront holds its whole list, the four lists of a target are evaluated
// together, their entries dealt out to the four wavefronts in turn.  A unit
// whose sources take several staging batches starts with an evaluation of
// every sum, which also serves as a Newton step.  The per-particle
// quantities of the force stage (Omega, P, c, A = P/(Omega rho^2), the
// Balsara switch of Sec. 4.1) are formed at the end.
// Force (Eqs. (4)-(5) + Sec. 4.1 viscosity): one sweep over r < max(h_i, h_j).
// A cell of more than shared_min particles is swept shared instead: each
// wavefront takes its own 64 targets and walks the sources staged by all four,
// so that a batch of sources is staged once per 256 targets rather than per 64.
// (The density stage keeps one layout: shared, its four wavefronts would run
// their Newton iterations in lockstep rounds, and on leaves of up to 256
// particles the waiting cost more than the staging it saves.)
//
// Arithmetic: pair terms in R (float or double); every per-particle sum and
// the Newton step in double.
#include "pairs.h"

#ifdef SPH_COUNT_WALK
// Counting build only: the walk tallies of the split density and force
// kernels (candidates tested, list entries), read and cleared by the host.
extern "C" int sph_walk_tally(unsigned long long out[4], int clear)
{
    if (hipMemcpyFromSymbol(out, HIP_SYMBOL(sph::g_walk_tally), 4 * sizeof(unsigned long long)) != hipSuccess)
        return 1;
    if (clear) {
        const unsigned long long z[4] = {0, 0, 0, 0};
        if (hipMemcpyToSymbol(HIP_SYMBOL(sph::g_walk_tally), z, sizeof(z)) != hipSuccess) return 1;
    }
    return 0;
}
#endif

namespace sph {
// ---------------------------------------------------------------- density
// waves per SIMD the register budget is held to: in FP32, four work-groups of
// four wavefronts per CU for configuration 0 (at most 128 VGPRs, the LDS of a
// work-group under 40 KiB), three for configuration 1 (its larger staging);
// three in FP64 (at most 168 VGPRs, under 53 KiB of LDS)
template <typename R, int CFG> constexpr int kDensWaves = sizeof(R) == 4 ? (CFG == 0 ? 4 : 3) : 3;

template <typename R, int CFG>
__global__ __launch_bounds__(WGS) __attribute__((amdgpu_waves_per_eu(kDensWaves<R, CFG>))) void k_density(Decomp dc, CellData<R> cd, Sorted<R> so, GhostData<R> gd,
                                                 DensityOut out, PassConsts pc)
{
    using R4 = typename Vec4T<R>::T;
    using SM = Smem<R, NACC_D, false, CFG>;
    __shared__ SM s;
    const int tid = threadIdx.x;
    const int w = __builtin_amdgcn_readfirstlane(tid >> 6);  // uniform: the wavefront index
    const int lane = tid & (kWave - 1);
    const int ncells = *dc.ncells;
    const double kNorm = 8.0 / kPi;
    // a decomposition flagged by the build (non-finite data, capacity, h too
    // large for the box) is not swept: its orderings need not be complete
    if (*dc.status & (ST_NONFINITE | ST_H_TOO_LARGE | ST_CAPACITY)) return;
    const int nunits = dc.nunits ? *dc.nunits : ncells;
    while (true) {
        if (tid == 0) s.unit = atomicAdd(dc.qhead, 1);
        __syncthreads();
        const int uidx = s.unit;
        __syncthreads();
        if (uidx >= nunits) break;
        const int unit = dc.units ? dc.units[uidx] : uidx;
        CellInfo T = dc.cells[unit];
        const BoxInfo B = dc.boxes[T.box];
        // the interaction lists cover h up to this, less the displacement
        // allowances of this cell and of the box since the cells were built; a
        // decomposition that has drifted by more than half of it is rebuilt
        // rather than swept: the unit is then swept as an empty cell (no early
        // exit from this loop, whose barriers every lane must reach together)
        const float dT = cell_dr(dc, unit);
        const double h_lim = (double)T.hlim - (double)dT - B.drift;
        const bool stale =
            __builtin_amdgcn_readfirstlane((double)dT + B.drift <= 0.5 * (double)T.hlim ? 0 : 1) != 0;
        if (stale) {
            if (tid == 0) atomicOr(dc.status, ST_REBUILD);
            T.count = 0;
        }
        // with multiple time-stepping, a cell without active particles stages
        // nothing and only passes its particles' stored quantities on
        bool any_on = !gd.active;
        if (gd.active)
            for (int t = lane; t < T.count; t += kWave) any_on |= gd.active[dc.perm[T.start + t]] != 0;
        const bool cell_on = __builtin_amdgcn_readfirstlane(__any(any_on) ? 1 : 0) != 0;
        const int nsrc = (stale || !cell_on) ? 0 : dc.src_count[unit];
        const double h_box = fmin(B.L[0], fmin(B.L[1], B.L[2])) / 3.0;
        // rounding margin of the sweeps; staging also covers targets that left
        // the cell by up to dT
        const float margin = 1e-5f * (float)fmax(B.e[0], fmax(B.e[1], B.e[2]));
        const float mstage = margin + dT;
        double hc = 0.0;
        for (int t = lane; t < T.count; t += kWave) hc = fmax(hc, cd.h[T.start + t]);
        hc = wave_max(hc);
        float Hst = (float)fmin(hc * (1.0 + pc.h_margin), h_lim);
        float cell_hmax = 0.0f;

        // staging of the first batch, kept while it holds every source of the wavefront
        int k = 0, p = 0;
        stage_wave<R, false>(s, w, dc, cd, so, gd, B, unit, T.level, nsrc, k, p, Hst, mstage);
        bool single = k >= nsrc;
        // every wavefront staged all of its sources at once (a uniform vote)
        auto vote_all = [&](bool mine) {
            if (lane == 0) s.done[w] = mine ? 1 : 0;
            __syncthreads();
            const bool all = (s.done[0] & s.done[1] & s.done[2] & s.done[3]) != 0;
            __syncthreads();   // read before done[] is written again
            return __builtin_amdgcn_readfirstlane(all ? 1 : 0) != 0;
        };
        bool all_single = vote_all(single);

        for (int c0 = 0; c0 < T.count; c0 += kWave) {
            const int ti = c0 + lane;
            const bool valid = ti < T.count;
            const uint32_t gi = (uint32_t)(T.start + (valid ? ti : 0));
            const uint32_t pi = dc.perm[gi];
            const bool on = valid && (!gd.active || gd.active[pi] != 0);   // a target of this pass
            const R4 ri = cd.rp[gi];
            const R xi = ri.x, yi = ri.y, zi = ri.z;
            const R4 vmi = cd.vm[gi];
            const float fxi = (float)xi, fyi = (float)yi, fzi = (float)zi;
            double h = fmin(cd.h[gi], h_lim);
            // Newton state (identical in every wavefront)
            double lo = 0.0, hi = INFINITY, h_rebuild = 0.0;
            int iters = 0;
            bool failed = false;
            bool conv = !on || pc.fixed_h;
            if (pc.fixed_h && on && cd.h[gi] > h_lim) {
                // a given h beyond what the cells allow: rebuilt for it, then swept again
                if (w == 0) atomicOr(dc.status, ST_REBUILD);
                h_rebuild = cd.h[gi];
            }
            // neighbour lists of this wavefront: valid while every lane's h <= hcache
            bool cached = false;
            // block-uniform: the lists of all four wavefronts are whole (evaluated
            // together), or some wavefront's list filled during the last walk
            // (each wavefront then keeps to its own lists, without votes)
            bool lists_all = false, own_mode = false;
            bool cached_all = false;  // the lists were built with every valid lane active
            float hcache = 0.0f;
            int cnt = 0;
            DensAcc acc;

            // Sums at the current h, for the lanes in `act`: the two of Eq. (3)
            // (full = false) or all of them (full = true).  Lists in hand are
            // evaluated by their own wavefront (a list that fills, or a batch of
            // sources staged in several), or, once every wavefront holds its whole
            // list, all four lists of a target together: wavefront w takes entries
            // w, w + 4, ... of their concatenation, so that the list loops of the
            // four run about equally long whatever the split of the neighbours
            // between the regions.
            auto evaluate = [&](bool act, bool full) {
                acc = DensAcc{};
                const R hr = (R)h, hinv = (R)(1.0 / h), h2 = hr * hr;
                // region and staged index of list entry k: of this wavefront's own
                // list, or (ALL) of the concatenation of the four
                auto process = [&](int n, auto all_tag) {
                    constexpr bool ALL = decltype(all_tag)::value;
                    int C1 = 0, C2 = 0, C3 = 0, tot = n;
                    if constexpr (ALL) {
                        C1 = s.lcount[0][lane];
                        C2 = C1 + s.lcount[1][lane];
                        C3 = C2 + s.lcount[2][lane];
                        tot = C3 + s.lcount[3][lane];
                    }
                    constexpr int t0s = ALL ? 1 : 0;   // start at w (ALL) or 0
                    constexpr int dt = ALL ? NW : 1;
                    auto entry = [&](int kk, int& r, int& j) {
                        if constexpr (ALL) {
                            // selects rather than a chain of branches on r
                            const bool b1 = kk >= C1, b2 = kk >= C2, b3 = kk >= C3;
                            int off = b1 ? C1 : 0;
                            off = b2 ? C2 : off;
                            off = b3 ? C3 : off;
                            r = (int)b1 + (int)b2 + (int)b3;
                            j = s.list[r][lane][kk - off];
                        } else {
                            r = w;
                            j = s.list[w][lane][kk];
                        }
                    };
                    if (full) {
                        DensPart<R> b = {};
                        for (int t = t0s * w;; t += 2 * dt) {
                            converge();
                            const bool v0 = act && t < tot, v1 = act && t + dt < tot;
                            if (!__any(v0)) break;
                            int r0, j0, r1, j1;
                            entry(v0 ? t : 0, r0, j0);
                            entry(v1 ? t + dt : 0, r1, j1);
                            j0 = v0 ? j0 : 0;
                            j1 = v1 ? j1 : 0;
                            const R4 e0 = s.st[r0][j0], e1 = s.st[r1][j1];
                            const R4 q0 = cd.vm[s.sg[r0][j0]], q1 = cd.vm[s.sg[r1][j1]];
                            density_pair<R>(b, v0, xi, yi, zi, vmi.x, vmi.y, vmi.z, hr, hinv, h2, e0, q0);
                            density_pair<R>(b, v1, xi, yi, zi, vmi.x, vmi.y, vmi.z, hr, hinv, h2, e1, q1);
                        }
                        acc.w += (double)b.w;
                        acc.qdw += (double)b.qdw;
                        acc.n += b.n;
                        // into the FP64 totals of the four wavefronts (cleared before
                        // the evaluation); nothing of them stays in registers
                        if (act) {
                            atomicAdd(&s.red[2][lane], (double)b.mw);
                            atomicAdd(&s.red[3][lane], (double)b.mqdw);
                            atomicAdd(&s.red[4][lane], (double)b.div);
                            atomicAdd(&s.red[5][lane], (double)b.cx);
                            atomicAdd(&s.red[6][lane], (double)b.cy);
                            atomicAdd(&s.red[7][lane], (double)b.cz);
                        }
                    } else {
                        // partial sums of these terms (at most LISTW of the lane's
                        // own list; about a quarter of four lists), then FP64
                        R sw = (R)0, sq = (R)0;
                        for (int t = t0s * w;; t += 2 * dt) {
                            converge();
                            const bool v0 = act && t < tot, v1 = act && t + dt < tot;
                            if (lanes(v0) == 0) break;
                            int r0, j0, r1, j1;
                            entry(v0 ? t : 0, r0, j0);
                            entry(v1 ? t + dt : 0, r1, j1);
                            const R4 e0 = s.st[r0][v0 ? j0 : 0], e1 = s.st[r1][v1 ? j1 : 0];
                            count_pair<R>(sw, sq, v0, xi, yi, zi, hinv, h2, e0);
                            count_pair<R>(sw, sq, v1, xi, yi, zi, hinv, h2, e1);
                        }
                        acc.w += (double)sw;
                        acc.qdw += (double)sq;
                    }
                };
                using Own = std::false_type;
                using All = std::true_type;
                const bool fit = (!full || cached_all) && __all(!act || (float)h <= hcache);
                if (lists_all && fit) {
                    process(0, All{});
                    return;
                }
                if (!lists_all && cached && fit) {
                    process(cnt, Own{});
                    return;
                }
                // sweep(s) with early exit; the lists keep r < h (1 + slack)
                hcache = fminf((float)h * (1.0f + kCacheSlack), Hst);
                const R rad = (R)hcache;
                const float fh = hcache + margin;
                bool flushed = false;
                lists_all = false;
                if (all_single && !own_mode) {
                    // every source is staged: walk, keeping the lists (one that fills
                    // is evaluated at once by its owner), then all four together
                    const int selfj = self_index(s, w, ti);
                    int seg = 0, jj = s.nseg[w] > 0 ? s.seg_b[w][0] : 0;
                    cnt = 0;
                    while (true) {
                        converge();
                        cnt = walk<R, false, NACC_D, CFG>(s, w, w, lane, act, xi, yi, zi, fxi, fyi, fzi, rad, fh,
                                                          margin, selfj, seg, jj, cnt);
                        if (seg >= s.nseg[w]) break;
                        process(cnt, Own{});
                        cnt = 0;
                        flushed = true;
                    }
                    s.lcount[w][lane] = (uint8_t)cnt;
                    // the vote's barriers also publish the lists and their counts
                    lists_all = vote_all(!flushed);
                    own_mode = !lists_all;
                    process(0, All{});
                    cached = !flushed;   // a wavefront's own list stays whole while it did not fill
                } else {
                    int kk = 0, pp = 0;
                    do {
                        if (!single)
                            stage_wave<R, false>(s, w, dc, cd, so, gd, B, unit, T.level, nsrc, kk, pp, Hst, mstage);
                        else kk = nsrc;
                        const int selfj = self_index(s, w, ti);
                        int seg = 0, jj = s.nseg[w] > 0 ? s.seg_b[w][0] : 0;
                        cnt = 0;
                        while (true) {
                            converge();
                            cnt = walk<R, false, NACC_D, CFG>(s, w, w, lane, act, xi, yi, zi, fxi, fyi, fzi, rad,
                                                              fh, margin, selfj, seg, jj, cnt);
                            if (seg >= s.nseg[w]) break;
                            process(cnt, Own{});  // a list is full: evaluate it and continue the walk
                            cnt = 0;
                            flushed = true;
                        }
                        if (!single) {
                            process(cnt, Own{});
                            cnt = 0;
                            flushed = true;
                        }
                    } while (kk < nsrc);
                    if (single) process(cnt, Own{});
                    cached = single && !flushed;
                }
                cached_all = __all(act || !on);
            };

            // ---- Newton iteration on h (Eq. (3)) in FP64, safeguarded by a bracket.
            // The iteration runs on g(h) = N(h)^(1/3) - n_ngb^(1/3), which is close
            // to linear in h (N grows like h^3), so it needs fewer steps than
            // Newton on N itself; the root is the same.  The two sums of each
            // evaluation are added across the wavefronts into one of three LDS
            // buffers, so one barrier per step suffices: every wavefront then
            // takes the same step for its 64 targets.
            const double cbrt_ngb = cbrt(pc.n_ngb);
            // A step so small that the next residual is predicted far below the
            // tolerance: the next evaluation takes every sum, and the iteration
            // ends there if it confirms convergence.  Once every lane has
            // converged, one evaluation with every sum ends it too.  An
            // evaluation with every sum also holds the two of Eq. (3), so the
            // lanes it does not confirm take their Newton step from it.
            const double step_final = sqrt(pc.tol / (10.0 * pc.n_ngb));
            // A given h goes straight to the full sums.  So does a unit whose
            // sources take several staging batches: each evaluation stages and
            // walks them all again, which costs far more than the extra sums,
            // and an h that is already converged is then confirmed by the first
            // evaluation rather than the second.
            bool full = pc.fixed_h != 0 || !all_single;
            int cit = 0;  // count steps since the buffers were last cleared
            // one Newton step of a lane not yet converged, from the sums w and
            // q dw/dq of Eq. (3) at the current h
            auto newton = [&](double ws, double qs, bool& restage, bool& close) {
                iters++;
                const double N = 32.0 / 3.0 * (ws + 1.0);
                const double dN = -32.0 / 3.0 / h * qs;
                const double f = N - pc.n_ngb;
                if (fabs(f) <= pc.tol) {
                    conv = true;
                } else if (iters >= pc.max_iter) {
                    conv = true; failed = true;
                } else {
                    if (f < 0.0) lo = h; else hi = h;
                    // Newton on g: h - g / g', g' = N' / (3 N^(2/3))
                    const double c = cbrt(N);
                    double hn = h - 3.0 * c * c * (c - cbrt_ngb) / dN;
                    const bool ok = (dN > 0.0) && (hn > lo) && (hn < hi) && (hn >= 0.5 * h) && (hn <= 2.0 * h);
                    if (!ok) hn = isinf(hi) ? 2.0 * h : 0.5 * (lo + hi);
                    if (hn > h_lim) {
                        if (h >= h_lim) {  // the root lies beyond what the cells allow
                            if (w == 0) atomicOr(dc.status, ST_REBUILD);
                            conv = true; failed = true;
                            // the next build takes it from here, within what a
                            // periodic box allows (three cells of edge >= h)
                            h_rebuild = fmin(hn, h_box);
                        } else {
                            hn = h_lim;
                        }
                    }
                    if (!conv) {
                        close = fabs(hn - h) <= step_final * h;
                        h = hn;
                        restage = (float)h > Hst;
                    }
                }
            };
            // staging again for an h beyond the staged reach (a block-uniform
            // vote: the four wavefronts hold the same lanes' states)
            auto restage_if = [&](bool restage) {
                if (!__any(restage)) return;
                const double hm = wave_max(conv ? 0.0 : h);
                Hst = (float)fmin(fmax((double)Hst, hm * (1.0 + pc.h_margin)), h_lim);
                k = 0; p = 0;
                stage_wave<R, false>(s, w, dc, cd, so, gd, B, unit, T.level, nsrc, k, p, Hst, mstage);
                single = k >= nsrc;
                all_single = vote_all(single);
                cached = false;
                lists_all = false;
                own_mode = false;
            };
            for (int a = w; a < 2; a += NW) s.red[a][lane] = 0.0;
            __syncthreads();
            while (true) {
                if (full) {
                    // ---- every sum at the current h, into s.red[0..8]
                    __syncthreads();  // every wavefront has read the last step's sums
                    for (int a = w; a < NACC_D; a += NW) s.red[a][lane] = 0.0;
                    __syncthreads();
                    evaluate(on, true);
                    if (on) {
                        atomicAdd(&s.red[0][lane], acc.w);
                        atomicAdd(&s.red[1][lane], acc.qdw);
                        atomicAdd(&s.red[8][lane], (double)acc.n);
                    }
                    __syncthreads();
                    bool restage = false;
                    bool close = true;
                    if (!conv) newton(s.red[0][lane], s.red[1][lane], restage, close);
                    if (__all(conv)) break;
                    // not yet: on from the step just taken, with cleared buffers
                    cit = 0;
                    __syncthreads();
                    for (int a = w; a < 2; a += NW) s.red[a][lane] = 0.0;
                    __syncthreads();
                    restage_if(restage);
                    full = __all(close);
                    continue;
                }
                const int rb = 2 * (cit % 3);        // this step's buffer
                const int zb = 2 * ((cit + 1) % 3);  // the next step's buffer: last read two steps ago
                cit++;
                if (w < 2) s.red[zb + w][lane] = 0.0;
                evaluate(!conv, false);
                if (!conv) {
                    atomicAdd(&s.red[rb][lane], acc.w);
                    atomicAdd(&s.red[rb + 1][lane], acc.qdw);
                }
                __syncthreads();
                bool restage = false;
                bool close = true;
                if (!conv) newton(s.red[rb][lane], s.red[rb + 1][lane], restage, close);
                restage_if(restage);
                full = __all(close);  // every lane converged, or its next residual is negligible
            }

            // ---- per-particle quantities between the stages (wavefront 0)
            if (w == 0 && valid && !on) {
                // not a target this time: its quantities of the last active step
                const double hh = cd.h[gi];
                const double k5 = kNorm / (hh * hh * hh * hh * hh);
                R4 g0, g1;
                g0.x = (R)(1.0 / hh); g0.y = (R)k5; g0.z = (R)gd.s_A[pi]; g0.w = (R)gd.s_rho[pi];
                g1.x = (R)gd.s_c[pi]; g1.y = (R)gd.s_f[pi]; g1.z = (R)hh; g1.w = (R)0;
                gd.g0[gi] = g0;
                gd.g1[gi] = g1;
                cell_hmax = fmaxf(cell_hmax, (float)hh * (1.0f + 1e-6f));
            }
            if (w == 0 && on) {
                struct { double w, qdw, mw, mqdw, div, cx, cy, cz, n; } tot;
                tot.w = s.red[0][lane]; tot.qdw = s.red[1][lane]; tot.mw = s.red[2][lane];
                tot.mqdw = s.red[3][lane]; tot.div = s.red[4][lane]; tot.cx = s.red[5][lane];
                tot.cy = s.red[6][lane]; tot.cz = s.red[7][lane]; tot.n = s.red[8][lane];
                const double m = (double)vmi.w;
                const double k3 = kNorm / (h * h * h);
                const double k5 = k3 / (h * h);
                const double rho = k3 * (tot.mw + m);
                const double drho = -kNorm / (h * h * h * h) * (3.0 * (tot.mw + m) + tot.mqdw);
                const double omega = 1.0 + h / (3.0 * rho) * drho;
                const double N = 32.0 / 3.0 * (tot.w + 1.0);
                const double div = k5 * tot.div / rho;
                const double cx = -k5 * tot.cx / rho, cy = -k5 * tot.cy / rho, cz = -k5 * tot.cz / rho;
                const double u = cd.u[gi];
                const double P = (pc.gamma - 1.0) * rho * u;
                const double c = sqrt(pc.gamma * P / rho);
                const double A = P / (omega * rho * rho);
                const double cm = sqrt(cx * cx + cy * cy + cz * cz);
                const double den = fabs(div) + cm + pc.beps * c / h;
                const double bal = den > 0.0 ? (pc.balsara_div ? fabs(div) : cm) / den : 0.0;
                cd.h[gi] = h;
                R4 g0, g1;
                g0.x = (R)(1.0 / h); g0.y = (R)k5; g0.z = (R)A; g0.w = (R)rho;
                g1.x = (R)c; g1.y = (R)bal; g1.z = (R)h; g1.w = (R)0;
                gd.g0[gi] = g0;
                gd.g1[gi] = g1;
                if (gd.sd0) {
                    gd.sd0[gi] = make_double4(tot.mw + m, tot.mqdw, -32.0 / 3.0 / h * tot.qdw, tot.div);
                    gd.sd1[gi] = make_double4(tot.cx, tot.cy, tot.cz, 0.0);
                }
                if (gd.s_rho) { gd.s_rho[pi] = rho; gd.s_A[pi] = A; gd.s_c[pi] = c; gd.s_f[pi] = bal; }
                if (out.h) out.h[pi] = h_rebuild > 0.0 ? h_rebuild : h;
                if (out.rho) out.rho[pi] = rho;
                if (out.omega) out.omega[pi] = omega;
                if (out.nngb) out.nngb[pi] = N;
                if (out.div) out.div[pi] = div;
                if (out.curl) {
                    out.curl[3 * (int64_t)pi] = cx; out.curl[3 * (int64_t)pi + 1] = cy; out.curl[3 * (int64_t)pi + 2] = cz;
                }
                if (out.balsara) out.balsara[pi] = bal;
                if (out.P) out.P[pi] = P;
                if (out.c) out.c[pi] = c;
                if (out.iters) out.iters[pi] = failed ? -1 : iters;
                if (out.ndens) out.ndens[pi] = (int32_t)tot.n;
                if (failed) atomicOr(dc.status, ST_NOT_CONVERGED);
                cell_hmax = fmaxf(cell_hmax, (float)h * (1.0f + 1e-6f));
            }
            __syncthreads();
        }
        if (w == 0) {
            cell_hmax = (float)wave_max((double)cell_hmax);
            if (lane == 0) gd.cell_hmax[unit] = cell_hmax;
        }
        __syncthreads();
    }
}

// ---------------------------------------------------------------- force
// FP64: three work-groups per CU (at most 168 VGPRs); FP32 needs no bound to fit four
template <typename R>
__global__ __launch_bounds__(WGS) __attribute__((amdgpu_waves_per_eu(sizeof(R) == 4 ? 1 : 3))) void k_force(Decomp dc, CellData<R> cd, Sorted<R> so, GhostData<R> gd,
                                               ForceOut out, PassConsts pc)
{
    using R4 = typename Vec4T<R>::T;
    using SM = Smem<R, NACC_F, true>;
    __shared__ SM s;
    const int tid = threadIdx.x;
    const int w = __builtin_amdgcn_readfirstlane(tid >> 6);  // uniform: the wavefront index
    const int lane = tid & (kWave - 1);
    const int ncells = *dc.ncells;
    const R alpha = (R)pc.alpha;
    if (*dc.status & (ST_NONFINITE | ST_H_TOO_LARGE | ST_CAPACITY)) return;
    const int nunits = dc.nunits ? *dc.nunits : ncells;
    while (true) {
        if (tid == 0) s.unit = atomicAdd(dc.qhead, 1);
        __syncthreads();
        const int uidx = s.unit;
        __syncthreads();
        if (uidx >= nunits) break;
        const int unit = dc.units ? dc.units[uidx] : uidx;
        const CellInfo T = dc.cells[unit];
        const BoxInfo B = dc.boxes[T.box];
        int nsrc = dc.src_count[unit];
        const float margin = 1e-5f * (float)fmax(B.e[0], fmax(B.e[1], B.e[2]));
        const float mstage = margin + cell_dr(dc, unit);   // targets may have left the cell by this
        const float Hst = gd.cell_hmax[unit];
        bool any_on = !gd.active;
        if (gd.active)
            for (int t = lane; t < T.count; t += kWave) any_on |= gd.active[dc.perm[T.start + t]] != 0;
        const bool cell_on = __builtin_amdgcn_readfirstlane(__any(any_on) ? 1 : 0) != 0;
        if (!cell_on) nsrc = 0;   // no target here: nothing to stage or sweep
        int k = 0, p = 0;
        stage_wave<R, true>(s, w, dc, cd, so, gd, B, unit, T.level, nsrc, k, p, Hst, mstage);
        const bool single = k >= nsrc;
        // Cells of more than shared_min particles are swept shared: each
        // wavefront takes its own 64 targets and walks the staged sources of all
        // four, so that a batch of sources is staged once for up to 256 targets
        // rather than once per 64.  Otherwise the four wavefronts hold the same
        // 64 targets, each walking its own sources, and add their sums in LDS.
        const bool shared = T.count > pc.shared_min;
        bool all_single = single;
        if (shared) {
            if (lane == 0) s.done[w] = single ? 1 : 0;
            __syncthreads();
            all_single = (s.done[0] & s.done[1] & s.done[2] & s.done[3]) != 0;
            __syncthreads();   // read before the sweeps write done[] again
        }
        const int gstep = shared ? NW * kWave : kWave;
        for (int c0 = 0; c0 < T.count; c0 += gstep) {
            const int ti_ = c0 + (shared ? w * kWave : 0) + lane;
            const bool valid = ti_ < T.count;
            const uint32_t gi = (uint32_t)(T.start + (valid ? ti_ : 0));
            const bool on = valid && (!gd.active || gd.active[dc.perm[gi]] != 0);   // a target of this pass
            ForceTarget<R> ti;
            const R4 ri = cd.rp[gi];
            ti.x = ri.x; ti.y = ri.y; ti.z = ri.z;
            const R4 vmi = cd.vm[gi], g0i = gd.g0[gi], g1i = gd.g1[gi];
            ti.vx = vmi.x; ti.vy = vmi.y; ti.vz = vmi.z;
            ti.hinv = g0i.x; ti.gk = g0i.y; ti.A = g0i.z; ti.rho = g0i.w;
            ti.c = g1i.x; ti.f = g1i.y; ti.h = g1i.z;
            const float fxi = (float)ti.x, fyi = (float)ti.y, fzi = (float)ti.z, fh = (float)ti.h;
            if (!shared)
                for (int a = w; a < NACC_F; a += NW) s.red[a][lane] = 0.0;
            __syncthreads();
            ForceAcc<R> acc = {};
            // the pairs of a list of staged indices of region r
            auto process = [&](int n, int r) {
                ForcePart<R> b = {};
                for (int t = 0;; t += 2) {
                    const bool v0 = t < n, v1 = t + 1 < n;
                    if (lanes(v0) == 0) break;
                    // slots t, t + 1 <= LISTW lie in the row; past the list: masked
                    const int r0 = s.list[w][lane][t], r1 = s.list[w][lane][t + 1];
                    const int j0 = v0 ? r0 : 0, j1 = v1 ? r1 : 0;
                    const uint32_t q0 = s.sg[r][j0], q1 = s.sg[r][j1];
                    const R4 e0 = s.st[r][j0], e1 = s.st[r][j1];
                    const R4 v0m = cd.vm[q0], v1m = cd.vm[q1];
                    const R4 a0 = gd.g0[q0], a1 = gd.g0[q1];
                    const R4 b0 = gd.g1[q0], b1 = gd.g1[q1];
                    force_pair<R>(acc, b, v0, ti, alpha, e0, v0m, a0, b0);
                    force_pair<R>(acc, b, v1, ti, alpha, e1, v1m, a1, b1);
                }
                acc.ax += (double)b.ax;
                acc.ay += (double)b.ay;
                acc.az += (double)b.az;
                acc.du += (double)b.du;
            };
            // walk of region r, its lists evaluated as they fill and at the end
            auto sweep = [&](int r) {
                const int selfj = self_index(s, r, ti_);
                int seg = 0, jj = s.nseg[r] > 0 ? s.seg_b[r][0] : 0;
                int cnt = 0;
                while (true) {
                    cnt = walk<R, true, NACC_F>(s, w, r, lane, on, ti.x, ti.y, ti.z, fxi, fyi, fzi, ti.h, fh, margin,
                                                selfj, seg, jj, cnt);
                    process(cnt, r);
                    cnt = 0;
                    if (seg >= s.nseg[r]) break;
                }
            };
            int kk = 0, pp = 0;
            if (shared) {
                // batch rounds: every wavefront stages its next batch, then all
                // walk the four regions; the rounds end together
                while (true) {
                    if (!all_single) {
                        stage_wave<R, true>(s, w, dc, cd, so, gd, B, unit, T.level, nsrc, kk, pp, Hst, mstage);
                        if (lane == 0) s.done[w] = kk >= nsrc ? 1 : 0;
                    }
                    __syncthreads();   // the four regions are staged
                    const bool last = all_single || (s.done[0] & s.done[1] & s.done[2] & s.done[3]) != 0;
                    for (int r = 0; r < NW; r++) sweep(r);
                    __syncthreads();   // every wavefront is done with the regions and with done[]
                    if (last) break;
                }
            } else {
                do {
                    if (!single) stage_wave<R, true>(s, w, dc, cd, so, gd, B, unit, T.level, nsrc, kk, pp, Hst, mstage);
                    else kk = nsrc;
                    sweep(w);
                } while (kk < nsrc);
                if (on) {
                    atomicAdd(&s.red[0][lane], acc.ax);
                    atomicAdd(&s.red[1][lane], acc.ay);
                    atomicAdd(&s.red[2][lane], acc.az);
                    atomicAdd(&s.red[3][lane], acc.du);
                    atomicAdd(&s.red[4][lane], (double)acc.n);
                    // signal speeds are >= 0, where the order of the bit patterns is the order of the values
                    atomicMax((unsigned long long*)&s.red[5][lane],
                              (unsigned long long)__double_as_longlong((double)acc.vsig));
                }
            }
            __syncthreads();
            if ((shared || w == 0) && on) {
                const uint32_t pi = dc.perm[gi];
                const double ax = shared ? acc.ax : s.red[0][lane], ay = shared ? acc.ay : s.red[1][lane];
                const double az = shared ? acc.az : s.red[2][lane], du = shared ? acc.du : s.red[3][lane];
                const double np_ = shared ? (double)acc.n : s.red[4][lane];
                const double vsg = shared ? (double)acc.vsig : s.red[5][lane];
                if (out.ax) out.ax[pi] = ax;
                if (out.ay) out.ay[pi] = ay;
                if (out.az) out.az[pi] = az;
                if (out.dudt) out.dudt[pi] = du;
                if (out.npairs) out.npairs[pi] = (int32_t)np_;
                if (out.dt) {
                    // j = i contributes 2 c_i (no approach speed)
                    const double vs = fmax(vsg, 2.0 * (double)ti.c);
                    out.dt[pi] = vs > 0.0 ? pc.cfl * 2.0 * (double)ti.h / vs : (double)INFINITY;
                }
            }
            __syncthreads();
        }
    }
}

// ---------------------------------------------------------------- multiple time-stepping
// Before the density stage of a base step: the force-stage records of the
// inactive particles from their last active step, and per cell whether it
// holds an active particle (flag) and its largest h (the sweeps of active
// cells read those of their sources).  Particle-parallel in cell order: the
// lanes of one cell are consecutive, so a segmented wavefront reduction
// leaves each cell's values in its last lane, which issues the atomics.
template <typename R>
__global__ void k_ghost_stash(const uint32_t* perm, const uint32_t* cell_of, CellData<R> cd, GhostData<R> gd,
                              uint32_t* cell_flag, int64_t n)
{
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k - (int64_t)(threadIdx.x & 63) >= n) return;   // the whole wavefront is past the end
    const bool valid = k < n;
    int c = -1;
    float hm = 0.0f;
    uint32_t on = 0;
    if (valid) {
        const uint32_t pi = perm[k];
        c = (int)cell_of[k];
        const double h = cd.h[k];
        hm = (float)h * (1.0f + 1e-6f);
        on = gd.active[pi] ? 1u : 0u;
        if (!on) {
            const double kNorm = 8.0 / kPi;
            typename Vec4T<R>::T g0, g1;
            g0.x = (R)(1.0 / h); g0.y = (R)(kNorm / (h * h * h * h * h)); g0.z = (R)gd.s_A[pi];
            g0.w = (R)gd.s_rho[pi];
            g1.x = (R)gd.s_c[pi]; g1.y = (R)gd.s_f[pi]; g1.z = (R)h; g1.w = (R)0;
            gd.g0[k] = g0;
            gd.g1[k] = g1;
        }
    }
    const int lane = threadIdx.x & 63;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const float ho = __shfl_up(hm, o, 64);
        const uint32_t oo = __shfl_up(on, o, 64);
        const int co = __shfl_up(c, o, 64);
        if (lane >= o && co == c) { hm = fmaxf(hm, ho); on |= oo; }
    }
    const int cn = __shfl_down(c, 1, 64);
    if (valid && (lane == 63 || cn != c)) {
        atomicMax((unsigned int*)&gd.cell_hmax[c], __float_as_uint(hm));
        if (on) atomicOr(&cell_flag[c], 1u);
    }
}

// The flagged cells appended to the unit list (order is irrelevant: each
// unit's result does not depend on the others); flags and maxima cleared for
// the next base step are done by the caller's fills.
__global__ void k_mts_units(const int32_t* ncells, const uint32_t* cell_flag, int32_t* units, int32_t* nunits)
{
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    const bool f = c < *ncells && cell_flag[c] != 0;
    const unsigned long long b = __ballot(f);
    if (!b) return;
    const int lane = threadIdx.x & 63;
    int base = 0;
    if (lane == __ffsll((long long)b) - 1) base = atomicAdd(nunits, __popcll(b));
    base = __shfl(base, __ffsll((long long)b) - 1, 64);
    if (f) units[base + __popcll(b & ((1ull << lane) - 1))] = c;
}

__global__ void k_clear_cells(const int32_t* ncells, float* cell_hmax, uint32_t* cell_flag)
{
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c < *ncells) { cell_hmax[c] = 0.0f; cell_flag[c] = 0u; }
}

__global__ void k_zero_i32(int32_t* a) { *a = 0; }

template <typename R>
void launch_mts_prepare(const Decomp& dc, const CellData<R>& cd, const GhostData<R>& gd, int32_t* units,
                        int32_t* nunits, uint32_t* cell_flag, const uint32_t* cell_of, int64_t n, hipStream_t st)
{
    hipLaunchKernelGGL(k_zero_i32, dim3(1), dim3(1), 0, st, nunits);
    if (n <= 0) return;
    // cells number at most n
    const unsigned g = (unsigned)((n + 255) / 256);
    hipLaunchKernelGGL(k_clear_cells, dim3(g), dim3(256), 0, st, dc.ncells, gd.cell_hmax, cell_flag);
    hipLaunchKernelGGL(k_ghost_stash<R>, dim3(g), dim3(256), 0, st, dc.perm, cell_of, cd, gd, cell_flag, n);
    hipLaunchKernelGGL(k_mts_units, dim3(g), dim3(256), 0, st, dc.ncells, (const uint32_t*)cell_flag, units, nunits);
}
template void launch_mts_prepare<float>(const Decomp&, const CellData<float>&, const GhostData<float>&, int32_t*,
                                        int32_t*, uint32_t*, const uint32_t*, int64_t, hipStream_t);
template void launch_mts_prepare<double>(const Decomp&, const CellData<double>&, const GhostData<double>&, int32_t*,
                                         int32_t*, uint32_t*, const uint32_t*, int64_t, hipStream_t);

// ---------------------------------------------------------------- launchers
__global__ void k_reset_counter(int32_t* c) { *c = 0; }

void launch_reset_counter(int32_t* c, hipStream_t st)
{
    hipLaunchKernelGGL(k_reset_counter, dim3(1), dim3(1), 0, st, c);
}

static int occupancy_grid(const void* fn)
{
    int dev = 0, ncu = 0, per = 0;
    (void)hipGetDevice(&dev);
    (void)hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev);
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, fn, WGS, 0) != hipSuccess || per < 1) per = 1;
    if (ncu < 1) ncu = 1;
    return ncu * per;
}

template <typename R>
void launch_density(const Decomp& dc, const CellData<R>& cd, const Sorted<R>& so, const GhostData<R>& gd,
                    const DensityOut& out, const PassConsts& pc, int staging, hipStream_t st)
{
    launch_reset_counter(dc.qhead, st);
    bool wide = false;
    if constexpr (sizeof(R) == 4) {
        // FP64 has one staging form
        wide = staging == SPH_STAGING_WIDE;
        if (wide)
            hipLaunchKernelGGL((k_density<R, 1>), dim3(occupancy_grid((const void*)k_density<R, 1>)), dim3(WGS), 0,
                               st, dc, cd, so, gd, out, pc);
    }
    if (!wide) {
        hipLaunchKernelGGL((k_density<R, 0>), dim3(occupancy_grid((const void*)k_density<R, 0>)), dim3(WGS), 0, st,
                           dc, cd, so, gd, out, pc);
    }
}

template <typename R>
void launch_force(const Decomp& dc, const CellData<R>& cd, const Sorted<R>& so, const GhostData<R>& gd,
                  const ForceOut& out, const PassConsts& pc, int grid, hipStream_t st)
{
    launch_reset_counter(dc.qhead, st);
    hipLaunchKernelGGL(k_force<R>, dim3(grid), dim3(WGS), 0, st, dc, cd, so, gd, out, pc);
}

template void launch_density<float>(const Decomp&, const CellData<float>&, const Sorted<float>&,
                                    const GhostData<float>&, const DensityOut&, const PassConsts&, int, hipStream_t);
template void launch_density<double>(const Decomp&, const CellData<double>&, const Sorted<double>&,
                                     const GhostData<double>&, const DensityOut&, const PassConsts&, int, hipStream_t);
template void launch_force<float>(const Decomp&, const CellData<float>&, const Sorted<float>&,
                                  const GhostData<float>&, const ForceOut&, const PassConsts&, int, hipStream_t);
template void launch_force<double>(const Decomp&, const CellData<double>&, const Sorted<double>&,
                                   const GhostData<double>&, const ForceOut&, const PassConsts&, int, hipStream_t);


int force_occupancy_grid(int precision)
{
    return precision == SPH_FP64 ? occupancy_grid((const void*)k_force<double>)
                                 : occupancy_grid((const void*)k_force<float>);
}

}  // namespace sph
