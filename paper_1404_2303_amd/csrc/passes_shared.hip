// passes_shared.hip -- the two interaction stages of Gonnet (2014), Sec. 2.1,
// with the sources of a target cell staged once for a whole work-group and
// four lanes per target, for gfx950.
//
// Work unit: one target cell T, processed by a work-group of four 64-lane
// wavefronts.  Each wavefront stages its share of T's interaction sources
// (a quarter of T itself, the self interaction, and a fixed share of the 26
// neighbour cells, the pair interactions of Sec. 3.3) as in the split layout
// of passes.hip; every wavefront then reads all four staging areas.  The
// targets are taken 64 at a time, 16 per wavefront, each served by a quad of
// four adjacent lanes:
//  - walk: lane b of a quad tests entries b and b + 4 of each step of eight
//    staged entries against its target; the hits of a step are appended to
//    the target's one neighbour list at offsets counted over the quad;
//  - early exit of the sorted sweep: per wavefront, from the largest bound of
//    its 16 targets.  They are consecutive in cell order (Morton order, a
//    compact block of about a quarter of the cell), so a wavefront leaves a
//    segment well before the bound of the whole cell;
//  - sums: lane b of a quad evaluates entries b, b + 4, ... of the list and
//    the quad adds its four partial sums with two data-parallel-primitive
//    moves, after which the four lanes hold bitwise equal totals and take
//    the same Newton steps.
// A list holds every neighbour of its target, and in SPH every particle has
// about n_ngb neighbours, so the lists of a wavefront have about the same
// length; each wavefront runs its Newton iteration on its own, and the
// work-group only votes (two barriers) when some h outgrows the staged reach.
//
// A cell whose sources do not fit into the four staging areas at once is not
// swept here: it is appended to a list of deferred cells, which the split
// layout's kernel sweeps right afterwards (staging in several batches).
//
// Density (Eqs. (2)-(3) with the divergence and curl of Sec. 4.1): lists over
// r < h (1 + slack), kept across Newton evaluations while h stays inside.
// Force (Eqs. (4)-(5) with the viscosity of Sec. 4.1): lists over
// r < max(h_i, h_j), evaluated whenever one fills and at the end.
// Arithmetic: pair terms in R (float or double); per-lane partial sums over
// one pass of a list in R, then FP64; per-particle sums and the Newton step
// in FP64.
#include "pairs.h"

namespace sph {
namespace shared {

constexpr int kQuad = 4;                 // lanes per target
constexpr int kTW = kWave / kQuad;       // targets per wavefront
constexpr int kTG = NW * kTW;            // targets per work-group round
constexpr int kQStep = 2 * kQuad;        // staged entries per walk step

// staged entries per wavefront area and list slots per target (density
// lists cover h (1 + slack) at the first h of the Newton iteration, which
// may lie well above the root, and should not overflow: a list that
// overflows is evaluated at once and built again at every later step)
template <typename R, bool FORCE> struct Cfg;
template <> struct Cfg<float, false> { static constexpr int CAPW = 192, LISTW = 90; };
template <> struct Cfg<float, true> { static constexpr int CAPW = 216, LISTW = 74; };
template <> struct Cfg<double, false> { static constexpr int CAPW = 256, LISTW = 90; };
template <> struct Cfg<double, true> { static constexpr int CAPW = 256, LISTW = 74; };

template <typename R, bool FORCE>
struct Smem {
    using R4 = typename Vec4T<R>::T;
    static constexpr int CAPW = Cfg<R, FORCE>::CAPW;
    static constexpr int MAXSEG = kMaxSegW;
    // entries per area: a walk step reads up to kQStep - 1 past a segment's end
    static constexpr int STRIDE = CAPW + kQStep;
    static constexpr int LISTW = Cfg<R, FORCE>::LISTW;
    // a list row holds LISTW slots and is read up to 2 kQuad - 1 past its last
    // (masked); its pitch is an odd number of dwords, so the rows of the 16
    // targets of a wavefront start in distinct banks
    static constexpr int LISTP = LISTW + 2 * kQuad;
    static_assert(LISTP % 2 == 0 && (LISTP / 2) % 2 == 1, "odd dword pitch");
    static_assert(NW * STRIDE <= 65536, "list entries are 16-bit");
    // staged (x, y, z in T's frame, |x|^2 / 2 less its rounding allowance),
    // force: h_j^2 / 2, projection on the segment axis, cell-order index;
    // a list entry is a flat index area * STRIDE + position
    R4 st[NW][STRIDE];
    R sh[NW][FORCE ? STRIDE : 1];
    float sp[NW][STRIDE];
    uint32_t sg[NW][STRIDE];
    uint16_t list[kTG][LISTP];
    // density: the mass-weighted sums of each target's last full evaluation
    double fin[FORCE ? 1 : kTG][6];
    int seg_b[NW][MAXSEG], seg_e[NW][MAXSEG];
    float seg_u[NW][MAXSEG][3];
    float seg_hx[NW][MAXSEG];
    float seg_dr[NW][MAXSEG];
    int nseg[NW];
    int self_b[NW], self_t0[NW], self_n[NW];
    int unit;
    float vote[NW];
};

// Cells left to the split layout (their sources need several staging batches)
struct Deferred {
    int32_t* units;
    int32_t* count;
};

// ---------------------------------------------------------------- quad operations
// data-parallel-primitive moves within quads of lanes: the value of lane ^ 1,
// of lane ^ 2 (quad permutations [1,0,3,2] and [2,3,0,1])
__device__ __forceinline__ int dpp_x1(int v) { return __builtin_amdgcn_mov_dpp(v, 0xB1, 0xF, 0xF, false); }
__device__ __forceinline__ int dpp_x2(int v) { return __builtin_amdgcn_mov_dpp(v, 0x4E, 0xF, 0xF, false); }

// the same move of a double (its two halves)
__device__ __forceinline__ double quad_mv(double x, bool two)
{
    const long long u = __double_as_longlong(x);
    int lo = (int)(uint32_t)u, hi = (int)(uint32_t)((unsigned long long)u >> 32);
    lo = two ? dpp_x2(lo) : dpp_x1(lo);
    hi = two ? dpp_x2(hi) : dpp_x1(hi);
    return __longlong_as_double((long long)(((unsigned long long)(uint32_t)hi << 32) | (uint32_t)lo));
}

// Sums over the quad, bitwise equal in its four lanes (the additions of the
// two rounds commute).  Every lane of the wavefront must be active.
__device__ __forceinline__ double quad_sum(double v)
{
    v += quad_mv(v, false);
    v += quad_mv(v, true);
    return v;
}
__device__ __forceinline__ int quad_sum(int v)
{
    v += dpp_x1(v);
    v += dpp_x2(v);
    return v;
}
// largest value over the quad
__device__ __forceinline__ float quad_max(float v)
{
    v = fmaxf(v, __int_as_float(dpp_x1(__float_as_int(v))));
    return fmaxf(v, __int_as_float(dpp_x2(__float_as_int(v))));
}
__device__ __forceinline__ double quad_max(double v)
{
    v = fmax(v, quad_mv(v, false));
    return fmax(v, quad_mv(v, true));
}

// Block-level votes, two barriers each.  The results are read into scalar
// registers, so that the branches taken on them (around further barriers)
// are uniform for the compiler too.
// all four wavefronts agree (ok is uniform within each)
template <typename SM>
__device__ __forceinline__ bool block_all(SM& s, int w, int lane, bool ok)
{
    if (lane == 0) s.vote[w] = ok ? 1.0f : 0.0f;
    __syncthreads();
    const bool all = (s.vote[0] != 0.0f) & (s.vote[1] != 0.0f) & (s.vote[2] != 0.0f) & (s.vote[3] != 0.0f);
    __syncthreads();
    return uniform(all ? 1 : 0) != 0;
}
// largest of the four wavefronts' values (uniform within each, >= 0)
template <typename SM>
__device__ __forceinline__ float block_max(SM& s, int w, int lane, float v)
{
    if (lane == 0) s.vote[w] = v;
    __syncthreads();
    const float m = fmaxf(fmaxf(s.vote[0], s.vote[1]), fmaxf(s.vote[2], s.vote[3]));
    __syncthreads();
    return __int_as_float(uniform(__float_as_int(m)));
}

// flat staged index of target ti (a particle of T) in the self segments, or -1
template <typename SM>
__device__ __forceinline__ int self_flat(const SM& s, int ti)
{
    int g = -1;
#pragma unroll
    for (int r = 0; r < NW; r++) {
        const int d = ti - s.self_t0[r];
        if (d >= 0 && d < s.self_n[r]) g = r * SM::STRIDE + s.self_b[r] + d;
    }
    return g;
}

// ---------------------------------------------------------------- walk
// Walk of one wavefront's quads over the staged segments of the four areas,
// from (r, seg, jj) on, one segment at a time for all lanes: a step covers
// eight staged entries, two per lane of each quad, every one tested against
// the quad's target.  A segment is left before the first step whose first
// entry lies beyond every lane's projected bound (the early exit of the
// sorted sweep; the self segments have none).  Returns the list length, early
// when a list might overflow in the next step, with (r, seg, jj) the place to
// resume; r == NW when the walk is complete.
//
// The in-range test is that of the split layout: r^2 / 2 = K_i + a_j - x_i . x_j
// with the halved squared norms reduced by their rounding allowance, so a
// list holds every pair in range and possibly a few just outside, which the
// pair arithmetic discards.
template <typename R, bool FORCE>
__device__ __forceinline__ int walk(Smem<R, FORCE>& s, const int lane, const bool act, const R xi, const R yi,
                                    const R zi, const float fxi, const float fyi, const float fzi, const R rad,
                                    const float fh, const float margin, const int selfg, uint16_t* const row,
                                    int& r_io, int& seg_io, int& jj_io, int wi)
{
    using SM = Smem<R, FORCE>;
    using R4 = typename Vec4T<R>::T;
    constexpr int LISTW = SM::LISTW;
    constexpr int STRIDE = SM::STRIDE;
    const int b = lane & (kQuad - 1);
    const int qsh = lane & ~(kQuad - 1);
    const uint32_t below = (1u << b) - 1u;
    const R ki = half_sq_lo(xi, yi, zi);
    const R c_half = (R)0.5 * rad * rad * ((R)1 + (R)8 * std::numeric_limits<R>::epsilon());
    const R d_half = c_half - ki;
    int r = uniform(r_io);
    int seg = uniform(seg_io);
    int jj = uniform(jj_io);
    bool full = false;
    auto test = [&](const R4& e, R hj2) {
        if constexpr (FORCE) {
            const R t = fma(-zi, e.z, fma(-yi, e.y, fma(-xi, e.x, e.w + ki)));
            return t < sq_max(c_half, hj2);
        } else {
            const R t = fma(-zi, e.z, fma(-yi, e.y, fma(-xi, e.x, e.w)));
            return t < d_half;
        }
    };
    // lanes whose quad position b is below d (uniform): those whose entry
    // jj + b lies before a segment end d entries on
    auto below_end = [](int d) -> uint64_t {
        return d >= kQuad ? ~0ull : (d <= 0 ? 0ull : ((1ull << d) - 1ull) * 0x1111111111111111ull);
    };
    const uint64_t mact = lanes(act);
    // a list slot that is never read unmasked: the writes of lanes without a hit
    const int trash = SM::LISTP - 1;
    // entries jj + b and jj + 4 + b of area r (past the segment end: masked);
    // excl is the flat index of the target itself in a self segment, else -1.
    // Hits are lane masks combined in scalar registers; every lane writes a
    // slot (its own next one on a hit, else the trash slot), so that the
    // stores need no branch.
    auto step = [&](int je, int jj, int excl, bool self) {
        const int j0 = jj + b, j1 = j0 + kQuad;
        const R4 e0 = s.st[r][j0], e1 = s.st[r][j1];
        const R hj0 = FORCE ? s.sh[r][FORCE ? j0 : 0] : (R)0;
        const R hj1 = FORCE ? s.sh[r][FORCE ? j1 : 0] : (R)0;
        const int g0 = r * STRIDE + j0, g1 = g0 + kQuad;
        uint64_t m0 = lanes(test(e0, hj0)) & mact & below_end(je - jj);
        uint64_t m1 = lanes(test(e1, hj1)) & mact & below_end(je - jj - kQuad);
        if (self) {
            m0 &= lanes(g0 != excl);
            m1 &= lanes(g1 != excl);
        }
        // the quad's hits of each entry
        const uint32_t q0 = (uint32_t)(m0 >> qsh) & 0xFu;
        const uint32_t q1 = (uint32_t)(m1 >> qsh) & 0xFu;
        const int n0 = __popc(q0) + wi;
        const bool h0 = (q0 >> b) & 1u, h1 = (q1 >> b) & 1u;
        row[h0 ? wi + __popc(q0 & below) : trash] = (uint16_t)g0;
        row[h1 ? n0 + __popc(q1 & below) : trash] = (uint16_t)g1;
        wi = n0 + __popc(q1);
    };
    while (r < NW) {
        converge();
        const int nseg = uniform(s.nseg[r]);
        while (seg < nseg) {
            converge();
            const int je = uniform(s.seg_e[r][seg]);
            const float ux = s.seg_u[r][seg][0], uy = s.seg_u[r][seg][1], uz = s.seg_u[r][seg][2];
            const float hx = s.seg_hx[r][seg];
            // the self segment has u = 0
            const bool self = uniform((ux == 0.0f) & (uy == 0.0f) & (uz == 0.0f)) != 0;
            // stored order of projections that moved by up to d since: an entry
            // beyond bound + 2d leaves every later one beyond bound
            const float bound =
                !act ? -INFINITY : ux * fxi + uy * fyi + uz * fzi + fmaxf(fh, hx) + margin + 2.0f * s.seg_dr[r][seg];
            if (self) {
                while (jj < je) {
                    converge();
                    if (wave_any(wi > LISTW - kQStep)) { full = true; break; }
                    step(je, jj, selfg, true);
                    jj += kQStep;
                }
            } else {
                while (jj < je) {
                    converge();
                    if (wave_any(wi > LISTW - kQStep)) { full = true; break; }
                    if (!wave_any(s.sp[r][jj] <= bound)) break;   // the rest is out of reach
                    step(je, jj, -1, false);
                    jj += kQStep;
                }
            }
            if (full) break;
            seg++;
            jj = seg < nseg ? uniform(s.seg_b[r][seg]) : 0;
        }
        if (full) break;
        r++;
        seg = 0;
        jj = (r < NW && s.nseg[r] > 0) ? uniform(s.seg_b[r][0]) : 0;
    }
    r_io = r;
    seg_io = seg;
    jj_io = jj;
    return wi;
}

// start of a walk: the first segment of the first area
template <typename SM>
__device__ __forceinline__ void walk_start(const SM& s, int& r, int& seg, int& jj)
{
    r = 0;
    seg = 0;
    jj = s.nseg[0] > 0 ? uniform(s.seg_b[0][0]) : 0;
}

// The next unit of the persistent loop, the same in every wavefront.  The
// barrier in front is part of the loop's top: the compiler cannot route the
// lanes other than thread 0 around thread 0's fetch on their way back to the
// top (a path that knows tid != 0, such as the end of a unit whose last store
// is thread 0's, would otherwise jump straight to the read below and leave
// those lanes in a loop of their own that re-reads the old unit).
template <typename SM>
__device__ __forceinline__ int next_unit(SM& s, const Decomp& dc, int tid)
{
    __syncthreads();   // every wavefront is done with the last unit and its index
    if (tid == 0) s.unit = atomicAdd(dc.qhead, 1);
    __syncthreads();
    return uniform(s.unit);
}

__device__ __forceinline__ void defer(const Deferred& df, int unit, int tid)
{
    if (tid == 0) df.units[atomicAdd(df.count, 1)] = unit;
}

// ---------------------------------------------------------------- density
// FP32: four work-groups per CU (at most 128 VGPRs); FP64: two, by LDS
template <typename R> constexpr int kWavesDens = sizeof(R) == 4 ? 4 : 2;

template <typename R>
__global__ __launch_bounds__(WGS) __attribute__((amdgpu_waves_per_eu(kWavesDens<R>))) void k_density(
    Decomp dc, CellData<R> cd, Sorted<R> so, GhostData<R> gd, DensityOut out, PassConsts pc, Deferred df)
{
    using R4 = typename Vec4T<R>::T;
    using SM = Smem<R, false>;
    __shared__ SM s;
    const int tid = threadIdx.x;
    const int w = uniform(tid >> 6);
    const int lane = tid & (kWave - 1);
    const int b = lane & (kQuad - 1);
    const int ts = w * kTW + (lane >> 2);   // the quad's target slot
    uint16_t* const row = &s.list[ts][0];
    const R4* const stf = &s.st[0][0];
    const uint32_t* const sgf = &s.sg[0][0];
    const int ncells = *dc.ncells;
    const double kNorm = 8.0 / kPi;
    if (*dc.status & (ST_NONFINITE | ST_H_TOO_LARGE | ST_CAPACITY)) return;
    const int nunits = dc.nunits ? *dc.nunits : ncells;
    while (true) {
        const int uidx = next_unit(s, dc, tid);
        if (uidx >= nunits) break;
        const int unit = dc.units ? dc.units[uidx] : uidx;
        CellInfo T = dc.cells[unit];
        const BoxInfo B = dc.boxes[T.box];
        // the lists cover h up to this, less the displacement allowances; a
        // decomposition that has drifted by more than half of it is rebuilt
        // rather than swept (the cell is then swept as an empty one)
        const float dT = cell_dr(dc, unit);
        const double h_lim = (double)T.hlim - (double)dT - B.drift;
        const bool stale = uniform((double)dT + B.drift <= 0.5 * (double)T.hlim ? 0 : 1) != 0;
        if (stale) {
            if (tid == 0) atomicOr(dc.status, ST_REBUILD);
            T.count = 0;
        }
        // with multiple time-stepping, a cell without active particles stages
        // nothing and only passes its particles' stored quantities on
        bool any_on = !gd.active;
        if (gd.active)
            for (int t = lane; t < T.count; t += kWave) any_on |= gd.active[dc.perm[T.start + t]] != 0;
        const bool cell_on = uniform(__any(any_on) ? 1 : 0) != 0;
        const int nsrc = (stale || !cell_on) ? 0 : dc.src_count[unit];
        const double h_box = fmin(B.L[0], fmin(B.L[1], B.L[2])) / 3.0;
        const float margin = 1e-5f * (float)fmax(B.e[0], fmax(B.e[1], B.e[2]));
        const float mstage = margin + dT;   // targets may have left the cell by dT
        double hc = 0.0;
        for (int t = lane; t < T.count; t += kWave) hc = fmax(hc, cd.h[T.start + t]);
        hc = wave_max(hc);
        float Hst = (float)fmin(hc * (1.0 + pc.h_margin), h_lim);

        int k = 0, p = 0;
        stage_wave<R, false>(s, w, dc, cd, so, gd, B, unit, T.level, nsrc, k, p, Hst, mstage);
        if (!block_all(s, w, lane, k >= nsrc)) {
            defer(df, unit, tid);
            continue;
        }
        bool deferred = false;
        float cell_hmax = 0.0f;

        for (int c0 = 0; c0 < T.count && !deferred; c0 += kTG) {
            converge();
            const int ti = c0 + ts;
            const bool valid = ti < T.count;
            const uint32_t gi = (uint32_t)(T.start + (valid ? ti : 0));
            const uint32_t pi = dc.perm[gi];
            const bool on = valid && (!gd.active || gd.active[pi] != 0);
            const R4 ri = cd.rp[gi];
            const R xi = ri.x, yi = ri.y, zi = ri.z;
            const R4 vmi = cd.vm[gi];
            const float fxi = (float)xi, fyi = (float)yi, fzi = (float)zi;
            double h = fmin(cd.h[gi], h_lim);
            double lo = 0.0, hi = INFINITY, h_rebuild = 0.0;
            int iters = 0;
            bool failed = false;
            bool conv = !on || pc.fixed_h;
            if (pc.fixed_h && on && cd.h[gi] > h_lim) {
                // a given h beyond what the cells allow: rebuilt for it, then swept again
                if (b == 0) atomicOr(dc.status, ST_REBUILD);
                h_rebuild = cd.h[gi];
            }
            const int selfg = valid ? self_flat(s, ti) : -1;
            bool cached = false, cached_all = false;
            float hcache = 0.0f;
            int cnt = 0;
            // the quad's totals of the last evaluation
            DensAcc acc = {};

            // The sums of the lane's target at the current h, for the lanes in
            // `act`: the two of Eq. (3) (full = false) or all of them (full = true).
            auto evaluate = [&](bool act, bool full) {
                acc = DensAcc{};
                double tm[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};   // full: the mass-weighted sums
                const R hr = (R)h, hinv = (R)(1.0 / h), h2 = hr * hr;
                // this lane's entries b, b + 4, ... of the first n of the list
                auto process = [&](int n) {
                    if (full) {
                        DensPart<R> bp = {};
                        for (int t = b;; t += kQuad) {
                            converge();
                            const bool v0 = act && t < n;
                            if (!wave_any(v0)) break;
                            const int j0 = v0 ? (int)row[t] : 0;
                            const R4 e0 = stf[j0];
                            const R4 q0 = cd.vm[sgf[j0]];
                            density_pair<R>(bp, v0, xi, yi, zi, vmi.x, vmi.y, vmi.z, hr, hinv, h2, e0, q0);
                        }
                        acc.w += (double)bp.w; acc.qdw += (double)bp.qdw; acc.n += bp.n;
                        tm[0] += (double)bp.mw; tm[1] += (double)bp.mqdw; tm[2] += (double)bp.div;
                        tm[3] += (double)bp.cx; tm[4] += (double)bp.cy; tm[5] += (double)bp.cz;
                    } else {
                        R sw = (R)0, sq = (R)0;
                        for (int t = b;; t += 2 * kQuad) {
                            converge();
                            const bool v0 = act && t < n, v1 = act && t + kQuad < n;
                            if (!wave_any(v0)) break;
                            // slots t, t + 4 lie in the row (its pitch); past the list: masked
                            const int r0 = row[t], r1 = row[t + kQuad];
                            const R4 e0 = stf[v0 ? r0 : 0], e1 = stf[v1 ? r1 : 0];
                            count_pair<R>(sw, sq, v0, xi, yi, zi, hinv, h2, e0);
                            count_pair<R>(sw, sq, v1, xi, yi, zi, hinv, h2, e1);
                        }
                        acc.w += (double)sw;
                        acc.qdw += (double)sq;
                    }
                };
                const bool reuse = cached && (!full || cached_all) && __all(!act || (float)h <= hcache);
                if (reuse) {
                    process(cnt);
                } else {
                    // a walk with early exit; the lists keep r < h (1 + slack)
                    hcache = fminf((float)h * (1.0f + kCacheSlack), Hst);
                    const R rad = (R)hcache;
                    const float fh = hcache + margin;
                    bool flushed = false;
                    int r, seg, jj;
                    walk_start(s, r, seg, jj);
                    cnt = 0;
                    while (true) {
                        converge();
                        cnt = walk<R, false>(s, lane, act, xi, yi, zi, fxi, fyi, fzi, rad, fh, margin, selfg, row, r,
                                             seg, jj, cnt);
                        if (r >= NW) break;
                        process(cnt);   // a list is full: evaluate it and continue the walk
                        cnt = 0;
                        flushed = true;
                    }
                    process(cnt);
                    cached = !flushed;
                    cached_all = __all(act || !on);
                }
                acc.w = quad_sum(acc.w);
                acc.qdw = quad_sum(acc.qdw);
                if (full) {
                    // kept in LDS for the per-particle quantities
                    acc.n = quad_sum(acc.n);
#pragma unroll
                    for (int a = 0; a < 6; a++) {
                        const double v = quad_sum(tm[a]);
                        if (b == 0) s.fin[ts][a] = v;
                    }
                }
            };

            // Newton iteration on h (Eq. (3)) in FP64, safeguarded by a bracket, on
            // g(h) = N(h)^(1/3) - n_ngb^(1/3) (close to linear in h: N grows like
            // h^3), whose root is the same.  A step so small that the next
            // residual is predicted far below the tolerance makes the next
            // evaluation one of every sum, which ends the iteration if it
            // confirms convergence.  A lane whose next h exceeds the staged
            // reach waits (blocked) for the work-group to stage again.
            const double cbrt_ngb = cbrt(pc.n_ngb);
            const double step_final = sqrt(pc.tol / (10.0 * pc.n_ngb));
            bool full = pc.fixed_h != 0;
            bool blocked = false;
            while (true) {
                converge();
                while (true) {
                    converge();
                    if (full) {
                        evaluate(on && !blocked, true);
                        if (!conv && !blocked) {
                            iters++;
                            const double N = 32.0 / 3.0 * (acc.w + 1.0);
                            if (fabs(N - pc.n_ngb) <= pc.tol) conv = true;
                        }
                        if (__all(conv || blocked)) break;
                        full = false;
                    }
                    const bool act = !conv && !blocked;
                    evaluate(act, false);
                    bool close = true;
                    if (act) {
                        iters++;
                        const double N = 32.0 / 3.0 * (acc.w + 1.0);
                        const double dN = -32.0 / 3.0 / h * acc.qdw;
                        const double f = N - pc.n_ngb;
                        if (fabs(f) <= pc.tol) {
                            conv = true;
                        } else if (iters >= pc.max_iter) {
                            conv = true; failed = true;
                        } else {
                            if (f < 0.0) lo = h; else hi = h;
                            const double c = cbrt(N);
                            double hn = h - 3.0 * c * c * (c - cbrt_ngb) / dN;
                            const bool ok = (dN > 0.0) && (hn > lo) && (hn < hi) && (hn >= 0.5 * h) && (hn <= 2.0 * h);
                            if (!ok) hn = isinf(hi) ? 2.0 * h : 0.5 * (lo + hi);
                            if (hn > h_lim) {
                                if (h >= h_lim) {   // the root lies beyond what the cells allow
                                    if (b == 0) atomicOr(dc.status, ST_REBUILD);
                                    conv = true; failed = true;
                                    h_rebuild = fmin(hn, h_box);
                                } else {
                                    hn = h_lim;
                                }
                            }
                            if (!conv) {
                                close = fabs(hn - h) <= step_final * h;
                                h = hn;
                                blocked = (float)h > Hst;
                            }
                        }
                    }
                    full = __all(close || blocked);
                }
                // restaging when some lane of the work-group waits for it
                const float hw = (float)wave_max(blocked ? h : 0.0);
                const float hreq = block_max(s, w, lane, hw);
                if (hreq == 0.0f) break;
                Hst = (float)fmin(fmax((double)Hst, (double)hreq * (1.0 + pc.h_margin)), h_lim);
                k = 0; p = 0;
                stage_wave<R, false>(s, w, dc, cd, so, gd, B, unit, T.level, nsrc, k, p, Hst, mstage);
                if (!block_all(s, w, lane, k >= nsrc)) {
                    deferred = true;
                    break;
                }
                blocked = false;
                cached = false;
                full = false;
            }
            if (deferred) break;

            // ---- per-particle quantities between the stages (lane 0 of each quad)
            if (b == 0 && valid && !on) {
                // not a target this time: its quantities of the last active step
                const double hh = cd.h[gi];
                const double k5 = kNorm / (hh * hh * hh * hh * hh);
                R4 g0, g1;
                g0.x = (R)(1.0 / hh); g0.y = (R)k5; g0.z = (R)gd.s_A[pi]; g0.w = (R)gd.s_rho[pi];
                g1.x = (R)gd.s_c[pi]; g1.y = (R)gd.s_f[pi]; g1.z = (R)hh; g1.w = (R)0;
                gd.g0[gi] = g0;
                gd.g1[gi] = g1;
            }
            if (valid && !on) cell_hmax = fmaxf(cell_hmax, (float)cd.h[gi] * (1.0f + 1e-6f));
            if (on) cell_hmax = fmaxf(cell_hmax, (float)h * (1.0f + 1e-6f));
            if (b == 0 && on) {
                const double tmw = s.fin[ts][0], tmqdw = s.fin[ts][1], tdiv = s.fin[ts][2];
                const double tcx = s.fin[ts][3], tcy = s.fin[ts][4], tcz = s.fin[ts][5];
                const double m = (double)vmi.w;
                const double k3 = kNorm / (h * h * h);
                const double k5 = k3 / (h * h);
                const double rho = k3 * (tmw + m);
                const double drho = -kNorm / (h * h * h * h) * (3.0 * (tmw + m) + tmqdw);
                const double omega = 1.0 + h / (3.0 * rho) * drho;
                const double N = 32.0 / 3.0 * (acc.w + 1.0);
                const double div = k5 * tdiv / rho;
                const double cx = -k5 * tcx / rho, cy = -k5 * tcy / rho, cz = -k5 * tcz / rho;
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
                    gd.sd0[gi] = make_double4(tmw + m, tmqdw, -32.0 / 3.0 / h * acc.qdw, tdiv);
                    gd.sd1[gi] = make_double4(tcx, tcy, tcz, 0.0);
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
                if (out.ndens) out.ndens[pi] = acc.n;
                if (failed) atomicOr(dc.status, ST_NOT_CONVERGED);
            }
        }
        if (deferred) {
            // the split layout sweeps the cell again from the start
            defer(df, unit, tid);
            continue;
        }
        const float hm = block_max(s, w, lane, (float)wave_max((double)cell_hmax));
        if (tid == 0) gd.cell_hmax[unit] = hm;
    }
}

// ---------------------------------------------------------------- force
template <typename R> constexpr int kWavesForce = sizeof(R) == 4 ? 4 : 2;

template <typename R>
__global__ __launch_bounds__(WGS) __attribute__((amdgpu_waves_per_eu(kWavesForce<R>))) void k_force(
    Decomp dc, CellData<R> cd, Sorted<R> so, GhostData<R> gd, ForceOut out, PassConsts pc, Deferred df)
{
    using R4 = typename Vec4T<R>::T;
    using SM = Smem<R, true>;
    __shared__ SM s;
    const int tid = threadIdx.x;
    const int w = uniform(tid >> 6);
    const int lane = tid & (kWave - 1);
    const int b = lane & (kQuad - 1);
    const int ts = w * kTW + (lane >> 2);
    uint16_t* const row = &s.list[ts][0];
    const R4* const stf = &s.st[0][0];
    const uint32_t* const sgf = &s.sg[0][0];
    const int ncells = *dc.ncells;
    const R alpha = (R)pc.alpha;
    if (*dc.status & (ST_NONFINITE | ST_H_TOO_LARGE | ST_CAPACITY)) return;
    const int nunits = dc.nunits ? *dc.nunits : ncells;
    while (true) {
        const int uidx = next_unit(s, dc, tid);
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
        const bool cell_on = uniform(__any(any_on) ? 1 : 0) != 0;
        if (!cell_on) nsrc = 0;   // no target here: nothing to stage or sweep
        int k = 0, p = 0;
        stage_wave<R, true>(s, w, dc, cd, so, gd, B, unit, T.level, nsrc, k, p, Hst, mstage);
        if (!block_all(s, w, lane, k >= nsrc)) {
            defer(df, unit, tid);
            continue;
        }
        for (int c0 = 0; c0 < T.count; c0 += kTG) {
            converge();
            const int ti_ = c0 + ts;
            const bool valid = ti_ < T.count;
            const uint32_t gi = (uint32_t)(T.start + (valid ? ti_ : 0));
            const bool on = valid && (!gd.active || gd.active[dc.perm[gi]] != 0);
            ForceTarget<R> ti;
            const R4 ri = cd.rp[gi];
            ti.x = ri.x; ti.y = ri.y; ti.z = ri.z;
            const R4 vmi = cd.vm[gi], g0i = gd.g0[gi], g1i = gd.g1[gi];
            ti.vx = vmi.x; ti.vy = vmi.y; ti.vz = vmi.z;
            ti.hinv = g0i.x; ti.gk = g0i.y; ti.A = g0i.z; ti.rho = g0i.w;
            ti.c = g1i.x; ti.f = g1i.y; ti.h = g1i.z;
            const float fxi = (float)ti.x, fyi = (float)ti.y, fzi = (float)ti.z, fh = (float)ti.h;
            const int selfg = valid ? self_flat(s, ti_) : -1;
            ForceAcc<R> acc = {};
            // this lane's entries b, b + 4, ... of the first n of the list
            auto process = [&](int n) {
                ForcePart<R> bp = {};
                for (int t = b;; t += 2 * kQuad) {
                    converge();
                    const bool v0 = t < n, v1 = t + kQuad < n;
                    if (!wave_any(v0)) break;
                    const int r0 = row[t], r1 = row[t + kQuad];
                    const int j0 = v0 ? r0 : 0, j1 = v1 ? r1 : 0;
                    const uint32_t q0 = sgf[j0], q1 = sgf[j1];
                    const R4 e0 = stf[j0], e1 = stf[j1];
                    const R4 v0m = cd.vm[q0], v1m = cd.vm[q1];
                    const R4 a0 = gd.g0[q0], a1 = gd.g0[q1];
                    const R4 b0 = gd.g1[q0], b1 = gd.g1[q1];
                    force_pair<R>(acc, bp, v0, ti, alpha, e0, v0m, a0, b0);
                    force_pair<R>(acc, bp, v1, ti, alpha, e1, v1m, a1, b1);
                }
                acc.ax += (double)bp.ax;
                acc.ay += (double)bp.ay;
                acc.az += (double)bp.az;
                acc.du += (double)bp.du;
            };
            int r, seg, jj;
            walk_start(s, r, seg, jj);
            int cnt = 0;
            while (true) {
                converge();
                cnt = walk<R, true>(s, lane, on, ti.x, ti.y, ti.z, fxi, fyi, fzi, ti.h, fh, margin, selfg, row, r, seg,
                                    jj, cnt);
                process(cnt);
                cnt = 0;
                if (r >= NW) break;
            }
            const double ax = quad_sum(acc.ax), ay = quad_sum(acc.ay), az = quad_sum(acc.az);
            const double du = quad_sum(acc.du);
            const int np_ = quad_sum(acc.n);
            const R vsg = quad_max(acc.vsig);
            if (b == 0 && on) {
                const uint32_t pi = dc.perm[gi];
                if (out.ax) out.ax[pi] = ax;
                if (out.ay) out.ay[pi] = ay;
                if (out.az) out.az[pi] = az;
                if (out.dudt) out.dudt[pi] = du;
                if (out.npairs) out.npairs[pi] = np_;
                if (out.dt) {
                    // j = i contributes 2 c_i (no approach speed)
                    const double vs = fmax((double)vsg, 2.0 * (double)ti.c);
                    out.dt[pi] = vs > 0.0 ? pc.cfl * 2.0 * (double)ti.h / vs : (double)INFINITY;
                }
            }
        }
    }
}

__global__ void k_reset_pair(int32_t* c)
{
    c[0] = 0;
    c[1] = 0;
}

}  // namespace shared

// ---------------------------------------------------------------- launchers
template <typename F>
static int shared_grid(F fn)
{
    int dev = 0, ncu = 0, per = 0;
    (void)hipGetDevice(&dev);
    (void)hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev);
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, (const void*)fn, WGS, 0) != hipSuccess || per < 1) per = 1;
    if (ncu < 1) ncu = 1;
    return ncu * per;
}

// counters: [0] the work counter of the shared launch, [1] the deferred cells,
// [2] the work counter of the split launch over them
template <typename R>
void launch_density_shared(const Decomp& dc, const CellData<R>& cd, const Sorted<R>& so, const GhostData<R>& gd,
                           const DensityOut& out, const PassConsts& pc, int staging, int32_t* deferred,
                           int32_t* counters, hipStream_t st)
{
    hipLaunchKernelGGL(shared::k_reset_pair, dim3(1), dim3(1), 0, st, counters);
    Decomp d1 = dc;
    d1.qhead = counters;
    hipLaunchKernelGGL(shared::k_density<R>, dim3(shared_grid(shared::k_density<R>)), dim3(WGS), 0, st, d1, cd, so,
                       gd, out, pc, shared::Deferred{deferred, counters + 1});
    Decomp d2 = dc;
    d2.units = deferred;
    d2.nunits = counters + 1;
    d2.qhead = counters + 2;
    launch_density<R>(d2, cd, so, gd, out, pc, staging, st);
}

template <typename R>
void launch_force_shared(const Decomp& dc, const CellData<R>& cd, const Sorted<R>& so, const GhostData<R>& gd,
                         const ForceOut& out, const PassConsts& pc, int split_grid, int32_t* deferred,
                         int32_t* counters, hipStream_t st)
{
    hipLaunchKernelGGL(shared::k_reset_pair, dim3(1), dim3(1), 0, st, counters);
    Decomp d1 = dc;
    d1.qhead = counters;
    hipLaunchKernelGGL(shared::k_force<R>, dim3(shared_grid(shared::k_force<R>)), dim3(WGS), 0, st, d1, cd, so, gd,
                       out, pc, shared::Deferred{deferred, counters + 1});
    Decomp d2 = dc;
    d2.units = deferred;
    d2.nunits = counters + 1;
    d2.qhead = counters + 2;
    launch_force<R>(d2, cd, so, gd, out, pc, split_grid, st);
}

template void launch_density_shared<float>(const Decomp&, const CellData<float>&, const Sorted<float>&,
                                           const GhostData<float>&, const DensityOut&, const PassConsts&, int,
                                           int32_t*, int32_t*, hipStream_t);
template void launch_density_shared<double>(const Decomp&, const CellData<double>&, const Sorted<double>&,
                                            const GhostData<double>&, const DensityOut&, const PassConsts&, int,
                                            int32_t*, int32_t*, hipStream_t);
template void launch_force_shared<float>(const Decomp&, const CellData<float>&, const Sorted<float>&,
                                         const GhostData<float>&, const ForceOut&, const PassConsts&, int, int32_t*,
                                         int32_t*, hipStream_t);
template void launch_force_shared<double>(const Decomp&, const CellData<double>&, const Sorted<double>&,
                                          const GhostData<double>&, const ForceOut&, const PassConsts&, int,
                                          int32_t*, int32_t*, hipStream_t);

}  // namespace sph
