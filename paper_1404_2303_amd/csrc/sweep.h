// sweep.h -- the staging and sorted-sweep machinery shared by the interaction
// kernels (density, force) and their adjoints, for gfx950.  See passes.hip
// for the description of the work unit, the staging and the walk.
#pragma once

#include <limits>
#include <type_traits>

#include "sph_internal.h"
#include "kernels.h"

namespace sph {


constexpr int NW = kSweepWaves;       // wavefronts per target cell
constexpr int WGS = NW * kWave;
constexpr int kMaxSegW = 28;          // staged segments per wavefront and batch
constexpr int NACC_D = 9;             // density partial sums per target
constexpr int NACC_F = 6;             // force partial sums per target
constexpr float kCacheSlack = 0.05f;  // neighbour lists cover h (1 + slack)
constexpr int WALK_STEP = 4;          // staged particles tested per walk step
constexpr int WALK_PAD = WALK_STEP - 1;

// staged particles per wavefront and list slots per lane (density lists also
// serve the Newton iteration, so they are longer)
// The FP32 density stage has two (SPH_STAGING_COMPACT and _WIDE): CFG 0 for
// cells of up to ~80 particles (four work-groups per CU), CFG 1 with room for
// cells of ~80-110 (three).  FP64 stages 192 per wavefront, so that three
// work-groups share a CU (under 53 KiB of LDS each).
template <typename R, bool FORCE, int CFG = 0> struct PCfg;
template <> struct PCfg<float, false, 0> { static constexpr int CAPW = 192, LISTW = 48; };
template <> struct PCfg<float, false, 1> { static constexpr int CAPW = 256, LISTW = 48; };
template <> struct PCfg<float, true, 0> { static constexpr int CAPW = 216, LISTW = 32; };
template <int CFG> struct PCfg<double, false, CFG> { static constexpr int CAPW = 192, LISTW = 48; };
template <> struct PCfg<double, true, 0> { static constexpr int CAPW = 192, LISTW = 32; };

// square root, reciprocal square root and reciprocal of the pair arithmetic:
// the hardware instructions in FP32 (about 1 ulp), correctly rounded in FP64
template <typename R> __device__ __forceinline__ R fast_sqrt(R x);
template <> __device__ __forceinline__ float fast_sqrt<float>(float x) { return __builtin_amdgcn_sqrtf(x); }
template <> __device__ __forceinline__ double fast_sqrt<double>(double x) { return sqrt(x); }
template <typename R> __device__ __forceinline__ R fast_rsqrt(R x);
template <> __device__ __forceinline__ float fast_rsqrt<float>(float x) { return __builtin_amdgcn_rsqf(x); }
template <> __device__ __forceinline__ double fast_rsqrt<double>(double x) { return 1.0 / sqrt(x); }
template <typename R> __device__ __forceinline__ R fast_rcp(R x);
template <> __device__ __forceinline__ float fast_rcp<float>(float x) { return __builtin_amdgcn_rcpf(x); }
template <> __device__ __forceinline__ double fast_rcp<double>(double x) { return 1.0 / x; }

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

__device__ __forceinline__ double wave_max(double v)
{
    for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
    return v;
}

#ifdef SPH_COUNT_WALK
// Counting build only: per translation unit, [density, force][candidate
// tests, list entries] over the walks of its kernels.
static __device__ unsigned long long g_walk_tally[2][2];
#endif

// LDS writes of one lane become visible to the other lanes of its wavefront
__device__ __forceinline__ void wave_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// |x|^2 / 2 reduced by 32 units of rounding, for the in-range test of the walk:
// with a_j and K_i from this, a_j + K_i - x_i . x_j evaluated by fused
// multiply-adds stays below r_ij^2 / 2 (the three roundings of the dot product
// and those of the two norms add up to less than the reduction), so the test
// never drops a pair in range; the pair arithmetic then decides exactly.
template <typename R> __device__ __forceinline__ R half_sq_lo(R x, R y, R z)
{
    constexpr R lo = (R)0.5 * ((R)1 - (R)32 * std::numeric_limits<R>::epsilon() / (R)2);
    return (x * x + y * y + z * z) * lo;
}

// Convergence point of the wavefront, free at run time (no instruction): it
// opens the body of every loop that holds wave-level operations (ballots,
// lane reads, shuffles).  Such a loop can have iterations without any side
// effect for some lanes, and the compiler may then take those lanes out of
// the loop early (a thread must make progress), leaving the wave-level
// operations with part of the wavefront; a wave barrier has a side effect in
// every lane and keeps them all in the loop together.
__device__ __forceinline__ void converge() { __builtin_amdgcn_wave_barrier(); }

__device__ __forceinline__ int uniform(int v) { return __builtin_amdgcn_readfirstlane(v); }
// the value of lane l (uniform) of v
__device__ __forceinline__ int lane_of(int v, int l) { return __builtin_amdgcn_readlane(v, l); }
__device__ __forceinline__ float lane_of(float v, int l)
{
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), l));
}

// ---------------------------------------------------------------- LDS layout
template <typename R, int NACC, bool STAGE_H, int CFG = 0>
struct Smem {
    using R4 = typename Vec4T<R>::T;
    static constexpr int CAPW = PCfg<R, STAGE_H, CFG>::CAPW;
    static constexpr int LISTW = PCfg<R, STAGE_H, CFG>::LISTW;
    static constexpr int MAXSEG = kMaxSegW;
    // staged (x, y, z in T's frame, |x|^2 / 2 less its rounding allowance); the
    // walk reads up to WALK_PAD entries past a segment's end (masked off)
    R4 st[NW][CAPW + WALK_PAD];
    R sh[NW][STAGE_H ? CAPW + WALK_PAD : 1];  // pair range max(h_i, h_j): h^2 / 2 of each staged particle
    float sp[NW][CAPW + WALK_PAD];    // projection on the segment axis (the early exit)
    uint32_t sg[NW][CAPW];            // cell-order index of each staged particle
    // per-lane neighbour lists (staged indices), each lane's slots contiguous;
    // the row pitch is an odd number of dwords, so that the 64 lanes of a
    // wavefront reading or writing slot t of their rows meet 64 distinct banks
    static constexpr int LISTP = LISTW + 4;
    static_assert(CAPW <= 256, "list entries are bytes");
    static_assert(LISTW % 8 == 0, "odd dword pitch");
    uint8_t list[NW][kWave][LISTP];
    uint8_t lcount[NW][kWave];        // density: list lengths, for evaluating all four lists together
    double red[NACC][kWave];          // partial sums of the four wavefronts
    int seg_b[NW][kMaxSegW], seg_e[NW][kMaxSegW];
    float seg_u[NW][kMaxSegW][3];
    float seg_hx[NW][kMaxSegW];       // force: largest h of the source cell
    float seg_dr[NW][kMaxSegW];       // staleness of the source cell's stored projections
    int nseg[NW];
    int self_b[NW], self_t0[NW], self_n[NW];  // self segment: staged start, first cell index, count
    int done[NW];                     // shared sweeps: every source of the wavefront staged
    int unit;
};

// Stage, for wavefront w, its sources from cursor (k, p) on; advance the
// cursor past what was staged (k == nsrc when every source is staged).  The
// sources of the target cell are read 64 at a time, one per lane.  SM is an
// LDS layout with this one's staging members (st, sh, sp, sg, seg_*, nseg,
// self_*), their capacity CAPW and segment count MAXSEG per wavefront.
template <typename R, bool FORCE, typename SM>
__device__ void stage_wave(SM& s, const int w, const Decomp& dc, const CellData<R>& cd,
                           const Sorted<R>& so, const GhostData<R>& gd, const BoxInfo& B, const int tcell,
                           const int tlevel, const int nsrc, int& k, int& p, const float Hst, const float margin)
{
    using R4 = typename Vec4T<R>::T;
    const int lane = threadIdx.x & (kWave - 1);
    const int CAPW = SM::CAPW;
    // edges of the target cell and the finest-level unit of the source offsets
    const float et[3] = {(float)ldexp(B.e[0], -tlevel), (float)ldexp(B.e[1], -tlevel),
                         (float)ldexp(B.e[2], -tlevel)};
    const double ef[3] = {ldexp(B.e[0], -B.depth), ldexp(B.e[1], -B.depth), ldexp(B.e[2], -B.depth)};
    const int64_t soff = dc.src_off[tcell];
    int fill = 0, nseg = 0;
    wave_sync();  // earlier readers of this wavefront's staging area are done
    int chunk = -1;
    Source my = {};
    uint64_t mask = 0;
    // per lane, for its source of the chunk: the cell's range, staleness and
    // (force) largest h, loaded for the whole chunk at once and broadcast
    // from the source's lane when it is staged
    int my_start = 0, my_count = 0;
    float my_ds = 0.f, my_hx = 0.f;
    if (lane == 0) s.self_n[w] = 0;
    while (true) {
        converge();
        if (k >= nsrc) { k = nsrc; p = 0; break; }
        if ((k & ~(kWave - 1)) != chunk) {  // lane-parallel view of the next 64 sources
            chunk = k & ~(kWave - 1);
            const bool in = chunk + lane < nsrc;
            my = in ? dc.src[soff + chunk + lane] : Source{};
            const bool mine = in && (my.wave == w || my.wave == kAllWaves);
            mask = __ballot(mine);
            if (mine) {
                const CellInfo S = dc.cells[my.cell];
                my_start = S.start;
                my_count = S.count;
                my_ds = key_dr(dc, my.cell);
                if constexpr (FORCE) my_hx = gd.cell_hmax[my.cell];
            }
        }
        const uint64_t m = mask & (~0ull << (k - chunk));
        if (m == 0) { k = chunk + kWave; p = 0; continue; }
        k = chunk + __builtin_ctzll(m);
        if (nseg == SM::MAXSEG || fill >= CAPW) break;
        const int sl = uniform(k - chunk);
        const int sdir = lane_of((int)my.dir, sl);
        const int sox = lane_of((int)my.ox, sl), soy = lane_of((int)my.oy, sl), soz = lane_of((int)my.oz, sl);
        const bool self = sdir == kSelfDir;
        struct { int start, count; } S = {lane_of(my_start, sl), lane_of(my_count, sl)};
        const int segb = fill;
        bool complete = true;
        float u[3] = {0.f, 0.f, 0.f};
        float hx = 0.f, ds = 0.f;
        if (self) {
            const int q0 = (S.count * w) / NW, q1 = (S.count * (w + 1)) / NW;
            const int n = q1 - q0 - p;
            const int take = min(n, CAPW - fill);
            for (int t = lane; t < take; t += kWave) {
                const int g = S.start + q0 + p + t;
                R4 e;
                e = cd.rp[g];
                e.w = half_sq_lo(e.x, e.y, e.z);
                s.st[w][fill + t] = e;
                if constexpr (FORCE) { const R hj = gd.g1[g].z; s.sh[w][fill + t] = (R)0.5 * hj * hj; }
                s.sg[w][fill + t] = (uint32_t)g;
            }
            if (lane == 0) { s.self_b[w] = fill; s.self_t0[w] = q0 + p; s.self_n[w] = take; }
            fill += take;
            if (take < n) { complete = false; p += take; }
        } else {
            dir_unit(sdir, u);
            const int sd = dir_sort(sdir);
            const bool flip = dir_flip(sdir);
            // source corner in the target's frame
            const double dxo = sox * ef[0], dyo = soy * ef[1], dzo = soz * ef[2];
            const R dox = (R)dxo, doy = (R)dyo, doz = (R)dzo;
            const float udo = u[0] * (float)dxo + u[1] * (float)dyo + u[2] * (float)dzo;
            float hs = Hst;
            if (FORCE) { hx = lane_of(my_hx, sl); hs = fmaxf(Hst, hx); }
            ds = lane_of(my_ds, sl);
            const float reach = fmaxf(u[0], 0.f) * et[0] + fmaxf(u[1], 0.f) * et[1] + fmaxf(u[2], 0.f) * et[2] +
                                hs + margin + ds;
            const int64_t sbase = (int64_t)sd * dc.n + S.start;
            while (p < S.count) {
                converge();
                const int pos = p + lane;
                bool ok = false;
                int l = 0;
                if (pos < S.count) {
                    const int idx = flip ? (S.count - 1 - pos) : pos;
                    const SortRec r = so.rec[sbase + idx];
                    l = (int)r.idx;
                    const float proj = (flip ? -r.key : r.key) + udo;
                    // a stored key may be its projection rounded down by less
                    // than 2^-15 of its magnitude (flipped: rounded up)
                    ok = proj <= reach + 0x1p-14f * fabsf(r.key);
                }
                const int cnt = __popcll(__ballot(ok));  // the keys are monotone: a prefix
                const int take = min(cnt, CAPW - fill);
                if (lane < take) {
                    // positions now (they may have moved since the ordering was made)
                    const int g = S.start + l;
                    R4 e;
                    e = cd.rp[g];
                    e.x += dox; e.y += doy; e.z += doz;
                    e.w = half_sq_lo(e.x, e.y, e.z);
                    s.st[w][fill + lane] = e;
                    // projection on the segment axis, recomputed from the shifted position
                    s.sp[w][fill + lane] = u[0] * (float)e.x + u[1] * (float)e.y + u[2] * (float)e.z;
                    if constexpr (FORCE) { const R hj = gd.g1[g].z; s.sh[w][fill + lane] = (R)0.5 * hj * hj; }
                    s.sg[w][fill + lane] = (uint32_t)g;
                }
                fill += take;
                p += take;
                if (take < cnt) { complete = false; break; }  // out of room
                if (cnt < kWave) { p = S.count; break; }       // the prefix ended
            }
        }
        if (lane == 0) {
            s.seg_b[w][nseg] = segb;
            s.seg_e[w][nseg] = fill;
            s.seg_u[w][nseg][0] = u[0]; s.seg_u[w][nseg][1] = u[1]; s.seg_u[w][nseg][2] = u[2];
            s.seg_hx[w][nseg] = hx;
            s.seg_dr[w][nseg] = ds;
        }
        nseg++;
        if (!complete) break;
        k++;
        p = 0;
    }
    if (lane == 0) s.nseg[w] = nseg;
    wave_sync();
}

// Staged index of the lane's own particle in wavefront w's self segment, or -1.
template <typename R, int NACC, bool F, int CFG>
__device__ __forceinline__ int self_index(const Smem<R, NACC, F, CFG>& s, int w, int ti)
{
    const int d = ti - s.self_t0[w];
    return (d >= 0 && d < s.self_n[w]) ? s.self_b[w] + d : -1;
}

__device__ __forceinline__ bool wave_any(bool p) { return __builtin_amdgcn_ballot_w64(p) != 0; }

// max of two squares (>= 0, no NaN): their bit patterns order like their values
__device__ __forceinline__ float sq_max(float a, float b)
{
    return __uint_as_float(max(__float_as_uint(a), __float_as_uint(b)));
}
__device__ __forceinline__ double sq_max(double a, double b)
{
    return __longlong_as_double((long long)max((unsigned long long)__double_as_longlong(a),
                                               (unsigned long long)__double_as_longlong(b)));
}
// p += 1 in the lanes of mask m, as one add with m as its carry-in (the
// compiler otherwise selects 0 or 1 into a register and adds that)
template <typename P> __device__ __forceinline__ void append(P& p, uint64_t m)
{
    uint64_t carry_out;
    asm volatile("v_addc_co_u32_e64 %0, %1, 0, %0, %2" : "+v"(p), "=s"(carry_out) : "s"(m));
}
__device__ __forceinline__ uint64_t lanes(bool p) { return __builtin_amdgcn_ballot_w64(p); }

// Walk of wavefront w over the staged segments of region r (its own, r = w,
// or in the shared sweeps any of the four), one segment at a time for
// all lanes together: every lane reads the same staged particle (an LDS
// broadcast), tests it against its own radius, and appends it to its list
// when in range.  The segment is left as soon as no lane is still within its
// projected bound (the early exit of the sorted sweep).  The walk state
// (seg, jj) is uniform and kept in scalar registers; four staged particles
// are tested per step.  The call returns early when some lane's list might
// overflow in the next step (lists hold at most LISTW entries), and resumes
// from (seg, jj).
//
// The in-range test takes r^2 / 2 = K_i + a_j - x_i . x_j, with the halved
// squared norms a_j (staged) and K_i (per lane) reduced by their rounding
// allowance (half_sq_lo): three fused multiply-adds per candidate, never
// below the exact r^2 / 2 by more than the allowance, so a list holds every
// pair in range and possibly a few just outside, which the pair arithmetic
// (its own tests of r against h) discards.
template <typename R, bool FORCE, int NACC, int CFG = 0>
__device__ __forceinline__ int walk(Smem<R, NACC, FORCE, CFG>& s, int w, int r, int lane, bool act, R xi, R yi, R zi, float fxi,
                                    float fyi, float fzi, R rad, float fh, float margin, int selfj, int& seg_io,
                                    int& jj_io, int cnt)
{
    constexpr int LISTW = Smem<R, NACC, FORCE, CFG>::LISTW;
    constexpr int STEP = WALK_STEP;
    const int nseg = uniform(s.nseg[r]);
    // lane constants of the test: K_i, and the range (rad^2 / 2, rounded up)
    const R ki = half_sq_lo(xi, yi, zi);
    const R c_half = (R)0.5 * rad * rad * ((R)1 + (R)8 * std::numeric_limits<R>::epsilon());
    const R d_half = c_half - ki;   // density: a_j - x_i . x_j < d_half
    const uint64_t mact = lanes(act);
    int seg = uniform(seg_io);
    int jj = uniform(jj_io);
    // list slots of this lane; wp is the next free one (an LDS pointer: the
    // append is one add of the hit flag, the pointer is the store address)
    using lds_u8 = __attribute__((address_space(3))) uint8_t;
    lds_u8* const lst = (lds_u8*)&s.list[w][lane][0];
    lds_u8* wp = lst + cnt;
    lds_u8* const wfull = lst + (LISTW - STEP);
    bool full = false;
    // in range: r^2 < h_i^2, or (force) r^2 < max(h_i^2, h_j^2); both halved
    // squares are >= 0, whose bit patterns order like their values (one integer max).
    // A step reads its STEP staged particles before it writes any list slot:
    // list entries are bytes, which may alias anything, so the reads could not
    // be moved ahead of the writes by the compiler.
#ifdef SPH_COUNT_WALK
    unsigned long long n_tests = 0;   // uniform: candidates tested by the active lanes
    const int cnt_in = cnt;
#endif
    using R4 = typename Vec4T<R>::T;
    auto test = [&](const R4& e, R hj2) {
        if constexpr (FORCE) {
            const R t = fma(-zi, e.z, fma(-yi, e.y, fma(-xi, e.x, e.w + ki)));
            return t < sq_max(c_half, hj2);
        } else {
            const R t = fma(-zi, e.z, fma(-yi, e.y, fma(-xi, e.x, e.w)));
            return t < d_half;
        }
    };
    // one step over staged entries jj .. jj + STEP - 1 (past the segment end:
    // any value, masked by j < je)
    auto step = [&](int je, int jj, bool self) {
        R4 e[STEP];
        R hj2[STEP];
#pragma unroll
        for (int k = 0; k < STEP; k++) {
            e[k] = s.st[r][jj + k];
            hj2[k] = FORCE ? s.sh[r][FORCE ? jj + k : 0] : (R)0;
        }
        // hits as lane masks, combined in scalar registers
        uint64_t hit[STEP];
#pragma unroll
        for (int k = 0; k < STEP; k++) {
            const int j = jj + k;
            hit[k] = lanes(test(e[k], hj2[k])) & (j < je ? mact : 0ull);
            if (self) hit[k] &= lanes(j != selfj);
        }
#pragma unroll
        for (int k = 0; k < STEP; k++) {
            *wp = (uint8_t)(jj + k);  // the free slot; kept only on a hit
            append(wp, hit[k]);
        }
#ifdef SPH_COUNT_WALK
        for (int k = 0; k < STEP; k++)
            if (jj + k < je) n_tests += (unsigned long long)__popcll(mact);
#endif
    };
    while (seg < nseg) {
        const int je = uniform(s.seg_e[r][seg]);
        const float ux = s.seg_u[r][seg][0], uy = s.seg_u[r][seg][1], uz = s.seg_u[r][seg][2];
        const float hx = s.seg_hx[r][seg];
        // the self segment has u = 0; a uniform flag
        const bool self = uniform((ux == 0.0f) & (uy == 0.0f) & (uz == 0.0f)) != 0;
        if (self) {
            // the whole self segment is within every bound; skip the target itself
            while (jj < je) {
                if (wave_any(wp > wfull)) { full = true; break; }
                step(je, jj, true);
                jj += STEP;
            }
        } else {
            // stored order of projections that moved by up to d since: an entry
            // beyond bound + 2d leaves every later one beyond bound.  A pair in
            // range is within the bound, so only the exit reads projections.
            const float bound =
                !act ? -INFINITY : ux * fxi + uy * fyi + uz * fzi + fmaxf(fh, hx) + margin + 2.0f * s.seg_dr[r][seg];
            while (jj < je) {
                if (wave_any(wp > wfull)) { full = true; break; }
                const int jl = jj + STEP - 1;
                const uint64_t in_last = jl < je ? lanes(s.sp[r][jl] <= bound) : 0ull;
                step(je, jj, false);
                jj += STEP;
                // projections grow along the segment: once the last entry of a step
                // is beyond every lane's bound, so is the rest of the segment
                if (in_last == 0) break;
            }
        }
        if (full) break;
        seg++;
        jj = seg < nseg ? uniform(s.seg_b[r][seg]) : 0;
    }
    cnt = (int)(wp - lst);
    seg_io = seg;
    jj_io = jj;
#ifdef SPH_COUNT_WALK
    {
        double added = (double)(cnt - cnt_in);
        for (int o = 32; o > 0; o >>= 1) added += __shfl_xor(added, o, 64);
        if (lane == 0) {
            atomicAdd(&g_walk_tally[FORCE ? 1 : 0][0], n_tests);
            atomicAdd(&g_walk_tally[FORCE ? 1 : 0][1], (unsigned long long)added);
        }
    }
#endif
    return cnt;
}

}  // namespace sph
