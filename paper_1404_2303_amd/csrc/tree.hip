// tree.hip -- hierarchical cell decomposition below the top grid (Gonnet
// 2014, Sec. 3.2) and the interaction lists of its leaves, for gfx950.
//
// The keys encode the particle's cell at the finest level (the top grid
// bisected `depth` times), so the cells of every level are runs of equal key
// prefixes in the sorted order.  Per level, the runs become a node table
// (first particle, split flag, largest h).  A node is split, as Sec. 3.2
// states, when it holds more than split_count particles and at least the
// fraction split_frac of them has h below half its edge; the leaves are the
// unsplit nodes whose parent is split.  The leaves are the cells of the
// interaction kernels.
//
// Interaction lists: for each leaf T, every leaf Q whose box lies within
// max(H_T, H_Q) of T's box, where H is the largest h a cell's lists cover
// (cells' hlim).  A pair of particles in range, r < max(h_i, h_j), is
// therefore always a pair of listed cells.  The lists are found by walking
// the tree from the 27 top cells around T and opening nodes whose box is
// within reach; each source is swept along the one of the 26 cell-pair axes
// closest to the direction from T to Q.
#include "sph_internal.h"
#include "kernels.h"

namespace sph {

__device__ inline void key_coords(uint64_t key, int tb, int depth, uint32_t c[3], int* box)
{
    const int bits = 3 * (tb + depth);
    const uint64_t mc = bits >= 64 ? key : (key & ((1ull << bits) - 1));
    c[0] = compact3(mc); c[1] = compact3(mc >> 1); c[2] = compact3(mc >> 2);
    *box = bits >= 64 ? 0 : (int)(key >> bits);
}

// first level at which the key prefix differs from the previous particle's
// (0: another top cell or box; depth + 1: the same finest cell)
__global__ void k_tree_chg(const uint64_t* keys, int64_t n, int depth, uint8_t* chg)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    if (i == 0) { chg[0] = 0; return; }
    const uint64_t x = keys[i] ^ keys[i - 1];
    if (x == 0) { chg[i] = (uint8_t)(depth + 1); return; }
    const int hb = 63 - __builtin_clzll(x);
    chg[i] = (uint8_t)(hb >= 3 * depth ? 0 : depth - hb / 3);
}

// per particle (cell order), the number of levels whose edge is more than
// twice its h: h is below half the edge at levels 0 .. count - 1 (the edges
// halve with each level).  Kept in tv.lev until the leaf levels replace it.
__global__ void k_small_levels(TreeView tv, const BoxInfo* boxes, const double* h)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= tv.n) return;
    uint32_t c[3];
    int b;
    key_coords(tv.keys[i], tv.top_bits, tv.depth, c, &b);
    const BoxInfo& B = boxes[b];
    const double e = fmin(B.e[0], fmin(B.e[1], B.e[2]));
    const double hi = h[tv.perm[i]];
    int cnt = 0;
    while (cnt <= tv.depth && hi < 0.5 * ldexp(e, -cnt)) cnt++;
    tv.lev[i] = (uint8_t)cnt;
}

// run heads at level l, and whether h is below half the level's edge
__global__ void k_lvl_prep(TreeView tv, int l)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= tv.n) return;
    tv.flag[i] = tv.chg[i] <= l ? 1u : 0u;
    tv.small[i] = l < (int)tv.lev[i] ? 1u : 0u;
}

__global__ void k_lvl_nodes(TreeView tv, int l)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= tv.n) return;
    const uint32_t f = tv.flag[i];
    const uint32_t m = tv.scan[i] + f - 1;
    tv.node_of[(int64_t)l * tv.n + i] = m;
    if (f) tv.node_start[(int64_t)l * tv.stride + m] = (uint32_t)i;
    if (i == tv.n - 1) tv.node_start[(int64_t)l * tv.stride + m + 1] = (uint32_t)tv.n;
}

__global__ void k_lvl_split(TreeView tv, int l, int split_count, double split_frac)
{
    const int64_t m = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (m >= tv.nnodes[l]) return;
    const uint32_t* ns = tv.node_start + (int64_t)l * tv.stride;
    const uint32_t start = ns[m], end = ns[m + 1];
    const uint32_t cnt = end - start;
    const uint32_t nsmall = tv.psmall[end] - tv.psmall[start];
    bool live = true;
    if (l > 0) {
        const uint32_t parent = tv.node_of[(int64_t)(l - 1) * tv.n + start];
        live = (tv.node_flag[(int64_t)(l - 1) * tv.stride + parent] & NODE_SPLIT) != 0;
    }
    const bool split = live && l < tv.depth && (int64_t)cnt > split_count &&
                       (double)nsmall >= split_frac * (double)cnt;
    tv.node_flag[(int64_t)l * tv.stride + m] = (uint8_t)((live ? NODE_LIVE : 0) | (split ? NODE_SPLIT : 0));
    tv.node_leaf[(int64_t)l * tv.stride + m] = -1;
}

// largest h per node, from the particles (finest level) or the children
__global__ void k_lvl_hmax(TreeView tv, const double* h, int l)
{
    const int64_t m = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (m >= tv.nnodes[l]) return;
    const uint32_t* ns = tv.node_start + (int64_t)l * tv.stride;
    const uint32_t start = ns[m], end = ns[m + 1];
    float hm = 0.0f;
    if (l == tv.depth) {
        for (uint32_t i = start; i < end; i++) hm = fmaxf(hm, (float)h[tv.perm[i]]);
    } else {
        const uint32_t* no = tv.node_of + (int64_t)(l + 1) * tv.n;
        const float* ch = tv.node_hmax + (int64_t)(l + 1) * tv.stride;
        for (uint32_t c = no[start]; c <= no[end - 1]; c++) hm = fmaxf(hm, ch[c]);
    }
    tv.node_hmax[(int64_t)l * tv.stride + m] = hm;
}

// leaf level of each particle: the first level at which its node is live and unsplit
__global__ void k_leaf_flags(TreeView tv)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= tv.n) return;
    int lev = tv.depth;
    for (int l = 0; l <= tv.depth; l++) {
        const uint32_t m = tv.node_of[(int64_t)l * tv.n + i];
        if (tv.node_flag[(int64_t)l * tv.stride + m] == NODE_LIVE) { lev = l; break; }
    }
    tv.lev[i] = (uint8_t)lev;
    tv.flag[i] = tv.chg[i] <= lev ? 1u : 0u;
}

__global__ void k_leaf_cells(TreeView tv, const BoxInfo* boxes, CellInfo* cells, uint32_t* cell_of, double h_margin)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= tv.n) return;
    const int l = tv.lev[i];
    const uint32_t f = tv.flag[i];
    const uint32_t c = tv.scan[i] + f - 1;
    cell_of[i] = c;
    if (!f) return;
    uint32_t cf[3];
    int b;
    key_coords(tv.keys[i], tv.top_bits, tv.depth, cf, &b);
    const BoxInfo& B = boxes[b];
    const int sh = tv.depth - l;
    const uint32_t m = tv.node_of[(int64_t)l * tv.n + i];
    const uint32_t end = tv.node_start[(int64_t)l * tv.stride + m + 1];
    CellInfo C;
    C.start = (int32_t)i;
    C.count = (int32_t)(end - i);
    C.box = b;
    for (int d = 0; d < 3; d++) C.c[d] = (int32_t)((cf[d] >> sh) << sh);
    C.level = l;
    // the lists cover h up to the cell's edge, or its largest h with the
    // margin if that is more, and never beyond the top-cell edge
    const double e0 = fmin(B.e[0], fmin(B.e[1], B.e[2]));
    const double hm = (double)tv.node_hmax[(int64_t)l * tv.stride + m];
    C.hlim = (float)fmin(e0, fmax(hm * (1.0 + h_margin), ldexp(e0, -l)));
    cells[c] = C;
    tv.node_leaf[(int64_t)l * tv.stride + m] = (int32_t)c;
}

// per node: the largest list bound of its leaves (0 below a leaf)
__global__ void k_lvl_H(TreeView tv, const CellInfo* cells, int l)
{
    const int64_t m = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (m >= tv.nnodes[l]) return;
    const int64_t o = (int64_t)l * tv.stride + m;
    const uint8_t fl = tv.node_flag[o];
    float H = 0.0f;
    if (fl & NODE_SPLIT) {
        const uint32_t* ns = tv.node_start + (int64_t)l * tv.stride;
        const uint32_t start = ns[m], end = ns[m + 1];
        const uint32_t* no = tv.node_of + (int64_t)(l + 1) * tv.n;
        const float* ch = tv.node_H + (int64_t)(l + 1) * tv.stride;
        for (uint32_t c = no[start]; c <= no[end - 1]; c++) H = fmaxf(H, ch[c]);
    } else if (fl & NODE_LIVE) {
        H = cells[tv.node_leaf[o]].hlim;
    }
    tv.node_H[o] = H;
}

// dense top-grid map of each box: top cell -> level-0 node
__global__ void k_top_map(TreeView tv, const BoxInfo* boxes, int32_t* cell_map)
{
    const int64_t m = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (m >= tv.nnodes[0]) return;
    uint32_t cf[3];
    int b;
    key_coords(tv.keys[tv.node_start[m]], tv.top_bits, tv.depth, cf, &b);
    const BoxInfo& B = boxes[b];
    const int64_t x = cf[0] >> tv.depth, y = cf[1] >> tv.depth, z = cf[2] >> tv.depth;
    cell_map[B.map_off + (x * B.nc[1] + y) * B.nc[2] + z] = (int32_t)m;
}

// ---------------------------------------------------------------- interaction lists
constexpr int kTreeStack = 112;

// The one of the 26 cell-pair axes closest to v: the unit vectors along one,
// two or three of v's largest components (with v's signs) are the only
// candidates; take the one with the largest projection of v.
__device__ inline int nearest_dir(double vx, double vy, double vz)
{
    const double v[3] = {vx, vy, vz};
    const double a[3] = {fabs(vx), fabs(vy), fabs(vz)};
    int i0 = 0, i1 = 1, i2 = 2;
    if (a[i1] > a[i0]) { const int t = i0; i0 = i1; i1 = t; }
    if (a[i2] > a[i0]) { const int t = i0; i0 = i2; i2 = t; }
    if (a[i2] > a[i1]) { const int t = i1; i1 = i2; i2 = t; }
    const double s1 = a[i0];
    const double s2 = (a[i0] + a[i1]) * 0.70710678118654752;
    const double s3 = (a[i0] + a[i1] + a[i2]) * 0.57735026918962576;
    int o[3] = {0, 0, 0};
    if (s3 >= s2 && s3 >= s1) {
        for (int k = 0; k < 3; k++) o[k] = v[k] >= 0.0 ? 1 : -1;
    } else if (s2 >= s1) {
        o[i0] = v[i0] >= 0.0 ? 1 : -1;
        o[i1] = v[i1] >= 0.0 ? 1 : -1;
    } else {
        o[i0] = v[i0] >= 0.0 ? 1 : -1;
    }
    const int idx = (o[0] + 1) * 9 + (o[1] + 1) * 3 + (o[2] + 1);  // 13 is the centre
    return idx < 13 ? idx : idx - 1;
}

// relative sweep cost of a source by direction type (face, edge, corner)
__device__ inline float dir_weight(int d)
{
    int o[3];
    dir_off(d, o);
    const int nz = (o[0] != 0) + (o[1] != 0) + (o[2] != 0);
    return nz == 1 ? 1.0f : (nz == 2 ? 0.7f : 0.5f);
}

// Each particle's finest-level cell coordinates, decoded from its key into
// the three per-particle arrays that are free once the leaves are built
// (flag, small, psmall), for the walks below.
__global__ void k_tree_coords(TreeView tv)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= tv.n) return;
    uint32_t c[3];
    int b;
    key_coords(tv.keys[i], tv.top_bits, tv.depth, c, &b);
    tv.flag[i] = c[0];
    tv.small[i] = c[1];
    tv.psmall[i] = c[2];
}

// One thread per (leaf T, top cell around T's): walk that top cell's subtree,
// opening nodes within reach, and count (FILL = false) or write the leaves
// found, in a group of 27 per leaf whose offsets come from a scan of the
// counts.  The wavefront of each source is assigned afterwards.
template <bool FILL>
__global__ void k_tree_sources(TreeView tv, const CellInfo* cells, const int32_t* ncells, const BoxInfo* boxes,
                               const int32_t* cell_map, Source* src, int64_t src_cap, uint32_t* group,
                               uint32_t* status, int64_t cell_cap)
{
    // threads run over the leaves for one neighbour offset at a time: the
    // lanes of a wavefront walk the same offset from consecutive (nearby)
    // leaves, so their walks are alike; the counts stay leaf-major (g)
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= 27 * cell_cap) return;
    const int oi = (int)(k / cell_cap);
    const int64_t t = k - (int64_t)oi * cell_cap;
    const int64_t g = t * 27 + oi;
    if (t >= *ncells) return;
    const CellInfo T = cells[t];
    const BoxInfo& B = boxes[T.box];
    const int D = tv.depth;
    // coordinates in finest-level units stay below 2^23 (at most 1023 top
    // cells of 2^12 finest units per axis, and one period of shift): int32
    const int sT = 1 << (D - T.level);
    const double ef[3] = {ldexp(B.e[0], -D), ldexp(B.e[1], -D), ldexp(B.e[2], -D)};
    const double HT = T.hlim;
    const int64_t base = FILL ? (int64_t)group[g] : 0;
    int cnt = 0;
    const int o[3] = {oi / 9 - 1, (oi / 3) % 3 - 1, oi % 3 - 1};
    int tc[3];
    int shift[3];
    for (int d = 0; d < 3; d++) {
        int v = (T.c[d] >> D) + o[d];
        shift[d] = 0;
        if (v < 0) { v += B.nc[d]; shift[d] = -(B.nc[d] << D); }
        else if (v >= B.nc[d]) { v -= B.nc[d]; shift[d] = B.nc[d] << D; }
        tc[d] = v;
    }
    const int32_t m0 = cell_map[B.map_off + ((int64_t)tc[0] * B.nc[1] + tc[1]) * B.nc[2] + tc[2]];
    if (m0 >= 0) {
        int stack[kTreeStack];
        int sp = 0;
        stack[sp++] = m0;  // node index in the low 27 bits, level above
        while (sp > 0) {
            const int e = stack[--sp];
            const int l = e >> 27, m = e & ((1 << 27) - 1);
            const int64_t lo = (int64_t)l * tv.stride + m;
            const uint32_t start = tv.node_start[lo], end = tv.node_start[lo + 1];
            // the node's finest-level coordinates, from its first particle's
            // (decoded once per build by k_tree_coords)
            const uint32_t cf[3] = {tv.flag[start], tv.small[start], tv.psmall[start]};
            const int sN = 1 << (D - l);
            double dist2 = 0.0;
            int cn[3];
            for (int d = 0; d < 3; d++) {
                cn[d] = (int)((cf[d] >> (D - l)) << (D - l)) + shift[d];
                const int a0 = T.c[d], a1 = T.c[d] + sT, b0 = cn[d], b1 = cn[d] + sN;
                const int gap = b0 > a1 ? b0 - a1 : (a0 > b1 ? a0 - b1 : 0);
                const double gd = (double)gap * ef[d];
                dist2 += gd * gd;
            }
            const double R = fmax(HT, (double)tv.node_H[lo]);
            if (dist2 >= R * R) continue;
            const uint8_t fl = tv.node_flag[lo];
            if (fl & NODE_SPLIT) {
                const uint32_t* no = tv.node_of + (int64_t)(l + 1) * tv.n;
                const uint32_t c0 = no[start], c1 = no[end - 1];
                if (sp + (int)(c1 - c0 + 1) > kTreeStack) { atomicOr(status, ST_CAPACITY); continue; }
                for (uint32_t c = c0; c <= c1; c++) stack[sp++] = ((l + 1) << 27) | (int)c;
                continue;
            }
            const int32_t q = tv.node_leaf[lo];
            if (q < 0) continue;  // not reachable for a live tree
            if (FILL) {
                Source s;
                s.cell = q;
                s.wave = 0;
                s.ox = (int16_t)(cn[0] - T.c[0]);
                s.oy = (int16_t)(cn[1] - T.c[1]);
                s.oz = (int16_t)(cn[2] - T.c[2]);
                if (q == (int32_t)t && oi == 13) {
                    s.dir = (int8_t)kSelfDir;
                    s.wave = (int8_t)kAllWaves;
                } else {
                    // direction between the centres, in length units
                    s.dir = (int8_t)nearest_dir((double)(2 * cn[0] + sN - 2 * T.c[0] - sT) * ef[0],
                                                (double)(2 * cn[1] + sN - 2 * T.c[1] - sT) * ef[1],
                                                (double)(2 * cn[2] + sN - 2 * T.c[2] - sT) * ef[2]);
                }
                if (base + cnt < src_cap) src[base + cnt] = s;
                else atomicOr(status, ST_CAPACITY);
            }
            cnt++;
        }
    }
    if (!FILL) group[g] = (uint32_t)cnt;
}

// Per leaf: its list's offset and length, and the wavefront of each source,
// greedily to the least loaded (cost: source count by direction type).  One
// wavefront per leaf: its lanes load the costs of 64 sources at once, then
// the greedy pass walks them in order from registers (readlane).
constexpr int FIN_THREADS = 256;
__global__ __launch_bounds__(FIN_THREADS) void k_src_finish(const CellInfo* cells, const int32_t* ncells,
                                                           const uint32_t* group, Source* src, int64_t src_cap,
                                                           int32_t* src_off, int32_t* src_count)
{
    const int lane = threadIdx.x & (kWave - 1);
    const int64_t nwaves = (int64_t)gridDim.x * (FIN_THREADS / kWave);
    const int64_t nc = *ncells;
    for (int64_t t = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / kWave; t < nc; t += nwaves) {
        const int64_t b = group[27 * t], e = group[27 * t + 27];
        if (lane == 0) {
            src_off[t] = (int32_t)b;
            src_count[t] = (int32_t)(e - b);
        }
        float cost[kSweepWaves] = {0.f, 0.f, 0.f, 0.f};   // the same in every lane
        const int64_t end = e < src_cap ? e : src_cap;
        for (int64_t c0 = b; c0 < end; c0 += kWave) {
            const int64_t k = c0 + lane;
            int dir = kSelfDir;
            float my = 0.f;
            if (k < end) {
                const Source sk = src[k];
                dir = sk.dir;
                if (dir != kSelfDir) my = (float)cells[sk.cell].count * dir_weight(dir);
            }
            const int m = (int)(end - c0 < kWave ? end - c0 : kWave);
            int mine = 0;
            for (int i = 0; i < m; i++) {
                if (__builtin_amdgcn_readlane(dir, i) == kSelfDir) continue;
                int wv = 0;
                for (int w = 1; w < kSweepWaves; w++) if (cost[w] < cost[wv]) wv = w;
                cost[wv] += __int_as_float(__builtin_amdgcn_readlane(__float_as_int(my), i));
                if (lane == i) mine = wv;
            }
            if (k < end && dir != kSelfDir) src[k].wave = (int8_t)mine;
        }
    }
}

// h from the local number density: the particle count of the deepest node
// around the particle holding at least 2 n_ngb particles, over its volume;
// the box's mean density where even its top cell holds fewer
__global__ void k_estimate_h(TreeView tv, const BoxInfo* boxes, double n_ngb, double* h)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= tv.n) return;
    uint32_t cf[3];
    int b;
    key_coords(tv.keys[i], tv.top_bits, tv.depth, cf, &b);
    const BoxInfo& B = boxes[b];
    double density = (double)B.n / (B.L[0] * B.L[1] * B.L[2]);
    for (int l = tv.depth; l >= 0; l--) {
        const uint32_t m = tv.node_of[(int64_t)l * tv.n + i];
        const uint32_t* ns = tv.node_start + (int64_t)l * tv.stride;
        const double cnt = (double)(ns[m + 1] - ns[m]);
        if (cnt >= 2.0 * n_ngb) {
            density = cnt / (ldexp(B.e[0], -l) * ldexp(B.e[1], -l) * ldexp(B.e[2], -l));
            break;
        }
    }
    // a periodic box holds three cells of edge >= h at most
    const double cap = 0.99 * fmin(B.L[0], fmin(B.L[1], B.L[2])) / 3.0;
    h[tv.perm[i]] = fmin(cbrt(3.0 * n_ngb / (4.0 * kPi * density)), cap);
}

// ---------------------------------------------------------------- host launchers
static inline dim3 grid_for(int64_t n) { return dim3((unsigned)((n + 255) / 256)); }

void launch_tree(const Particles& p, const TreeView& tv, const BoxInfo* boxes, int split_count, double split_frac,
                 double h_margin, uint32_t* scan_scratch, hipStream_t st)
{
    (void)h_margin;
    const int64_t n = tv.n;
    if (n <= 0) return;
    hipLaunchKernelGGL(k_tree_chg, grid_for(n), dim3(256), 0, st, tv.keys, n, tv.depth, tv.chg);
    hipLaunchKernelGGL(k_small_levels, grid_for(n), dim3(256), 0, st, tv, boxes, p.h);
    for (int l = 0; l <= tv.depth; l++) {
        hipLaunchKernelGGL(k_lvl_prep, grid_for(n), dim3(256), 0, st, tv, l);
        exclusive_scan2(tv.flag, tv.scan, (uint32_t*)(tv.nnodes + l), tv.small, tv.psmall, tv.psmall + n, n,
                        scan_scratch, st);
        hipLaunchKernelGGL(k_lvl_nodes, grid_for(n), dim3(256), 0, st, tv, l);
        hipLaunchKernelGGL(k_lvl_split, grid_for(n), dim3(256), 0, st, tv, l, split_count, split_frac);
    }
    for (int l = tv.depth; l >= 0; l--)
        hipLaunchKernelGGL(k_lvl_hmax, grid_for(n), dim3(256), 0, st, tv, p.h, l);
}

void launch_tree_cells(const TreeView& tv, const BoxInfo* boxes, CellInfo* cells, int32_t* cell_map,
                       int64_t map_total, uint32_t* cell_of, int32_t* ncells, double h_margin,
                       uint32_t* scan_scratch, hipStream_t st)
{
    const int64_t n = tv.n;
    if (n <= 0) return;
    hipLaunchKernelGGL(k_leaf_flags, grid_for(n), dim3(256), 0, st, tv);
    exclusive_scan(tv.flag, tv.scan, n, scan_scratch, (uint32_t*)ncells, st);
    hipLaunchKernelGGL(k_leaf_cells, grid_for(n), dim3(256), 0, st, tv, boxes, cells, cell_of, h_margin);
    for (int l = tv.depth; l >= 0; l--)
        hipLaunchKernelGGL(k_lvl_H, grid_for(n), dim3(256), 0, st, tv, cells, l);
    launch_fill_i32(cell_map, map_total, -1, st);
    hipLaunchKernelGGL(k_top_map, grid_for(n), dim3(256), 0, st, tv, boxes, cell_map);
}

void launch_tree_sources(const TreeView& tv, const CellInfo* cells, const int32_t* ncells, const BoxInfo* boxes,
                         const int32_t* cell_map, Source* src, int64_t src_cap, int32_t* src_off,
                         int32_t* src_count, uint32_t* group, uint32_t* status, uint32_t* scan_scratch,
                         int64_t cell_cap, hipStream_t st)
{
    if (cell_cap <= 0) return;
    hipLaunchKernelGGL(k_tree_coords, grid_for(tv.n), dim3(256), 0, st, tv);
    const int64_t ng = 27 * cell_cap;
    hipLaunchKernelGGL(k_tree_sources<false>, grid_for(ng), dim3(256), 0, st, tv, cells, ncells, boxes, cell_map,
                       src, src_cap, group, status, cell_cap);
    exclusive_scan(group, group, ng, scan_scratch, group + ng, st);
    hipLaunchKernelGGL(k_tree_sources<true>, grid_for(ng), dim3(256), 0, st, tv, cells, ncells, boxes, cell_map,
                       src, src_cap, group, status, cell_cap);
    // one wavefront per leaf; leaves number at most cell_cap, the grid strides over them
    const int64_t fb = (cell_cap + FIN_THREADS / kWave - 1) / (FIN_THREADS / kWave);
    hipLaunchKernelGGL(k_src_finish, dim3((unsigned)(fb < 2048 ? fb : 2048)), dim3(FIN_THREADS), 0, st, cells,
                       ncells, group, src, src_cap, src_off, src_count);
}

void launch_estimate_h(const TreeView& tv, const BoxInfo* boxes, double n_ngb, double* h, int64_t n,
                       hipStream_t st)
{
    if (n <= 0) return;
    hipLaunchKernelGGL(k_estimate_h, grid_for(n), dim3(256), 0, st, tv, boxes, n_ngb, h);
}

}  // namespace sph
