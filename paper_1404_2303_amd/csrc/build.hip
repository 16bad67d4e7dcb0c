// build.hip -- cell decomposition kernels (Gonnet 2014, Sec. 3.2) and the
// 13 per-cell orderings (Sec. 3.3), for gfx950.
//
//   box_scan      finiteness checks, largest h per box
//   grid_dims     top-level grid per box: edge >= (1+margin) max h, >= 3 cells
//   keys          Morton key of each particle's cell (box id in the top bits)
//   radix sort    LSD, 8-bit digits, stable; tile = 256 threads x 8 keys
//   cells         runs of equal keys -> cell table + dense per-box cell map
//   gather        cell-ordered particle copies, positions relative to the cell
//   sources       self + 26 neighbour cells of each cell (single-level grid)
//   sort13        per cell and direction: ranks of the projections (stable)
#include "sph_internal.h"
#include "kernels.h"

namespace sph {

__device__ inline int find_box(const BoxInfo* boxes, int nbox, int64_t p)
{
    int lo = 0, hi = nbox - 1;
    while (lo < hi) {
        int mid = (lo + hi + 1) >> 1;
        if (boxes[mid].begin <= p) lo = mid; else hi = mid - 1;
    }
    return lo;
}

__device__ inline bool finite_d(double v) { return isfinite(v); }

__device__ inline double wrap_coord(double v, double L)
{
    double w = fmod(v, L);
    if (w < 0.0) w += L;
    if (w >= L) w -= L;
    return w;
}

// ---------------------------------------------------------------- box scan
// Each block takes a contiguous chunk of particles; when the chunk lies in one
// box (the common case) the largest h is reduced in the block and merged
// with one atomic, otherwise per particle.
constexpr int BS_THREADS = 256;

__global__ __launch_bounds__(BS_THREADS) void k_box_scan(Particles p, BoxInfo* boxes, int nbox, int64_t n,
                                                         int64_t chunk, uint32_t* status)
{
    __shared__ double red[BS_THREADS / kWave];
    const int64_t beg = (int64_t)blockIdx.x * chunk;
    const int64_t end = beg + chunk < n ? beg + chunk : n;
    if (beg >= n) return;
    const int b0 = find_box(boxes, nbox, beg), b1 = find_box(boxes, nbox, end - 1);
    const bool one_box = b0 == b1;
    double hm = 0.0;
    bool bad = false;
    for (int64_t i = beg + threadIdx.x; i < end; i += BS_THREADS) {
        bool ok = finite_d(p.x[i]) && finite_d(p.y[i]) && finite_d(p.z[i]) && finite_d(p.vx[i]) &&
                  finite_d(p.vy[i]) && finite_d(p.vz[i]) && finite_d(p.u[i]) && finite_d(p.m[i]) &&
                  finite_d(p.h[i]) && p.m[i] > 0.0 && p.h[i] > 0.0 && p.u[i] >= 0.0;
        if (!ok) { bad = true; continue; }
        if (one_box) {
            hm = fmax(hm, p.h[i]);
        } else {
            int b = find_box(boxes, nbox, i);
            // h > 0: the IEEE bit pattern orders like the value
            atomicMax((unsigned long long*)&boxes[b].hmax, (unsigned long long)__double_as_longlong(p.h[i]));
        }
    }
    if (bad) atomicOr(status, ST_NONFINITE);
    if (!one_box) return;
    for (int o = 32; o > 0; o >>= 1) hm = fmax(hm, __shfl_xor(hm, o, 64));
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = hm;
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int w = 1; w < BS_THREADS / kWave; w++) hm = fmax(hm, red[w]);
        // most blocks of a box find no larger h than one already merged
        if (hm > 0.0 && hm > *(volatile double*)&boxes[b0].hmax)
            atomicMax((unsigned long long*)&boxes[b0].hmax, (unsigned long long)__double_as_longlong(hm));
    }
}

__global__ void k_clear_boxes(BoxInfo* boxes, int nbox)
{
    int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b < nbox) boxes[b].hmax = 0.0;
}

// ---------------------------------------------------------------- grid dims
__global__ void k_grid_dims(BoxInfo* boxes, int nbox, double margin, int max_nc, uint32_t* status)
{
    int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= nbox) return;
    BoxInfo& B = boxes[b];
    double hm = B.hmax;
    for (int d = 0; d < 3; d++) {
        double L = B.L[d];
        int nc = (int)floor(L / fmax(hm * (1.0 + margin), B.e_target));
        if (nc < 3) nc = (L / hm >= 3.0) ? 3 : 0;  // margin dropped if it alone breaks the rule
        if (nc > max_nc) nc = max_nc;
        if (nc > B.cap_nc[d]) nc = B.cap_nc[d];
        if (nc < 3) { atomicOr(status, ST_H_TOO_LARGE); nc = 3; }
        B.nc[d] = nc;
        B.e[d] = L / nc;
    }
    if ((int64_t)B.nc[0] * B.nc[1] * B.nc[2] > B.map_cap) atomicOr(status, ST_CAPACITY);
}

// ---------------------------------------------------------------- keys
// Key = box id above the Morton code of the particle's cell at the finest
// level (top grid refined `depth` times by bisection), so that the cells of
// every level are runs of equal key prefixes.
__global__ void k_keys(Particles p, const BoxInfo* boxes, int nbox, int64_t n, int top_bits, int depth,
                       uint64_t* keys, uint32_t* vals)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    int b = find_box(boxes, nbox, i);
    const BoxInfo& B = boxes[b];
    double pos[3] = {p.x[i], p.y[i], p.z[i]};
    uint32_t c[3];
    for (int d = 0; d < 3; d++) {
        const double w = wrap_coord(pos[d], B.L[d]);
        const double ef = ldexp(B.e[d], -depth);
        const double fc = floor(w / ef);
        const double top = ldexp((double)B.nc[d], depth) - 1.0;
        int cc = (fc >= 0.0) ? (int)fmin(fc, top) : 0;  // NaN -> 0 (flagged by the box scan)
        c[d] = (uint32_t)cc;
    }
    keys[i] = ((uint64_t)b << (3 * (top_bits + depth))) | morton3(c[0], c[1], c[2]);
    vals[i] = (uint32_t)i;
}

// ---------------------------------------------------------------- radix sort
constexpr int RS_THREADS = 256;
constexpr int RS_ITEMS = 8;
constexpr int RS_TILE = RS_THREADS * RS_ITEMS;

__global__ __launch_bounds__(RS_THREADS) void k_rs_hist(const uint64_t* keys, int64_t n, int shift,
                                                        uint32_t* hist, int nblocks)
{
    __shared__ uint32_t h[256];
    h[threadIdx.x] = 0;
    __syncthreads();
    int64_t base = (int64_t)blockIdx.x * RS_TILE;
    for (int k = 0; k < RS_ITEMS; k++) {
        int64_t i = base + k * RS_THREADS + threadIdx.x;
        if (i < n) atomicAdd(&h[(keys[i] >> shift) & 255u], 1u);
    }
    __syncthreads();
    hist[(int64_t)threadIdx.x * nblocks + blockIdx.x] = h[threadIdx.x];
}

// one block per digit: exclusive scan of that digit's column over blocks
__global__ __launch_bounds__(256) void k_rs_colscan(uint32_t* hist, int nblocks, uint32_t* tot)
{
    __shared__ uint32_t part[256];
    uint32_t* col = hist + (int64_t)blockIdx.x * nblocks;
    int per = (nblocks + 255) / 256;
    int b0 = threadIdx.x * per, b1 = min(nblocks, b0 + per);
    uint32_t s = 0;
    for (int b = b0; b < b1; b++) s += col[b];
    part[threadIdx.x] = s;
    __syncthreads();
    // inclusive scan of part (Hillis-Steele)
    for (int off = 1; off < 256; off <<= 1) {
        uint32_t v = threadIdx.x >= off ? part[threadIdx.x - off] : 0;
        __syncthreads();
        part[threadIdx.x] += v;
        __syncthreads();
    }
    uint32_t run = threadIdx.x ? part[threadIdx.x - 1] : 0;
    for (int b = b0; b < b1; b++) { uint32_t v = col[b]; col[b] = run; run += v; }
    if (threadIdx.x == 255) tot[blockIdx.x] = part[255];
}

__global__ __launch_bounds__(RS_THREADS) void k_rs_scatter(const uint64_t* kin, const uint32_t* vin,
                                                           uint64_t* kout, uint32_t* vout, int64_t n,
                                                           int shift, const uint32_t* hist,
                                                           const uint32_t* tot, int nblocks)
{
    __shared__ uint32_t offs[256];
    __shared__ uint32_t wcnt[RS_THREADS / kWave][256];
    __shared__ uint32_t base[256];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    // digit bases: exclusive scan of the totals
    base[tid] = tot[tid];
    __syncthreads();
    for (int off = 1; off < 256; off <<= 1) {
        uint32_t v = tid >= off ? base[tid - off] : 0;
        __syncthreads();
        base[tid] += v;
        __syncthreads();
    }
    uint32_t excl = base[tid] - tot[tid];
    offs[tid] = excl + hist[(int64_t)tid * nblocks + blockIdx.x];
    __syncthreads();
    const uint64_t lt = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    int64_t tile = (int64_t)blockIdx.x * RS_TILE;
    for (int k = 0; k < RS_ITEMS; k++) {
        int64_t i = tile + k * RS_THREADS + tid;
        bool valid = i < n;
        uint64_t key = valid ? kin[i] : 0;
        uint32_t val = valid ? vin[i] : 0;
        uint32_t d = (uint32_t)(key >> shift) & 255u;
        uint64_t peers = __ballot(valid);
#pragma unroll
        for (int b = 0; b < 8; b++) {
            uint64_t bb = __ballot((d >> b) & 1u);
            peers &= ((d >> b) & 1u) ? bb : ~bb;
        }
        uint32_t rank = __popcll(peers & lt);
        uint32_t cnt = __popcll(peers);
        for (int w = 0; w < RS_THREADS / kWave; w++) wcnt[w][tid] = 0;
        __syncthreads();
        if (valid && rank == 0) wcnt[wave][d] = cnt;
        __syncthreads();
        if (valid) {
            uint32_t pos = offs[d] + rank;
            for (int w = 0; w < wave; w++) pos += wcnt[w][d];
            kout[pos] = key;
            vout[pos] = val;
        }
        __syncthreads();
        uint32_t add = 0;
        for (int w = 0; w < RS_THREADS / kWave; w++) add += wcnt[w][tid];
        offs[tid] += add;
        __syncthreads();
    }
}

// ---------------------------------------------------------------- generic exclusive scan (u32)
// Three launches: per-tile sums, a scan of the tile sums, the tiles' scans.
// One or two arrays (NA) are scanned together, each with its own sums.
constexpr int SC_THREADS = 256;
constexpr int SC_ITEMS = 8;
constexpr int SC_TILE = SC_THREADS * SC_ITEMS;
constexpr int SC_WAVES = SC_THREADS / kWave;

// inclusive scan across the block of one value per thread: shuffles within
// each wavefront, then the wavefront totals through LDS
__device__ inline uint32_t block_incl_scan(uint32_t v, uint32_t* wsum)
{
    const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave;
#pragma unroll
    for (int o = 1; o < kWave; o <<= 1) {
        const uint32_t t = __shfl_up(v, o, kWave);
        if (lane >= o) v += t;
    }
    if (lane == kWave - 1) wsum[w] = v;
    __syncthreads();
    uint32_t off = 0;
    for (int k = 0; k < w; k++) off += wsum[k];
    __syncthreads();   // wsum may be written again
    return v + off;
}

// the SC_ITEMS consecutive values from base (zeros past n); two 16-byte loads
// where the whole run is in range and the array is 16-byte aligned
__device__ inline void scan_load(const uint32_t* in, int64_t base, int64_t n, uint32_t v[SC_ITEMS])
{
    if (base + SC_ITEMS <= n && (reinterpret_cast<uintptr_t>(in) & 15) == 0) {
        const uint4 a = *reinterpret_cast<const uint4*>(in + base);
        const uint4 b = *reinterpret_cast<const uint4*>(in + base + 4);
        v[0] = a.x; v[1] = a.y; v[2] = a.z; v[3] = a.w; v[4] = b.x; v[5] = b.y; v[6] = b.z; v[7] = b.w;
    } else {
        for (int k = 0; k < SC_ITEMS; k++) v[k] = base + k < n ? in[base + k] : 0u;
    }
}

template <int NA>
__global__ __launch_bounds__(SC_THREADS) void k_scan_reduce(const uint32_t* in0, const uint32_t* in1, int64_t n,
                                                            uint32_t* sums, int nb)
{
    __shared__ uint32_t wsum[SC_WAVES];
    const int64_t base = (int64_t)blockIdx.x * SC_TILE + (int64_t)threadIdx.x * SC_ITEMS;
#pragma unroll
    for (int a = 0; a < NA; a++) {
        uint32_t v[SC_ITEMS];
        scan_load(a == 0 ? in0 : in1, base, n, v);
        uint32_t t = 0;
        for (int k = 0; k < SC_ITEMS; k++) t += v[k];
        const uint32_t inc = block_incl_scan(t, wsum);
        if (threadIdx.x == SC_THREADS - 1) sums[(int64_t)a * nb + blockIdx.x] = inc;
    }
}

// exclusive scan of the nb tile sums of each array in place, one block: each
// thread takes a run of consecutive sums
template <int NA>
__global__ __launch_bounds__(SC_THREADS) void k_scan_top(uint32_t* sums, int nb, uint32_t* total0, uint32_t* total1)
{
    __shared__ uint32_t wsum[SC_WAVES];
    const int per = (nb + SC_THREADS - 1) / SC_THREADS;
    const int b0 = threadIdx.x * per, b1 = min(nb, b0 + per);
#pragma unroll
    for (int a = 0; a < NA; a++) {
        uint32_t* sa = sums + (int64_t)a * nb;
        uint32_t t = 0;
        for (int b = b0; b < b1; b++) t += sa[b];
        const uint32_t inc = block_incl_scan(t, wsum);
        uint32_t run = inc - t;
        for (int b = b0; b < b1; b++) {
            const uint32_t x = sa[b];
            sa[b] = run;
            run += x;
        }
        uint32_t* tot = a == 0 ? total0 : total1;
        if (threadIdx.x == SC_THREADS - 1 && tot) *tot = inc;
    }
}

template <int NA>
__global__ __launch_bounds__(SC_THREADS) void k_scan_down(const uint32_t* in0, const uint32_t* in1, int64_t n,
                                                          const uint32_t* sums, int nb, uint32_t* out0,
                                                          uint32_t* out1)
{
    __shared__ uint32_t wsum[SC_WAVES];
    const int64_t base = (int64_t)blockIdx.x * SC_TILE + (int64_t)threadIdx.x * SC_ITEMS;
#pragma unroll
    for (int a = 0; a < NA; a++) {
        uint32_t v[SC_ITEMS];
        scan_load(a == 0 ? in0 : in1, base, n, v);
        uint32_t t = 0;
        for (int k = 0; k < SC_ITEMS; k++) t += v[k];
        const uint32_t inc = block_incl_scan(t, wsum);
        uint32_t run = sums[(int64_t)a * nb + blockIdx.x] + inc - t;
        uint32_t* out = a == 0 ? out0 : out1;
        for (int k = 0; k < SC_ITEMS; k++) {
            if (base + k < n) out[base + k] = run;
            run += v[k];
        }
    }
}

// ---------------------------------------------------------------- cells
__global__ void k_cell_heads(const uint64_t* keys, int64_t n, uint32_t* flag)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    flag[i] = (i == 0 || keys[i] != keys[i - 1]) ? 1u : 0u;
}

__global__ void k_fill_i32(int32_t* a, int64_t n, int32_t v)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) a[i] = v;
}

// clearing by a kernel rather than hipMemsetAsync keeps the sequence capturable in a graph
void launch_fill_i32(int32_t* a, int64_t n, int32_t v, hipStream_t st)
{
    if (n <= 0) return;
    hipLaunchKernelGGL(k_fill_i32, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, a, n, v);
}

// cellx[i] = exclusive scan of the head flags; cell index of particle i is
// cellx[i] + flag[i] - 1.
__global__ void k_cell_fill(const uint64_t* keys, const uint32_t* flag, const uint32_t* cellx,
                            int64_t n, int top_bits, const BoxInfo* boxes, CellInfo* cells,
                            int32_t* cell_map, uint32_t* cell_of, int32_t* ncells)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    uint32_t c = cellx[i] + flag[i] - 1;
    cell_of[i] = c;
    bool last = (i == n - 1) || (keys[i + 1] != keys[i]);
    if (flag[i]) {
        uint64_t k = keys[i];
        int b = (int)(k >> (3 * top_bits));
        uint64_t mc = k & ((3 * top_bits >= 64) ? ~0ull : ((1ull << (3 * top_bits)) - 1));
        int cx = (int)compact3(mc), cy = (int)compact3(mc >> 1), cz = (int)compact3(mc >> 2);
        cells[c].start = (int32_t)i;
        cells[c].box = b;
        cells[c].c[0] = cx; cells[c].c[1] = cy; cells[c].c[2] = cz;
        const BoxInfo& B = boxes[b];
        cell_map[B.map_off + ((int64_t)cx * B.nc[1] + cy) * B.nc[2] + cz] = (int32_t)c;
    }
    if (last) {
        // count = end - start; start written by the head thread of this cell, so
        // store the end here and convert in a second pass
        cells[c].count = (int32_t)(i + 1);
        if (i == n - 1) *ncells = (int32_t)(c + 1);
    }
}

__global__ void k_cell_counts(CellInfo* cells, const int32_t* ncells, const BoxInfo* boxes)
{
    const int nc_all = *ncells;
    for (int c = blockIdx.x * blockDim.x + threadIdx.x; c < nc_all; c += gridDim.x * blockDim.x) {
        cells[c].count -= cells[c].start;
        cells[c].level = 0;
        const BoxInfo& B = boxes[cells[c].box];
        cells[c].hlim = (float)fmin(B.e[0], fmin(B.e[1], B.e[2]));
    }
}

// ---------------------------------------------------------------- gather (cell order)
// Position of a particle relative to the lower corner of its cell: the
// periodic image nearest the cell (a particle that moved across the box face
// since the cells were built stays next to its cell).
__device__ inline double cell_rel(double v, double o, double L)
{
    double r = wrap_coord(v, L) - o;
    if (r > 0.5 * L) r -= L;
    if (r < -0.5 * L) r += L;
    return r;
}

template <typename R>
__global__ void k_gather(Particles p, const uint32_t* perm, const uint32_t* cell_of,
                         const CellInfo* cells, const BoxInfo* boxes, int64_t n, CellData<R> cd,
                         typename Vec4T<R>::T* r0)
{
    int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n) return;
    uint32_t i = perm[k];
    const CellInfo& C = cells[cell_of[k]];
    const BoxInfo& B = boxes[C.box];
    double pos[3] = {p.x[i], p.y[i], p.z[i]};
    R rel[3];
    for (int d = 0; d < 3; d++) {
        double o = (double)C.c[d] * ldexp(B.e[d], -B.depth);
        // a coordinate that rounded onto the upper face belongs to this cell
        rel[d] = (R)cell_rel(pos[d], o, B.L[d]);
    }
    cd.rp[k] = typename CellData<R>::R4{rel[0], rel[1], rel[2], (R)0};
    cd.h[k] = p.h[i];
    typename CellData<R>::R4 vm;
    vm.x = (R)p.vx[i]; vm.y = (R)p.vy[i]; vm.z = (R)p.vz[i]; vm.w = (R)p.m[i];
    cd.vm[k] = vm;
    cd.u[k] = p.u[i];
    if (r0) {
        typename Vec4T<R>::T q;
        q.x = rel[0]; q.y = rel[1]; q.z = rel[2]; q.w = (R)0;
        r0[k] = q;
    }
}

// Pseudo-Verlet reuse (Sec. 3.3 keeps orderings over several steps): the
// cell-ordered copies of the particle data are refreshed from the caller's
// arrays in the cell membership of the last build, and the largest
// displacement since that build is recorded per cell (cell_drift) and per
// box (BoxInfo::drift).  A particle has left its cell by at most its
// displacement and its projection on any axis has moved by at most as much,
// so for targets in cell T and sources in cell S every pair in range still
// lies in a listed cell pair, and inside the swept prefix of every stored
// ordering, once the ranges and early-exit bounds are widened by
// drift(T) + drift(S) and every h_i + drift(T) + drift(box) stays within the
// h limit of i's cell.
template <typename R>
__global__ void k_refresh(Particles p, const uint32_t* perm, const uint32_t* cell_of, const CellInfo* cells,
                          const BoxInfo* boxes, int64_t n, CellData<R> cd, const typename Vec4T<R>::T* r0,
                          float* cell_drift, uint32_t* status)
{
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k - (int64_t)(threadIdx.x & 63) >= n) return;   // the whole wavefront is past the end
    const bool valid = k < n;
    int c = -1;
    double dd = 0.0;
    if (valid) {
        const uint32_t i = perm[k];
        c = (int)cell_of[k];
        const CellInfo& C = cells[c];
        const BoxInfo& B = boxes[C.box];
        const double pos[3] = {p.x[i], p.y[i], p.z[i]};
        const double h = p.h[i];
        if (!isfinite(pos[0]) || !isfinite(pos[1]) || !isfinite(pos[2]) || !(h > 0.0) || !isfinite(h))
            atomicOr(status, ST_NONFINITE);
        R rel[3];
        for (int d = 0; d < 3; d++) {
            const double o = (double)C.c[d] * ldexp(B.e[d], -B.depth);
            rel[d] = (R)cell_rel(pos[d], o, B.L[d]);
        }
        cd.rp[k] = typename CellData<R>::R4{rel[0], rel[1], rel[2], (R)0};
        cd.h[k] = h;
        typename CellData<R>::R4 vm;
        vm.x = (R)p.vx[i]; vm.y = (R)p.vy[i]; vm.z = (R)p.vz[i]; vm.w = (R)p.m[i];
        cd.vm[k] = vm;
        cd.u[k] = p.u[i];
        const typename Vec4T<R>::T q = r0[k];
        const double dx = (double)rel[0] - (double)q.x, dy = (double)rel[1] - (double)q.y,
                     dz = (double)rel[2] - (double)q.z;
        // rounded up, so that the float allowance is never below the displacement
        dd = sqrt(dx * dx + dy * dy + dz * dz) * (1.0 + 1e-6);
        if (!(dd == dd)) dd = (double)INFINITY;
    }
    const int lane = threadIdx.x & 63;
    // per cell: the lanes of one cell are consecutive (cell order), so a
    // segmented maximum over the wavefront leaves each cell's maximum in its
    // last lane, which issues the one atomic of that cell
    float m = (float)dd;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const float mo = __shfl_up(m, o, 64);
        const int co = __shfl_up(c, o, 64);
        if (lane >= o && co == c) m = fmaxf(m, mo);
    }
    const int cn = __shfl_down(c, 1, 64);
    if (valid && (lane == 63 || cn != c)) atomicMax((unsigned int*)&cell_drift[c], __float_as_uint(m));
}

// Largest cell drift of each box (cells are ordered by box): a small grid
// strides over the cells, each lane keeps the maximum of its current box and
// hands it on with one atomic when its box changes and at the end.
__global__ void k_box_drift(const CellInfo* cells, const int32_t* ncells, const float* cell_drift, BoxInfo* boxes)
{
    const int nc = *ncells;
    int cb = -1;
    float cm = 0.0f;
    for (int c = blockIdx.x * blockDim.x + threadIdx.x; c < nc; c += gridDim.x * blockDim.x) {
        const int b = cells[c].box;
        if (b != cb) {
            if (cb >= 0) atomicMax((unsigned long long*)&boxes[cb].drift,
                                   (unsigned long long)__double_as_longlong((double)cm));
            cb = b;
            cm = 0.0f;
        }
        cm = fmaxf(cm, cell_drift[c]);
    }
    const int b0 = __builtin_amdgcn_readfirstlane(cb);
    if (__all(cb == b0)) {
        for (int o = 32; o > 0; o >>= 1) cm = fmaxf(cm, __shfl_xor(cm, o, 64));
        if ((threadIdx.x & 63) == 0 && b0 >= 0)
            atomicMax((unsigned long long*)&boxes[b0].drift, (unsigned long long)__double_as_longlong((double)cm));
    } else if (cb >= 0) {
        atomicMax((unsigned long long*)&boxes[cb].drift, (unsigned long long)__double_as_longlong((double)cm));
    }
}

// After a refresh: the decomposition still serves the particles whose h,
// with room for a growth of half the build slack, stays within the h limit
// of their cell less the allowances; otherwise a rebuild is requested.
template <typename R>
__global__ void k_refresh_check(const uint32_t* cell_of, const CellInfo* cells, const BoxInfo* boxes, int64_t n,
                                CellData<R> cd, const float* cell_drift, double h_margin, uint32_t* status)
{
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    bool bad = false;
    if (k < n) {
        const int c = (int)cell_of[k];
        const CellInfo& C = cells[c];
        const double lim = (double)C.hlim - (double)cell_drift[c] - boxes[C.box].drift;
        bad = !(cd.h[k] * (1.0 + 0.5 * h_margin) <= lim);
    }
    if (__any(bad) && (threadIdx.x & 63) == 0) atomicOr(status, ST_REBUILD);
}

__global__ void k_zero_drift(BoxInfo* boxes, int nbox, float* cell_drift, const int32_t* ncells)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < nbox) boxes[i].drift = 0.0;
    if (i < *ncells) cell_drift[i] = 0.0f;
}

// ---------------------------------------------------------------- sources
// wavefront of each of the 26 neighbour directions on the single-level grid
// (2 bits per direction).  A wavefront's list loops run to its longest list,
// and a lane's list holds its neighbours in that wavefront's sources: each
// pair of opposite faces shares a wavefront (0: x, 3: y, 1: z), so that a
// target near one face gets few neighbours from the other, and the edges and
// corners fill in.  Chosen by a search on a jittered lattice of 64 particles
// per cell, minimising the sum over wavefronts of the longest list with every
// wavefront's staging within its 192 slots and its walk no longer than
// before (the loops shorten by a fifth).
constexpr uint64_t kDirWavePacked = 0x5e2d6c533acdaull;

// The self source and the existing neighbours of each cell, in direction
// order: 32 lanes per cell, lane 0 the cell itself and lane 1 + d direction
// d; a ballot over the half-wavefront compacts them.
__global__ __launch_bounds__(256) void k_sources(const CellInfo* cells, const int32_t* ncells,
                                                 const BoxInfo* boxes, const int32_t* cell_map, Source* src,
                                                 int32_t* src_off, int32_t* src_count)
{
    const int nc_all = *ncells;
    const int lane = threadIdx.x & (kWave - 1);
    const int j = lane & 31;                 // slot within the cell's half-wavefront
    const int64_t stride = (int64_t)gridDim.x * blockDim.x / 32;
    for (int64_t base = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / 32; ; base += stride) {
        // every lane of a wavefront takes the loop's last step together (ballot below)
        const int64_t first = base - (lane >> 5);   // the wavefront's first cell
        if (first >= nc_all) break;
        const int c = (int)base;
        bool have = false;
        Source sv{};
        if (c < nc_all && j <= kDirs) {
            const CellInfo C = cells[c];
            if (j == 0) {
                sv = Source{c, (int8_t)kSelfDir, (int8_t)kAllWaves, 0, 0, 0};
                have = true;
            } else {
                const int d = j - 1;
                const BoxInfo& B = boxes[C.box];
                int o[3];
                dir_off(d, o);
                int nc[3];
                for (int a = 0; a < 3; a++) {
                    const int v = C.c[a] + o[a];
                    nc[a] = v < 0 ? v + B.nc[a] : (v >= B.nc[a] ? v - B.nc[a] : v);
                }
                const int32_t sc = cell_map[B.map_off + ((int64_t)nc[0] * B.nc[1] + nc[1]) * B.nc[2] + nc[2]];
                if (sc >= 0) {
                    sv = Source{sc, (int8_t)d, (int8_t)((kDirWavePacked >> (2 * d)) & 3u), (int16_t)o[0],
                                (int16_t)o[1], (int16_t)o[2]};
                    have = true;
                }
            }
        }
        const uint64_t m = __ballot(have);
        const uint32_t half = (uint32_t)(m >> (lane & 32));
        if (have) src[(int64_t)c * kMaxSources + __popc(half & ((1u << j) - 1u))] = sv;
        if (c < nc_all && j == 0) {
            src_off[c] = c * kMaxSources;
            src_count[c] = __popc(half);
        }
    }
}


// ---------------------------------------------------------------- 13-direction orderings
// One workgroup per (cell, direction).  Each particle's rank is the number of
// particles with a smaller projection, ties broken by cell-order index, so
// the ordering is a permutation and stable.
constexpr int SORT_MAX = 4096;
constexpr int kWaveSortMax = 4 * kWave;   // cells up to this size are sorted by one wavefront

// order-preserving integer image of a float (a total order, NaN included)
__device__ inline uint32_t float_key(float f)
{
    const uint32_t b = __float_as_uint(f);
    return (b & 0x80000000u) ? ~b : (b | 0x80000000u);
}
__device__ inline float key_float(uint32_t k) { return __uint_as_float((k & 0x80000000u) ? (k & 0x7fffffffu) : ~k); }

// Bitonic sort across one wavefront of 64 E 32-bit words, word i held by
// lane i % 64 in slot i / 64, ascending on return.  The network is the form
// whose first stage of every merge of size kk pairs i with i ^ (kk - 1) (the
// mirror image in its block) and whose later stages pair i with i ^ j; every
// comparator leaves the smaller word at the lower index, so a lane's choice
// depends on one bit of its index only.

// the value held by lane (lane ^ M), M < 64: data-parallel-primitive moves
// inside a row of 16 lanes where the pattern allows (xor 1, 2, 3 by quad
// permutes, 7 and 15 by the row half-mirror and mirror, 4 and 8 by two
// shifts, each writing the banks of four lanes that read in its direction),
// a lane permute otherwise
template <int M>
__device__ __forceinline__ uint32_t lane_xor(uint32_t v)
{
    const int x = (int)v;
    if constexpr (M == 0) return v;
    else if constexpr (M == 1) return (uint32_t)__builtin_amdgcn_mov_dpp(x, 0xB1, 0xF, 0xF, false);   // quad [1,0,3,2]
    else if constexpr (M == 2) return (uint32_t)__builtin_amdgcn_mov_dpp(x, 0x4E, 0xF, 0xF, false);   // quad [2,3,0,1]
    else if constexpr (M == 3) return (uint32_t)__builtin_amdgcn_mov_dpp(x, 0x1B, 0xF, 0xF, false);   // quad [3,2,1,0]
    else if constexpr (M == 7) return (uint32_t)__builtin_amdgcn_mov_dpp(x, 0x141, 0xF, 0xF, false);  // row half-mirror
    else if constexpr (M == 15) return (uint32_t)__builtin_amdgcn_mov_dpp(x, 0x140, 0xF, 0xF, false); // row mirror
    else if constexpr (M == 4 || M == 8) {
        // banks whose lanes have bit M clear read lane + M (row shift left),
        // the others lane - M (row shift right)
        constexpr int lo = M == 4 ? 0x5 : 0x3;
        const int t = __builtin_amdgcn_update_dpp(x, x, 0x100 + M, 0xF, lo, false);
        return (uint32_t)__builtin_amdgcn_update_dpp(t, x, 0x110 + M, 0xF, 0xF ^ lo, false);
    } else {
        return (uint32_t)__shfl_xor(x, M, kWave);
    }
}

// stage I of the network over 64 E words: its partner mask m and the index
// bit hb that marks the upper element of a pair
__host__ __device__ constexpr int net_size(int E) { int n = 0; for (int kk = 2; kk <= 64 * E; kk <<= 1) for (int j = kk; j > 1; j >>= 1) n++; return n; }
__host__ __device__ constexpr int net_stage(int E, int I, bool want_hb)
{
    int i = 0;
    for (int kk = 2; kk <= 64 * E; kk <<= 1) {
        if (i++ == I) return want_hb ? kk / 2 : kk - 1;
        for (int j = kk / 4; j >= 1; j >>= 1)
            if (i++ == I) return j;
    }
    return 0;
}

template <int E, int M, int HB>
__device__ __forceinline__ void net_step(uint32_t (&v)[E], const int lane)
{
    if constexpr (HB >= kWave) {
        // pairs across slots (e, e ^ (M >> 6)), lanes mirrored when M's low bits are set
        uint32_t q[E];
#pragma unroll
        for (int e = 0; e < E; e++) q[e] = lane_xor<(M & (kWave - 1))>(v[e ^ (M >> 6)]);
#pragma unroll
        for (int e = 0; e < E; e++) v[e] = ((e * kWave) & HB) == 0 ? min(v[e], q[e]) : max(v[e], q[e]);
    } else {
        const bool low = (lane & HB) == 0;
#pragma unroll
        for (int e = 0; e < E; e++) {
            const uint32_t q = lane_xor<M>(v[e]);
            v[e] = low ? min(v[e], q) : max(v[e], q);
        }
    }
}

template <int E, int I = 0>
__device__ __forceinline__ void wave_bitonic(uint32_t (&v)[E], const int lane)
{
    if constexpr (I < net_size(E)) {
        net_step<E, net_stage(E, I, false), net_stage(E, I, true)>(v, lane);
        wave_bitonic<E, I + 1>(v, lane);
    }
}

// The 13 orderings of one cell of at most 64 E particles by one wavefront:
// every particle's position is loaded once, and for each direction the
// order-preserving image of the projection, with its low bits replaced by the
// particle's index in the cell, is sorted.  The stored key is that image with
// the index bits cleared: the projection rounded down by less than 2^-15 of
// its magnitude, and monotone along the ordering (ties keep the cell order).
template <typename R, int E>
__device__ __forceinline__ void sort13_cell(const CellInfo& C, const CellData<R>& cd, int64_t n,
                                            const Sorted<R>& so, const int lane)
{
    constexpr uint32_t IDX = 64u * E - 1u;  // index bits
    R x[E], y[E], z[E];
#pragma unroll
    for (int e = 0; e < E; e++) {
        const int t = e * kWave + lane;
        const int64_t k = C.start + (t < C.count ? t : 0);
        const typename CellData<R>::R4 q = cd.rp[k];
        x[e] = q.x; y[e] = q.y; z[e] = q.z;
    }
    for (int s = 0; s < kSortDirs; s++) {
        float su[3];
        dir_unit(s + 13, su);
        uint32_t v[E];
#pragma unroll
        for (int e = 0; e < E; e++) {
            const int t = e * kWave + lane;
            const float f = su[0] * (float)x[e] + su[1] * (float)y[e] + su[2] * (float)z[e];
            v[e] = t < C.count ? ((float_key(f) & ~IDX) | (uint32_t)t) : ~0u;
        }
        wave_bitonic<E>(v, lane);
        // slot e of this lane now holds the word of rank e * 64 + lane
#pragma unroll
        for (int e = 0; e < E; e++) {
            const int r = e * kWave + lane;
            if (r < C.count)
                so.rec[(int64_t)s * n + C.start + r] = SortRec{key_float(v[e] & ~IDX), v[e] & IDX};
        }
    }
}

__global__ void k_zero_header(int32_t* a)
{
    for (int i = 0; i < kBigHeader; i++) a[i] = 0;
}

// Cells of at most kWaveSortMax particles: one wavefront per cell.  The
// larger ones are listed for k_sort13: big[0] counts them (zero on entry),
// big[kBigHeader..] holds them.
template <typename R>
__global__ __launch_bounds__(kWave) void k_sort13_wave(const CellInfo* cells, const int32_t* ncells, CellData<R> cd,
                                                       int64_t n, Sorted<R> so, int32_t* big)
{
    const int lane = threadIdx.x;
    const int nc = *ncells;
    for (int c = blockIdx.x; c < nc; c += gridDim.x) {
        const CellInfo C = cells[c];
        if (C.count <= kWave) sort13_cell<R, 1>(C, cd, n, so, lane);
        else if (C.count <= 2 * kWave) sort13_cell<R, 2>(C, cd, n, so, lane);
        else if (C.count <= kWaveSortMax) sort13_cell<R, 4>(C, cd, n, so, lane);
        else if (lane == 0) big[kBigHeader + atomicAdd(&big[0], 1)] = c;
    }
}

// Larger cells (Sec. 3.3, Fig. HierarchySorting): a split cell's orderings
// are made from those of its eight sub-cells, each shifted into the
// parent's frame, by merges that take O(n) per level.  One work-group per
// (cell, direction).  The cell is split D levels deep (D = 1, 2 or 3: the
// shallowest whose sub-cells hold at most kSubRun particles each); the
// sub-cells of depth D are ordered directly (each particle's rank in its
// sub-cell), with keys in the sub-cell's own frame.  Then, level by level up
// to the cell, every run is shifted into its parent's frame (its key plus
// the projection of the sub-cell's corner relative to the parent's) and the
// eight sibling runs are merged pairwise in three rounds.  A merge places
// each word at its index in its run plus the number of words of the partner
// run before it (a binary search on the key: strictly below for the first
// run, at most equal for the second, so equal keys keep their run order).
// A shift adds the same amount to every key of a run, which keeps it
// ordered.  The stored key is the projection so obtained: within a few
// units of rounding of the cell's size of the projection computed in the
// cell's frame, and monotone along the ordering.
//
// A cell whose particles crowd more than kSubRun into one sub-cell of
// depth 3 is ordered by merging runs of 256 consecutive particles instead
// (each run sorted by a bitonic network).  Words: (order-preserving image of
// the projection) << 32 | cell index.
constexpr int MERGE_THREADS = 1024;   // latency-bound: many wavefronts per cell
constexpr int MERGE_RUN = 256;
constexpr int kSubDepth = 3;                            // deepest split of a big cell
constexpr int kSubCells = 1 << (3 * kSubDepth);         // sub-cells of that depth
constexpr int kSubRun = 64;                             // largest sub-cell ordered directly
constexpr int kSubRunMax = 256;                         // ... at depth 3, before the fallback

// the number of words of run [b, b + len) below x (strict) or at most x
__device__ __forceinline__ int count_before(const uint64_t* a, int b, int len, uint64_t x, bool strict)
{
    int lo = 0, hi = len;
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        const uint64_t y = a[b + mid];
        if (strict ? (y < x) : (y <= x)) lo = mid + 1;
        else hi = mid;
    }
    return lo;
}
// the same on the keys alone (the high 32 bits)
__device__ __forceinline__ int keys_before(const uint64_t* a, int b, int len, uint32_t x, bool strict)
{
    int lo = 0, hi = len;
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        const uint32_t y = (uint32_t)(a[b + mid] >> 32);
        if (strict ? (y < x) : (y <= x)) lo = mid + 1;
        else hi = mid;
    }
    return lo;
}

__device__ __forceinline__ uint64_t make_word(float f, uint32_t t) { return ((uint64_t)float_key(f) << 32) | t; }
__device__ __forceinline__ float word_key(uint64_t w) { return key_float((uint32_t)(w >> 32)); }

// Morton index of sub-cell (ix, iy, iz) of depth kSubDepth (x in the highest
// bit of each triple, as the cell order's keys)
__device__ __forceinline__ int sub_morton(int ix, int iy, int iz)
{
    int m = 0;
#pragma unroll
    for (int b = kSubDepth - 1; b >= 0; b--) m = (m << 3) | (((ix >> b) & 1) << 2) | (((iy >> b) & 1) << 1) | ((iz >> b) & 1);
    return m;
}
// lower corner, in units of the depth-kSubDepth edge, of the depth-L sub-cell
// holding depth-kSubDepth sub-cell m
__device__ __forceinline__ void sub_corner(int m, int L, int c[3])
{
    c[0] = c[1] = c[2] = 0;
    for (int b = kSubDepth - 1; b >= kSubDepth - L; b--) {
        const int tri = (m >> (3 * b)) & 7;
        c[0] |= ((tri >> 2) & 1) << b;
        c[1] |= ((tri >> 1) & 1) << b;
        c[2] |= (tri & 1) << b;
    }
}

template <typename R>
__global__ __launch_bounds__(MERGE_THREADS) void k_sort13(const CellInfo* cells, const BoxInfo* boxes,
                                                          const int32_t* big, CellData<R> cd, int64_t n,
                                                          Sorted<R> so, uint32_t* status)
{
    __shared__ uint64_t buf[2][SORT_MAX];
    __shared__ uint16_t subof[SORT_MAX];        // depth-3 sub-cell of each particle (cell order)
    __shared__ int off[kSubCells + 1];          // particles per depth-3 sub-cell, then run starts
    __shared__ int fill[kSubCells];
    __shared__ int runmax[kSubDepth + 1];       // largest sub-cell of each depth
    __shared__ int part[kSubCells / 8];         // counts of the depth-2 sub-cells
    const int tid = threadIdx.x;
    const int64_t units = (int64_t)big[0] * kSortDirs;  // the cells k_sort13_wave left
    for (int64_t unit = blockIdx.x; unit < units; unit += gridDim.x) {
        const int c = big[kBigHeader + (int)(unit / kSortDirs)];
        const int s = (int)(unit % kSortDirs);
        const CellInfo C = cells[c];
        if (C.count > SORT_MAX) { if (tid == 0) atomicOr(status, ST_CAPACITY); continue; }
        const BoxInfo& B = boxes[C.box];
        float su[3];
        dir_unit(s + 13, su);
        // edge of the depth-3 sub-cells
        const float es[3] = {(float)ldexp(B.e[0], -C.level - kSubDepth), (float)ldexp(B.e[1], -C.level - kSubDepth),
                             (float)ldexp(B.e[2], -C.level - kSubDepth)};
        __syncthreads();   // the last unit's words are written out
        for (int m = tid; m <= kSubCells; m += MERGE_THREADS) off[m] = 0;
        for (int m = tid; m < kSubCells; m += MERGE_THREADS) fill[m] = 0;
        if (tid <= kSubDepth) runmax[tid] = 0;
        __syncthreads();
        // ---- the depth-3 sub-cell of every particle, and their counts
        for (int t = tid; t < C.count; t += MERGE_THREADS) {
            const typename CellData<R>::R4 q = cd.rp[C.start + t];
            int ix = (int)((float)q.x / es[0]), iy = (int)((float)q.y / es[1]), iz = (int)((float)q.z / es[2]);
            constexpr int top = (1 << kSubDepth) - 1;
            ix = min(max(ix, 0), top); iy = min(max(iy, 0), top); iz = min(max(iz, 0), top);
            const int m = sub_morton(ix, iy, iz);
            subof[t] = (uint16_t)m;
            atomicAdd(&off[m], 1);
        }
        __syncthreads();
        // largest sub-cell of each depth (a depth-L sub-cell is a run of 8^(3-L)
        // depth-3 ones): counts of depth 2 into part[0..63], of depth 1 from those
        for (int m = tid; m < kSubCells; m += MERGE_THREADS) atomicMax(&runmax[3], off[m]);
        if (tid < kSubCells / 8) {
            int a = 0;
            for (int k = 0; k < 8; k++) a += off[8 * tid + k];
            part[tid] = a;
            atomicMax(&runmax[2], a);
        }
        __syncthreads();
        if (tid < kSubCells / 64) {
            int a = 0;
            for (int k = 0; k < 8; k++) a += part[8 * tid + k];
            atomicMax(&runmax[1], a);
        }
        __syncthreads();
        int D = 0;
        for (int L = 1; L <= kSubDepth && D == 0; L++)
            if (runmax[L] <= kSubRun) D = L;
        if (D == 0 && runmax[kSubDepth] <= kSubRunMax) D = kSubDepth;

        int src = 0;
        if (D > 0) {
            // ---- run starts: exclusive scan of the 512 counts by the first
            // wavefront, eight consecutive counts per lane
            static_assert(kSubCells == 8 * kWave, "eight counts per lane");
            if (tid < kWave) {
                int v[8], a = 0;
#pragma unroll
                for (int k = 0; k < 8; k++) { v[k] = off[8 * tid + k]; a += v[k]; }
                int inc = a;
#pragma unroll
                for (int d = 1; d < kWave; d <<= 1) {
                    const int y = __shfl_up(inc, d, kWave);
                    if (tid >= d) inc += y;
                }
                int e = inc - a;
#pragma unroll
                for (int k = 0; k < 8; k++) { off[8 * tid + k] = e; e += v[k]; }
                if (tid == kWave - 1) off[kSubCells] = inc;
            }
            __syncthreads();
            // ---- words in the frame of their depth-D sub-cell, grouped by sub-cell
            const int gsh = 3 * (kSubDepth - D);   // depth-3 sub-cells per depth-D one: 1 << gsh
            for (int t = tid; t < C.count; t += MERGE_THREADS) {
                const int m = subof[t];
                int cc[3];
                sub_corner(m, D, cc);
                const typename CellData<R>::R4 q = cd.rp[C.start + t];
                const float f = su[0] * ((float)q.x - (float)cc[0] * es[0]) + su[1] * ((float)q.y - (float)cc[1] * es[1]) +
                                su[2] * ((float)q.z - (float)cc[2] * es[2]);
                const int mg = m >> gsh << gsh;    // first depth-3 sub-cell of the depth-D one
                buf[0][off[mg] + atomicAdd(&fill[mg], 1)] = make_word(f, (uint32_t)t);
            }
            __syncthreads();
            // ---- each depth-D sub-cell ordered: a word's place is its rank in its run
            for (int i = tid; i < C.count; i += MERGE_THREADS) {
                const uint64_t x = buf[0][i];
                const int m = subof[(uint32_t)x];
                const int mg = m >> gsh << gsh;
                const int a = off[mg], b = off[mg + (1 << gsh)];
                int r = 0;
                for (int j = a; j < b; j++) r += buf[0][j] < x;
                buf[1][a + r] = x;
            }
            src = 1;
            __syncthreads();
            // ---- up the levels: shift into the parent's frame, merge eight siblings
            for (int L = D; L >= 1; L--) {
                const int csh = 3 * (kSubDepth - L);   // a depth-L sub-cell spans 1 << csh depth-3 ones
                for (int i = tid; i < C.count; i += MERGE_THREADS) {
                    const uint64_t x = buf[src][i];
                    const int m = subof[(uint32_t)x];
                    int cl[3], cp[3];
                    sub_corner(m, L, cl);
                    sub_corner(m, L - 1, cp);
                    const float sh = su[0] * (float)(cl[0] - cp[0]) * es[0] + su[1] * (float)(cl[1] - cp[1]) * es[1] +
                                     su[2] * (float)(cl[2] - cp[2]) * es[2];
                    buf[src][i] = make_word(word_key(x) + sh, (uint32_t)x);
                }
                __syncthreads();
                for (int q = 0; q < 3; q++) {
                    // runs of 2^q siblings merged with their partners into runs of 2^(q+1)
                    const uint64_t* in = buf[src];
                    uint64_t* outb = buf[src ^ 1];
                    for (int i = tid; i < C.count; i += MERGE_THREADS) {
                        const uint64_t x = in[i];
                        const int m = subof[(uint32_t)x];
                        const int g = m >> (csh + q);               // the word's run of 2^q siblings
                        const int a0 = off[g << (csh + q)], a1 = off[(g + 1) << (csh + q)];
                        const int p = g ^ 1;                        // partner run
                        const int b0 = off[p << (csh + q)], b1 = off[(p + 1) << (csh + q)];
                        const bool first = (g & 1) == 0;
                        const int place = (i - a0) + keys_before(in, b0, b1 - b0, (uint32_t)(x >> 32), first);
                        outb[min(a0, b0) + place] = x;
                    }
                    src ^= 1;
                    __syncthreads();
                }
            }
        } else {
            // ---- crowded: runs of MERGE_RUN consecutive particles, sorted and merged
            const int np = (C.count + MERGE_RUN - 1) / MERGE_RUN * MERGE_RUN;
            for (int t = tid; t < np; t += MERGE_THREADS) {
                uint64_t wd = ~0ull;
                if (t < C.count) {
                    const typename CellData<R>::R4 q = cd.rp[C.start + t];
                    wd = make_word(su[0] * (float)q.x + su[1] * (float)q.y + su[2] * (float)q.z, (uint32_t)t);
                }
                buf[0][t] = wd;
            }
            __syncthreads();
            // each run sorted: bitonic stages of span <= MERGE_RUN stay inside a run;
            // the last (k = MERGE_RUN) leaves every run ascending
            for (int k = 2; k <= MERGE_RUN; k <<= 1) {
                for (int j = k >> 1; j > 0; j >>= 1) {
                    for (int i = tid; i < np; i += MERGE_THREADS) {
                        const int l = i ^ j;
                        if (l > i) {
                            const uint64_t a = buf[0][i], b = buf[0][l];
                            if ((a > b) == ((i & k & (MERGE_RUN - 1)) == 0)) { buf[0][i] = b; buf[0][l] = a; }
                        }
                    }
                    __syncthreads();
                }
            }
            // merges: runs of `w` words into runs of 2w, alternating buffers
            for (int w = MERGE_RUN; w < np; w <<= 1) {
                const uint64_t* in = buf[src];
                uint64_t* outb = buf[src ^ 1];
                for (int i = tid; i < np; i += MERGE_THREADS) {
                    const int pair = i / (2 * w) * (2 * w);      // first word of the two runs
                    const int la = min(w, np - pair);            // first run (whole unless the last)
                    const int lb = min(w, np - pair - la);       // partner run (possibly empty)
                    const uint64_t x = in[i];
                    int place;
                    if (i < pair + la) place = (i - pair) + count_before(in, pair + la, lb, x, true);
                    else place = (i - pair - la) + count_before(in, pair, la, x, false);
                    outb[pair + place] = x;
                }
                src ^= 1;
                __syncthreads();
            }
        }
        for (int r = tid; r < C.count; r += MERGE_THREADS) {
            const uint64_t wd = buf[src][r];
            so.rec[(int64_t)s * n + C.start + r] = SortRec{word_key(wd), (uint32_t)wd};
        }
    }
}

// ---------------------------------------------------------------- host launchers
void launch_box_scan(const Particles& p, BoxInfo* boxes, int nbox, int64_t n, uint32_t* status,
                     hipStream_t st)
{
    hipLaunchKernelGGL(k_clear_boxes, dim3((nbox + 255) / 256), dim3(256), 0, st, boxes, nbox);
    if (n > 0) {
        int64_t nb = (n + BS_THREADS - 1) / BS_THREADS;
        if (nb > 4096) nb = 4096;
        int64_t chunk = (n + nb - 1) / nb;
        nb = (n + chunk - 1) / chunk;
        hipLaunchKernelGGL(k_box_scan, dim3((unsigned)nb), dim3(BS_THREADS), 0, st, p, boxes, nbox, n, chunk,
                           status);
    }
}

void launch_grid_dims(BoxInfo* boxes, int nbox, double margin, int max_nc, uint32_t* status,
                      hipStream_t st)
{
    hipLaunchKernelGGL(k_grid_dims, dim3((nbox + 63) / 64), dim3(64), 0, st, boxes, nbox, margin,
                       max_nc, status);
}

void launch_keys(const Particles& p, const BoxInfo* boxes, int nbox, int64_t n, int top_bits,
                 uint64_t* keys, uint32_t* vals, hipStream_t st)
{
    launch_keys_depth(p, boxes, nbox, n, top_bits, 0, keys, vals, st);
}

void launch_keys_depth(const Particles& p, const BoxInfo* boxes, int nbox, int64_t n, int top_bits, int depth,
                       uint64_t* keys, uint32_t* vals, hipStream_t st)
{
    hipLaunchKernelGGL(k_keys, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, p, boxes, nbox,
                       n, top_bits, depth, keys, vals);
}

size_t radix_scratch_words(int64_t n)
{
    int64_t nb = (n + RS_TILE - 1) / RS_TILE;
    return (size_t)(256 * nb + 256);
}

// Sorts (keys, vals) in place over the low `bits` bits; k2/v2 are scratch.
void radix_sort(uint64_t* keys, uint32_t* vals, uint64_t* k2, uint32_t* v2, int64_t n, int bits,
                uint32_t* scratch, hipStream_t st)
{
    int nb = (int)((n + RS_TILE - 1) / RS_TILE);
    uint32_t* hist = scratch;
    uint32_t* tot = scratch + (size_t)256 * nb;
    uint64_t *ka = keys, *kb = k2;
    uint32_t *va = vals, *vb = v2;
    int passes = (bits + 7) / 8;
    for (int ps = 0; ps < passes; ps++) {
        int shift = ps * 8;
        hipLaunchKernelGGL(k_rs_hist, dim3(nb), dim3(RS_THREADS), 0, st, ka, n, shift, hist, nb);
        hipLaunchKernelGGL(k_rs_colscan, dim3(256), dim3(256), 0, st, hist, nb, tot);
        hipLaunchKernelGGL(k_rs_scatter, dim3(nb), dim3(RS_THREADS), 0, st, ka, va, kb, vb, n, shift,
                           hist, tot, nb);
        uint64_t* tk = ka; ka = kb; kb = tk;
        uint32_t* tv = va; va = vb; vb = tv;
    }
    if (ka != keys) {
        (void)hipMemcpyAsync(keys, ka, sizeof(uint64_t) * n, hipMemcpyDeviceToDevice, st);
        (void)hipMemcpyAsync(vals, va, sizeof(uint32_t) * n, hipMemcpyDeviceToDevice, st);
    }
}

// tile sums of two arrays scanned together
size_t scan_scratch_words(int64_t n) { return 2 * (size_t)((n + SC_TILE - 1) / SC_TILE) + 1; }

void exclusive_scan(const uint32_t* in, uint32_t* out, int64_t n, uint32_t* scratch, uint32_t* total,
                    hipStream_t st)
{
    const int nb = (int)((n + SC_TILE - 1) / SC_TILE);
    if (nb > 0) hipLaunchKernelGGL(k_scan_reduce<1>, dim3(nb), dim3(SC_THREADS), 0, st, in, in, n, scratch, nb);
    hipLaunchKernelGGL(k_scan_top<1>, dim3(1), dim3(SC_THREADS), 0, st, scratch, nb, total, total);   // total 0 if empty
    if (nb > 0) hipLaunchKernelGGL(k_scan_down<1>, dim3(nb), dim3(SC_THREADS), 0, st, in, in, n, scratch, nb, out, out);
}

void exclusive_scan2(const uint32_t* in0, uint32_t* out0, uint32_t* total0, const uint32_t* in1, uint32_t* out1,
                     uint32_t* total1, int64_t n, uint32_t* scratch, hipStream_t st)
{
    const int nb = (int)((n + SC_TILE - 1) / SC_TILE);
    if (nb > 0) hipLaunchKernelGGL(k_scan_reduce<2>, dim3(nb), dim3(SC_THREADS), 0, st, in0, in1, n, scratch, nb);
    hipLaunchKernelGGL(k_scan_top<2>, dim3(1), dim3(SC_THREADS), 0, st, scratch, nb, total0, total1);
    if (nb > 0)
        hipLaunchKernelGGL(k_scan_down<2>, dim3(nb), dim3(SC_THREADS), 0, st, in0, in1, n, scratch, nb, out0, out1);
}

void launch_cells(const uint64_t* keys, uint32_t* flag, uint32_t* cellx, int64_t n, int top_bits,
                  const BoxInfo* boxes, CellInfo* cells, int32_t* cell_map, int64_t map_total,
                  uint32_t* cell_of, int32_t* ncells, uint32_t* scan_scratch, int64_t cell_cap,
                  hipStream_t st)
{
    unsigned g = (unsigned)((n + 255) / 256);
    hipLaunchKernelGGL(k_fill_i32, dim3((unsigned)((map_total + 255) / 256)), dim3(256), 0, st,
                       cell_map, map_total, -1);
    hipLaunchKernelGGL(k_cell_heads, dim3(g), dim3(256), 0, st, keys, n, flag);
    exclusive_scan(flag, cellx, n, scan_scratch, nullptr, st);
    hipLaunchKernelGGL(k_cell_fill, dim3(g), dim3(256), 0, st, keys, flag, cellx, n, top_bits, boxes,
                       cells, cell_map, cell_of, ncells);
    const int64_t cb = (cell_cap + 255) / 256;   // cells number at most cell_cap: the grid strides
    hipLaunchKernelGGL(k_cell_counts, dim3((unsigned)(cb < 1024 ? cb : 1024)), dim3(256), 0, st,
                       cells, ncells, boxes);
}

template <typename R>
void launch_gather(const Particles& p, const uint32_t* perm, const uint32_t* cell_of, const CellInfo* cells,
                   const BoxInfo* boxes, int64_t n, const CellData<R>& cd, typename Vec4T<R>::T* r0,
                   hipStream_t st)
{
    hipLaunchKernelGGL(k_gather<R>, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, p, perm,
                       cell_of, cells, boxes, n, cd, r0);
}
template void launch_gather<float>(const Particles&, const uint32_t*, const uint32_t*, const CellInfo*,
                                   const BoxInfo*, int64_t, const CellData<float>&, float4*, hipStream_t);
template void launch_gather<double>(const Particles&, const uint32_t*, const uint32_t*,
                                    const CellInfo*, const BoxInfo*, int64_t,
                                    const CellData<double>&, double4*, hipStream_t);

template <typename R>
void launch_refresh(const Particles& p, const uint32_t* perm, const uint32_t* cell_of, const CellInfo* cells,
                    const int32_t* ncells, BoxInfo* boxes, int nbox, int64_t n, const CellData<R>& cd,
                    const typename Vec4T<R>::T* r0, float* cell_drift, double h_margin, uint32_t* status,
                    hipStream_t st)
{
    // cells number at most n (and at least one per box)
    const int64_t zn = n > nbox ? n : nbox;
    hipLaunchKernelGGL(k_zero_drift, dim3((unsigned)((zn + 255) / 256)), dim3(256), 0, st, boxes, nbox, cell_drift,
                       ncells);
    if (n > 0) {
        hipLaunchKernelGGL(k_refresh<R>, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, p, perm, cell_of,
                           cells, (const BoxInfo*)boxes, n, cd, r0, cell_drift, status);
        hipLaunchKernelGGL(k_box_drift, dim3(64), dim3(256), 0, st, cells, ncells, (const float*)cell_drift, boxes);
        hipLaunchKernelGGL(k_refresh_check<R>, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, cell_of, cells,
                           (const BoxInfo*)boxes, n, cd, (const float*)cell_drift, h_margin, status);
    }
}
template void launch_refresh<float>(const Particles&, const uint32_t*, const uint32_t*, const CellInfo*,
                                    const int32_t*, BoxInfo*, int, int64_t, const CellData<float>&, const float4*,
                                    float*, double, uint32_t*, hipStream_t);
template void launch_refresh<double>(const Particles&, const uint32_t*, const uint32_t*, const CellInfo*,
                                     const int32_t*, BoxInfo*, int, int64_t, const CellData<double>&,
                                     const double4*, float*, double, uint32_t*, hipStream_t);

void launch_sources(const CellInfo* cells, const int32_t* ncells, const BoxInfo* boxes,
                    const int32_t* cell_map, Source* src, int32_t* src_off, int32_t* src_count,
                    int64_t cell_cap, hipStream_t st)
{
    // cells number at most cell_cap (not known here); 8 cells per block, the grid strides over them
    const int64_t blocks = (cell_cap + 7) / 8;
    hipLaunchKernelGGL(k_sources, dim3((unsigned)(blocks < 4096 ? blocks : 4096)), dim3(256), 0, st, cells,
                       ncells, boxes, cell_map, src, src_off, src_count);
}

template <typename R>
void launch_sort13(const CellInfo* cells, const int32_t* ncells, const BoxInfo* boxes, const CellData<R>& cd,
                   int64_t n, const Sorted<R>& so, int32_t* big, uint32_t* status, int64_t cell_cap, hipStream_t st)
{
    hipLaunchKernelGGL(k_zero_header, dim3(1), dim3(1), 0, st, big);
    unsigned gw = (unsigned)(cell_cap < 65536 ? cell_cap : 65536);
    if (gw < 1) gw = 1;
    hipLaunchKernelGGL(k_sort13_wave<R>, dim3(gw), dim3(kWave), 0, st, cells, ncells, cd, n, so, big);
    // at most n / (kWaveSortMax + 1) cells are left; the grid strides over them
    const int64_t units = (cell_cap / (kWaveSortMax + 1) + 1) * kSortDirs;
    const unsigned grid = (unsigned)(units < 2048 ? units : 2048);
    hipLaunchKernelGGL(k_sort13<R>, dim3(grid), dim3(MERGE_THREADS), 0, st, cells, boxes, big, cd, n, so, status);
}
template void launch_sort13<float>(const CellInfo*, const int32_t*, const BoxInfo*, const CellData<float>&, int64_t,
                                   const Sorted<float>&, int32_t*, uint32_t*, int64_t, hipStream_t);
template void launch_sort13<double>(const CellInfo*, const int32_t*, const BoxInfo*, const CellData<double>&, int64_t,
                                    const Sorted<double>&, int32_t*, uint32_t*, int64_t, hipStream_t);

}  // namespace sph
