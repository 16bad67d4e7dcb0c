// api.cpp -- C ABI of the SPH library: context, workspace and the launch
// sequence of each entry point (declared in include/sph.h).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <new>
#include <vector>

#include "kernels.h"
#include "sph_internal.h"

using namespace sph;

namespace {

// A fixed region of device memory handed out front to back (256-byte
// aligned pieces); nothing is returned before the region is reset.
struct Arena {
    char* base = nullptr;
    size_t cap = 0, used = 0;
};

// grow-only device buffer: its own allocation, or a piece of an arena
struct DBuf {
    void* p = nullptr;
    size_t bytes = 0;
    Arena* arena = nullptr;
    bool ensure(size_t nb)
    {
        if (nb <= bytes) return true;
        if (arena) {
            const size_t off = (arena->used + 255) & ~(size_t)255;
            if (off > arena->cap || nb > arena->cap - off) return false;
            p = arena->base + off;
            bytes = nb;
            arena->used = off + nb;
            return true;
        }
        if (p) (void)hipFree(p);
        p = nullptr;
        bytes = 0;
        if (hipMalloc(&p, nb) != hipSuccess) { p = nullptr; return false; }
        bytes = nb;
        return true;
    }
    void release()
    {
        if (p && !arena) (void)hipFree(p);
        p = nullptr;
        bytes = 0;
    }
    template <typename T> T* as() const { return static_cast<T*>(p); }
};

inline size_t rsz(int prec) { return prec == SPH_FP64 ? sizeof(double) : sizeof(float); }

}  // namespace

struct sph_ctx {
    sph_params prm;
    int device = 0;
    // workspace
    DBuf boxes, keys, keys2, vals, vals2, rs_scratch, flag, cellx, cell_of, sc_scratch;
    DBuf cells, ncells, cell_map, src, src_count, srec;
    DBuf deferred;                                   // cells the shared sweep leaves to the split one
    DBuf big_cells;                                  // count, then the cells the wavefront sort leaves
    DBuf rp, h, vm, u;                               // cell order
    DBuf r0;                                         // cell-relative positions at the last build
    DBuf cell_drift;                                 // largest displacement per cell since that build
    bool refreshed = false;                          // a refresh followed the last build
    bool keys_stale = false;                         // ... and the orderings predate it
    bool refresh_checked = false;                    // its rebuild request was already acted on
    int step_rebuilds = 0;                           // rebuilds a step did before its sph_density
    DBuf g0, g1, cell_hmax;                          // ghost quantities, cell order
    DBuf sd0, sd1;                                   // density sums kept for the adjoint
    DBuf src_off;                                    // first source of each cell
    // hierarchy (max_depth > 0)
    DBuf t_chg, t_node_of, t_node_start, t_node_flag, t_node_hmax, t_node_H, t_node_leaf, t_nnodes;
    DBuf t_flag, t_scan, t_small, t_psmall, t_lev, t_group;
    int depth = 0;                                   // levels below the top grid of the current build
    int64_t src_cap = 0;
    DBuf adj_ab, adj_sb0, adj_sb1, adj_x, adj_h, adj_fg;  // adjoint workspace
    DBuf qhead, status;
    DBuf step_tmp;                                   // predicted v, u; new a, du/dt
    DBuf dt_box, dt_min, t_box;                      // per-box step length, minimum of Eq. (6), time
    // multiple time-stepping: activity of the current base step, the density-stage
    // quantities of every particle's last active step (caller order), counters
    DBuf mts_active, mts_rho, mts_A, mts_c, mts_f, mts_count, mts_units, mts_flag;
    bool mts_ready = false, mts_masked = false, mts_store = false;
    int64_t mts_n = 0, mts_np = 0;
    double mts_dtb = 0.0;
    int mts_max_bin = 0;
    uint32_t* status_host = nullptr;                 // pinned
    int32_t* ncells_host = nullptr;                  // pinned
    // allocation-free context (sph_pass_noalloc): every buffer is a piece of
    // the arena, and host copies go through the static arrays below
    bool noalloc = false;
    Arena arena;
    uint32_t status_static[4] = {};
    int32_t ncells_static[4] = {};
    BoxInfo box_static = {};
    // state of the current decomposition
    int64_t n = 0;
    int nbox = 0;
    int top_bits = 1;
    int64_t map_total = 0;
    std::vector<BoxInfo> box_host;
    BoxInfo* box_pinned = nullptr;                   // pinned copy uploaded to the device
    int box_pinned_cap = 0;
    hipStream_t cap_stream = nullptr;                // stream used for graph capture
    hipGraph_t graph = nullptr;
    hipGraphExec_t graph_exec = nullptr;
    std::vector<int64_t> batch_off;
    std::vector<double> batch_len;
    bool built = false, sorted = false, have_density = false;
    bool adjoint_ready = false;                      // the last density kept the reverse-pass sums
    uint64_t generation = 0;                         // density evaluations so far
    unsigned ev_recorded = 0;                        // events recorded at least once (bit per event)
    sph_stats stats{};
    // optional kernel timing
    bool timing = false;
    hipEvent_t ev[10] = {};
    float dens_ms_acc = 0.0f;
    bool adj_timed = false;
    bool dens_async_timed = false;  // the last density call was sph_density_async (events not yet read)
};

enum { EV_BUILD0, EV_BUILD1, EV_SORT0, EV_SORT1, EV_DENS0, EV_DENS1, EV_FORCE0, EV_FORCE1, EV_ADJ0, EV_ADJ1 };

static void ev_record(sph_ctx* c, int k, hipStream_t st)
{
    if (c->timing && hipEventRecord(c->ev[k], st) == hipSuccess) c->ev_recorded |= 1u << k;
}

// Elapsed milliseconds between two recorded events (0 when either was never
// recorded: querying such a pair would leave a HIP error behind).
static float ev_elapsed(sph_ctx* c, int a, int b)
{
    const unsigned need = (1u << a) | (1u << b);
    float ms = 0.0f;
    if ((c->ev_recorded & need) != need) return 0.0f;
    if (hipEventSynchronize(c->ev[b]) != hipSuccess || hipEventElapsedTime(&ms, c->ev[a], c->ev[b]) != hipSuccess) {
        (void)hipGetLastError();
        return 0.0f;
    }
    return ms;
}

static sph_status hip_status(hipError_t e) { return e == hipSuccess ? SPH_OK : SPH_E_HIP; }

template <typename R>
static CellData<R> cell_data(sph_ctx* c)
{
    using R4 = typename Vec4T<R>::T;
    CellData<R> d;
    d.rp = c->rp.as<R4>();
    d.h = c->h.as<double>();
    d.vm = c->vm.as<R4>();
    d.u = c->u.as<double>();
    return d;
}

template <typename R>
static Sorted<R> sorted_data(sph_ctx* c)
{
    using R4 = typename Vec4T<R>::T;
    Sorted<R> so;
    so.rec = c->srec.as<SortRec>();
    return so;
}

template <typename R>
static GhostData<R> ghost_data(sph_ctx* c)
{
    using R4 = typename Vec4T<R>::T;
    GhostData<R> g;
    g.g0 = c->g0.as<R4>(); g.g1 = c->g1.as<R4>();
    g.cell_hmax = c->cell_hmax.as<float>();
    g.sd0 = c->prm.keep_adjoint ? c->sd0.as<double4>() : nullptr;
    g.sd1 = c->prm.keep_adjoint ? c->sd1.as<double4>() : nullptr;
    g.active = c->mts_masked ? c->mts_active.as<uint8_t>() : nullptr;
    const bool st = c->mts_masked || c->mts_store;
    g.s_rho = st ? c->mts_rho.as<double>() : nullptr;
    g.s_A = st ? c->mts_A.as<double>() : nullptr;
    g.s_c = st ? c->mts_c.as<double>() : nullptr;
    g.s_f = st ? c->mts_f.as<double>() : nullptr;
    return g;
}

static Decomp decomp(sph_ctx* c)
{
    Decomp d;
    d.cells = c->cells.as<CellInfo>();
    d.ncells = c->ncells.as<int32_t>();
    d.boxes = c->boxes.as<BoxInfo>();
    d.src = c->src.as<Source>();
    d.src_off = c->src_off.as<int32_t>();
    d.src_count = c->src_count.as<int32_t>();
    d.perm = c->vals.as<uint32_t>();
    d.n = c->n;
    d.qhead = c->qhead.as<int32_t>();
    d.status = c->status.as<uint32_t>();
    d.cell_drift = c->refreshed ? c->cell_drift.as<float>() : nullptr;
    d.keys_stale = c->keys_stale ? 1 : 0;
    d.units = c->mts_masked ? c->mts_units.as<int32_t>() : nullptr;
    d.nunits = c->mts_masked ? c->mts_count.as<int32_t>() + 1 : nullptr;
    return d;
}

static PassConsts pass_consts(const sph_params& p)
{
    PassConsts pc;
    pc.n_ngb = p.n_ngb;
    pc.tol = p.ngb_tol > 0 ? p.ngb_tol : (p.precision == SPH_FP64 ? 1e-10 : 1e-4);
    pc.gamma = p.gamma;
    pc.alpha = p.alpha;
    pc.beps = p.balsara_eps;
    pc.max_iter = p.max_iter;
    pc.h_margin = p.h_margin;
    pc.cfl = p.cfl;
    pc.balsara_div = p.balsara_form == SPH_BALSARA_DIV ? 1 : 0;
    pc.shared_min = p.shared_min;
    pc.fixed_h = p.fixed_h;
    return pc;
}

// particle-count dependent workspace
static bool ensure_particles(sph_ctx* c, int64_t n)
{
    size_t N = (size_t)std::max<int64_t>(n, 1);
    size_t R = rsz(c->prm.precision);
    bool ok = true;
    ok &= c->keys.ensure(N * 8) && c->keys2.ensure(N * 8);
    ok &= c->vals.ensure(N * 4) && c->vals2.ensure(N * 4);
    ok &= c->rs_scratch.ensure(radix_scratch_words((int64_t)N) * 4);
    ok &= c->flag.ensure(N * 4) && c->cellx.ensure(N * 4) && c->cell_of.ensure(N * 4);
    ok &= c->sc_scratch.ensure(scan_scratch_words((int64_t)N) * 4 + 16);
    ok &= c->cells.ensure(N * sizeof(CellInfo)) && c->ncells.ensure(16) && c->deferred.ensure(N * 4);
    ok &= c->big_cells.ensure((N / 256 + 1 + kBigHeader) * 4);
    // interaction lists: 27 per cell on the single-level grid; on the hierarchy
    // a bound per particle (exceeding it sets SPH_E_CAPACITY)
    c->src_cap = (int64_t)N * (c->depth > 0 ? kTreeSourcesPerParticle : kMaxSources);
    ok &= c->src.ensure((size_t)c->src_cap * sizeof(Source)) && c->src_count.ensure(N * 4);
    ok &= c->src_off.ensure(N * 4);
    if (c->depth > 0) {
        const size_t L = (size_t)c->depth + 1, S = N + 1;
        ok &= c->t_chg.ensure(N) && c->t_lev.ensure(N);
        ok &= c->t_node_of.ensure(L * N * 4) && c->t_node_start.ensure(L * S * 4);
        ok &= c->t_node_flag.ensure(L * S) && c->t_node_hmax.ensure(L * S * 4) && c->t_node_H.ensure(L * S * 4);
        ok &= c->t_node_leaf.ensure(L * S * 4) && c->t_nnodes.ensure(L * 4 + 16);
        ok &= c->t_flag.ensure(N * 4) && c->t_scan.ensure(S * 4);
        ok &= c->t_small.ensure(N * 4) && c->t_psmall.ensure(S * 4);
        ok &= c->t_group.ensure((27 * N + 1) * 4) && c->sc_scratch.ensure(scan_scratch_words((int64_t)(27 * N)) * 4 + 16);
    }
    ok &= c->srec.ensure(N * kSortDirs * sizeof(SortRec));
    ok &= c->rp.ensure(N * 4 * R) && c->r0.ensure(N * 4 * R);
    ok &= c->cell_drift.ensure(N * sizeof(float));
    ok &= c->h.ensure(N * 8) && c->u.ensure(N * 8);
    ok &= c->vm.ensure(N * 4 * R);
    ok &= c->g0.ensure(N * 4 * R) && c->g1.ensure(N * 4 * R);
    ok &= c->cell_hmax.ensure(N * 4);
    if (c->prm.keep_adjoint) ok &= c->sd0.ensure(N * sizeof(double4)) && c->sd1.ensure(N * sizeof(double4));
    ok &= c->qhead.ensure(16) && c->status.ensure(16);
    return ok;
}

extern "C" {

void sph_default_params(sph_params* p)
{
    if (!p) return;
    std::memset(p, 0, sizeof(*p));
    p->box[0] = p->box[1] = p->box[2] = 1.0;
    p->n_ngb = 48.0;
    p->ngb_tol = 0.0;
    p->max_iter = 64;
    p->gamma = 5.0 / 3.0;
    p->alpha = 0.8;
    p->balsara_eps = 1e-4;
    p->precision = SPH_FP32_ACC64;
    p->cell_target = 64;
    p->h_margin = 0.1;
    p->max_rebuilds = 4;
    p->max_depth = 0;
    p->split_count = 64;
    p->split_frac = 0.875;
    p->cfl = 0.25;
    p->balsara_form = SPH_BALSARA_CURL;
    p->reuse = 0;
    p->staging = SPH_STAGING_COMPACT;
    p->shared_min = 128;
    p->fixed_h = 0;
    p->keep_adjoint = 0;
    p->sweep = SPH_SWEEP_AUTO;
}

const char* sph_status_string(sph_status s)
{
    switch (s) {
    case SPH_OK: return "ok";
    case SPH_E_INVALID_ARG: return "invalid argument";
    case SPH_E_NONFINITE: return "non-finite or non-positive particle data";
    case SPH_E_H_TOO_LARGE: return "smoothing length too large for the periodic box (need >= 3 cells of edge >= h)";
    case SPH_E_NOT_CONVERGED: return "smoothing-length iteration did not converge";
    case SPH_E_CAPACITY: return "workspace capacity exceeded (cell too large or grid too fine)";
    case SPH_E_OOM: return "device allocation failed";
    case SPH_E_HIP: return "HIP runtime error";
    case SPH_E_STATE: return "calls out of order";
    }
    return "unknown status";
}

static bool params_ok(const sph_params& p)
{
    for (int d = 0; d < 3; d++) if (!(p.box[d] > 0) || !std::isfinite(p.box[d])) return false;
    if (!(p.n_ngb > 32.0 / 3.0) || !std::isfinite(p.n_ngb)) return false;
    if (!(p.ngb_tol >= 0)) return false;
    if (p.max_iter < 1) return false;
    if (!(p.gamma > 1.0)) return false;
    if (!(p.alpha >= 0)) return false;
    if (!(p.balsara_eps >= 0)) return false;
    if (p.precision != SPH_FP64 && p.precision != SPH_FP32_ACC64) return false;
    if (p.cell_target < 1) return false;
    if (!(p.h_margin >= 0) || !(p.h_margin < 10)) return false;
    if (p.max_rebuilds < 0) return false;
    if (p.max_depth < 0 || p.split_count < 1 || !(p.split_frac >= 0.0) || !(p.split_frac <= 1.0)) return false;
    if (!(p.cfl > 0.0) || !std::isfinite(p.cfl)) return false;
    if (p.balsara_form != SPH_BALSARA_CURL && p.balsara_form != SPH_BALSARA_DIV) return false;
    if (p.reuse != SPH_REUSE_OFF && p.reuse != SPH_REUSE_ORDERINGS && p.reuse != SPH_REUSE_CELLS) return false;
    if (p.staging != SPH_STAGING_COMPACT && p.staging != SPH_STAGING_WIDE) return false;
    if (p.shared_min < 64) return false;
    if (p.fixed_h != 0 && p.fixed_h != 1) return false;
    if (p.keep_adjoint != 0 && p.keep_adjoint != 1) return false;
    if (p.sweep != SPH_SWEEP_AUTO && p.sweep != SPH_SWEEP_SHARED && p.sweep != SPH_SWEEP_SPLIT) return false;
    return true;
}

sph_status sph_create(const sph_params* params, sph_ctx** out)
{
    if (!out) return SPH_E_INVALID_ARG;
    *out = nullptr;
    sph_params p;
    if (params) p = *params; else sph_default_params(&p);
    if (!params_ok(p)) return SPH_E_INVALID_ARG;
    sph_ctx* c = new (std::nothrow) sph_ctx();
    if (!c) return SPH_E_OOM;
    c->prm = p;
    if (hipGetDevice(&c->device) != hipSuccess) { delete c; return SPH_E_HIP; }
    if (hipHostMalloc((void**)&c->status_host, 16, hipHostMallocDefault) != hipSuccess ||
        hipHostMalloc((void**)&c->ncells_host, 16, hipHostMallocDefault) != hipSuccess) {
        if (c->status_host) (void)hipHostFree(c->status_host);
        delete c;
        return SPH_E_HIP;
    }
    *out = c;
    return SPH_OK;
}

// every workspace buffer of a context
extern "C++" template <typename F> static void for_each_buf(sph_ctx* c, F f)
{
    DBuf* all[] = {&c->boxes, &c->keys, &c->keys2, &c->vals, &c->vals2, &c->rs_scratch, &c->flag,
                   &c->cellx, &c->cell_of, &c->sc_scratch, &c->deferred, &c->cells, &c->ncells, &c->big_cells, &c->cell_map,
                   &c->src, &c->src_count, &c->srec, &c->r0, &c->cell_drift, &c->rp, &c->h,
                   &c->vm, &c->u, &c->g0, &c->g1, &c->cell_hmax, &c->qhead, &c->status, &c->step_tmp, &c->dt_box, &c->dt_min, &c->t_box, &c->mts_active, &c->mts_rho, &c->mts_A,
                   &c->mts_c, &c->mts_f, &c->mts_count, &c->mts_units, &c->mts_flag,
                   &c->sd0, &c->sd1, &c->adj_ab, &c->adj_sb0, &c->adj_sb1, &c->adj_x, &c->adj_h, &c->adj_fg,
                   &c->src_off, &c->t_chg, &c->t_node_of, &c->t_node_start, &c->t_node_flag, &c->t_node_hmax,
                   &c->t_node_H, &c->t_node_leaf, &c->t_nnodes, &c->t_flag, &c->t_scan, &c->t_small,
                   &c->t_psmall, &c->t_lev, &c->t_group};
    for (DBuf* b : all) f(b);
}

sph_status sph_destroy(sph_ctx* c)
{
    if (!c) return SPH_OK;
    if (c->noalloc) return SPH_E_INVALID_ARG;   // the library's own, never destroyed
    for_each_buf(c, [](DBuf* b) { b->release(); });
    if (c->status_host) (void)hipHostFree(c->status_host);
    if (c->ncells_host) (void)hipHostFree(c->ncells_host);
    for (hipEvent_t& e : c->ev) if (e) (void)hipEventDestroy(e);
    if (c->graph_exec) (void)hipGraphExecDestroy(c->graph_exec);
    if (c->graph) (void)hipGraphDestroy(c->graph);
    if (c->cap_stream) (void)hipStreamDestroy(c->cap_stream);
    if (c->box_pinned) (void)hipHostFree(c->box_pinned);
    delete c;
    return SPH_OK;
}

static bool particles_ok(const sph_particles* p)
{
    if (!p || p->n < 0 || p->n > (int64_t)0x7fffffff) return false;
    if (p->n == 0) return true;
    return p->x && p->y && p->z && p->vx && p->vy && p->vz && p->u && p->m && p->h;
}

static Particles view(const sph_particles* p)
{
    return Particles{p->x, p->y, p->z, p->vx, p->vy, p->vz, p->u, p->m, p->h};
}

// Host part of the box table: per-box target edge and dense-map capacity.
static sph_status setup_boxes(sph_ctx* c, int64_t n, const sph_batch* batch)
{
    int nbox = batch ? batch->nbox : 1;
    if (nbox < 1) return SPH_E_INVALID_ARG;
    // the allocation-free context keeps its one box in the context itself
    if (c->noalloc && nbox != 1) return SPH_E_INVALID_ARG;
    if (!c->noalloc) c->box_host.assign(nbox, BoxInfo{});
    BoxInfo* const boxes = c->noalloc ? &c->box_static : c->box_host.data();
    int64_t map_total = 0;
    int max_nc = 1;
    for (int b = 0; b < nbox; b++) {
        BoxInfo& B = boxes[b];
        std::memset(&B, 0, sizeof(B));
        int64_t beg = batch ? batch->box_offsets[b] : 0;
        int64_t end = batch ? batch->box_offsets[b + 1] : n;
        if (beg < 0 || end < beg || end > n) return SPH_E_INVALID_ARG;
        if (batch && b == 0 && beg != 0) return SPH_E_INVALID_ARG;
        for (int d = 0; d < 3; d++) {
            B.L[d] = batch ? batch->box_len[3 * b + d] : c->prm.box[d];
            if (!(B.L[d] > 0) || !std::isfinite(B.L[d])) return SPH_E_INVALID_ARG;
        }
        B.begin = beg;
        B.n = end - beg;
        double vol = B.L[0] * B.L[1] * B.L[2];
        B.e_target = B.n > 0 ? std::cbrt((double)c->prm.cell_target * vol / (double)B.n)
                             : std::max(B.L[0], std::max(B.L[1], B.L[2]));
        int64_t cap = 1;
        for (int d = 0; d < 3; d++) {
            int nc = (int)std::floor(B.L[d] / B.e_target);
            nc = std::max(3, std::min(nc, 1023));
            B.cap_nc[d] = nc;
            cap *= nc;
            max_nc = std::max(max_nc, nc);
        }
        B.map_off = (int32_t)map_total;
        B.map_cap = (int32_t)cap;
        map_total += cap;
        if (map_total > (int64_t)0x7fffffff) return SPH_E_CAPACITY;
    }
    if (batch && batch->box_offsets[nbox] != n) return SPH_E_INVALID_ARG;
    int tb = 1;
    while ((1 << tb) < max_nc) tb++;
    int box_bits = 0;
    while ((1 << box_bits) < nbox) box_bits++;
    if (3 * tb + box_bits > 64) return SPH_E_CAPACITY;
    // levels of the hierarchy: bounded by the key width and the 21 bits per
    // dimension of the Morton code
    int depth = std::min(c->prm.max_depth, kMaxDepth);
    depth = std::min(depth, (64 - box_bits) / 3 - tb);
    depth = std::min(depth, 21 - tb);
    if (depth < 0) depth = 0;
    if (depth > 0 && n >= ((int64_t)1 << 27)) return SPH_E_CAPACITY;
    for (int b = 0; b < nbox; b++) boxes[b].depth = depth;
    c->depth = depth;
    c->nbox = nbox;
    c->top_bits = tb;
    c->map_total = map_total;
    return SPH_OK;
}

// Copies the host box table to the device through a pinned buffer (so the
// copy can be part of a captured graph).
static bool upload_boxes(sph_ctx* c, hipStream_t st)
{
    if (c->noalloc) {
        // one box, copied from host memory of the context (the copy waits for it)
        if (c->nbox != 1) return false;
        return hipMemcpyAsync(c->boxes.p, &c->box_static, sizeof(BoxInfo), hipMemcpyHostToDevice, st) == hipSuccess;
    }
    if (c->box_pinned_cap < c->nbox) {
        if (c->box_pinned) (void)hipHostFree(c->box_pinned);
        c->box_pinned = nullptr;
        c->box_pinned_cap = 0;
        if (hipHostMalloc((void**)&c->box_pinned, sizeof(BoxInfo) * c->nbox, hipHostMallocDefault) != hipSuccess)
            return false;
        c->box_pinned_cap = c->nbox;
    }
    std::memcpy(c->box_pinned, c->box_host.data(), sizeof(BoxInfo) * c->nbox);
    return hipMemcpyAsync(c->boxes.p, c->box_pinned, sizeof(BoxInfo) * c->nbox, hipMemcpyHostToDevice, st) ==
           hipSuccess;
}

static TreeView tree_view(sph_ctx* c)
{
    TreeView tv;
    tv.depth = c->depth;
    tv.top_bits = c->top_bits;
    tv.n = c->n;
    tv.stride = c->n + 1;
    tv.keys = c->keys.as<uint64_t>();
    tv.perm = c->vals.as<uint32_t>();
    tv.chg = c->t_chg.as<uint8_t>();
    tv.node_of = c->t_node_of.as<uint32_t>();
    tv.node_start = c->t_node_start.as<uint32_t>();
    tv.node_flag = c->t_node_flag.as<uint8_t>();
    tv.node_hmax = c->t_node_hmax.as<float>();
    tv.node_H = c->t_node_H.as<float>();
    tv.node_leaf = c->t_node_leaf.as<int32_t>();
    tv.nnodes = c->t_nnodes.as<int32_t>();
    tv.flag = c->t_flag.as<uint32_t>();
    tv.scan = c->t_scan.as<uint32_t>();
    tv.small = c->t_small.as<uint32_t>();
    tv.psmall = c->t_psmall.as<uint32_t>();
    tv.lev = c->t_lev.as<uint8_t>();
    return tv;
}

// box scan, top grid, keys (down to the current depth) and their sort
static void key_launches(sph_ctx* c, const Particles& pv, hipStream_t st)
{
    const int64_t n = c->n;
    BoxInfo* boxes = c->boxes.as<BoxInfo>();
    uint32_t* status = c->status.as<uint32_t>();
    launch_box_scan(pv, boxes, c->nbox, n, status, st);
    launch_grid_dims(boxes, c->nbox, c->prm.h_margin, 1023, status, st);
    launch_keys_depth(pv, boxes, c->nbox, n, c->top_bits, c->depth, c->keys.as<uint64_t>(), c->vals.as<uint32_t>(),
                      st);
    int box_bits = 0;
    while ((1 << box_bits) < c->nbox) box_bits++;
    radix_sort(c->keys.as<uint64_t>(), c->vals.as<uint32_t>(), c->keys2.as<uint64_t>(),
               c->vals2.as<uint32_t>(), n, 3 * (c->top_bits + c->depth) + box_bits, c->rs_scratch.as<uint32_t>(),
               st);
}

extern "C++" {
template <typename R>
static void build_launches(sph_ctx* c, const Particles& pv, hipStream_t st)
{
    const int64_t n = c->n;
    BoxInfo* boxes = c->boxes.as<BoxInfo>();
    key_launches(c, pv, st);
    if (c->depth == 0) {
        launch_cells(c->keys.as<uint64_t>(), c->flag.as<uint32_t>(), c->cellx.as<uint32_t>(), n, c->top_bits,
                     boxes, c->cells.as<CellInfo>(), c->cell_map.as<int32_t>(), c->map_total,
                     c->cell_of.as<uint32_t>(), c->ncells.as<int32_t>(), c->sc_scratch.as<uint32_t>(), n, st);
    } else {
        const TreeView tv = tree_view(c);
        launch_tree(pv, tv, boxes, c->prm.split_count, c->prm.split_frac, c->prm.h_margin,
                    c->sc_scratch.as<uint32_t>(), st);
        launch_tree_cells(tv, boxes, c->cells.as<CellInfo>(), c->cell_map.as<int32_t>(), c->map_total,
                          c->cell_of.as<uint32_t>(), c->ncells.as<int32_t>(), c->prm.h_margin,
                          c->sc_scratch.as<uint32_t>(), st);
    }
    launch_gather<R>(pv, c->vals.as<uint32_t>(), c->cell_of.as<uint32_t>(), c->cells.as<CellInfo>(), boxes,
                     n, cell_data<R>(c), c->r0.as<typename Vec4T<R>::T>(), st);
    if (c->depth == 0)
        launch_sources(c->cells.as<CellInfo>(), c->ncells.as<int32_t>(), boxes, c->cell_map.as<int32_t>(),
                       c->src.as<Source>(), c->src_off.as<int32_t>(), c->src_count.as<int32_t>(), n, st);
    else
        launch_tree_sources(tree_view(c), c->cells.as<CellInfo>(), c->ncells.as<int32_t>(), boxes,
                            c->cell_map.as<int32_t>(), c->src.as<Source>(), c->src_cap, c->src_off.as<int32_t>(),
                            c->src_count.as<int32_t>(), c->t_group.as<uint32_t>(), c->status.as<uint32_t>(),
                            c->sc_scratch.as<uint32_t>(), n, st);
}
}  // extern "C++"

sph_status sph_build_cells(sph_ctx* c, const sph_particles* p, const sph_batch* batch, void* stream)
{
    if (!c || !particles_ok(p)) return SPH_E_INVALID_ARG;
    if (batch && (batch->nbox < 1 || !batch->box_offsets || !batch->box_len)) return SPH_E_INVALID_ARG;
    hipStream_t st = (hipStream_t)stream;
    if (hipSetDevice(c->device) != hipSuccess) return SPH_E_HIP;
    sph_status s = setup_boxes(c, p->n, batch);
    if (s != SPH_OK) return s;
    if (batch) {
        c->batch_off.assign(batch->box_offsets, batch->box_offsets + batch->nbox + 1);
        c->batch_len.assign(batch->box_len, batch->box_len + 3 * batch->nbox);
    } else {
        c->batch_off.clear();
        c->batch_len.clear();
    }
    c->n = p->n;
    c->built = c->sorted = c->have_density = false;
    c->stats.refreshes = 0;
    c->refreshed = c->keys_stale = c->refresh_checked = false;
    if (!ensure_particles(c, p->n)) return SPH_E_OOM;
    if (!c->boxes.ensure(sizeof(BoxInfo) * c->nbox)) return SPH_E_OOM;
    if (!c->cell_map.ensure(sizeof(int32_t) * std::max<int64_t>(c->map_total, 1))) return SPH_E_OOM;
    if (!upload_boxes(c, st)) return SPH_E_HIP;
    launch_fill_i32(c->status.as<int32_t>(), 4, 0, st);
    launch_fill_i32(c->ncells.as<int32_t>(), 4, 0, st);
    if (p->n > 0) {
        Particles pv = view(p);
        ev_record(c, EV_BUILD0, st);
        if (c->prm.precision == SPH_FP64) build_launches<double>(c, pv, st);
        else build_launches<float>(c, pv, st);
        ev_record(c, EV_BUILD1, st);
    }
    if (hipGetLastError() != hipSuccess) return SPH_E_HIP;
    c->built = true;
    return SPH_OK;
}

// The batch layout of the last build equals `batch` (NULL: one box of params.box).
static bool same_layout(const sph_ctx* c, const sph_batch* batch)
{
    if (!batch) return c->batch_off.empty();
    if ((int)c->batch_off.size() != batch->nbox + 1 || !batch->box_offsets || !batch->box_len) return false;
    for (int b = 0; b <= batch->nbox; b++)
        if (c->batch_off[(size_t)b] != batch->box_offsets[b]) return false;
    for (int k = 0; k < 3 * batch->nbox; k++)
        if (c->batch_len[(size_t)k] != batch->box_len[k]) return false;
    return true;
}

sph_status sph_refresh(sph_ctx* c, const sph_particles* p, void* stream)
{
    if (!c || !particles_ok(p)) return SPH_E_INVALID_ARG;
    if (!c->built || !c->sorted || p->n != c->n) return SPH_E_STATE;
    hipStream_t st = (hipStream_t)stream;
    if (hipSetDevice(c->device) != hipSuccess) return SPH_E_HIP;
    c->have_density = false;
    launch_fill_i32(c->status.as<int32_t>(), 4, 0, st);
    if (p->n > 0) {
        Particles pv = view(p);
        if (c->prm.precision == SPH_FP64)
            launch_refresh<double>(pv, c->vals.as<uint32_t>(), c->cell_of.as<uint32_t>(), c->cells.as<CellInfo>(),
                                   c->ncells.as<int32_t>(), c->boxes.as<BoxInfo>(), c->nbox, c->n,
                                   cell_data<double>(c), c->r0.as<double4>(), c->cell_drift.as<float>(),
                                   c->prm.h_margin, c->status.as<uint32_t>(), st);
        else
            launch_refresh<float>(pv, c->vals.as<uint32_t>(), c->cell_of.as<uint32_t>(), c->cells.as<CellInfo>(),
                                  c->ncells.as<int32_t>(), c->boxes.as<BoxInfo>(), c->nbox, c->n,
                                  cell_data<float>(c), c->r0.as<float4>(), c->cell_drift.as<float>(),
                                  c->prm.h_margin, c->status.as<uint32_t>(), st);
    }
    if (hipGetLastError() != hipSuccess) return SPH_E_HIP;
    c->refreshed = true;
    c->keys_stale = true;
    c->refresh_checked = false;
    c->stats.refreshes++;
    return SPH_OK;
}

sph_status sph_estimate_h(sph_ctx* c, sph_particles* p, const sph_batch* batch, void* stream)
{
    if (!c || !particles_ok(p) || c->prm.max_depth < 1) return SPH_E_INVALID_ARG;
    if (batch && (batch->nbox < 1 || !batch->box_offsets || !batch->box_len)) return SPH_E_INVALID_ARG;
    hipStream_t st = (hipStream_t)stream;
    if (hipSetDevice(c->device) != hipSuccess) return SPH_E_HIP;
    sph_status s = setup_boxes(c, p->n, batch);
    if (s != SPH_OK) return s;
    if (c->depth < 1) return SPH_E_CAPACITY;
    c->n = p->n;
    c->built = c->sorted = c->have_density = false;
    if (!ensure_particles(c, p->n)) return SPH_E_OOM;
    if (!c->boxes.ensure(sizeof(BoxInfo) * c->nbox)) return SPH_E_OOM;
    if (!upload_boxes(c, st)) return SPH_E_HIP;
    launch_fill_i32(c->status.as<int32_t>(), 4, 0, st);
    if (p->n > 0) {
        Particles pv = view(p);
        key_launches(c, pv, st);
        const TreeView tv = tree_view(c);
        launch_tree(pv, tv, c->boxes.as<BoxInfo>(), c->prm.split_count, c->prm.split_frac, c->prm.h_margin,
                    c->sc_scratch.as<uint32_t>(), st);
        launch_estimate_h(tv, c->boxes.as<BoxInfo>(), c->prm.n_ngb, p->h, p->n, st);
    }
    return hipGetLastError() == hipSuccess ? SPH_OK : SPH_E_HIP;
}

sph_status sph_sort(sph_ctx* c, void* stream)
{
    if (!c) return SPH_E_INVALID_ARG;
    if (!c->built) return SPH_E_STATE;
    hipStream_t st = (hipStream_t)stream;
    if (c->n > 0) {
        ev_record(c, EV_SORT0, st);
        if (c->prm.precision == SPH_FP64)
            launch_sort13<double>(c->cells.as<CellInfo>(), c->ncells.as<int32_t>(), decomp(c).boxes, cell_data<double>(c), c->n,
                                  sorted_data<double>(c), c->big_cells.as<int32_t>(), c->status.as<uint32_t>(),
                                  c->n, st);
        else
            launch_sort13<float>(c->cells.as<CellInfo>(), c->ncells.as<int32_t>(), decomp(c).boxes, cell_data<float>(c), c->n,
                                 sorted_data<float>(c), c->big_cells.as<int32_t>(), c->status.as<uint32_t>(),
                                 c->n, st);
        ev_record(c, EV_SORT1, st);
    }
    if (hipGetLastError() != hipSuccess) return SPH_E_HIP;
    c->sorted = true;
    c->keys_stale = false;
    return SPH_OK;
}

static sph_status read_status(sph_ctx* c, hipStream_t st, uint32_t* bits)
{
    if (hipMemcpyAsync(c->status_host, c->status.p, 4, hipMemcpyDeviceToHost, st) != hipSuccess) return SPH_E_HIP;
    if (hipMemcpyAsync(c->ncells_host, c->ncells.p, 4, hipMemcpyDeviceToHost, st) != hipSuccess) return SPH_E_HIP;
    if (hipStreamSynchronize(st) != hipSuccess) return SPH_E_HIP;
    *bits = *c->status_host;
    c->stats.n_cells = *c->ncells_host;
    c->stats.n_units = *c->ncells_host;
    return SPH_OK;
}

static sph_status status_error(uint32_t bits)
{
    if (bits & ST_NONFINITE) return SPH_E_NONFINITE;
    if (bits & ST_H_TOO_LARGE) return SPH_E_H_TOO_LARGE;
    if (bits & ST_CAPACITY) return SPH_E_CAPACITY;
    return SPH_OK;
}

// the shared sweep (params.sweep; AUTO takes the split one)
static bool shared_sweep(const sph_ctx* c) { return c->prm.sweep == SPH_SWEEP_SHARED; }

extern "C++" {
template <typename R>
static void density_launch(sph_ctx* c, const sph_particles* p, const sph_density_out* o, hipStream_t st)
{
    DensityOut out{};
    out.h = p->h;
    if (o) {
        out.rho = o->rho; out.omega = o->omega; out.nngb = o->n_ngb; out.div = o->div_v;
        out.curl = o->curl_v; out.balsara = o->balsara; out.P = o->pressure; out.c = o->sound;
        out.iters = o->n_iter;
        out.ndens = o->n_dens;
    }
    if (shared_sweep(c))
        launch_density_shared<R>(decomp(c), cell_data<R>(c), sorted_data<R>(c), ghost_data<R>(c), out,
                                 pass_consts(c->prm), c->prm.staging, c->deferred.as<int32_t>(),
                                 c->qhead.as<int32_t>(), st);
    else
        launch_density<R>(decomp(c), cell_data<R>(c), sorted_data<R>(c), ghost_data<R>(c), out,
                          pass_consts(c->prm), c->prm.staging, st);
}
}  // extern "C++"

// Cells and orderings rebuilt for p with the boxes of the last build.
static sph_status rebuild_same_boxes(sph_ctx* c, sph_particles* p, void* stream)
{
    sph_batch b{}, *bp = nullptr;
    std::vector<int64_t> off = c->batch_off;
    std::vector<double> len = c->batch_len;
    if (!off.empty()) {
        b.nbox = (int)off.size() - 1;
        b.box_offsets = off.data();
        b.box_len = len.data();
        bp = &b;
    }
    sph_status s = sph_build_cells(c, p, bp, stream);
    if (s == SPH_OK) s = sph_sort(c, stream);
    return s;
}

// Multiple time-stepping: the active cells and the inactive particles' records
// for the decomposition as it stands (again after any rebuild).
static void mts_prepare(sph_ctx* c, hipStream_t st)
{
    if (c->prm.precision == SPH_FP64)
        launch_mts_prepare<double>(decomp(c), cell_data<double>(c), ghost_data<double>(c), c->mts_units.as<int32_t>(),
                                   c->mts_count.as<int32_t>() + 1, c->mts_flag.as<uint32_t>(),
                                   c->cell_of.as<uint32_t>(), c->n, st);
    else
        launch_mts_prepare<float>(decomp(c), cell_data<float>(c), ghost_data<float>(c), c->mts_units.as<int32_t>(),
                                  c->mts_count.as<int32_t>() + 1, c->mts_flag.as<uint32_t>(),
                                  c->cell_of.as<uint32_t>(), c->n, st);
}

sph_status sph_density(sph_ctx* c, sph_particles* p, sph_density_out* o, void* stream)
{
    if (!c || !particles_ok(p)) return SPH_E_INVALID_ARG;
    if (!c->built || !c->sorted) return SPH_E_STATE;
    if (p->n != c->n) return SPH_E_STATE;
    hipStream_t st = (hipStream_t)stream;
    c->stats.rebuilds = c->step_rebuilds;   // a rebuild the step did just before
    c->step_rebuilds = 0;
    c->have_density = false;
    c->dens_ms_acc = 0.0f;
    c->dens_async_timed = false;
    if (c->refreshed && !c->refresh_checked && c->n > 0) {
        // a refresh that found its decomposition no longer valid asked for a
        // rebuild: do it before sweeping rather than after
        uint32_t bits = 0;
        sph_status s = read_status(c, st, &bits);
        if (s == SPH_OK) s = status_error(bits);
        if (s != SPH_OK) return s;
        if (bits & ST_REBUILD) {
            s = rebuild_same_boxes(c, p, stream);
            if (s != SPH_OK) return s;
            c->stats.rebuilds++;
        }
    }
    if (c->mts_masked) mts_prepare(c, st);
    for (int attempt = 0;; attempt++) {
        uint32_t bits = 0;
        if (c->n > 0) {
            ev_record(c, EV_DENS0, st);
            if (c->prm.precision == SPH_FP64) density_launch<double>(c, p, o, st);
            else density_launch<float>(c, p, o, st);
            ev_record(c, EV_DENS1, st);
            if (hipGetLastError() != hipSuccess) return SPH_E_HIP;
        }
        sph_status s = read_status(c, st, &bits);
        if (c->timing && c->n > 0) {
            float ms = 0.0f;
            ms = ev_elapsed(c, EV_DENS0, EV_DENS1);
            c->dens_ms_acc += ms;
        }
        if (s != SPH_OK) return s;
        s = status_error(bits);
        if (s != SPH_OK) return s;
        if ((bits & ST_REBUILD) && attempt < c->prm.max_rebuilds) {
            // some smoothing length outgrew its cells: rebuild from the current h
            s = rebuild_same_boxes(c, p, stream);
            if (s != SPH_OK) return s;
            c->stats.rebuilds++;
            if (c->mts_masked) mts_prepare(c, st);
            continue;
        }
        if (bits & ST_REBUILD) return SPH_E_H_TOO_LARGE;
        c->have_density = true;
        c->adjoint_ready = c->prm.keep_adjoint != 0;
        c->generation++;
        if (bits & ST_NOT_CONVERGED) return SPH_E_NOT_CONVERGED;
        return SPH_OK;
    }
}

sph_status sph_density_async(sph_ctx* c, sph_particles* p, sph_density_out* o, void* stream)
{
    if (!c || !particles_ok(p)) return SPH_E_INVALID_ARG;
    if (!c->built || !c->sorted) return SPH_E_STATE;
    if (p->n != c->n) return SPH_E_STATE;
    hipStream_t st = (hipStream_t)stream;
    c->stats.rebuilds = 0;
    c->dens_ms_acc = 0.0f;
    if (c->n > 0) {
        ev_record(c, EV_DENS0, st);
        if (c->prm.precision == SPH_FP64) density_launch<double>(c, p, o, st);
        else density_launch<float>(c, p, o, st);
        ev_record(c, EV_DENS1, st);
        if (hipGetLastError() != hipSuccess) return SPH_E_HIP;
    }
    c->have_density = true;
    c->adjoint_ready = c->prm.keep_adjoint != 0;
    c->generation++;
    c->dens_async_timed = c->timing && c->n > 0;
    return SPH_OK;
}

sph_status sph_check(sph_ctx* c, void* stream)
{
    if (!c) return SPH_E_INVALID_ARG;
    uint32_t bits = 0;
    sph_status s = read_status(c, (hipStream_t)stream, &bits);
    if (s != SPH_OK) return s;
    s = status_error(bits);
    if (s != SPH_OK) return s;
    if (bits & ST_REBUILD) return SPH_E_H_TOO_LARGE;
    if (bits & ST_NOT_CONVERGED) return SPH_E_NOT_CONVERGED;
    return SPH_OK;
}

sph_status sph_force(sph_ctx* c, const sph_particles* p, sph_force_out* o, void* stream)
{
    if (!c || !particles_ok(p) || !o) return SPH_E_INVALID_ARG;
    if (!c->have_density || p->n != c->n) return SPH_E_STATE;
    hipStream_t st = (hipStream_t)stream;
    if (c->n == 0) return SPH_OK;
    ForceOut out{};
    out.ax = o->ax; out.ay = o->ay; out.az = o->az; out.dudt = o->dudt; out.npairs = o->n_pairs;
    out.dt = o->dt;
    ev_record(c, EV_FORCE0, st);
    const int grid = force_occupancy_grid(c->prm.precision);
    if (shared_sweep(c)) {
        if (c->prm.precision == SPH_FP64)
            launch_force_shared<double>(decomp(c), cell_data<double>(c), sorted_data<double>(c),
                                        ghost_data<double>(c), out, pass_consts(c->prm), grid,
                                        c->deferred.as<int32_t>(), c->qhead.as<int32_t>(), st);
        else
            launch_force_shared<float>(decomp(c), cell_data<float>(c), sorted_data<float>(c), ghost_data<float>(c),
                                       out, pass_consts(c->prm), grid, c->deferred.as<int32_t>(),
                                       c->qhead.as<int32_t>(), st);
        ev_record(c, EV_FORCE1, st);
        return hipGetLastError() == hipSuccess ? SPH_OK : SPH_E_HIP;
    }
    if (c->prm.precision == SPH_FP64)
        launch_force<double>(decomp(c), cell_data<double>(c), sorted_data<double>(c), ghost_data<double>(c), out,
                             pass_consts(c->prm), grid, st);
    else
        launch_force<float>(decomp(c), cell_data<float>(c), sorted_data<float>(c), ghost_data<float>(c), out,
                            pass_consts(c->prm), grid, st);
    ev_record(c, EV_FORCE1, st);
    return hipGetLastError() == hipSuccess ? SPH_OK : SPH_E_HIP;
}

extern "C++" {
template <typename R>
static sph_status backward_launch(sph_ctx* c, const sph_grad_in* gi, sph_grad_out* go, bool implicit_h,
                                  hipStream_t st)
{
    using R4 = typename Vec4T<R>::T;
    const size_t N = (size_t)c->n;
    bool ok = c->adj_ab.ensure(N * sizeof(R4)) && c->adj_sb0.ensure(N * sizeof(R4)) &&
              c->adj_sb1.ensure(N * sizeof(R4)) && c->adj_x.ensure(N * 3 * sizeof(double)) &&
              c->adj_h.ensure(N * sizeof(double)) && c->adj_fg.ensure(N * sizeof(double4));
    if (!ok) return SPH_E_OOM;
    AdjData<R> ad;
    ad.ab = c->adj_ab.as<R4>(); ad.sb0 = c->adj_sb0.as<R4>(); ad.sb1 = c->adj_sb1.as<R4>();
    ad.xbar = c->adj_x.as<double>(); ad.hbar = c->adj_h.as<double>(); ad.fg = c->adj_fg.as<double4>();
    AdjIO io;
    io.g_rho = gi->rho; io.g_ax = gi->ax; io.g_ay = gi->ay; io.g_az = gi->az; io.g_dudt = gi->dudt;
    io.gx = go->x; io.gy = go->y; io.gz = go->z; io.gh = go->h;
    launch_adjoint<R>(decomp(c), cell_data<R>(c), sorted_data<R>(c), ghost_data<R>(c), ad, io, pass_consts(c->prm),
                      implicit_h, c->n, st);
    return SPH_OK;
}
}  // extern "C++"

sph_status sph_backward(sph_ctx* c, const sph_particles* p, const sph_grad_in* gi, sph_grad_out* go,
                        int implicit_h, uint64_t generation, void* stream)
{
    if (!c || !particles_ok(p) || !gi || !go) return SPH_E_INVALID_ARG;
    if (!c->have_density || p->n != c->n) return SPH_E_STATE;
    if (!c->adjoint_ready) return SPH_E_STATE;                          // nothing kept to differentiate
    if (generation != 0 && generation != c->generation) return SPH_E_STATE;   // that state is gone
    if (implicit_h && c->prm.fixed_h) return SPH_E_STATE;                // h was given, not solved
    hipStream_t st = (hipStream_t)stream;
    c->adj_timed = false;
    if (c->n == 0) return SPH_OK;
    ev_record(c, EV_ADJ0, st);
    sph_status s = c->prm.precision == SPH_FP64 ? backward_launch<double>(c, gi, go, implicit_h != 0, st)
                                                : backward_launch<float>(c, gi, go, implicit_h != 0, st);
    if (s != SPH_OK) return s;
    ev_record(c, EV_ADJ1, st);
    c->adj_timed = c->timing;
    return hipGetLastError() == hipSuccess ? SPH_OK : SPH_E_HIP;
}

// The step proper, with the step length of each box in c->dt_box (device).
static sph_status step_core(sph_ctx* c, sph_particles* p, const sph_batch* batch, sph_force_out* acc,
                            bool reuse, hipStream_t st)
{
    const int64_t n = p->n;
    if (!c->step_tmp.ensure(sizeof(double) * 4 * (size_t)n)) return SPH_E_OOM;
    double* vp = c->step_tmp.as<double>();
    StepArrays sa;
    sa.x = p->x; sa.y = p->y; sa.z = p->z; sa.vx = p->vx; sa.vy = p->vy; sa.vz = p->vz; sa.u = p->u;
    sa.ax = acc->ax; sa.ay = acc->ay; sa.az = acc->az; sa.dudt = acc->dudt;
    sa.pvx = vp; sa.pvy = vp + n; sa.pvz = vp + 2 * n; sa.pu = vp + 3 * n;
    const double* dtb = c->dt_box.as<double>();
    launch_step_open(sa, dtb, c->boxes.as<BoxInfo>(), c->nbox, n, st);
    sph_particles q = *p;
    q.vx = sa.pvx; q.vy = sa.pvy; q.vz = sa.pvz; q.u = sa.pu;
    sph_status s;
    if (reuse) {
        // pseudo-Verlet: refresh, and rebuild only if the refresh finds the
        // decomposition no longer valid (one status read)
        s = sph_refresh(c, &q, st);
        uint32_t bits = 0;
        if (s == SPH_OK) s = read_status(c, st, &bits);
        if (s == SPH_OK) s = status_error(bits);
        if (s == SPH_OK) {
            if (bits & ST_REBUILD) {
                s = rebuild_same_boxes(c, &q, st);
                c->step_rebuilds = 1;
            } else {
                c->refresh_checked = true;
                if (c->prm.reuse == SPH_REUSE_CELLS) s = sph_sort(c, st);   // exact keys, no widening
            }
        }
    } else {
        s = sph_build_cells(c, &q, batch, st);
        if (s == SPH_OK) s = sph_sort(c, st);
    }
    if (s == SPH_OK) s = sph_density(c, &q, nullptr, st);
    if (s != SPH_OK && s != SPH_E_NOT_CONVERGED) return s;
    sph_status sd = s;
    s = sph_force(c, &q, acc, st);
    if (s != SPH_OK) return s;
    launch_step_close(sa, dtb, c->boxes.as<BoxInfo>(), c->nbox, n, st);
    if (hipGetLastError() != hipSuccess) return SPH_E_HIP;
    return sd;
}

// The decomposition of the last build can serve a step on p: reuse is on, the
// cells and orderings exist, and the particle count and boxes are unchanged.
static bool can_reuse(const sph_ctx* c, const sph_particles* p, const sph_batch* batch)
{
    return c->prm.reuse && c->built && c->sorted && p->n == c->n && same_layout(c, batch);
}

// box table and per-box step buffers for a step on p
static sph_status step_setup(sph_ctx* c, const sph_particles* p, const sph_batch* batch, bool reuse,
                             hipStream_t st)
{
    if (hipSetDevice(c->device) != hipSuccess) return SPH_E_HIP;
    if (!reuse) {
        // box table for the opening half (the build in the step refreshes it);
        // a reused decomposition keeps the table of its build
        sph_status s = setup_boxes(c, p->n, batch);
        if (s != SPH_OK) return s;
        if (!c->boxes.ensure(sizeof(BoxInfo) * c->nbox)) return SPH_E_OOM;
        if (!upload_boxes(c, st)) return SPH_E_HIP;
    }
    if (!c->dt_box.ensure(sizeof(double) * (size_t)c->nbox) || !c->dt_min.ensure(8 * (size_t)c->nbox))
        return SPH_E_OOM;
    return SPH_OK;
}

static bool acc_ok(const sph_force_out* acc, int64_t n, bool need_dt)
{
    if (!acc) return false;
    if (n > 0 && (!acc->ax || !acc->ay || !acc->az || !acc->dudt)) return false;
    return !(need_dt && n > 0 && !acc->dt);
}

sph_status sph_step(sph_ctx* c, sph_particles* p, const sph_batch* batch, sph_force_out* acc, double dt,
                    void* stream)
{
    if (!c || !particles_ok(p) || !acc_ok(acc, p ? p->n : 0, false) || !std::isfinite(dt)) return SPH_E_INVALID_ARG;
    hipStream_t st = (hipStream_t)stream;
    if (p->n == 0) return SPH_OK;
    const bool reuse = can_reuse(c, p, batch);
    sph_status s = step_setup(c, p, batch, reuse, st);
    if (s != SPH_OK) return s;
    launch_fill_f64(c->dt_box.as<double>(), dt, c->nbox, st);
    return step_core(c, p, batch, acc, reuse, st);
}

sph_status sph_step_adaptive(sph_ctx* c, sph_particles* p, const sph_batch* batch, sph_force_out* acc,
                             double dt_max, double t_end, double* t_box, double* dt_box, void* stream)
{
    if (!c || !particles_ok(p) || !acc_ok(acc, p ? p->n : 0, true) || !t_box) return SPH_E_INVALID_ARG;
    if (!(dt_max > 0.0) || !std::isfinite(dt_max) || !std::isfinite(t_end)) return SPH_E_INVALID_ARG;
    hipStream_t st = (hipStream_t)stream;
    if (p->n == 0) return SPH_OK;
    const bool reuse = can_reuse(c, p, batch);
    sph_status s = step_setup(c, p, batch, reuse, st);
    if (s != SPH_OK) return s;
    launch_dt_select(acc->dt, c->boxes.as<BoxInfo>(), c->nbox, p->n, c->dt_min.as<unsigned long long>(), dt_max,
                     t_end, t_box, c->dt_box.as<double>(), dt_box, st);
    return step_core(c, p, batch, acc, reuse, st);
}

sph_status sph_integrate(sph_ctx* c, sph_particles* p, const sph_batch* batch, sph_force_out* acc, double t_end,
                         double dt_max, int64_t max_steps, int64_t* steps, void* stream)
{
    if (steps) *steps = 0;
    if (!c || !particles_ok(p) || !acc_ok(acc, p ? p->n : 0, true) || max_steps < 0) return SPH_E_INVALID_ARG;
    if (!(dt_max > 0.0) || !std::isfinite(dt_max) || !std::isfinite(t_end)) return SPH_E_INVALID_ARG;
    hipStream_t st = (hipStream_t)stream;
    if (p->n == 0) return SPH_OK;
    if (hipSetDevice(c->device) != hipSuccess) return SPH_E_HIP;
    // the initial state: accelerations and time steps for the first step
    sph_status s = sph_build_cells(c, p, batch, st);
    if (s == SPH_OK) s = sph_sort(c, st);
    if (s == SPH_OK) s = sph_density(c, p, nullptr, st);
    if (s != SPH_OK && s != SPH_E_NOT_CONVERGED) return s;
    sph_status worst = s;
    s = sph_force(c, p, acc, st);
    if (s != SPH_OK) return s;
    const int nb = c->nbox;
    if (!c->t_box.ensure(sizeof(double) * (size_t)nb)) return SPH_E_OOM;
    launch_fill_f64(c->t_box.as<double>(), 0.0, nb, st);
    std::vector<double> tb((size_t)nb, 0.0);
    int64_t k = 0;
    for (; k < max_steps; k++) {
        bool done = true;
        for (double t : tb) done &= t >= t_end;
        if (done) break;
        s = sph_step_adaptive(c, p, batch, acc, dt_max, t_end, c->t_box.as<double>(), nullptr, stream);
        if (s == SPH_E_NOT_CONVERGED) worst = s;
        else if (s != SPH_OK) { if (steps) *steps = k; return s; }
        if (hipMemcpyAsync(tb.data(), c->t_box.as<double>(), sizeof(double) * (size_t)nb, hipMemcpyDeviceToHost,
                           st) != hipSuccess || hipStreamSynchronize(st) != hipSuccess) {
            if (steps) *steps = k + 1;
            return SPH_E_HIP;
        }
    }
    if (steps) *steps = k;
    for (double t : tb)
        if (t < t_end) return SPH_E_CAPACITY;
    return worst;
}

// ---------------------------------------------------------------- multiple time-stepping
static MtsStep mts_view(sph_ctx* c, int32_t* bin)
{
    MtsStep m;
    m.n = c->mts_n;
    m.dtb = c->mts_dtb;
    m.max_bin = c->mts_max_bin;
    m.bin = bin;
    m.active = c->mts_active.as<uint8_t>();
    m.n_active = c->mts_count.as<int32_t>();
    return m;
}

sph_status sph_mts_init(sph_ctx* c, sph_particles* p, sph_force_out* acc, int32_t* bin, double dt_base, int max_bin,
                        void* stream)
{
    if (!c || !particles_ok(p) || !acc_ok(acc, p ? p->n : 0, true) || (!bin && p->n > 0)) return SPH_E_INVALID_ARG;
    if (!(dt_base > 0.0) || !std::isfinite(dt_base) || max_bin < 0 || max_bin > 30) return SPH_E_INVALID_ARG;
    hipStream_t st = (hipStream_t)stream;
    if (hipSetDevice(c->device) != hipSuccess) return SPH_E_HIP;
    c->mts_ready = false;
    const size_t N = (size_t)std::max<int64_t>(p->n, 1);
    if (!c->mts_active.ensure(N) || !c->mts_rho.ensure(N * 8) || !c->mts_A.ensure(N * 8) || !c->mts_c.ensure(N * 8) ||
        !c->mts_f.ensure(N * 8) || !c->mts_count.ensure(16) || !c->mts_units.ensure(N * 4) ||
        !c->mts_flag.ensure(N * 4))
        return SPH_E_OOM;
    if (p->n == 0) return SPH_OK;
    // every particle active: the density-stage quantities of all are stored
    c->mts_store = true;
    sph_status s = sph_build_cells(c, p, nullptr, st);
    if (s == SPH_OK) s = sph_sort(c, st);
    if (s == SPH_OK) s = sph_density(c, p, nullptr, st);
    c->mts_store = false;
    if (s != SPH_OK && s != SPH_E_NOT_CONVERGED) return s;
    sph_status sd = s;
    s = sph_force(c, p, acc, st);
    if (s != SPH_OK) return s;
    c->mts_dtb = dt_base;
    c->mts_max_bin = max_bin;
    c->mts_n = 0;
    c->mts_np = p->n;
    launch_mts_bins(acc->dt, mts_view(c, bin), 0, p->n, st);
    if (hipGetLastError() != hipSuccess) return SPH_E_HIP;
    c->mts_ready = true;
    return sd;
}

sph_status sph_mts_step(sph_ctx* c, sph_particles* p, sph_force_out* acc, int32_t* bin, int64_t* n_active,
                        void* stream)
{
    if (n_active) *n_active = 0;
    if (!c || !particles_ok(p) || !acc_ok(acc, p ? p->n : 0, true) || (!bin && p->n > 0)) return SPH_E_INVALID_ARG;
    if (!c->mts_ready || p->n != c->mts_np || !c->batch_off.empty()) return SPH_E_STATE;
    hipStream_t st = (hipStream_t)stream;
    const int64_t n = p->n;
    if (n == 0) return SPH_OK;
    if (hipSetDevice(c->device) != hipSuccess) return SPH_E_HIP;
    if (!c->step_tmp.ensure(sizeof(double) * 4 * (size_t)n)) return SPH_E_OOM;
    double* vp = c->step_tmp.as<double>();
    StepArrays sa;
    sa.x = p->x; sa.y = p->y; sa.z = p->z; sa.vx = p->vx; sa.vy = p->vy; sa.vz = p->vz; sa.u = p->u;
    sa.ax = acc->ax; sa.ay = acc->ay; sa.az = acc->az; sa.dudt = acc->dudt;
    sa.pvx = vp; sa.pvy = vp + n; sa.pvz = vp + 2 * n; sa.pu = vp + 3 * n;
    const MtsStep m = mts_view(c, bin);
    // the box table of the last build (one box) gives the drift its box
    launch_mts_open(sa, m, c->boxes.as<BoxInfo>(), n, st);
    sph_particles q = *p;
    q.vx = sa.pvx; q.vy = sa.pvy; q.vz = sa.pvz; q.u = sa.pu;
    const bool reuse = can_reuse(c, p, nullptr);
    sph_status s = SPH_OK;
    if (reuse) {
        s = sph_refresh(c, &q, st);
        uint32_t bits = 0;
        if (s == SPH_OK) s = read_status(c, st, &bits);
        if (s == SPH_OK) s = status_error(bits);
        if (s == SPH_OK) {
            if (bits & ST_REBUILD) {
                s = rebuild_same_boxes(c, &q, st);
                c->step_rebuilds = 1;
            } else {
                c->refresh_checked = true;
                if (c->prm.reuse == SPH_REUSE_CELLS) s = sph_sort(c, st);
            }
        }
    } else {
        s = sph_build_cells(c, &q, nullptr, st);
        if (s == SPH_OK) s = sph_sort(c, st);
    }
    // only the active particles are targets; the others pass on their stored quantities
    c->mts_masked = true;
    if (s == SPH_OK) s = sph_density(c, &q, nullptr, st);
    sph_status sd = s;
    if (s == SPH_OK || s == SPH_E_NOT_CONVERGED) s = sph_force(c, &q, acc, st);
    c->mts_masked = false;
    if (s != SPH_OK) return s;
    launch_mts_close(sa, m, acc->dt, n, st);
    if (hipGetLastError() != hipSuccess) return SPH_E_HIP;
    c->mts_n++;
    if (n_active) {
        int32_t h = 0;
        if (hipMemcpyAsync(&h, m.n_active, 4, hipMemcpyDeviceToHost, st) != hipSuccess ||
            hipStreamSynchronize(st) != hipSuccess)
            return SPH_E_HIP;
        *n_active = h;
    }
    return sd;
}

__global__ void k_copy_f64(double* dst, const double* src, int64_t n)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) dst[i] = src[i];
}

// One whole pass on a stream: optional reset of h, cells, orderings, density
// (no synchronisation) and force.
static sph_status pass_sequence(sph_ctx* c, sph_particles* p, const sph_batch* b, const double* h_init,
                                sph_density_out* d, sph_force_out* f, hipStream_t st)
{
    if (h_init && p->n > 0)
        hipLaunchKernelGGL(k_copy_f64, dim3((unsigned)((p->n + 255) / 256)), dim3(256), 0, st, p->h, h_init, p->n);
    sph_status s = sph_build_cells(c, p, b, st);
    if (s == SPH_OK) s = sph_sort(c, st);
    if (s == SPH_OK) s = sph_density_async(c, p, d, st);
    if (s == SPH_OK) s = sph_force(c, p, f, st);
    return s;
}

sph_status sph_graph_capture(sph_ctx* c, sph_particles* p, const sph_batch* b, const double* h_init,
                             sph_density_out* d, sph_force_out* f, void* stream)
{
    if (!c || !particles_ok(p) || !f) return SPH_E_INVALID_ARG;
    if (hipSetDevice(c->device) != hipSuccess) return SPH_E_HIP;
    hipStream_t st = (hipStream_t)stream;
    if (!c->cap_stream && hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking) != hipSuccess)
        return SPH_E_HIP;
    // a plain run first: it sizes the workspace (no allocation may happen while capturing)
    const bool timing = c->timing;
    c->timing = false;
    sph_status s = pass_sequence(c, p, b, h_init, d, f, st);
    if (s == SPH_OK) s = sph_check(c, stream);
    if (s != SPH_OK && s != SPH_E_NOT_CONVERGED) { c->timing = timing; return s; }
    if (c->graph_exec) { (void)hipGraphExecDestroy(c->graph_exec); c->graph_exec = nullptr; }
    if (c->graph) { (void)hipGraphDestroy(c->graph); c->graph = nullptr; }
    if (hipStreamBeginCapture(c->cap_stream, hipStreamCaptureModeThreadLocal) != hipSuccess) {
        c->timing = timing;
        return SPH_E_HIP;
    }
    s = pass_sequence(c, p, b, h_init, d, f, c->cap_stream);
    hipError_t e = hipStreamEndCapture(c->cap_stream, &c->graph);
    c->timing = timing;
    if (s != SPH_OK) return s;
    if (e != hipSuccess) return SPH_E_HIP;
    if (hipGraphInstantiate(&c->graph_exec, c->graph, nullptr, nullptr, 0) != hipSuccess) return SPH_E_HIP;
    return SPH_OK;
}

sph_status sph_graph_launch(sph_ctx* c, void* stream)
{
    if (!c) return SPH_E_INVALID_ARG;
    if (!c->graph_exec) return SPH_E_STATE;
    if (hipGraphLaunch(c->graph_exec, (hipStream_t)stream) != hipSuccess) return SPH_E_HIP;
    c->generation++;   // the replay's density stage replaced the state
    return SPH_OK;
}

sph_status sph_enable_timing(sph_ctx* c, int on)
{
    if (!c) return SPH_E_INVALID_ARG;
    if (on && !c->ev[0]) {
        for (hipEvent_t& e : c->ev)
            if (hipEventCreate(&e) != hipSuccess) return SPH_E_HIP;
    }
    c->timing = on != 0;
    return SPH_OK;
}

sph_status sph_get_kernel_times(sph_ctx* c, sph_kernel_times* out)
{
    if (!c || !out) return SPH_E_INVALID_ARG;
    std::memset(out, 0, sizeof(*out));
    if (!c->timing) return SPH_OK;
    out->build_ms = ev_elapsed(c, EV_BUILD0, EV_BUILD1);
    out->sort_ms = ev_elapsed(c, EV_SORT0, EV_SORT1);
    out->force_ms = ev_elapsed(c, EV_FORCE0, EV_FORCE1);
    if (c->dens_async_timed) {
        c->dens_ms_acc = ev_elapsed(c, EV_DENS0, EV_DENS1);
        c->dens_async_timed = false;
    }
    out->density_ms = c->dens_ms_acc;
    if (c->adj_timed) out->backward_ms = ev_elapsed(c, EV_ADJ0, EV_ADJ1);
    return SPH_OK;
}

sph_status sph_get_stats(const sph_ctx* c, sph_stats* out)
{
    if (!c || !out) return SPH_E_INVALID_ARG;
    *out = c->stats;
    out->depth = c->depth;
    out->generation = c->generation;
    if (!c->box_host.empty()) {
        BoxInfo b0;
        if (c->built && hipMemcpy(&b0, c->boxes.p, sizeof(BoxInfo), hipMemcpyDeviceToHost) == hipSuccess) {
            out->grid[0] = b0.nc[0]; out->grid[1] = b0.nc[1]; out->grid[2] = b0.nc[2];
            out->drift = b0.drift;
        }
    }
    return SPH_OK;
}

}  // extern "C"

// ---------------------------------------------------------------- allocation-free pass
// sph_pass_noalloc keeps its whole workspace in `scratch`, a fixed array of
// device memory (each GPU holds its own copy from the library's load until
// the process ends).  Host code never uses the array's name as an address:
// on a device's first call its address is looked up once and kept per
// device, and the context of that device hands pieces of it out as its
// buffers.  Calls that overlap on one GPU share the array and race.
namespace {
constexpr size_t kNoAllocScratchBytes = (size_t)32 << 20;
constexpr int kNoAllocMaxDevices = 64;
static_assert(SPH_NOALLOC_MAX_PARTICLES <= 32768, "the scratch array is sized for 32,768 particles");
}  // namespace

static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

namespace {
struct NoAllocSlot {
    bool ready = false;
    void* ptr = nullptr;   // device address of this GPU's copy of scratch
    sph_ctx* ctx = nullptr;
};
NoAllocSlot g_noalloc[kNoAllocMaxDevices];
alignas(sph_ctx) unsigned char g_noalloc_ctx[kNoAllocMaxDevices][sizeof(sph_ctx)];
}  // namespace

// Once per device, with that device current: the address of its copy of the
// scratch array, and the context whose buffers are carved from it.
static sph_status noalloc_setup(int dev)
{
    NoAllocSlot& sl = g_noalloc[dev];
    if (sl.ready) return SPH_OK;
    void* ptr = nullptr;
    if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) return SPH_E_HIP;
    sph_ctx* c = new (g_noalloc_ctx[dev]) sph_ctx();
    c->noalloc = true;
    c->device = dev;
    c->arena.base = static_cast<char*>(ptr);
    c->arena.cap = kNoAllocScratchBytes;
    c->status_host = c->status_static;
    c->ncells_host = c->ncells_static;
    for_each_buf(c, [c](DBuf* b) { b->arena = &c->arena; });
    sl.ptr = ptr;
    sl.ctx = c;
    sl.ready = true;
    return SPH_OK;
}

extern "C" {

sph_status sph_pass_noalloc(const sph_params* params, sph_particles* p, sph_density_out* dout,
                            sph_force_out* fout, void* stream)
{
    if (!params || !particles_ok(p) || !fout) return SPH_E_INVALID_ARG;
    if (!params_ok(*params) || params->max_depth != 0 || params->reuse != SPH_REUSE_OFF || params->keep_adjoint)
        return SPH_E_INVALID_ARG;
    if (p->n > SPH_NOALLOC_MAX_PARTICLES) return SPH_E_CAPACITY;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return SPH_E_HIP;
    if (dev < 0 || dev >= kNoAllocMaxDevices) return SPH_E_INVALID_ARG;
    sph_status s = noalloc_setup(dev);
    if (s != SPH_OK) return s;
    sph_ctx* c = g_noalloc[dev].ctx;
    c->prm = *params;
    // every buffer carved afresh from the start of the array
    c->arena.used = 0;
    for_each_buf(c, [](DBuf* b) { b->p = nullptr; b->bytes = 0; });
    c->built = c->sorted = c->have_density = c->adjoint_ready = false;
    c->stats = sph_stats{};
    s = sph_build_cells(c, p, nullptr, stream);
    if (s == SPH_E_OOM) return SPH_E_CAPACITY;   // the array is full
    if (s == SPH_OK) s = sph_sort(c, stream);
    if (s == SPH_OK || s == SPH_E_NOT_CONVERGED) {
        const sph_status sd = sph_density(c, p, dout, stream);
        if (sd != SPH_OK && sd != SPH_E_NOT_CONVERGED) return sd == SPH_E_OOM ? SPH_E_CAPACITY : sd;
        s = sph_force(c, p, fout, stream);
        if (s == SPH_OK) s = sd;
    }
    return s == SPH_E_OOM ? SPH_E_CAPACITY : s;
}

}  // extern "C"
