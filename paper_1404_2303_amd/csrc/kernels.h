// kernels.h -- host-side launchers of the SPH kernels and the device views
// they take.  Not part of the public ABI.
#pragma once

#include "sph_internal.h"

namespace sph {

// Caller arrays (caller order, FP64).
struct Particles {
    const double *x, *y, *z, *vx, *vy, *vz, *u, *m, *h;
};

template <typename R> struct Vec4T;
template <> struct Vec4T<float> { using T = float4; };
template <> struct Vec4T<double> { using T = double4; };

// Cell-ordered particle copies.  Positions are relative to the lower corner
// of the particle's cell, in the pair-arithmetic type R.
template <typename R>
struct CellData {
    using R4 = typename Vec4T<R>::T;
    R4* rp;              // (x, y, z, 0) relative to the cell's lower corner: one load
    double* h;           // smoothing length (FP64 master copy)
    R4* vm;              // (vx, vy, vz, m)
    double* u;
};

// The 13 orderings of every cell: for stored direction s and rank k within
// cell C, entry s*n + C.start + k holds the projection on the direction (the
// sort key) and the particle's cell-local index.
template <typename R>
struct Sorted {
    SortRec* rec;   // [direction][cell-order slot]: the cell's particles by ascending projection
};

// Per-particle results of the density stage needed by the force stage, in
// cell order: g0 = (1/h, 8/(pi h^5), A = P/(Omega rho^2), rho),
// g1 = (c, Balsara f, h, 0).
template <typename R>
struct GhostData {
    using R4 = typename Vec4T<R>::T;
    R4 *g0, *g1;
    float* cell_hmax;    // largest h of each cell
    // sums kept for the adjoint (FP64, cell order; may be null):
    // sd0 = (sum m w incl. self, sum m q w', dN/dh, sum m g dv.r), sd1 = (sum m g dv x r, 0)
    double4 *sd0, *sd1;
    // multiple time-stepping (caller order; null when every particle is active):
    // a particle is a target of the density and force stages only where active[i] != 0;
    // the others enter as sources with the rho, A, c, f of their last active step
    const uint8_t* active;
    double *s_rho, *s_A, *s_c, *s_f;
};

// Per-particle adjoint data (cell order).
template <typename R>
struct AdjData {
    using R4 = typename Vec4T<R>::T;
    R4* ab;              // (dL/da_x, dL/da_y, dL/da_z, dL/d(du/dt))
    R4* sb0;             // (dL/dS_mw, dL/dS_mqw', dL/dD, lambda)
    R4* sb1;             // (dL/dC_x, dL/dC_y, dL/dC_z, 0)
    double* xbar;        // dL/dx, 3 per particle
    double* hbar;        // dL/dh (explicit)
    double4* fg;         // (dL/dA, dL/drho from the force stage, dL/df, dL/drho from the caller)
};

// Caller-order upstream gradients and outputs of the adjoint.
struct AdjIO {
    const double *g_rho, *g_ax, *g_ay, *g_az, *g_dudt;
    double *gx, *gy, *gz, *gh;
};

// Caller-order outputs of the density stage (any may be null).
struct DensityOut {
    double *h, *rho, *omega, *nngb, *div, *curl, *balsara, *P, *c;
    int32_t *iters, *ndens;
};

struct ForceOut {
    double *ax, *ay, *az, *dudt;
    int32_t* npairs;
    double* dt;                            // time step of Eq. (6)
    double *ax_c, *ay_c, *az_c, *dudt_c;   // optional cell-order copies (FP64)
};

// Shared view of the decomposition used by the interaction kernels.
struct Decomp {
    const CellInfo* cells;
    const int32_t* ncells;
    const BoxInfo* boxes;
    const Source* src;
    const int32_t* src_off;     // first source of each cell
    const int32_t* src_count;
    const uint32_t* perm;   // cell order -> caller index
    int64_t n;
    int32_t* qhead;         // work counter of the persistent launches
    uint32_t* status;
    const float* cell_drift;  // largest displacement in each cell since the build (null: none)
    int keys_stale;           // the orderings predate that displacement (made before it)
    const int32_t* units;     // the cells to process (null: every cell)
    const int32_t* nunits;    // their number (device)
};

// displacement of cell c's particles since the cells were built
__device__ __forceinline__ float cell_dr(const Decomp& dc, int c) { return dc.cell_drift ? dc.cell_drift[c] : 0.0f; }
// how far the stored projections of cell c may be from the current ones
__device__ __forceinline__ float key_dr(const Decomp& dc, int c)
{
    return (dc.cell_drift && dc.keys_stale) ? dc.cell_drift[c] : 0.0f;
}

// build.hip
void launch_fill_i32(int32_t* a, int64_t n, int32_t v, hipStream_t st);
void launch_box_scan(const Particles& p, BoxInfo* boxes, int nbox, int64_t n, uint32_t* status,
                     hipStream_t st);
void launch_grid_dims(BoxInfo* boxes, int nbox, double margin, int max_nc, uint32_t* status,
                      hipStream_t st);
void launch_keys(const Particles& p, const BoxInfo* boxes, int nbox, int64_t n, int top_bits,
                 uint64_t* keys, uint32_t* vals, hipStream_t st);
size_t radix_scratch_words(int64_t n);
void radix_sort(uint64_t* keys, uint32_t* vals, uint64_t* k2, uint32_t* v2, int64_t n, int bits,
                uint32_t* scratch, hipStream_t st);
size_t scan_scratch_words(int64_t n);
void exclusive_scan(const uint32_t* in, uint32_t* out, int64_t n, uint32_t* scratch, uint32_t* total,
                    hipStream_t st);
// two arrays of n scanned together, each with its own output and total (scratch of scan_scratch_words(n))
void exclusive_scan2(const uint32_t* in0, uint32_t* out0, uint32_t* total0, const uint32_t* in1, uint32_t* out1,
                     uint32_t* total1, int64_t n, uint32_t* scratch, hipStream_t st);
void launch_cells(const uint64_t* keys, uint32_t* flag, uint32_t* cellx, int64_t n, int top_bits,
                  const BoxInfo* boxes, CellInfo* cells, int32_t* cell_map, int64_t map_total,
                  uint32_t* cell_of, int32_t* ncells, uint32_t* scan_scratch, int64_t cell_cap,
                  hipStream_t st);
template <typename R>
void launch_gather(const Particles& p, const uint32_t* perm, const uint32_t* cell_of,
                   const CellInfo* cells, const BoxInfo* boxes, int64_t n, const CellData<R>& cd,
                   typename Vec4T<R>::T* r0, hipStream_t st);
template <typename R>
void launch_refresh(const Particles& p, const uint32_t* perm, const uint32_t* cell_of, const CellInfo* cells,
                    const int32_t* ncells, BoxInfo* boxes, int nbox, int64_t n, const CellData<R>& cd,
                    const typename Vec4T<R>::T* r0, float* cell_drift, double h_margin, uint32_t* status,
                    hipStream_t st);
void launch_sources(const CellInfo* cells, const int32_t* ncells, const BoxInfo* boxes,
                    const int32_t* cell_map, Source* src, int32_t* src_off, int32_t* src_count,
                    int64_t cell_cap, hipStream_t st);
template <typename R>
void launch_sort13(const CellInfo* cells, const int32_t* ncells, const BoxInfo* boxes, const CellData<R>& cd,
                   int64_t n, const Sorted<R>& so, int32_t* big, uint32_t* status, int64_t cell_cap, hipStream_t st);
// big[0]: the number of cells left to the rank sort, big[kBigHeader..]: those cells
constexpr int kBigHeader = 1;

// tree.hip -- hierarchical decomposition below the top grid
struct TreeView {
    int depth;                  // levels below the top grid (>= 1)
    int top_bits;
    int64_t n;
    int64_t stride;             // per-level stride of the node arrays (n + 1)
    const uint64_t* keys;       // sorted keys
    const uint32_t* perm;       // cell order -> caller index
    uint8_t* chg;               // first level whose prefix differs from the previous particle
    uint32_t* node_of;          // [level * n + i]: node of particle i at that level
    uint32_t* node_start;       // [level * stride + m]: first particle of node m (sentinel n)
    uint8_t* node_flag;         // bit 0: live (parent split), bit 1: split
    float* node_hmax;           // largest h of the node's particles at build time
    float* node_H;              // largest interaction bound (cell hlim) of the node's leaves
    int32_t* node_leaf;         // cell index of a leaf node, else -1
    int32_t* nnodes;            // nodes per level
    uint32_t* flag;             // scratch (n)
    uint32_t* scan;             // scratch (n + 1)
    uint32_t* small;            // scratch (n)
    uint32_t* psmall;           // scratch (n + 1)
    uint8_t* lev;               // leaf level of each particle
};
enum : uint8_t { NODE_LIVE = 1, NODE_SPLIT = 2 };

void launch_keys_depth(const Particles& p, const BoxInfo* boxes, int nbox, int64_t n, int top_bits, int depth,
                       uint64_t* keys, uint32_t* vals, hipStream_t st);
void launch_tree(const Particles& p, const TreeView& tv, const BoxInfo* boxes, int split_count, double split_frac,
                 double h_margin, uint32_t* scan_scratch, hipStream_t st);
void launch_tree_cells(const TreeView& tv, const BoxInfo* boxes, CellInfo* cells, int32_t* cell_map,
                       int64_t map_total, uint32_t* cell_of, int32_t* ncells, double h_margin,
                       uint32_t* scan_scratch, hipStream_t st);
void launch_tree_sources(const TreeView& tv, const CellInfo* cells, const int32_t* ncells, const BoxInfo* boxes,
                         const int32_t* cell_map, Source* src, int64_t src_cap, int32_t* src_off,
                         int32_t* src_count, uint32_t* group, uint32_t* status, uint32_t* scan_scratch,
                         int64_t cell_cap, hipStream_t st);
void launch_estimate_h(const TreeView& tv, const BoxInfo* boxes, double n_ngb, double* h, int64_t n,
                       hipStream_t st);

// passes.hip
void launch_reset_counter(int32_t* c, hipStream_t st);
template <typename R>
void launch_density(const Decomp& dc, const CellData<R>& cd, const Sorted<R>& so, const GhostData<R>& gd,
                    const DensityOut& out, const PassConsts& pc, int staging, hipStream_t st);
template <typename R>
void launch_force(const Decomp& dc, const CellData<R>& cd, const Sorted<R>& so, const GhostData<R>& gd,
                  const ForceOut& out, const PassConsts& pc, int grid, hipStream_t st);
template <typename R>
void launch_mts_prepare(const Decomp& dc, const CellData<R>& cd, const GhostData<R>& gd, int32_t* units,
                        int32_t* nunits, uint32_t* cell_flag, const uint32_t* cell_of, int64_t n, hipStream_t st);
int force_occupancy_grid(int precision);

// passes_shared.hip -- sources staged once per work-group, four lanes per
// target; cells whose sources need several batches are left to the split
// kernels above, launched right after over the deferred list.  counters: three
// ints (work counters and the deferred count).
template <typename R>
void launch_density_shared(const Decomp& dc, const CellData<R>& cd, const Sorted<R>& so, const GhostData<R>& gd,
                           const DensityOut& out, const PassConsts& pc, int staging, int32_t* deferred,
                           int32_t* counters, hipStream_t st);
template <typename R>
void launch_force_shared(const Decomp& dc, const CellData<R>& cd, const Sorted<R>& so, const GhostData<R>& gd,
                         const ForceOut& out, const PassConsts& pc, int split_grid, int32_t* deferred,
                         int32_t* counters, hipStream_t st);

// adjoint.hip
template <typename R>
void launch_adjoint(const Decomp& dc, const CellData<R>& cd, const Sorted<R>& so, const GhostData<R>& gd,
                    const AdjData<R>& ad, const AdjIO& io, const PassConsts& pc, bool implicit_h, int64_t n,
                    hipStream_t st);

// step.hip
struct StepArrays {
    double *x, *y, *z, *vx, *vy, *vz, *u;      // caller's state
    const double *ax, *ay, *az, *dudt;         // accelerations of the last force evaluation
    double *pvx, *pvy, *pvz, *pu;              // predicted v, u at the end of the step
};
void launch_step_open(const StepArrays& s, const double* dtb, const BoxInfo* boxes, int nbox, int64_t n,
                      hipStream_t st);
void launch_step_close(const StepArrays& s, const double* dtb, const BoxInfo* boxes, int nbox, int64_t n,
                       hipStream_t st);
void launch_fill_f64(double* a, double v, int n, hipStream_t st);
struct MtsStep {
    int64_t n;          // index of the base step
    double dtb;         // base step
    int max_bin;
    int32_t* bin;       // time bin per particle (caller order)
    uint8_t* active;    // active at the end of base step n
    int32_t* n_active;  // count of active particles (device)
};
void launch_mts_open(const StepArrays& s, const MtsStep& m, const BoxInfo* boxes, int64_t n, hipStream_t st);
void launch_mts_close(const StepArrays& s, const MtsStep& m, const double* dt, int64_t n, hipStream_t st);
void launch_mts_bins(const double* dt, const MtsStep& m, int64_t n_next, int64_t n, hipStream_t st);
void launch_dt_select(const double* dt, const BoxInfo* boxes, int nbox, int64_t n, unsigned long long* mn,
                      double dt_max, double t_end, double* t_box, double* dtb, double* dt_out, hipStream_t st);

}  // namespace sph
