/*
 * sph.h -- C ABI of the MI355X (gfx950) SPH density/force library.
 *
 * The library evaluates the two interaction stages of smoothed particle
 * hydrodynamics as described by P. Gonnet (2014), "Efficient and Scalable
 * Algorithms for Smoothed Particle Hydrodynamics on Hybrid Shared/Distributed-
 * Memory Architectures":
 *
 *   density stage  Sec. 2.1, Eq. (2): rho_i = sum_{r_ij < h_i} m_j W(r_ij, h_i),
 *                  with h_i solved by Newton iteration so that the weighted
 *                  neighbour count of Eq. (3) equals n_ngb;
 *   force stage    Sec. 2.1, Eqs. (4)-(5), plus the Monaghan-Balsara viscosity
 *                  and Balsara switch of Sec. 4.1, over r_ij < max(h_i, h_j);
 *
 * over the cell decomposition of Sec. 3.2 (cells of edge >= the largest h,
 * self and pair interactions between neighbouring cells, periodic images)
 * with the per-cell particle orderings along the 13 cell-pair axes of
 * Sec. 3.3.  W is the cubic spline of Sec. 2.1 with compact support h.
 *
 * Conventions for every entry point
 * ---------------------------------
 * - Particle, output and gradient arrays are DEVICE pointers owned by the
 *   caller, one value per particle, in the caller's particle order, FP64
 *   unless stated.  The library never frees or retains them past the call.
 * - `stream` is a hipStream_t passed as void*; NULL means the default stream.
 *   All work is enqueued asynchronously on it.  Calls that must inspect a
 *   device-side status (convergence, rebuild requests) synchronise that stream
 *   once per call, and say so.
 * - Every call returns an sph_status; nothing is thrown across the ABI.  On
 *   an argument error nothing is launched.
 * - A context (sph_ctx) owns the device workspace (cell table, sorted
 *   orderings, cell-ordered particle copies, queues).  It grows on demand and
 *   is freed by sph_destroy.  A context is bound to the device that was
 *   current at sph_create and must not be used from two host threads at once.
 */
#ifndef SPH_MI355X_H
#define SPH_MI355X_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    SPH_OK = 0,
    SPH_E_INVALID_ARG = 1,   /* null pointer, n < 0, bad parameter, inconsistent batch */
    SPH_E_NONFINITE = 2,     /* a position, velocity, mass, u or h is NaN/Inf, or m, h <= 0 */
    SPH_E_H_TOO_LARGE = 3,   /* some h >= box/3: a periodic box cannot hold three cells of edge >= h */
    SPH_E_NOT_CONVERGED = 4, /* the h iteration hit max_iter for some particle (outputs still written) */
    SPH_E_CAPACITY = 5,      /* a workspace limit was exceeded (see sph_status_string) */
    SPH_E_OOM = 6,           /* device allocation failed */
    SPH_E_HIP = 7,           /* a HIP runtime call failed */
    SPH_E_STATE = 8          /* call order violated (e.g. sph_force before sph_density) */
} sph_status;

/* Arithmetic of the pair interactions. */
enum {
    SPH_FP64 = 0,        /* every pair term and every sum in FP64 ("plain" form) */
    SPH_FP32_ACC64 = 1   /* pair terms in FP32 on cell-relative coordinates; per-particle
                            sums and the Newton step on h in FP64 (the sums reach FP64
                            through FP32 partial sums over one neighbour list, of at
                            most 48 pairs in the density stage and 32 in the force stage) */
};

typedef struct {
    double box[3];       /* periodic box lengths for single-box calls */
    double n_ngb;        /* target weighted neighbour count of Eq. (3); the paper uses 48 */
    double ngb_tol;      /* convergence: |N_i - n_ngb| <= ngb_tol; 0 selects 1e-10 (FP64)
                            or 1e-4 (FP32_ACC64) */
    int max_iter;        /* Newton evaluations per particle before SPH_E_NOT_CONVERGED */
    double gamma;        /* adiabatic index, P = (gamma-1) rho u; the paper uses 5/3 */
    double alpha;        /* viscosity coefficient of Sec. 4.1; the paper uses 0.8 */
    double balsara_eps;  /* the 1e-4 in the Balsara switch denominator of Sec. 4.1 */
    int precision;       /* SPH_FP64 or SPH_FP32_ACC64 */
    int cell_target;     /* top-cell edge is the larger of (1+h_margin)*max h and the edge that
                            holds cell_target particles at the mean density (Sec. 3.2 only
                            requires edge >= max h) */
    double h_margin;     /* relative slack on h when cells are built, so that h may grow by
                            this fraction during the iteration without a rebuild */
    int max_rebuilds;    /* sph_density rebuilds the cells at most this often when an h
                            outgrows them */
    int max_depth;       /* hierarchical decomposition (Sec. 3.2): levels of bisection allowed
                            below the top grid; 0 keeps the single-level grid.  Capped at 12
                            and by the 64-bit keys. */
    int split_count;     /* a cell is split when it holds more than this many particles ... */
    double split_frac;   /* ... and at least this fraction of them has h below half its edge */
    double cfl;          /* C_CFL of the time-step criterion, Eq. (6); the paper uses 1/4 */
    int balsara_form;    /* numerator of the Balsara switch f_i of Sec. 4.1:
                            SPH_BALSARA_CURL as printed there, or SPH_BALSARA_DIV */
    int reuse;           /* reuse of the decomposition across steps by sph_step and
                            sph_step_adaptive (SPH_REUSE_*) */
    int staging;         /* FP32 density stage: sources staged per wavefront and work-groups
                            per compute unit (SPH_STAGING_*); FP64 has one form */
    int shared_min;      /* force stage: cells of more than this many particles are swept
                            shared (each wavefront takes 64 targets and walks the sources
                            staged by all four, so that a batch of sources is staged once
                            per 256 targets rather than per 64); >= 64; results agree
                            with the other sweep up to summation order */
    int fixed_h;         /* 0: sph_density solves h (Eq. (3)); 1: sph_density evaluates every
                            sum at the caller's h as given (no Newton iteration, n_iter = 0),
                            the forward pass of the fixed-h derivative of sph_backward; cells
                            are rebuilt when a given h outgrows them */
    int keep_adjoint;    /* 1: sph_density also keeps the per-particle sums the reverse pass
                            needs (64 bytes per particle), which sph_backward requires;
                            0 (default): forward-only passes write nothing of the kind */
    int sweep;           /* work layout of the density and force kernels (SPH_SWEEP_*) */
} sph_params;

/* Work layout of the density and force kernels.  Both sweep the same sorted
 * segments of Sec. 3.3 with the same early exit and give the same results up
 * to the order of summation. */
enum {
    SPH_SWEEP_AUTO = 0,   /* SPLIT (the faster of the two on every workload measured) */
    SPH_SWEEP_SHARED = 1, /* four wavefronts per target cell: each stages a share of the sources
                             and all of them read every share; each target is served by four
                             lanes holding its whole neighbour list.  Cells whose sources do not
                             fit in one staging batch are swept by SPLIT right after */
    SPH_SWEEP_SPLIT = 2   /* four wavefronts per target cell, each staging a share of the
                             sources and sweeping only its own (the staging and shared_min
                             parameters apply) */
};

/* Staging of the FP32 density stage.  A target cell's sources are copied into
 * LDS per wavefront; when they do not fit, every Newton step stages and walks
 * them again.  Compact staging keeps four work-groups per compute unit and
 * suits cells of up to ~80 particles at the usual h / edge (the lattice and
 * hierarchy workloads); wide staging holds a third more at three work-groups
 * per compute unit, for single-level grids whose cells hold ~80-110 (a dense
 * region under cells sized for the largest h, as in the Sod tube).  Both
 * give the same results up to summation order. */
enum {
    SPH_STAGING_COMPACT = 0,  /* 192 sources per wavefront, 4 work-groups per CU */
    SPH_STAGING_WIDE = 1      /* 256 sources per wavefront, 3 work-groups per CU */
};

/* Decomposition reuse across steps (the pseudo-Verlet scheme of Sec. 3.3 and
 * Sec. 4.1).  While the particle count and boxes are unchanged and the
 * refresh finds the cells still valid, a step calls sph_refresh instead of
 * sph_build_cells + sph_sort; otherwise it rebuilds. */
enum {
    SPH_REUSE_OFF = 0,        /* rebuild cells and orderings every step */
    SPH_REUSE_ORDERINGS = 1,  /* keep cells and orderings (the paper's scheme): the sweeps widen
                                 by the displacement since the orderings were made */
    SPH_REUSE_CELLS = 2       /* keep the cells, make the orderings again (sph_sort) every step:
                                 exact orderings, only the staging reach and the h limit
                                 carry the displacement */
};

/* Numerator of the Balsara switch f = X / (|div v| + |curl v| + eps c/h). */
enum {
    SPH_BALSARA_CURL = 0,  /* X = |curl v|, the formula as printed in Sec. 4.1 */
    SPH_BALSARA_DIV = 1    /* X = |div v|, the switch of Balsara (1995) that Sec. 4.1 cites:
                              full viscosity in compressions, none in pure shear */
};

/* Default parameters: the paper's constants (48, 5/3, 0.8, 1e-4, C_CFL 1/4),
 * FP32_ACC64, cell_target 64, h_margin 0.1, max_iter 64, max_rebuilds 4, unit
 * box, max_depth 0 (single-level grid), split_count 64, split_frac 0.875,
 * balsara_form SPH_BALSARA_CURL, reuse SPH_REUSE_OFF, staging SPH_STAGING_COMPACT,
 * shared_min 128. */
void sph_default_params(sph_params *p);

typedef struct {
    int64_t n;
    double *x, *y, *z;        /* positions; wrapped into [0, box) by sph_step */
    double *vx, *vy, *vz;     /* velocities */
    double *u;                /* internal energy per unit mass */
    double *m;                /* masses */
    double *h;                /* smoothing lengths: initial guess in, solved value out (sph_density) */
} sph_particles;

/* Batched form: nbox independent periodic boxes in one set of arrays.  The
 * particles of box b are [box_offsets[b], box_offsets[b+1]).  box_offsets
 * (nbox+1 entries) and box_len (3*nbox) are HOST arrays, copied at the call. */
typedef struct {
    int nbox;
    const int64_t *box_offsets;
    const double *box_len;
} sph_batch;

/* Density-stage outputs (any pointer may be NULL to skip that output). */
typedef struct {
    double *rho;       /* Eq. (2) */
    double *omega;     /* Omega_i = 1 + h_i/(3 rho_i) d rho_i/d h_i (Sec. 2.1) */
    double *n_ngb;     /* weighted neighbour count of Eq. (3) at the solved h */
    double *div_v;     /* velocity divergence of Sec. 4.1 */
    double *curl_v;    /* velocity curl of Sec. 4.1, 3 values per particle (x,y,z interleaved) */
    double *balsara;   /* Balsara switch f_i of Sec. 4.1 */
    double *pressure;  /* P_i = (gamma-1) rho_i u_i */
    double *sound;     /* c_i = sqrt(gamma P_i / rho_i) */
    int32_t *n_iter;   /* Newton evaluations used, -1 if not converged */
    int32_t *n_dens;   /* number of j != i with r_ij < h_i at the solved h */
} sph_density_out;

/* Force-stage outputs (any pointer may be NULL). */
typedef struct {
    double *ax, *ay, *az;   /* dv/dt, Eq. (4) plus viscosity */
    double *dudt;           /* du/dt, Eq. (5) plus viscosity */
    int32_t *n_pairs;       /* number of j != i with r_ij < max(h_i, h_j) */
    double *dt;             /* time step of Eq. (6): C_CFL 2 h_i / vsig_i with
                               vsig_i = max_j (c_i + c_j + max(0, -3 v_ij.r_ij / r_ij)) over
                               the j with r_ij < max(h_i, h_j) and over j = i (term 2 c_i);
                               +inf where vsig_i = 0 */
} sph_force_out;

typedef struct sph_ctx sph_ctx;

/* Create a context on the current HIP device.  params may be NULL (defaults).
 * Errors: SPH_E_INVALID_ARG (bad parameter), SPH_E_HIP. */
sph_status sph_create(const sph_params *params, sph_ctx **ctx);

/* Free the context and all its device memory. NULL is accepted. */
sph_status sph_destroy(sph_ctx *ctx);

/* Cell decomposition (Sec. 3.2): wraps positions into the box, takes the
 * largest h (per box), builds the top-level grid of cells with edge >=
 * (1+h_margin) max h, keys each particle by the Morton code of its cell,
 * radix-sorts the keys, and forms cells as runs of equal keys, their
 * neighbour lists (self + 26 neighbours, periodic images included) and
 * cell-ordered copies of the particle data.  With max_depth > 0 the keys
 * encode cells down to max_depth bisections of the top cells, a cell is split
 * while it holds more than split_count particles of which at least split_frac
 * have h below half its edge, and the cells are the leaves of that
 * hierarchy; each leaf's list then holds every leaf whose box lies within
 * the largest h either cell covers (so every pair in range is listed).
 * batch may be NULL (one box of params.box).  Reads x, y, z, v, u, m, h.  Does not synchronise: the
 * checks that run on the device (non-finite data, h too large for the box,
 * capacity) are reported by the next sph_density.  Errors returned here:
 * SPH_E_INVALID_ARG, SPH_E_CAPACITY (key or map too large), SPH_E_OOM,
 * SPH_E_HIP. */
sph_status sph_build_cells(sph_ctx *ctx, const sph_particles *p, const sph_batch *batch,
                           void *stream);

/* Pseudo-Verlet reuse of the decomposition (Sec. 3.3 and Sec. 4.1: cells and
 * orderings kept over several steps until particle motion invalidates them):
 * refreshes the cell-ordered copies of x, v, u, m, h from p in the cell
 * membership and orderings of the last sph_build_cells + sph_sort, and
 * records the largest displacement since that build per cell, d(cell), and
 * per box, d(box).  The next sph_density, sph_force and sph_backward keep
 * h_i + d(T) + d(box) within the h limit of i's cell T (every pair in range
 * then lies in a listed cell pair), widen the staging reach of every cell
 * pair (T, S) by d(T) + d(S) and the early exit of a sweep over S by 2 d(S)
 * (the stored order of projections that moved by up to d(S)); an sph_sort
 * after the refresh makes the orderings exact again, which leaves d(T) in
 * the reach and nothing in the early exit.  The refresh requests a rebuild
 * when some h_i (1 + h_margin/2) exceeds that limit; sph_density then
 * rebuilds the cells from p before sweeping (as it also does when a solved
 * h outgrows its cell).  Requires a build and sort on the same particle
 * count and boxes.  Does not synchronise.  Errors: SPH_E_INVALID_ARG,
 * SPH_E_STATE, SPH_E_HIP (non-finite data is reported by the next
 * sph_density). */
sph_status sph_refresh(sph_ctx *ctx, const sph_particles *p, void *stream);

/* Initial smoothing lengths for particles without a usable guess: builds the
 * hierarchy of cells down to max_depth levels (params.max_depth >= 1) with
 * the current h only for the top grid, and sets every h from the local
 * number density n_loc: h = (3 n_ngb / (4 pi n_loc))^(1/3), n_loc being the
 * count over the volume of the smallest cell around the particle that holds
 * at least 2 n_ngb particles.  Writes p->h; the decomposition it builds is
 * not kept (call sph_build_cells afterwards).  Does not synchronise.
 * Errors: SPH_E_INVALID_ARG (also max_depth == 0), SPH_E_CAPACITY, SPH_E_OOM,
 * SPH_E_HIP. */
sph_status sph_estimate_h(sph_ctx *ctx, sph_particles *p, const sph_batch *batch, void *stream);

/* The 13 per-cell orderings of Sec. 3.3: for each cell and each of the 13
 * axis directions d (the other 13 of the 26 cell-pair axes are their
 * negatives), the particle order by ascending projection onto d.  Requires
 * sph_build_cells.  Errors: SPH_E_STATE, SPH_E_HIP. */
sph_status sph_sort(sph_ctx *ctx, void *stream);

/* Density stage with the smoothing-length iteration (Sec. 2.1, Eqs. (2)-(3)):
 * for every particle, Newton iteration on h_i until |N_i - n_ngb| <= ngb_tol,
 * then the per-particle quantities the force stage needs (Omega, P, c, the
 * Balsara switch).  Writes the solved h into p->h.  If an h outgrows the
 * cells, the cells and orderings are rebuilt (at most max_rebuilds times).
 * Requires sph_build_cells and sph_sort on the same particles.  Synchronises
 * `stream` once per (re)build to read the status.  Errors: SPH_E_STATE,
 * SPH_E_NOT_CONVERGED (outputs written, n_iter = -1 where unconverged),
 * SPH_E_H_TOO_LARGE, SPH_E_HIP. */
sph_status sph_density(sph_ctx *ctx, sph_particles *p, sph_density_out *out, void *stream);

/* Density stage without synchronisation: as sph_density, but the device
 * status is not read back and cells are never rebuilt, so the call can be
 * captured in a graph.  Problems found on the device (non-finite data, an h
 * that outgrows its cells, no convergence) are returned by the next
 * sph_check.  Errors returned here: SPH_E_INVALID_ARG, SPH_E_STATE, SPH_E_HIP. */
sph_status sph_density_async(sph_ctx *ctx, sph_particles *p, sph_density_out *out, void *stream);

/* Waits for `stream` and returns the device-side status accumulated since the
 * last sph_build_cells: SPH_OK, SPH_E_NONFINITE, SPH_E_H_TOO_LARGE (also when
 * an h outgrew its cells during sph_density_async), SPH_E_CAPACITY,
 * SPH_E_NOT_CONVERGED, or SPH_E_HIP. */
sph_status sph_check(sph_ctx *ctx, void *stream);

/* Force stage (Sec. 2.1 Eqs. (4)-(5), Sec. 4.1 viscosity) with the densities,
 * h and per-particle quantities of the last sph_density on this context.
 * Requires the particles of that call, unchanged.  Does not synchronise.
 * Errors: SPH_E_STATE, SPH_E_HIP. */
sph_status sph_force(sph_ctx *ctx, const sph_particles *p, sph_force_out *out, void *stream);

/* Upstream gradients of a scalar loss L (caller order; any may be NULL = 0). */
typedef struct {
    const double *rho;          /* dL/d rho_i */
    const double *ax, *ay, *az; /* dL/d a_i */
    const double *dudt;         /* dL/d (du/dt)_i */
} sph_grad_in;

/* Gradients of L (caller order; any may be NULL to skip it). */
typedef struct {
    double *x, *y, *z;   /* dL/dx_i (total: through rho, Omega, div, curl, f, A and every pair term) */
    double *h;           /* dL/dh_i with h held fixed; zeros when implicit_h != 0 */
} sph_grad_out;

/* Reverse mode of the density and force stages (Sec. 2.1 Eqs. (2)-(5) with
 * the Sec. 4.1 viscosity and Balsara switch) at the state of the last
 * sph_density on this context: positions, velocities, masses and u as
 * gathered by the last sph_build_cells, and the solved h.  Given dL/d rho,
 * dL/da and dL/d(du/dt), writes dL/dx and (fixed h) dL/dh.  Velocities,
 * masses and u are constants.
 *   implicit_h = 0: h is an independent input (the fixed-h derivative);
 *   implicit_h = 1: h_i is the solved root of N_i(h_i) = n_ngb (Eq. (3)), so
 *     dh_i/dx = -(dN_i/dx)/(dN_i/dh_i) is included in dL/dx (implicit
 *     function theorem; exact at the root, up to the ngb_tol of the solve).
 * `generation` names the density evaluation the caller means (the
 * sph_stats.generation read after it); 0 takes whichever ran last.  A
 * nonzero value that is not the last one (another forward pass ran on ctx
 * since) is refused, since its state is gone.  With implicit_h = 1 the h of
 * that evaluation must have been solved (params.fixed_h = 0).
 * Pair arithmetic in the context's precision, sums in FP64.  Does not
 * synchronise.  Errors: SPH_E_INVALID_ARG, SPH_E_STATE (no sph_density yet,
 * a different particle count, a stale generation, a context without
 * params.keep_adjoint, or implicit_h with a fixed h), SPH_E_OOM, SPH_E_HIP. */
sph_status sph_backward(sph_ctx *ctx, const sph_particles *p, const sph_grad_in *grad_in,
                        sph_grad_out *grad_out, int implicit_h, uint64_t generation, void *stream);

/* One kick-drift-kick velocity-Verlet step (Sec. 4.1) with fixed dt:
 *   v += dt/2 a, u += dt/2 du/dt  (a, du/dt of the previous step, from `acc`),
 *   x += dt v (wrapped into the box),
 *   cells, orderings, density and force at the new positions, using the
 *   predicted v + dt/2 a_old and u + dt/2 du_old,
 *   v += dt/2 a_new, u += dt/2 du_new, and `acc` overwritten with a_new, du_new.
 * acc->ax..dudt must hold the previous step's values (zeros for a cold start).
 * With params.reuse the cells (and orderings) of the last build are
 * refreshed (sph_refresh, then sph_sort for SPH_REUSE_CELLS) instead of
 * rebuilt, while the particle count and boxes are unchanged and the refresh
 * finds them valid; the step then reads the device status once more.
 * Errors: as sph_build_cells, sph_density. */
sph_status sph_step(sph_ctx *ctx, sph_particles *p, const sph_batch *batch, sph_force_out *acc,
                    double dt, void *stream);

/* Kick-drift-kick step whose length comes from the time-step criterion,
 * Eq. (6): per box b,
 *   dt_b = min(min_{i in b} acc->dt[i], dt_max, t_end - t_box[b])   (>= 0),
 * the smallest particle time step of the previous force evaluation, as the
 * blast-wave test of Sec. 4.2 steps.  Then the step of sph_step with dt_b for
 * the particles of box b, after which acc (a, du/dt and dt) holds the new
 * force evaluation.  t_box (device, nbox values) is advanced by dt_b, and set
 * to t_end exactly when the step was clipped to it; dt_box (device, nbox
 * values, may be NULL) receives dt_b.  A box with t_box >= t_end takes a step
 * of length 0.  acc->dt must hold the time steps of the last force
 * evaluation (run sph_density and sph_force with dt set for a cold start).
 * dt_max must be finite and > 0.  No synchronisation.  Errors: as sph_step. */
sph_status sph_step_adaptive(sph_ctx *ctx, sph_particles *p, const sph_batch *batch, sph_force_out *acc,
                             double dt_max, double t_end, double *t_box, double *dt_box, void *stream);

/* Time integration from t = 0 to t_end (Sec. 4.1 integrator, steps limited by
 * Eq. (6)): the cells, orderings, density and force of the initial state
 * (written to acc, which needs ax..dudt and dt), then sph_step_adaptive
 * steps until every box has reached t_end or max_steps steps were taken.
 * Synchronises `stream` once per step to read the box times.  *steps (may be
 * NULL) receives the number of steps taken.  Errors: as sph_step_adaptive;
 * SPH_E_CAPACITY when max_steps ends the run before t_end. */
sph_status sph_integrate(sph_ctx *ctx, sph_particles *p, const sph_batch *batch, sph_force_out *acc,
                         double t_end, double dt_max, int64_t max_steps, int64_t *steps, void *stream);

/* Multiple time-stepping (Sec. 4.1), one box (batch NULL).  Particle i sits
 * in time bin k_i: the largest k with 2^k dt_base <= its time step of
 * Eq. (6) (k >= 0, at most max_bin, infinite steps in max_bin), lowered until
 * its step starts on a multiple of its length; it takes kick-drift-kick steps
 * of 2^k_i dt_base and is active, a target of the density and force stages,
 * only at the end of each of them.  The other particles are sources with the
 * rho, A, c and f of their last active step (kept by the context).
 *
 * sph_mts_init: a full pass with every particle active (cells, orderings,
 * density, force with dt into acc), the stored quantities of every particle,
 * and bin[i] (device, n values, written) from acc->dt; the base step counter
 * is set to 0.  acc needs ax..dudt and dt.  dt_base > 0, 0 <= max_bin <= 30.
 *
 * sph_mts_step: base step n -> n+1: particles starting a step take the
 * opening half kick v += T_i/2 a_i, u += T_i/2 du_i; every particle drifts
 * by dt_base; velocities and energies are predicted at the end of the base
 * step from each particle's last kick; cells (params.reuse applies),
 * orderings, then density and force for the particles ending their step
 * there (acc, including dt, is written for them only); their closing half
 * kick and their new bin.  *n_active (may be NULL; it costs one stream
 * synchronisation) receives the number of active particles.  Errors: as
 * sph_step; SPH_E_STATE without sph_mts_init on the same particle count, or
 * after a batched build. */
sph_status sph_mts_init(sph_ctx *ctx, sph_particles *p, sph_force_out *acc, int32_t *bin, double dt_base,
                        int max_bin, void *stream);
sph_status sph_mts_step(sph_ctx *ctx, sph_particles *p, sph_force_out *acc, int32_t *bin, int64_t *n_active,
                        void *stream);

/* Graph of one whole pass (the batched persistent form): optional copy of
 * h_init (device, n values; may be NULL) into p->h, then sph_build_cells,
 * sph_sort, sph_density_async and sph_force, captured once into a HIP graph
 * on a stream owned by the context.  The call first runs the pass once
 * without capture (to size the workspace; its results are written) and
 * synchronises `stream`.  The graph keeps every pointer and size given here:
 * replay it with sph_graph_launch only while those buffers stay alive and
 * unchanged in size; a later sph_graph_capture replaces it.  Errors: as the
 * calls it contains, and SPH_E_HIP if capture fails. */
sph_status sph_graph_capture(sph_ctx *ctx, sph_particles *p, const sph_batch *batch, const double *h_init,
                             sph_density_out *dout, sph_force_out *fout, void *stream);

/* Replays the captured pass on `stream` (asynchronous).  Check the outcome
 * with sph_check.  Errors: SPH_E_STATE (nothing captured), SPH_E_HIP. */
sph_status sph_graph_launch(sph_ctx *ctx, void *stream);

/* Statistics of the last calls on ctx (host values, valid after the call
 * that produced them has completed on its stream). */
typedef struct {
    int64_t n_cells;         /* non-empty cells */
    int64_t n_units;         /* work units of the interaction kernels */
    int32_t grid[3];         /* top-level grid of box 0 */
    int32_t rebuilds;        /* rebuilds done by the last sph_density */
    int32_t max_iter_used;   /* largest Newton count of the last sph_density */
    int32_t unconverged;     /* particles left unconverged by the last sph_density */
    int32_t depth;           /* levels below the top grid in the keys of the last build */
    int32_t refreshes;       /* sph_refresh calls since the last build */
    double drift;            /* box 0: the largest displacement since the last build
                                (as of the last sph_refresh) */
    uint64_t generation;     /* count of density evaluations on ctx: sph_density,
                                sph_density_async and every sph_graph_launch add one; the
                                state sph_backward differentiates is that of this one */
} sph_stats;

sph_status sph_get_stats(const sph_ctx *ctx, sph_stats *out);

/* Kernel timing.  While enabled, the library records HIP events on the
 * call's stream immediately around its interaction kernels (and around the
 * build and sort launch sequences); sph_get_kernel_times waits for those
 * events and returns the elapsed milliseconds of the last sph_build_cells,
 * sph_sort, density kernel (every Newton evaluation, summed over rebuild
 * attempts) and force kernel.  Errors: SPH_E_INVALID_ARG, SPH_E_HIP. */
typedef struct {
    float build_ms, sort_ms, density_ms, force_ms;
    float backward_ms;       /* the last sph_backward (0 if none since timing was enabled) */
} sph_kernel_times;

sph_status sph_enable_timing(sph_ctx *ctx, int on);
sph_status sph_get_kernel_times(sph_ctx *ctx, sph_kernel_times *out);

/* Allocation-free pass, for callers that cannot allocate device memory
 * (code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc).  The same as sph_build_cells + sph_sort + sph_density +
 * sph_force on a context created with *params, for one periodic box
 * (params->box) of p->n <= SPH_NOALLOC_MAX_PARTICLES particles, with every
 * device buffer taken from a fixed array of 32 MiB inside the library (one per
 * GPU, held from the library's load until the process ends) instead of being
 * allocated: it calls no device or host allocation routine (its first call on
 * a device looks the array's address up, once).  p->h is the initial guess and receives
 * the solved h; dout (may be NULL, and any field of it) and fout (required;
 * any field may be NULL) are caller-owned device arrays as in sph_density and
 * sph_force.  Synchronises `stream` as sph_density does.  Calls on one GPU
 * share the array: calls that overlap on one GPU (two host threads, two
 * streams) race, and each call overwrites what the last one left there.
 * Requires params->max_depth == 0, params->reuse == SPH_REUSE_OFF and
 * params->keep_adjoint == 0 (no reverse pass).
 * Errors: SPH_E_INVALID_ARG, SPH_E_CAPACITY (p->n above the maximum, or a
 * workspace that would not fit the array), and those of the four calls. */
#define SPH_NOALLOC_MAX_PARTICLES 32768
sph_status sph_pass_noalloc(const sph_params *params, sph_particles *p, sph_density_out *dout,
                            sph_force_out *fout, void *stream);

/* Human-readable text of a status (static storage). */
const char *sph_status_string(sph_status s);

#ifdef __cplusplus
}
#endif
#endif /* SPH_MI355X_H */
