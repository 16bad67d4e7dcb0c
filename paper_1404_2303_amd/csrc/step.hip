// step.hip -- kick-drift-kick velocity Verlet (Gonnet 2014, Sec. 4.1) on the
// caller's FP64 arrays, with one step length per box: a fixed step, or the
// smallest particle time step of Eq. (6) (Sec. 4.2 runs its blast wave so).
#include "sph_internal.h"
#include "kernels.h"

namespace sph {

// box of caller-order particle i (boxes sorted by begin)
__device__ __forceinline__ int box_of(const BoxInfo* boxes, int nbox, int64_t i)
{
    int lo = 0, hi = nbox - 1;
    while (lo < hi) {
        int mid = (lo + hi + 1) >> 1;
        if (boxes[mid].begin <= i) lo = mid; else hi = mid - 1;
    }
    return lo;
}

// Opening half of the step, per particle with dt of its box:
//   v += dt/2 a_old, u += dt/2 du_old, x += dt v (wrapped into [0, L)),
//   predictions for the force evaluation at the new positions:
//   pv = v + dt/2 a_old, pu = u + dt/2 du_old.
__global__ void k_open(StepArrays s, const double* dtb, const BoxInfo* boxes, int nbox, int64_t n)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int b = box_of(boxes, nbox, i);
    const double dt = dtb[b], hdt = 0.5 * dt;
    const double ax = s.ax[i], ay = s.ay[i], az = s.az[i], du = s.dudt[i];
    const double vx = s.vx[i] + hdt * ax, vy = s.vy[i] + hdt * ay, vz = s.vz[i] + hdt * az;
    const double u = s.u[i] + hdt * du;
    s.vx[i] = vx; s.vy[i] = vy; s.vz[i] = vz; s.u[i] = u;
    s.pvx[i] = vx + hdt * ax; s.pvy[i] = vy + hdt * ay; s.pvz[i] = vz + hdt * az; s.pu[i] = u + hdt * du;
    const BoxInfo& B = boxes[b];
    double p[3] = {s.x[i] + dt * vx, s.y[i] + dt * vy, s.z[i] + dt * vz};
    for (int d = 0; d < 3; d++) {
        double w = fmod(p[d], B.L[d]);
        if (w < 0.0) w += B.L[d];
        if (w >= B.L[d]) w -= B.L[d];
        p[d] = w;
    }
    s.x[i] = p[0]; s.y[i] = p[1]; s.z[i] = p[2];
}

// Closing kick with the new accelerations: v += dt/2 a, u += dt/2 du/dt.
__global__ void k_close(StepArrays s, const double* dtb, const BoxInfo* boxes, int nbox, int64_t n)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double hdt = 0.5 * dtb[box_of(boxes, nbox, i)];
    s.vx[i] += hdt * s.ax[i];
    s.vy[i] += hdt * s.ay[i];
    s.vz[i] += hdt * s.az[i];
    s.u[i] += hdt * s.dudt[i];
}

__global__ void k_fill_f64(double* a, double v, int n)
{
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) a[i] = v;
}

__global__ void k_fill_i32_1(int32_t* a) { *a = 0; }

__global__ void k_fill_u64(unsigned long long* a, unsigned long long v, int n)
{
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) a[i] = v;
}

__device__ __forceinline__ double wave_min(double v)
{
    for (int o = 32; o > 0; o >>= 1) v = fmin(v, __shfl_xor(v, o, 64));
    return v;
}

// Per-box minimum of the particle time steps (values >= 0, so the order of
// their bit patterns is their order).  A small grid strides over the
// particles (ordered by box); each lane keeps the minimum of its current box
// and hands it on with one atomic when its box changes and at the end.
__global__ void k_box_min(const double* dt, const BoxInfo* boxes, int nbox, int64_t n, unsigned long long* mn)
{
    int cb = -1;
    double cm = (double)INFINITY;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int b = i < n ? box_of(boxes, nbox, i) : -1;
    for (; i < n; i += stride) {
        while (b + 1 < nbox && boxes[b + 1].begin <= i) b++;
        if (b != cb) {
            if (cb >= 0) atomicMin(&mn[cb], (unsigned long long)__double_as_longlong(cm));
            cb = b;
            cm = (double)INFINITY;
        }
        cm = fmin(cm, dt[i]);
    }
    const int b0 = __builtin_amdgcn_readfirstlane(cb);
    if (__all(cb == b0)) {
        const double m = wave_min(cm);
        if ((threadIdx.x & 63) == 0 && b0 >= 0) atomicMin(&mn[b0], (unsigned long long)__double_as_longlong(m));
    } else if (cb >= 0) {
        atomicMin(&mn[cb], (unsigned long long)__double_as_longlong(cm));
    }
}

// dt_b = min(smallest particle step, dt_max, t_end - t_b), and the box times
__global__ void k_dt_select(const unsigned long long* mn, int nbox, double dt_max, double t_end, double* t_box,
                            double* dtb, double* dt_out)
{
    int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= nbox) return;
    double dt = fmin(__longlong_as_double((long long)mn[b]), dt_max);
    const double rem = t_end - t_box[b];
    if (!(rem > 0.0)) {
        dt = 0.0;
    } else if (dt >= rem) {
        dt = rem;
        t_box[b] = t_end;
    } else {
        t_box[b] += dt;
    }
    dtb[b] = dt;
    if (dt_out) dt_out[b] = dt;
}

// ---------------------------------------------------------------- multiple time-stepping
// Time bin of a particle whose time step of Eq. (6) is dt: the largest k with
// 2^k dtb <= dt (at least 0, at most max_bin; max_bin where dt is infinite),
// lowered until its next step, starting at base step n_next, starts on a
// multiple of its length.
__device__ __forceinline__ int time_bin(double dt, double dtb, int max_bin, int64_t n_next)
{
    int k;
    if (isinf(dt)) {
        k = max_bin;
    } else {
        int e = 0;
        (void)frexp((dt > 0.0) ? dt / dtb : 1.0, &e);   // dt / dtb = mant 2^e, mant in [1/2, 1)
        k = min(max(e - 1, 0), max_bin);
    }
    while (k > 0 && (n_next & ((1ll << k) - 1)) != 0) k--;
    return k;
}

// Opening half of base step n for every particle (bin k, own step T = 2^k dtb):
// particles starting a step (n % 2^k == 0) take the half kick with T; every
// particle drifts by dtb; v and u are predicted at the end of the base step
// from each particle's last kick; the particles ending a step there are
// flagged active and counted.
__global__ void k_mts_open(StepArrays s, MtsStep m, const BoxInfo* boxes, int64_t n)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    bool act = false;
    if (i < n) {
        const int k = m.bin[i];
        const int64_t span = 1ll << k;
        const int64_t ph = m.n & (span - 1);   // base steps since this particle's step began
        const double T = (double)span * m.dtb;
        const double ax = s.ax[i], ay = s.ay[i], az = s.az[i], du = s.dudt[i];
        double vx = s.vx[i], vy = s.vy[i], vz = s.vz[i], u = s.u[i];
        if (ph == 0) {
            const double hk = 0.5 * T;
            vx += hk * ax; vy += hk * ay; vz += hk * az; u += hk * du;
            s.vx[i] = vx; s.vy[i] = vy; s.vz[i] = vz; s.u[i] = u;
        }
        const double tau = (double)(ph + 1) * m.dtb - 0.5 * T;
        s.pvx[i] = vx + tau * ax; s.pvy[i] = vy + tau * ay; s.pvz[i] = vz + tau * az; s.pu[i] = u + tau * du;
        const BoxInfo& B = boxes[0];
        double p[3] = {s.x[i] + m.dtb * vx, s.y[i] + m.dtb * vy, s.z[i] + m.dtb * vz};
        for (int d = 0; d < 3; d++) {
            double w = fmod(p[d], B.L[d]);
            if (w < 0.0) w += B.L[d];
            if (w >= B.L[d]) w -= B.L[d];
            p[d] = w;
        }
        s.x[i] = p[0]; s.y[i] = p[1]; s.z[i] = p[2];
        act = ph + 1 == span;
        m.active[i] = act ? 1 : 0;
    }
    const unsigned long long b = __ballot(act);
    if ((threadIdx.x & 63) == 0 && b) atomicAdd(m.n_active, (int32_t)__popcll(b));
}

// Closing half of base step n for the active particles: the half kick with
// the new accelerations and the bin of the next step.
__global__ void k_mts_close(StepArrays s, MtsStep m, const double* dt, int64_t n)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n || !m.active[i]) return;
    const double hk = 0.5 * (double)(1ll << m.bin[i]) * m.dtb;
    s.vx[i] += hk * s.ax[i];
    s.vy[i] += hk * s.ay[i];
    s.vz[i] += hk * s.az[i];
    s.u[i] += hk * s.dudt[i];
    m.bin[i] = time_bin(dt[i], m.dtb, m.max_bin, m.n + 1);
}

__global__ void k_mts_bins(const double* dt, MtsStep m, int64_t n_next, int64_t n)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) m.bin[i] = time_bin(dt[i], m.dtb, m.max_bin, n_next);
}

static unsigned blocks(int64_t n) { return (unsigned)((n + 255) / 256); }

void launch_mts_open(const StepArrays& s, const MtsStep& m, const BoxInfo* boxes, int64_t n, hipStream_t st)
{
    hipLaunchKernelGGL(k_fill_i32_1, dim3(1), dim3(1), 0, st, m.n_active);
    if (n > 0) hipLaunchKernelGGL(k_mts_open, dim3(blocks(n)), dim3(256), 0, st, s, m, boxes, n);
}

void launch_mts_close(const StepArrays& s, const MtsStep& m, const double* dt, int64_t n, hipStream_t st)
{
    if (n > 0) hipLaunchKernelGGL(k_mts_close, dim3(blocks(n)), dim3(256), 0, st, s, m, dt, n);
}

void launch_mts_bins(const double* dt, const MtsStep& m, int64_t n_next, int64_t n, hipStream_t st)
{
    if (n > 0) hipLaunchKernelGGL(k_mts_bins, dim3(blocks(n)), dim3(256), 0, st, dt, m, n_next, n);
}

void launch_step_open(const StepArrays& s, const double* dtb, const BoxInfo* boxes, int nbox, int64_t n,
                      hipStream_t st)
{
    if (n <= 0) return;
    hipLaunchKernelGGL(k_open, dim3(blocks(n)), dim3(256), 0, st, s, dtb, boxes, nbox, n);
}

void launch_step_close(const StepArrays& s, const double* dtb, const BoxInfo* boxes, int nbox, int64_t n,
                       hipStream_t st)
{
    if (n <= 0) return;
    hipLaunchKernelGGL(k_close, dim3(blocks(n)), dim3(256), 0, st, s, dtb, boxes, nbox, n);
}

void launch_fill_f64(double* a, double v, int n, hipStream_t st)
{
    if (n <= 0) return;
    hipLaunchKernelGGL(k_fill_f64, dim3(blocks(n)), dim3(256), 0, st, a, v, n);
}

void launch_dt_select(const double* dt, const BoxInfo* boxes, int nbox, int64_t n, unsigned long long* mn,
                      double dt_max, double t_end, double* t_box, double* dtb, double* dt_out, hipStream_t st)
{
    hipLaunchKernelGGL(k_fill_u64, dim3(blocks(nbox)), dim3(256), 0, st, mn, 0x7FF0000000000000ull, nbox);
    if (n > 0) {
        const unsigned g = blocks(n) < 256 ? blocks(n) : 256;
        hipLaunchKernelGGL(k_box_min, dim3(g), dim3(256), 0, st, dt, boxes, nbox, n, mn);
    }
    hipLaunchKernelGGL(k_dt_select, dim3(blocks(nbox)), dim3(256), 0, st, mn, nbox, dt_max, t_end, t_box, dtb,
                       dt_out);
}

}  // namespace sph
