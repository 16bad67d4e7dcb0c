// step.hip -- kick-drift-kick velocity Verlet (Gonnet 2014, Sec. 4.1) with a
// fixed step, on the caller's FP64 arrays.
#include "sph_internal.h"
#include "kernels.h"

namespace sph {

// v += hdt a, u += hdt du/dt
__global__ void k_kick(double* vx, double* vy, double* vz, double* u, const double* ax,
                       const double* ay, const double* az, const double* dudt, double hdt, int64_t n)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    vx[i] += hdt * ax[i];
    vy[i] += hdt * ay[i];
    vz[i] += hdt * az[i];
    u[i] += hdt * dudt[i];
}

// x += dt v, wrapped into [0, L) of the particle's box
__global__ void k_drift(double* x, double* y, double* z, const double* vx, const double* vy,
                        const double* vz, double dt, const BoxInfo* boxes, int nbox, int64_t n)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    int lo = 0, hi = nbox - 1;
    while (lo < hi) {
        int mid = (lo + hi + 1) >> 1;
        if (boxes[mid].begin <= i) lo = mid; else hi = mid - 1;
    }
    const BoxInfo& B = boxes[lo];
    double p[3] = {x[i] + dt * vx[i], y[i] + dt * vy[i], z[i] + dt * vz[i]};
    for (int d = 0; d < 3; d++) {
        double w = fmod(p[d], B.L[d]);
        if (w < 0.0) w += B.L[d];
        if (w >= B.L[d]) w -= B.L[d];
        p[d] = w;
    }
    x[i] = p[0]; y[i] = p[1]; z[i] = p[2];
}

// out = v + hdt a
__global__ void k_predict(const double* v, const double* a, double hdt, double* out, int64_t n)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) out[i] = v[i] + hdt * a[i];
}

void launch_kick(double* vx, double* vy, double* vz, double* u, const double* ax, const double* ay,
                 const double* az, const double* dudt, double hdt, int64_t n, hipStream_t st)
{
    if (n <= 0) return;
    hipLaunchKernelGGL(k_kick, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, vx, vy, vz, u, ax,
                       ay, az, dudt, hdt, n);
}

void launch_drift(double* x, double* y, double* z, const double* vx, const double* vy,
                  const double* vz, double dt, const int64_t*, const BoxInfo* boxes, int nbox,
                  int64_t n, hipStream_t st)
{
    if (n <= 0) return;
    hipLaunchKernelGGL(k_drift, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, x, y, z, vx, vy,
                       vz, dt, boxes, nbox, n);
}

void launch_predict(const double* v, const double* a, double hdt, double* out, int64_t n,
                    hipStream_t st)
{
    if (n <= 0) return;
    hipLaunchKernelGGL(k_predict, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, v, a, hdt, out, n);
}

}  // namespace sph
