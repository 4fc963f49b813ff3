// gfx950 auxiliary kernels of the PVD phase-field library: the seeded
// initial condition, inflow accumulators and the FP64 diagnostics (masses,
// inflow, discrete free energy).  The stepper is in pf_step.hip.

#include "pf_kernels.h"

#include <math.h>

namespace pfk {
namespace {

// ---------------------------------------------------------------- init

__device__ __forceinline__ uint64_t splitmix64(uint64_t seed, uint64_t n)
{
    // SplitMix64 (Steele, Lea & Flood 2014): output n of the stream of seed
    uint64_t z = seed + (n + 1ull) * 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

template <typename T>
__global__ __launch_bounds__(256) void init_kernel(T* c, T* phi, T* rho, InitArgs a)
{
    const int b = blockIdx.y;
    const size_t plane = (size_t)a.nx * a.ny;
    for (size_t k = (size_t)blockIdx.x * 256 + threadIdx.x; k < plane; k += (size_t)gridDim.x * 256) {
        const int j = (int)(k / a.nx);
        const double U = (double)(splitmix64(a.seed + (uint64_t)b, (uint64_t)k) >> 11) * 0x1.0p-53;
        const double cv = a.c0[b] + a.c_noise * (2.0 * U - 1.0);
        const double ph = tanh((a.H0 - (j + 0.5) * a.h) / a.width);
        const double rv = a.rho_in * (1.0 - ph) / 2.0;
        c[b * plane + k] = (T)cv;
        phi[b * plane + k] = (T)ph;
        rho[b * plane + k] = (T)rv;
    }
}

__global__ __launch_bounds__(256) void set_inflow_kernel(double* Qcol, const double* q, int nx)
{
    const int b = blockIdx.y;
    for (int i = blockIdx.x * 256 + threadIdx.x; i < nx; i += gridDim.x * 256)
        Qcol[(size_t)b * nx + i] = (i == 0 && q) ? q[b] : 0.0;
}

// ---------------------------------------------------------- reductions

__device__ __forceinline__ double wave_sum(double v)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// Per-block FP64 partial sums (c, phi, rho, energy) over rows j = blockIdx.x,
// blockIdx.x + gridDim.x, ...; fixed assignment and tree, so deterministic.
template <typename T>
__global__ __launch_bounds__(256) void reduce_kernel(const T* c, const T* phi, const T* rho,
                                                     double* partials, RedArgs a)
{
    const int b = blockIdx.y;
    const int nx = a.nx, ny = a.ny;
    const size_t plane = (size_t)nx * ny;
    c += b * plane;
    phi += b * plane;
    rho += b * plane;
    double sc = 0, sp = 0, sr = 0, se = 0;
    for (int j = blockIdx.x; j < ny; j += gridDim.x) {
        const bool has_n = a.pvd ? (j + 1 < ny) : true;
        const int jn = j + 1 < ny ? j + 1 : 0;
        for (int i = threadIdx.x; i < nx; i += 256) {
            const size_t k = (size_t)j * nx + i;
            const int ie = i + 1 < nx ? i + 1 : 0;
            const double cv = (double)c[k], pv = (double)phi[k], rv = (double)rho[k];
            sc += cv;
            sp += pv;
            sr += rv;
            const double q1 = 1.0 + pv, w = 1.0 - pv * pv;
            const double pf = 0.25 * (2.0 - pv) * q1 * q1;
            const double cg = cv * (1.0 - cv);
            const double f = a.Wc * pf * (cg * cg) + 0.25 * a.Wphi * w * w;
            const double dcE = (double)c[(size_t)j * nx + ie] - cv;
            const double dpE = (double)phi[(size_t)j * nx + ie] - pv;
            double gc = dcE * dcE, gp = dpE * dpE;
            if (has_n) {
                const double dcN = (double)c[(size_t)jn * nx + i] - cv;
                const double dpN = (double)phi[(size_t)jn * nx + i] - pv;
                gc += dcN * dcN;
                gp += dpN * dpN;
            }
            se += a.h2 * f + a.half_kc * gc + a.half_kp * gp;
        }
    }
    __shared__ double red[4][4];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    sc = wave_sum(sc);
    sp = wave_sum(sp);
    sr = wave_sum(sr);
    se = wave_sum(se);
    if (lane == 0) {
        red[wv][0] = sc;
        red[wv][1] = sp;
        red[wv][2] = sr;
        red[wv][3] = se;
    }
    __syncthreads();
    if (threadIdx.x < 4) {
        const int m = threadIdx.x;
        const double v = (red[0][m] + red[1][m]) + (red[2][m] + red[3][m]);
        partials[((size_t)b * gridDim.x + blockIdx.x) * 4 + m] = v;
    }
}

// One block per realisation: sum the partials and the inflow columns.
__global__ __launch_bounds__(256) void finish_kernel(const double* partials, const double* Qcol,
                                                     double* out, int nblk, int nx, double h2)
{
    const int b = blockIdx.x;
    double s[5] = {0, 0, 0, 0, 0};
    for (int i = threadIdx.x; i < nblk; i += 256)
        for (int m = 0; m < 4; ++m) s[m] += partials[((size_t)b * nblk + i) * 4 + m];
    for (int i = threadIdx.x; i < nx; i += 256) s[4] += Qcol[(size_t)b * nx + i];
    __shared__ double red[4][5];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    for (int m = 0; m < 5; ++m) {
        const double v = wave_sum(s[m]);
        if (lane == 0) red[wv][m] = v;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double t[5];
        for (int m = 0; m < 5; ++m) t[m] = (red[0][m] + red[1][m]) + (red[2][m] + red[3][m]);
        out[b * 5 + 0] = h2 * t[0];
        out[b * 5 + 1] = h2 * t[1];
        out[b * 5 + 2] = h2 * t[2];
        out[b * 5 + 3] = t[4];
        out[b * 5 + 4] = t[3];
    }
}

}  // namespace

template <typename T>
hipError_t launch_init(T* c, T* phi, T* rho, const InitArgs& a, int batch, hipStream_t s)
{
    const size_t plane = (size_t)a.nx * a.ny;
    const unsigned gx = (unsigned)((plane + 255) / 256 < 4096 ? (plane + 255) / 256 : 4096);
    hipLaunchKernelGGL(init_kernel<T>, dim3(gx, batch), dim3(256), 0, s, c, phi, rho, a);
    return hipGetLastError();
}
template hipError_t launch_init<float>(float*, float*, float*, const InitArgs&, int, hipStream_t);
template hipError_t launch_init<double>(double*, double*, double*, const InitArgs&, int, hipStream_t);

hipError_t launch_set_inflow(double* Qcol, const double* q, int nx, int batch, hipStream_t s)
{
    const unsigned gx = (unsigned)((nx + 255) / 256);
    hipLaunchKernelGGL(set_inflow_kernel, dim3(gx, batch), dim3(256), 0, s, Qcol, q, nx);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_reduce(const T* c, const T* phi, const T* rho, const double* Qcol,
                         double* partials, double* out, const RedArgs& a, int batch,
                         int nblk, hipStream_t s)
{
    hipLaunchKernelGGL(reduce_kernel<T>, dim3(nblk, batch), dim3(256), 0, s, c, phi, rho, partials, a);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(finish_kernel, dim3(batch), dim3(256), 0, s, partials, Qcol, out, nblk, a.nx, a.h2);
    return hipGetLastError();
}
template hipError_t launch_reduce<float>(const float*, const float*, const float*, const double*,
                                         double*, double*, const RedArgs&, int, int, hipStream_t);
template hipError_t launch_reduce<double>(const double*, const double*, const double*, const double*,
                                          double*, double*, const RedArgs&, int, int, hipStream_t);

}  // namespace pfk
