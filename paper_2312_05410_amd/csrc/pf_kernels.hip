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

// Loads of V consecutive elements (one 16-byte load when V > 1).
template <typename T, int V>
struct Vec {
    T v[V];
};
template <typename T, int V>
__device__ __forceinline__ Vec<T, V> load_vec(const T* p)
{
    Vec<T, V> r;
    if constexpr (V == 4) {
        const float4 q = *reinterpret_cast<const float4*>(p);
        r.v[0] = q.x;
        r.v[1] = q.y;
        r.v[2] = q.z;
        r.v[3] = q.w;
    } else if constexpr (V == 2) {
        const double2 q = *reinterpret_cast<const double2*>(p);
        r.v[0] = q.x;
        r.v[1] = q.y;
    } else {
        r.v[0] = p[0];
    }
    return r;
}

// Per-workgroup FP64 partial sums (c, phi, rho, energy) of one band of rows
// [j0, j0 + rows) and one chunk of 256 V columns of realisation blockIdx.z.
// Each thread owns V consecutive columns and walks down its band keeping the
// current row of c and phi in registers: the next row is loaded once, as the
// north neighbour, and becomes the current row (each row is read once per
// band); the east neighbour of the last column is the next thread's first,
// a cache hit.  Energy terms: the double well at every cell, the gradient
// energy of every x face (periodic wrap included) and of the y faces to
// the row above (interior faces only for the PVD boundaries; the wrap face
// too when y is periodic).  Fixed assignment and tree: deterministic.
template <typename T, int V>
__global__ __launch_bounds__(256) void reduce_kernel(const T* c, const T* phi, const T* rho,
                                                     double* partials, RedArgs a, int rows)
{
    const int b = blockIdx.z;
    const int nx = a.nx, ny = a.ny;
    const size_t plane = (size_t)nx * ny;
    c += b * plane;
    phi += b * plane;
    rho += b * plane;
    const int i0 = (blockIdx.x * 256 + threadIdx.x) * V;
    const int j0 = blockIdx.y * rows;
    const int j1 = j0 + rows < ny ? j0 + rows : ny;
    double sc = 0, sp = 0, sr = 0, se = 0;
    if (i0 < nx) {
        const int ie = i0 + V < nx ? i0 + V : 0;
        Vec<T, V> cc = load_vec<T, V>(c + (size_t)j0 * nx + i0);
        Vec<T, V> pc = load_vec<T, V>(phi + (size_t)j0 * nx + i0);
        for (int j = j0; j < j1; ++j) {
            const bool has_n = a.pvd ? (j + 1 < ny) : true;
            const int jn = j + 1 < ny ? j + 1 : 0;
            const size_t row = (size_t)j * nx, rown = (size_t)jn * nx;
            const Vec<T, V> rr = load_vec<T, V>(rho + row + i0);
            const Vec<T, V> cn = load_vec<T, V>(c + rown + i0);
            const Vec<T, V> pn = load_vec<T, V>(phi + rown + i0);
            const double ceE = (double)c[row + ie], peE = (double)phi[row + ie];
#pragma unroll
            for (int v = 0; v < V; ++v) {
                const double cv = (double)cc.v[v], pv = (double)pc.v[v], rv = (double)rr.v[v];
                sc += cv;
                sp += pv;
                sr += rv;
                const double q1 = 1.0 + pv, w = 1.0 - pv * pv;
                const double pf = 0.25 * (2.0 - pv) * q1 * q1;
                const double cg = cv * (1.0 - cv);
                const double f = a.Wc * pf * (cg * cg) + 0.25 * a.Wphi * w * w;
                const double dcE = (v + 1 < V ? (double)cc.v[v + 1 < V ? v + 1 : 0] : ceE) - cv;
                const double dpE = (v + 1 < V ? (double)pc.v[v + 1 < V ? v + 1 : 0] : peE) - pv;
                double gc = dcE * dcE, gp = dpE * dpE;
                if (has_n) {
                    const double dcN = (double)cn.v[v] - cv;
                    const double dpN = (double)pn.v[v] - pv;
                    gc += dcN * dcN;
                    gp += dpN * dpN;
                }
                se += a.h2 * f + a.half_kc * gc + a.half_kp * gp;
            }
            cc = cn;
            pc = pn;
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
        const size_t part = ((size_t)b * gridDim.y + blockIdx.y) * gridDim.x + blockIdx.x;
        partials[part * 4 + m] = v;
    }
}

// One block per realisation: sum the partials and the inflow columns
// (out[b][5]); without inflow columns (Qcol null) the masses and the energy
// only (out[b][4]).  Each
// thread in a fixed order; the loops are unrolled so that a thread's loads
// are in flight together rather than one latency per element).
__global__ __launch_bounds__(256) void finish_kernel(const double* partials, const double* Qcol,
                                                     double* out, int nblk, int nx, double h2)
{
    const int b = blockIdx.x;
    double s[5] = {0, 0, 0, 0, 0};
    const double4* pp = reinterpret_cast<const double4*>(partials) + (size_t)b * nblk;
#pragma unroll 8
    for (int i = threadIdx.x; i < nblk; i += 256) {
        const double4 q = pp[i];
        s[0] += q.x;
        s[1] += q.y;
        s[2] += q.z;
        s[3] += q.w;
    }
    if (Qcol) {
        const double* qc = Qcol + (size_t)b * nx;
#pragma unroll 8
        for (int i = threadIdx.x; i < nx; i += 256) s[4] += qc[i];
    }
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
        if (Qcol) {
            out[b * 5 + 0] = h2 * t[0];
            out[b * 5 + 1] = h2 * t[1];
            out[b * 5 + 2] = h2 * t[2];
            out[b * 5 + 3] = t[4];
            out[b * 5 + 4] = t[3];
        } else {
            out[b * 4 + 0] = h2 * t[0];
            out[b * 4 + 1] = h2 * t[1];
            out[b * 4 + 2] = h2 * t[2];
            out[b * 4 + 3] = t[3];
        }
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

RedGeo reduce_geometry(int nx, int ny, int batch, int elem_bytes)
{
    // about 2048 workgroups per launch (8 per compute unit on MI355X; the
    // count is a fixed function of the shape so that sums keep one order)
    RedGeo g{};
    const int v16 = 16 / elem_bytes;
    g.vec = nx % v16 == 0 ? v16 : 1;
    const long cw = 256L * g.vec;
    g.chunks = (int)((nx + cw - 1) / cw);
    long want = 2048L / ((long)g.chunks * (batch > 0 ? batch : 1));
    if (want < 1) want = 1;
    if (want > ny) want = ny;
    g.rows = (int)((ny + want - 1) / want);
    g.bands = (ny + g.rows - 1) / g.rows;
    return g;
}

template <typename T>
hipError_t launch_reduce(const T* c, const T* phi, const T* rho, const double* Qcol,
                         double* partials, double* out, const RedArgs& a, const RedGeo& g, int batch,
                         hipStream_t s)
{
    const dim3 grid((unsigned)g.chunks, (unsigned)g.bands, (unsigned)batch);
    constexpr int V16 = 16 / (int)sizeof(T);
    if (g.vec == V16)
        hipLaunchKernelGGL((reduce_kernel<T, V16>), grid, dim3(256), 0, s, c, phi, rho, partials, a, g.rows);
    else
        hipLaunchKernelGGL((reduce_kernel<T, 1>), grid, dim3(256), 0, s, c, phi, rho, partials, a, g.rows);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(finish_kernel, dim3(batch), dim3(256), 0, s, partials, Qcol, out, g.parts(), a.nx, a.h2);
    return hipGetLastError();
}
template hipError_t launch_reduce<float>(const float*, const float*, const float*, const double*,
                                         double*, double*, const RedArgs&, const RedGeo&, int, hipStream_t);
template hipError_t launch_reduce<double>(const double*, const double*, const double*, const double*,
                                          double*, double*, const RedArgs&, const RedGeo&, int, hipStream_t);

}  // namespace pfk
