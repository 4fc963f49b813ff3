// gfx950 kernels of the explicit PVD phase-field step (Materials and
// Methods, "Phase-field modeling of physical vapor deposition"; central
// differences as stated in "Dataset").
//
// step_kernel: one launch advances a TX x TY output tile of one realisation
// by up to K explicit Euler sub-steps.  The tile plus a halo of 2K cells of
// c, phi and rho is loaded once from HBM into LDS (x wrapped, y mirrored or
// the inlet value), then every sub-step runs two fused stencil stages out of
// LDS: stage 1 computes mu_c, mu_phi and M_c on the region one cell wider
// than the update region; stage 2 computes the flux-form conserved updates,
// the deposition source and vapour transport.  The valid region shrinks by
// two cells per sub-step.  Only the TX x TY tile is written back, so HBM
// traffic per launch is one read and one write of the state.  Every cell is
// computed by the same inlined code with a fixed expression order
// (-ffp-contract=off plus explicit fma), so any K and any tile shape give
// bitwise-identical states.
#include "pf_kernels.h"

#include <math.h>

namespace pfk {
namespace {

__device__ __forceinline__ float fmaT(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__device__ __forceinline__ double fmaT(double a, double b, double c) { return __builtin_fma(a, b, c); }

// exp(-phi^2 / sigma^2): float uses the hardware base-2 exponential with
// log2(e)/sigma^2 folded on the host; double uses the device math library.
__device__ __forceinline__ float surf_exp(float ph2, float e) { return __builtin_amdgcn_exp2f(-(ph2 * e)); }
__device__ __forceinline__ double surf_exp(double ph2, double e) { return exp(-(ph2 * e)); }

template <typename T>
__device__ __forceinline__ T clampT(T x, T lo, T hi)
{
    return x < lo ? lo : (x > hi ? hi : x);
}

// Stage 1 at one cell: chemical potentials and composition mobility.
//   mu_c   = W_c p(phi) g'(c) - kappa_c Lap c
//   mu_phi = W_c p'(phi) g(c) - W_phi phi (1 - phi^2) - kappa_phi Lap phi
//   M_c    = p(phi~)(MB + H dM)_bulk + exp(-(phi~/sigma)^2)(MB + H dM)_surf
// Neighbour sums are formed as (E + W) + (N + S) so that mirrored ghost
// rows reproduce the interior values exactly.
template <typename T>
__device__ __forceinline__ void potentials(const Coef<T>& k, T c, T cE, T cW, T cN, T cS,
                                           T p, T pE, T pW, T pN, T pS,
                                           T& mu_c, T& mu_p, T& M)
{
    const T lapc = fmaT(T(-4), c, (cE + cW) + (cN + cS));
    const T lapp = fmaT(T(-4), p, (pE + pW) + (pN + pS));
    const T q1 = T(1) + p;
    const T pf = (T(0.25) * (T(2) - p)) * (q1 * q1);
    const T w = fmaT(-p, p, T(1));
    const T dpf = T(0.75) * w;
    const T cg = c * (T(1) - c);
    const T g = cg * cg;
    const T dg = cg * fmaT(T(-4), c, T(2));
    mu_c = fmaT(k.Wc * pf, dg, -(k.kc * lapc));
    mu_p = fmaT(k.Wc * dpf, g, fmaT(-(k.Wphi * p), w, -(k.kp * lapp)));
    const T x = clampT(c, T(0), T(1));
    const T H = ((x * x) * x) * fmaT(fmaT(T(6), x, T(-15)), x, T(10));
    const T ph = clampT(p, T(-1), T(1));
    const T r1 = T(1) + ph;
    const T pb = (T(0.25) * (T(2) - ph)) * (r1 * r1);
    const T e = surf_exp(ph * ph, k.esurf);
    M = fmaT(pb, fmaT(H, k.dMb, k.MBb), e * fmaT(H, k.dMs, k.MBs));
}

// Shared-memory tile of one launch.
template <typename T, int LN>
struct Tile {
    T c[LN], p[LN], r[LN], mc[LN], mp[LN], M[LN];
};

// One sub-step S (compile-time) of the tile; recursion over S unrolls the
// sub-steps with compile-time region sizes.
template <typename T, int K, int TX, int TY, int NT, int S>
__device__ __forceinline__ void substep(const StepArgs<T>& a, Tile<T, (TX + 4 * K) * (TY + 4 * K)>& t,
                                        double* s_q, int b, int x0, int y0, T vx2h, T vy2h,
                                        double qa, double qb)
{
    constexpr int R = 2 * K;
    constexpr int LW = TX + 2 * R, LH = TY + 2 * R;
    const int tid = threadIdx.x;
    const int nx = a.nx, ny = a.ny;
    const Coef<T>& k = a.k;

    // ---- stage 1: potentials and mobility on the region of offset 2S+1
    {
        constexpr int o = 2 * S + 1, W = LW - 2 * o, H = LH - 2 * o, N = W * H;
        constexpr int Q = (N + NT - 1) / NT;
#pragma unroll
        for (int q = 0; q < Q; ++q) {
            const int idx = tid + q * NT;
            if (idx < N) {
                const int ly = idx / W + o, lx = idx % W + o;
                const int l = ly * LW + lx;
                T mc, mp, M;
                potentials(k, t.c[l], t.c[l + 1], t.c[l - 1], t.c[l + LW], t.c[l - LW],
                           t.p[l], t.p[l + 1], t.p[l - 1], t.p[l + LW], t.p[l - LW], mc, mp, M);
                t.mc[l] = mc;
                t.mp[l] = mp;
                t.M[l] = M;
            }
        }
    }
    __syncthreads();

    // ---- stage 2: conserved updates, deposition, vapour transport
    constexpr int o = 2 * S + 2, W = LW - 2 * o, H = LH - 2 * o, N = W * H;
    constexpr int Q = (N + NT - 1) / NT;
    T nc[Q], np[Q], nr[Q];
    const bool last = (S == a.nsub - 1);
#pragma unroll
    for (int q = 0; q < Q; ++q) {
        const int idx = tid + q * NT;
        if (idx < N) {
            const int ly = idx / W + o, lx = idx % W + o;
            const int l = ly * LW + lx;
            const int gj = y0 - R + ly;
            const T M0 = t.M[l], m0 = t.mc[l];
            const T fx = (t.M[l + 1] + M0) * (t.mc[l + 1] - m0) + (t.M[l - 1] + M0) * (t.mc[l - 1] - m0);
            const T fy = (t.M[l + LW] + M0) * (t.mc[l + LW] - m0) + (t.M[l - LW] + M0) * (t.mc[l - LW] - m0);
            const T divc = k.half_ih2 * (fx + fy);
            const T mp0 = t.mp[l];
            const T divp = k.mphi_h2 * fmaT(T(-4), mp0, (t.mp[l + 1] + t.mp[l - 1]) + (t.mp[l + LW] + t.mp[l - LW]));
            const T r0 = t.r[l];
            const T src = r0 * fmaT(vx2h, t.p[l + 1] - t.p[l - 1], vy2h * (t.p[l + LW] - t.p[l - LW]));
            const T rE = t.r[l + 1], rW = t.r[l - 1], rN = t.r[l + LW], rS = t.r[l - LW];
            const T lapr = fmaT(T(-4), r0, (rE + rW) + (rN + rS));
            // no advective flux through the substrate: the south face flux is 0
            const T rSa = (a.pvd && gj == 0) ? -r0 : rS;
            const T adv = fmaT(vx2h, rE - rW, vy2h * (rN - rSa));
            const T Tr = fmaT(k.D_h2, lapr, -adv);
            nc[q] = fmaT(k.dt, divc, t.c[l]);
            np[q] = fmaT(k.dt, divp + src, t.p[l]);
            nr[q] = fmaT(k.dt, Tr - src, r0);
            if (a.pvd && gj == ny - 1 && lx >= R && lx < R + TX && ly >= R && ly < R + TY) {
                // inflow through the top face: advective + diffusive flux
                const int ix = lx - R;
                if (x0 + ix < nx) {
                    const double rin = (double)k.rho_in, rr = (double)r0;
                    s_q[ix] += qa * (rr + rin) + qb * (rin - rr);
                }
            }
        }
    }

    if (last) {
        const size_t plane = (size_t)nx * ny;
        T* oc = a.c_out + (size_t)b * plane;
        T* op = a.phi_out + (size_t)b * plane;
        T* orr = a.rho_out + (size_t)b * plane;
#pragma unroll
        for (int q = 0; q < Q; ++q) {
            const int idx = tid + q * NT;
            if (idx < N) {
                const int ly = idx / W + o, lx = idx % W + o;
                if (lx >= R && lx < R + TX && ly >= R && ly < R + TY) {
                    const int gi = x0 + lx - R, gj = y0 + ly - R;
                    if (gi < nx && gj < ny) {
                        const size_t g = (size_t)gj * nx + gi;
                        oc[g] = nc[q];
                        op[g] = np[q];
                        orr[g] = nr[q];
                    }
                }
            }
        }
        return;
    }

    __syncthreads();
#pragma unroll
    for (int q = 0; q < Q; ++q) {
        const int idx = tid + q * NT;
        if (idx < N) {
            const int l = (idx / W + o) * LW + idx % W + o;
            t.c[l] = nc[q];
            t.p[l] = np[q];
            t.r[l] = nr[q];
        }
    }
    __syncthreads();

    // Ghost rows (PVD): refill from the mirrored interior rows, to the depth
    // the remaining sub-steps can still reach (R - o); rho above the top is
    // the inlet value.
    if (a.pvd) {
        const bool lo = (y0 - R + o) < 0;
        const bool hi = (y0 - R + LH - o - 1) >= ny;
        if (lo || hi) {
            for (int idx = tid; idx < N; idx += NT) {
                const int ly = idx / W + o, lx = idx % W + o;
                const int gj = y0 - R + ly;
                int gm;
                bool rin = false;
                if (gj < 0) {
                    if (-gj > R - o) continue;
                    gm = -1 - gj;
                } else if (gj >= ny) {
                    if (gj - ny + 1 > R - o) continue;
                    gm = 2 * ny - 1 - gj;
                    rin = true;
                } else {
                    continue;
                }
                const int l = ly * LW + lx, m = (gm - (y0 - R)) * LW + lx;
                t.c[l] = t.c[m];
                t.p[l] = t.p[m];
                t.r[l] = rin ? k.rho_in : t.r[m];
            }
            __syncthreads();
        }
    }

    if constexpr (S + 1 < K) {
        if (S + 1 < a.nsub)
            substep<T, K, TX, TY, NT, S + 1>(a, t, s_q, b, x0, y0, vx2h, vy2h, qa, qb);
    }
}

template <typename T, int K, int TX, int TY, int NT>
__global__ __launch_bounds__(NT) void step_kernel(StepArgs<T> a)
{
    constexpr int R = 2 * K;
    constexpr int LW = TX + 2 * R, LH = TY + 2 * R, LN = LW * LH;
    __shared__ Tile<T, LN> t;
    __shared__ double s_q[TX];

    const int tid = threadIdx.x;
    const int b = blockIdx.y;
    const int nx = a.nx, ny = a.ny;

    // Tile order: consecutive workgroup ids go round-robin over the 8 XCDs,
    // so give XCD x a contiguous band of tiles (shared halos stay in its L2).
    const int nblk = a.tiles_x * a.tiles_y;
    const int bid = blockIdx.x;
    const int xcd = bid & 7, slot = bid >> 3;
    const int q8 = nblk >> 3, r8 = nblk & 7;
    const int tileid = xcd * q8 + (xcd < r8 ? xcd : r8) + slot;
    const int x0 = (tileid % a.tiles_x) * TX;
    const int y0 = (tileid / a.tiles_x) * TY;

    const size_t plane = (size_t)nx * ny;
    const T* gc = a.c + (size_t)b * plane;
    const T* gp = a.phi + (size_t)b * plane;
    const T* gr = a.rho + (size_t)b * plane;

    // ---- load tile + halo: all loads of a thread are issued before any
    // LDS store so they are in flight together
    constexpr int NL = (LN + NT - 1) / NT;
    T vc[NL], vp[NL], vr[NL];
#pragma unroll
    for (int q = 0; q < NL; ++q) {
        const int idx = tid + q * NT;
        if (idx < LN) {
            const int ly = idx / LW, lx = idx % LW;
            int gi = x0 - R + lx;
            while (gi < 0) gi += nx;
            while (gi >= nx) gi -= nx;
            const int gj = y0 - R + ly;
            int jj = gj;
            if (a.pvd) {
                while (jj < 0 || jj >= ny) jj = jj < 0 ? -1 - jj : 2 * ny - 1 - jj;
            } else {
                while (jj < 0) jj += ny;
                while (jj >= ny) jj -= ny;
            }
            const size_t g = (size_t)jj * nx + gi;
            vc[q] = gc[g];
            vp[q] = gp[g];
            vr[q] = (a.pvd && gj >= ny) ? a.k.rho_in : gr[g];
        }
    }
#pragma unroll
    for (int q = 0; q < NL; ++q) {
        const int idx = tid + q * NT;
        if (idx < LN) {
            t.c[idx] = vc[q];
            t.p[idx] = vp[q];
            t.r[idx] = vr[q];
        }
    }
    const bool top = a.pvd && y0 <= ny - 1 && ny - 1 < y0 + TY;
    if (top) {
        for (int i = tid; i < TX; i += NT)
            if (x0 + i < nx) s_q[i] = a.Qcol[(size_t)b * nx + x0 + i];
    }
    __syncthreads();

    const Real rl = a.real[b];
    substep<T, K, TX, TY, NT, 0>(a, t, s_q, b, x0, y0, (T)rl.vx2h, (T)rl.vy2h, rl.qa, rl.qb);

    if (top) {
        __syncthreads();
        for (int i = tid; i < TX; i += NT)
            if (x0 + i < nx) a.Qcol[(size_t)b * nx + x0 + i] = s_q[i];
    }
}

// Tile shapes per precision and fused-step count.
template <typename T, int K> struct Shape;
template <> struct Shape<float, 1> { static constexpr int TX = 64, TY = 16, NT = 256; };
template <> struct Shape<float, 2> { static constexpr int TX = 64, TY = 32, NT = 256; };
template <> struct Shape<float, 3> { static constexpr int TX = 64, TY = 32, NT = 256; };
template <> struct Shape<float, 4> { static constexpr int TX = 64, TY = 32, NT = 256; };
template <> struct Shape<double, 1> { static constexpr int TX = 64, TY = 16, NT = 256; };
template <> struct Shape<double, 2> { static constexpr int TX = 64, TY = 16, NT = 256; };

template <typename T, int K>
hipError_t launch_k(const StepArgs<T>& a, int batch, hipStream_t s)
{
    using Sh = Shape<T, K>;
    dim3 grid(a.tiles_x * a.tiles_y, batch);
    hipLaunchKernelGGL((step_kernel<T, K, Sh::TX, Sh::TY, Sh::NT>), grid, dim3(Sh::NT), 0, s, a);
    return hipGetLastError();
}

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

template <>
TileCfg tile_cfg<float>(int k)
{
    switch (k) {
    case 1: return {Shape<float, 1>::TX, Shape<float, 1>::TY, 1, Shape<float, 1>::NT};
    case 2: return {Shape<float, 2>::TX, Shape<float, 2>::TY, 2, Shape<float, 2>::NT};
    case 3: return {Shape<float, 3>::TX, Shape<float, 3>::TY, 3, Shape<float, 3>::NT};
    case 4: return {Shape<float, 4>::TX, Shape<float, 4>::TY, 4, Shape<float, 4>::NT};
    default: return {0, 0, 0, 0};
    }
}

template <>
TileCfg tile_cfg<double>(int k)
{
    switch (k) {
    case 1: return {Shape<double, 1>::TX, Shape<double, 1>::TY, 1, Shape<double, 1>::NT};
    case 2: return {Shape<double, 2>::TX, Shape<double, 2>::TY, 2, Shape<double, 2>::NT};
    default: return {0, 0, 0, 0};
    }
}

template <>
hipError_t launch_step<float>(const StepArgs<float>& a, int k, int batch, hipStream_t s)
{
    switch (k) {
    case 1: return launch_k<float, 1>(a, batch, s);
    case 2: return launch_k<float, 2>(a, batch, s);
    case 3: return launch_k<float, 3>(a, batch, s);
    case 4: return launch_k<float, 4>(a, batch, s);
    default: return hipErrorInvalidValue;
    }
}

template <>
hipError_t launch_step<double>(const StepArgs<double>& a, int k, int batch, hipStream_t s)
{
    switch (k) {
    case 1: return launch_k<double, 1>(a, batch, s);
    case 2: return launch_k<double, 2>(a, batch, s);
    default: return hipErrorInvalidValue;
    }
}

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
