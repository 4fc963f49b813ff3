// gfx950 discrete adjoint of the explicit PVD phase-field step.
//
// For u' = u + dt R(u; M_scale, v0) and a cotangent lambda' = dL/du', one
// adjoint step produces lambda = lambda' + (dR/du)^T w with w = dt lambda',
// and accumulates w . dR/dM_scale and w . dR/dv0 per cell in FP64.  The
// transpose is taken as a gather (each thread owns one output cell, no
// atomics) in three passes, all in one launch per step:
//   pass 0  forward potentials mu_c and M_c (the shared per-cell code of the
//           stepper), and at the output cell the mobility partials dM/dc,
//           dM/dphi;
//   pass A  cotangents of the intermediates:
//             mubar = sum_n (M + M_n)(w_c,n - w_c) / 2h^2   (CH operator on w_c)
//             Mbar  = sum_n (mu_n - mu)(w_c - w_c,n) / 2h^2
//             nubar = M_phi Lap w_phi,  Sbar = w_phi - w_rho;
//   pass B  chain rule back to (c, phi, rho): the pointwise derivatives of
//           mu_c, mu_phi and M_c, the symmetric Laplacians of mubar and
//           nubar, the transposed deposition stencil (an anti-mirrored
//           ghost in y for Sbar rho) and the transposed vapour
//           transport (inlet ghost is a constant; the substrate row keeps
//           its own mirror coefficient).
// A block forms pass 0 for its tile and two rings of cells around it and
// pass A for the tile and one ring in LDS, then runs pass B on its tile.
// The boundary rules are the transposes of the forward step's.
#include "pf_cell.h"

namespace pfk {
namespace {

using namespace cell;

template <typename T>
struct AdjArgs {
    const T* c;
    const T* phi;
    const T* rho;
    const T* lc;       // lambda' (in)
    const T* lp;
    const T* lr;
    T* oc;             // lambda (out)
    T* op;
    T* orr;
    double* gacc;      // [2][B][ny][nx] accumulated parameter gradients
    const Real* real;
    Coef<T> k;
    T Mscale_inv;      // 1 / M_scale (0 if M_scale == 0)
    T cosx, siny;      // d vx/d v0 = cos(theta), d vy/d v0 = -sin(theta) (0 if flux off)
    T inv2h;
    int nx, ny, pvd, batch;
};

__device__ __forceinline__ int wrapi(int i, int n) { return i < 0 ? i + n : (i >= n ? i - n : i); }

// neighbour row under the forward rule for c and phi: mirror (PVD) or wrap
__device__ __forceinline__ int nrow(int j, int n, int pvd)
{
    if (pvd) return j < 0 ? 0 : (j >= n ? n - 1 : j);
    return wrapi(j, n);
}

template <typename T>
__device__ __forceinline__ T ld(const T* a, int i, int j, int nx) { return a[(size_t)j * nx + i]; }

// dM_c/dc and dM_c/dphi (the coefficients in Coef are already scaled by
// M_scale), zero where the clamps are active
template <typename T>
__device__ __forceinline__ void mobility_grad(const Coef<T>& k, T c, T p, T& dmc, T& dmp)
{
    const T x = clampT(c, T(0), T(1));
    const T ph = clampT(p, T(-1), T(1));
    const T H = ((x * x) * x) * fmaT(fmaT(T(6), x, T(-15)), x, T(10));
    const T om = T(1) - x;
    const T dH = T(30) * (x * x) * (om * om);
    const T r1 = T(1) + ph;
    const T pb = (T(0.25) * (T(2) - ph)) * (r1 * r1);
    const T dpb = T(0.75) * (T(1) - ph * ph);
    const T e = surf_exp(ph * ph, k.esurf);
    // d e / d phi = -2 phi / sigma^2 e; esurf holds 1/sigma^2 (double) or
    // log2(e)/sigma^2 (float)
    const T inv_s2 = sizeof(T) == 4 ? k.esurf * T(0.6931471805599453) : k.esurf;
    const T de = T(-2) * ph * inv_s2 * e;
    const T bulk = fmaT(H, k.dMb, k.MBb), surf = fmaT(H, k.dMs, k.MBs);
    dmc = (c > T(0) && c < T(1)) ? (pb * k.dMb + e * k.dMs) * dH : T(0);
    dmp = (p > T(-1) && p < T(1)) ? fmaT(dpb, bulk, de * surf) : T(0);
}

__device__ __forceinline__ int modi(int i, int n) { return ((i % n) + n) % n; }

constexpr int kAdjRows = 8;   // tile rows of the adjoint step (one wave per row)

// One adjoint step for a block's 64 x kAdjRows cells.  Pass 0's mu_c and M_c are
// formed in LDS for the tile and two rings of cells around it, pass A's
// cotangents for the tile and one ring, and pass B reads both there.  A ring
// entry holds the value of the cell that the forward's neighbour rule reads
// at that place (x wraps; y mirrors under PVD, else wraps); per cell the
// arithmetic is that of three separate passes over the grid.
template <typename T>
__global__ __launch_bounds__(64 * kAdjRows) void adj_step(AdjArgs<T> a)
{
    constexpr int TW = 64, TH = kAdjRows, NT = 64 * kAdjRows;
    constexpr int AW = TW + 2, AH = TH + 2;   // pass A tile: one ring
    constexpr int ZW = TW + 4, ZH = TH + 4;   // pass 0 tile: two rings
    __shared__ T z[2][ZH][ZW];                // mu_c, M_c
    __shared__ T sm[4][AH][AW];               // mbar, nbar, Mbar, sig
    const int x0 = blockIdx.x * TW, y0 = blockIdx.y * TH;
    const int b = blockIdx.z;
    const int nx = a.nx, ny = a.ny, pvd = a.pvd;
    const size_t o = (size_t)b * nx * ny;
    const T* c = a.c + o;
    const T* phi = a.phi + o;
    const T* rho = a.rho + o;
    const T* lc = a.lc + o;
    const T* lp = a.lp + o;
    const T* lr = a.lr + o;
    const Coef<T>& k = a.k;
    const T dt = k.dt;

    // pass 0: entry (zj, zi) is the cell at column x0 - 2 + zi, row y0 - 2 + zj
    for (int e = threadIdx.x; e < ZH * ZW; e += NT) {
        const int zj = e / ZW, zi = e - zj * ZW;
        const int i = modi(x0 - 2 + zi, nx);
        const int gy = y0 - 2 + zj, j = pvd ? min(max(gy, 0), ny - 1) : modi(gy, ny);
        const int iE = wrapi(i + 1, nx), iW = wrapi(i - 1, nx);
        const int jN = nrow(j + 1, ny, pvd), jS = nrow(j - 1, ny, pvd);
        T mu, nu, M;
        potentials(k, ld(c, i, j, nx), ld(c, iE, j, nx), ld(c, iW, j, nx), ld(c, i, jN, nx), ld(c, i, jS, nx),
                   ld(phi, i, j, nx), ld(phi, iE, j, nx), ld(phi, iW, j, nx), ld(phi, i, jN, nx),
                   ld(phi, i, jS, nx), mu, nu, M);
        z[0][zj][zi] = mu;
        z[1][zj][zi] = M;
    }
    __syncthreads();

    // pass A: entry (hj, hi) is the cell at column x0 - 1 + hi, row y0 - 1 + hj
    for (int e = threadIdx.x; e < AH * AW; e += NT) {
        const int hj = e / AW, hi = e - hj * AW;
        const int i = modi(x0 - 1 + hi, nx);
        const int gy = y0 - 1 + hj, j = pvd ? min(max(gy, 0), ny - 1) : modi(gy, ny);
        const int iE = wrapi(i + 1, nx), iW = wrapi(i - 1, nx);
        const int jN = nrow(j + 1, ny, pvd), jS = nrow(j - 1, ny, pvd);
        // pass-0 rows of this cell and of its N and S neighbours: the tile's
        // row offsets follow the wrap rule, at a mirrored edge the row is the
        // neighbour's own; the columns follow the wrap rule in x
        const int zc = pvd ? j - y0 + 2 : hj + 1;
        const int zN = pvd ? jN - y0 + 2 : hj + 2;
        const int zS = pvd ? jS - y0 + 2 : hj;
        const int zr[4] = {zc, zc, zN, zS}, zq[4] = {hi + 2, hi, hi + 1, hi + 1};
        const int ni[4] = {iE, iW, i, i}, nj[4] = {j, j, jN, jS};
        const T wc = dt * ld(lc, i, j, nx), wp = dt * ld(lp, i, j, nx), wr = dt * ld(lr, i, j, nx);
        const T M0 = z[1][zc][hi + 1], m0 = z[0][zc][hi + 1];
        T mb = 0, Mb = 0, lapw = 0;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const T wn = dt * ld(lc, ni[q], nj[q], nx);
            mb += (M0 + z[1][zr[q]][zq[q]]) * (wn - wc);
            Mb += (z[0][zr[q]][zq[q]] - m0) * (wc - wn);
            lapw += dt * ld(lp, ni[q], nj[q], nx) - wp;
        }
        sm[0][hj][hi] = k.half_ih2 * mb;
        sm[1][hj][hi] = k.mphi_h2 * lapw;
        sm[2][hj][hi] = k.half_ih2 * Mb;
        sm[3][hj][hi] = (wp - wr) * ld(rho, i, j, nx);
    }
    __syncthreads();

    // pass B on the block's own cells
    const int li = threadIdx.x & 63, lj = threadIdx.x >> 6;
    const int i = x0 + li, j = y0 + lj;
    if (i >= nx || j >= ny) return;
    const Real rl = a.real[b];
    const T vx2h = (T)rl.vx2h, vy2h = (T)rl.vy2h;
    const int iE = wrapi(i + 1, nx), iW = wrapi(i - 1, nx);
    const bool top = pvd && j == ny - 1, bottom = pvd && j == 0;
    const int jN = nrow(j + 1, ny, pvd), jS = nrow(j - 1, ny, pvd);
    const size_t g = o + (size_t)j * nx + i;
    const T cc = a.c[g], pp = a.phi[g], rr = a.rho[g];
    const int hi = li + 1, hj = lj + 1;   // this cell in the pass A tile
    const T mb = sm[0][hj][hi], nb = sm[1][hj][hi], Mb = sm[2][hj][hi];
    T dmc, dmp;
    mobility_grad(k, cc, pp, dmc, dmp);

    // pointwise derivatives of mu_c = W_c p g' - ... and mu_phi = W_c p' g - W_phi phi (1-phi^2) - ...
    const T cg = cc * (T(1) - cc);
    const T g0 = cg * cg;
    const T g1 = cg * fmaT(T(-4), cc, T(2));
    const T g2 = T(2) * fmaT(T(6) * cc, cc, fmaT(T(-6), cc, T(1)));
    const T q1 = T(1) + pp;
    const T p0 = (T(0.25) * (T(2) - pp)) * (q1 * q1);
    const T p1 = T(0.75) * (T(1) - pp * pp);
    const T p2 = T(-1.5) * pp;
    T gc = mb * k.Wc * p0 * g2 + nb * k.Wc * p1 * g1;
    T gp = mb * k.Wc * p1 * g1 + nb * (k.Wc * p2 * g0 - k.Wphi * (T(1) - T(3) * pp * pp));
    // the Laplacians inside mu_c and mu_phi are symmetric (mirror rule)
    const T mE = sm[0][hj][hi + 1], mW = sm[0][hj][hi - 1], mN = sm[0][hj + 1][hi], mS = sm[0][hj - 1][hi];
    const T nE = sm[1][hj][hi + 1], nW = sm[1][hj][hi - 1], nN = sm[1][hj + 1][hi], nS = sm[1][hj - 1][hi];
    gc += k.kc * (T(4) * mb - ((mE + mW) + (mN + mS)));
    gp += k.kp * (T(4) * nb - ((nE + nW) + (nN + nS)));
    // mobility M_c (its host-scaled coefficients make dMc, dMp derivatives of M_c)
    gc += Mb * dmc;
    gp += Mb * dmp;
    // deposition: sig = Sbar rho of every cell whose stencil reads phi here;
    // the mirror ghost row in y turns into an anti-mirrored sig
    const T s0 = sm[3][hj][hi];
    const T sE = sm[3][hj][hi + 1], sW = sm[3][hj][hi - 1];
    const T sN = top ? -s0 : sm[3][hj + 1][hi];
    const T sS = bottom ? -s0 : sm[3][hj - 1][hi];
    gp += fmaT(vx2h, sW - sE, vy2h * (sS - sN));
    // rho: deposition, then the transposed transport stencil
    const T wp = dt * a.lp[g], wr = dt * a.lr[g];
    const T dphx = ld(phi, iE, j, nx) - ld(phi, iW, j, nx), dphy = ld(phi, i, jN, nx) - ld(phi, i, jS, nx);
    T gr = (wp - wr) * fmaT(vx2h, dphx, vy2h * dphy);
    const T D = k.D_h2;
    gr += (D - vx2h) * (dt * ld(lr, iW, j, nx)) + (D + vx2h) * (dt * ld(lr, iE, j, nx));
    if (!pvd) {
        gr += (D - vy2h) * (dt * ld(lr, i, jS, nx)) + (D + vy2h) * (dt * ld(lr, i, jN, nx));
    } else {
        if (j > 0) gr += (D - vy2h) * (dt * ld(lr, i, j - 1, nx));       // north coefficient of the cell below
        if (j < ny - 1) gr += (D + vy2h) * (dt * ld(lr, i, j + 1, nx));  // south coefficient of the cell above
        if (bottom) gr += (D - vy2h) * wr;                               // own mirror ghost, no advective flux
    }
    gr += T(-4) * D * wr;
    // parameter gradients (FP64 per cell): w . dR/dM_scale and w . dR/dv0
    const T rN = top ? k.rho_in : ld(rho, i, jN, nx);
    const T rSa = bottom ? -rr : ld(rho, i, jS, nx);
    const T dTv = -(a.cosx * (ld(rho, iE, j, nx) - ld(rho, iW, j, nx)) + a.siny * (rN - rSa)) * a.inv2h;
    const T dSv = rr * (a.cosx * dphx + a.siny * dphy) * a.inv2h;
    const size_t cells = (size_t)a.batch * nx * ny;
    a.gacc[g] += (double)Mb * (double)(z[1][lj + 2][li + 2] * a.Mscale_inv);
    a.gacc[cells + g] += (double)(wp - wr) * (double)dSv + (double)wr * (double)dTv;
    a.oc[g] = a.lc[g] + gc;
    a.op[g] = a.lp[g] + gp;
    a.orr[g] = a.lr[g] + gr;
}

__global__ __launch_bounds__(256) void fill_kernel(double* x, size_t n)
{
    for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (size_t)gridDim.x * 256) x[i] = 0.0;
}

__device__ __forceinline__ double wave_sum64(double v)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// out[b*2 + comp] = sum over the cells of realisation b of gacc[comp] (fixed order)
__global__ __launch_bounds__(256) void gsum_kernel(const double* gacc, double* out, size_t cells_per, int batch)
{
    const int b = blockIdx.x, comp = blockIdx.y;
    const double* x = gacc + (size_t)comp * batch * cells_per + (size_t)b * cells_per;
    double s = 0.0;
    for (size_t i = threadIdx.x; i < cells_per; i += 256) s += x[i];
    __shared__ double red[4];
    s = wave_sum64(s);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) out[b * 2 + comp] = (red[0] + red[1]) + (red[2] + red[3]);
}

template <typename T>
AdjArgs<T> adj_args(const AdjointIO<T>& io, const StepArgs<T>& st, double Mscale, double cos_th, double msin_th,
                    double h, int batch)
{
    AdjArgs<T> a{};
    a.c = io.c;
    a.phi = io.phi;
    a.rho = io.rho;
    a.lc = io.lc;
    a.lp = io.lp;
    a.lr = io.lr;
    a.oc = io.oc;
    a.op = io.op;
    a.orr = io.orr;
    a.gacc = io.gacc;
    a.real = st.real;
    a.k = st.k;
    a.Mscale_inv = (T)(1.0 / Mscale);
    a.cosx = (T)cos_th;
    a.siny = (T)msin_th;
    a.inv2h = (T)(0.5 / h);
    a.nx = st.nx;
    a.ny = st.ny;
    a.pvd = st.pvd;
    a.batch = batch;
    return a;
}

template <typename T>
dim3 adj_grid(const AdjArgs<T>& a) { return dim3((a.nx + 63) / 64, (a.ny + kAdjRows - 1) / kAdjRows, a.batch); }

}  // namespace

template <typename T>
hipError_t launch_adjoint(const AdjointIO<T>& io, const StepArgs<T>& st, double Mscale, double cos_th,
                          double msin_th, double h, int batch, hipStream_t s)
{
    const AdjArgs<T> a = adj_args<T>(io, st, Mscale, cos_th, msin_th, h, batch);
    hipLaunchKernelGGL(adj_step<T>, adj_grid(a), dim3(64 * kAdjRows), 0, s, a);
    return hipGetLastError();
}
template hipError_t launch_adjoint<float>(const AdjointIO<float>&, const StepArgs<float>&, double, double, double,
                                          double, int, hipStream_t);
template hipError_t launch_adjoint<double>(const AdjointIO<double>&, const StepArgs<double>&, double, double,
                                           double, double, int, hipStream_t);

hipError_t launch_gacc_zero(double* gacc, size_t n, hipStream_t s)
{
    hipLaunchKernelGGL(fill_kernel, dim3(256), dim3(256), 0, s, gacc, n);
    return hipGetLastError();
}

hipError_t launch_gacc_sum(const double* gacc, double* out, size_t cells_per, int batch, hipStream_t s)
{
    hipLaunchKernelGGL(gsum_kernel, dim3(batch, 2), dim3(256), 0, s, gacc, out, cells_per, batch);
    return hipGetLastError();
}

}  // namespace pfk
