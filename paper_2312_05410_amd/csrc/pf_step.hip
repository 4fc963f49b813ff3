// gfx950 stepper of the explicit PVD phase-field model (Materials and
// Methods, "Phase-field modeling of physical vapor deposition"; second-order
// central differences as stated in "Dataset"; explicit Euler in time).
//
// One launch advances a 64 x TY output tile of one realisation by up to K
// sub-steps.  Layout of a workgroup (256 threads = 4 wave64s):
//
//  * load: the tile plus a halo of R = 2K cells (radius 2 per sub-step) of
//    c, phi, rho is read from HBM once, as 16-byte vectors (row-contiguous,
//    x wrapped periodically, y mirrored or the inlet value), into LDS;
//  * every sub-step runs two stencil stages out of LDS.  Stage 1 computes
//    mu_c, mu_phi, M_c on the region one cell wider than the update region;
//    stage 2 computes the flux-form conserved updates, the deposition
//    source and vapour transport.  In both stages the 64 output columns map
//    to the 64 lanes of a wave and each wave marches down a contiguous run
//    of rows, so north/south neighbours stay in registers and east/west pairs
//    come from one ds_read2; the narrower margins of the halo are done as a
//    flattened remainder pass;
//  * only the 64 x TY tile is written back: one HBM read and one write of
//    the state per launch, whatever K is.
//
// Every cell, in the main block or a margin, in any K or tile shape, is
// evaluated by the same two inline functions with a fixed expression order
// (contraction off, explicit fma), so all variants give bitwise-identical
// states.
#include "pf_cell.h"

namespace pfk {
namespace {

using namespace cell;

// 16-byte vectors as native clang vector types (kept in registers)
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef double f64x2 __attribute__((ext_vector_type(2)));
template <typename T> struct VecT;
template <> struct VecT<float> {
    using type = f32x4;
    __device__ static type pick(bool c, float v, type x) { return c ? (type){v, v, v, v} : x; }
};
template <> struct VecT<double> {
    using type = f64x2;
    __device__ static type pick(bool c, double v, type x) { return c ? (type){v, v} : x; }
};

// Compile-time geometry of one instantiation.
template <typename T, int K, int TY>
struct Geo {
    static constexpr int NT = 256;
    static constexpr int V = 16 / (int)sizeof(T);          // elements per 16-byte vector
    static constexpr int R = 2 * K;                         // halo: radius 2 per sub-step
    static constexpr int A = ((R + V - 1) / V) * V;         // left pad, >= R, multiple of V
    static constexpr int LW = 64 + 2 * A;                   // LDS row length
    static constexpr int P = LW;                            // LDS row pitch
    static constexpr int LH = TY + 2 * R;                   // LDS rows
    static constexpr int N = LH * P;
    static constexpr int NV = LW / V;                       // vectors per row
};

template <typename T, int N>
struct alignas(16) Tile {
    T c[N], p[N], r[N], mc[N], mp[N], M[N];
};

__device__ __forceinline__ int reflect_clamp(int j, int n, int pvd)
{
    // one mirror (PVD) or wrap (periodic) step, then clamp so that rows
    // beyond every dependency cone still address memory inside the grid
    if (pvd) j = j < 0 ? -1 - j : (j >= n ? 2 * n - 1 - j : j);
    else j = j < 0 ? j + n : (j >= n ? j - n : j);
    return j < 0 ? 0 : (j >= n ? n - 1 : j);
}

template <typename T, int K, int TY>
struct Stepper {
    using G = Geo<T, K, TY>;
    static constexpr int NT = G::NT, R = G::R, A = G::A, LW = G::LW, P = G::P, LH = G::LH, V = G::V;
    using Tl = Tile<T, G::N>;

    const StepArgs<T> a;
    Tl& t;
    double* s_q;
    int b, x0, y0, tid, lane, wv;
    T vx2h, vy2h;
    double qa, qb;
    RhoCoef<T> rc;

    // ------------------------------------------------------------ load
    __device__ __forceinline__ void load()
    {
        const int nx = a.nx, ny = a.ny;
        const size_t plane = (size_t)nx * ny;
        const T* gc = a.c + (size_t)b * plane;
        const T* gp = a.phi + (size_t)b * plane;
        const T* gr = a.rho + (size_t)b * plane;
        const T rin = a.k.rho_in;
        if (a.fast) {
            // 16-byte vectors: nx % V == 0 and nx >= 64 + A, so each vector
            // lies wholly inside the grid after one periodic wrap
            using VT = typename VecT<T>::type;
            constexpr int NVEC = LH * G::NV;
            constexpr int QL = (NVEC + NT - 1) / NT;
            VT vc[QL], vp[QL], vr[QL];
            // every load is issued (indices clamped into the tile) before any
            // LDS store, so all of a thread's loads are in flight together
#pragma unroll
            for (int q = 0; q < QL; ++q) {
                const int idx = min(tid + q * NT, NVEC - 1);
                const int r = idx / G::NV, v = idx % G::NV;
                const int gj = y0 - R + r;
                const int jj = reflect_clamp(gj, ny, a.pvd);
                int gi = x0 - A + v * V;
                gi = gi < 0 ? gi + nx : (gi >= nx ? gi - nx : gi);
                const size_t g = (size_t)jj * nx + gi;
                vc[q] = *(const VT*)(gc + g);
                vp[q] = *(const VT*)(gp + g);
                vr[q] = VecT<T>::pick(a.pvd && gj >= ny, rin, *(const VT*)(gr + g));
            }
            // surplus threads (idx clamped) rewrite the last vector with the
            // same values, which keeps this phase free of branches
#pragma unroll
            for (int q = 0; q < QL; ++q) {
                const int idx = min(tid + q * NT, NVEC - 1);
                const int r = idx / G::NV, v = idx % G::NV;
                const int l = r * P + v * V;
                *(VT*)&t.c[l] = vc[q];
                *(VT*)&t.p[l] = vp[q];
                *(VT*)&t.r[l] = vr[q];
            }
        } else {
            // any grid: element loads with exact periodic wrap and mirror
            for (int idx = tid; idx < LH * LW; idx += NT) {
                const int r = idx / LW, lx = idx % LW;
                int gi = x0 - A + lx;
                while (gi < 0) gi += nx;
                while (gi >= nx) gi -= nx;
                const int gj = y0 - R + r;
                int jj = gj;
                if (a.pvd) {
                    while (jj < 0 || jj >= ny) jj = jj < 0 ? -1 - jj : 2 * ny - 1 - jj;
                } else {
                    while (jj < 0) jj += ny;
                    while (jj >= ny) jj -= ny;
                }
                const size_t g = (size_t)jj * nx + gi;
                const int l = r * P + lx;
                t.c[l] = gc[g];
                t.p[l] = gp[g];
                t.r[l] = (a.pvd && gj >= ny) ? rin : gr[g];
            }
        }
    }

    // ------------------------------------------------------- stage 1
    __device__ __forceinline__ void pot_cell(int l)
    {
        T mc, mp, M;
        potentials(a.k, t.c[l], t.c[l + 1], t.c[l - 1], t.c[l + P], t.c[l - P],
                   t.p[l], t.p[l + 1], t.p[l - 1], t.p[l + P], t.p[l - P], mc, mp, M);
        t.mc[l] = mc;
        t.mp[l] = mp;
        t.M[l] = M;
    }

    template <int S>
    __device__ __forceinline__ void stage1()
    {
        constexpr int rb = 2 * S + 1, re = LH - 2 * S - 1, nr = re - rb;
        constexpr int RPW = (nr + 3) / 4;
        // main block: the 64 output columns, a run of rows per wave
        const int r0 = rb + wv * RPW;
        if (r0 < re) {
            const int lx = A + lane;
            T cS = t.c[(r0 - 1) * P + lx], cC = t.c[r0 * P + lx];
            T pS = t.p[(r0 - 1) * P + lx], pC = t.p[r0 * P + lx];
#pragma unroll
            for (int i = 0; i < RPW; ++i) {
                const int r = r0 + i;
                if (r < re) {
                    const int l = r * P + lx;
                    const T cN = t.c[l + P], pN = t.p[l + P];
                    T mc, mp, M;
                    potentials(a.k, cC, t.c[l + 1], t.c[l - 1], cN, cS,
                               pC, t.p[l + 1], t.p[l - 1], pN, pS, mc, mp, M);
                    t.mc[l] = mc;
                    t.mp[l] = mp;
                    t.M[l] = M;
                    cS = cC;
                    cC = cN;
                    pS = pC;
                    pC = pN;
                }
            }
        }
        // margins: MW columns left and right of the output columns
        constexpr int MW = R - 2 * S - 1;
        if constexpr (MW > 0) {
            constexpr int NM = 2 * MW * nr;
            // reversed thread order puts the margin work on the last wave,
            // whose row run is the shortest
            for (int idx = NT - 1 - tid; idx < NM; idx += NT) {
                const int side = idx / (MW * nr), rem = idx % (MW * nr);
                const int r = rb + rem / MW, m = rem % MW;
                const int lx = side ? A + 64 + m : A - MW + m;
                pot_cell(r * P + lx);
            }
        }
    }

    // ------------------------------------------------------- stage 2
    __device__ __forceinline__ void upd_cell(int l, bool bottom, T& nc, T& np, T& nr)
    {
        const T M0 = t.M[l], m0 = t.mc[l];
        update(a.k, rc, vx2h, vy2h, bottom, t.c[l],
               t.p[l], t.p[l + 1], t.p[l - 1], t.p[l + P], t.p[l - P],
               t.r[l], t.r[l + 1], t.r[l - 1], t.r[l + P], t.r[l - P],
               cflux(M0, m0, t.M[l + 1], t.mc[l + 1]), cflux(t.M[l - 1], t.mc[l - 1], M0, m0),
               cflux(M0, m0, t.M[l + P], t.mc[l + P]), cflux(t.M[l - P], t.mc[l - P], M0, m0),
               t.mp[l], t.mp[l + 1], t.mp[l - 1], t.mp[l + P], t.mp[l - P], nc, np, nr);
    }

    // inflow through the top face of an output cell in row ny-1
    __device__ __forceinline__ void inflow(int r, int lx, T r0)
    {
        const int gj = y0 - R + r;
        if (a.pvd && gj == a.ny - 1 && r >= R && r < R + TY && lx >= A && lx < A + 64) {
            const int ix = lx - A;
            if (x0 + ix < a.nx) {
                const double rin = (double)a.k.rho_in, rr = (double)r0;
                s_q[ix] += qa * (rr + rin) + qb * (rin - rr);
            }
        }
    }

    template <int S>
    __device__ __forceinline__ void stage2(bool last)
    {
        constexpr int rb = 2 * S + 2, re = LH - 2 * S - 2, nr = re - rb;
        constexpr int RPW = (nr + 3) / 4;
        constexpr int MW = R - 2 * S - 2;
        constexpr int NM = 2 * MW * nr;
        constexpr int QM = (NM + NT - 1) / NT;
        T mc_[RPW], mp_[RPW], mr_[RPW];
        T xc_[QM > 0 ? QM : 1], xp_[QM > 0 ? QM : 1], xr_[QM > 0 ? QM : 1];
        const int r0 = rb + wv * RPW;
        const int lx = A + lane;
        if (r0 < re) {
            T pS = t.p[(r0 - 1) * P + lx], pC = t.p[r0 * P + lx];
            T rS = t.r[(r0 - 1) * P + lx], rC = t.r[r0 * P + lx];
            T MS = t.M[(r0 - 1) * P + lx], MC = t.M[r0 * P + lx];
            T mS = t.mc[(r0 - 1) * P + lx], mC = t.mc[r0 * P + lx];
            T qS = t.mp[(r0 - 1) * P + lx], qC = t.mp[r0 * P + lx];
#pragma unroll
            for (int i = 0; i < RPW; ++i) {
                const int r = r0 + i;
                if (r < re) {
                    const int l = r * P + lx;
                    const T pN = t.p[l + P], rN = t.r[l + P], MN = t.M[l + P], mN = t.mc[l + P], qN = t.mp[l + P];
                    const bool bottom = a.pvd && (y0 - R + r) == 0;
                    update(a.k, rc, vx2h, vy2h, bottom, t.c[l],
                           pC, t.p[l + 1], t.p[l - 1], pN, pS,
                           rC, t.r[l + 1], t.r[l - 1], rN, rS,
                           cflux(MC, mC, t.M[l + 1], t.mc[l + 1]), cflux(t.M[l - 1], t.mc[l - 1], MC, mC),
                           cflux(MC, mC, MN, mN), cflux(MS, mS, MC, mC),
                           qC, t.mp[l + 1], t.mp[l - 1], qN, qS, mc_[i], mp_[i], mr_[i]);
                    inflow(r, lx, rC);
                    pS = pC; pC = pN;
                    rS = rC; rC = rN;
                    MS = MC; MC = MN;
                    mS = mC; mC = mN;
                    qS = qC; qC = qN;
                }
            }
        }
        if constexpr (MW > 0) {
#pragma unroll
            for (int q = 0; q < QM; ++q) {
                const int idx = NT - 1 - tid + q * NT;
                if (idx < NM) {
                    const int side = idx / (MW * nr), rem = idx % (MW * nr);
                    const int r = rb + rem / MW, m = rem % MW;
                    const int mx = side ? A + 64 + m : A - MW + m;
                    const bool bottom = a.pvd && (y0 - R + r) == 0;
                    upd_cell(r * P + mx, bottom, xc_[q], xp_[q], xr_[q]);
                }
            }
        }

        if (last) {
            // store the output tile only: when this launch runs fewer
            // sub-steps than its capacity K, the region still holds halo rows
            const int nx = a.nx, ny = a.ny;
            const size_t plane = (size_t)nx * ny;
            const int gi = x0 + lane;
            if (gi < nx) {
                T* oc = a.c_out + (size_t)b * plane;
                T* op = a.phi_out + (size_t)b * plane;
                T* orr = a.rho_out + (size_t)b * plane;
#pragma unroll
                for (int i = 0; i < RPW; ++i) {
                    const int r = r0 + i;
                    const int gj = y0 - R + r;
                    if (r < re && r >= R && r < R + TY && gj < ny) {
                        const size_t g = (size_t)gj * nx + gi;
                        oc[g] = mc_[i];
                        op[g] = mp_[i];
                        orr[g] = mr_[i];
                    }
                }
            }
            return;
        }

        __syncthreads();
#pragma unroll
        for (int i = 0; i < RPW; ++i) {
            const int r = r0 + i;
            if (r < re) {
                const int l = r * P + lx;
                t.c[l] = mc_[i];
                t.p[l] = mp_[i];
                t.r[l] = mr_[i];
            }
        }
        if constexpr (MW > 0) {
#pragma unroll
            for (int q = 0; q < QM; ++q) {
                const int idx = NT - 1 - tid + q * NT;
                if (idx < NM) {
                    const int side = idx / (MW * nr), rem = idx % (MW * nr);
                    const int r = rb + rem / MW, m = rem % MW;
                    const int mx = side ? A + 64 + m : A - MW + m;
                    const int l = r * P + mx;
                    t.c[l] = xc_[q];
                    t.p[l] = xp_[q];
                    t.r[l] = xr_[q];
                }
            }
        }
        __syncthreads();
        ghost_fix<S>();
    }

    // PVD: rows outside the grid that later sub-steps still read are refilled
    // from their mirror rows (rho above the top: the inlet value).
    template <int S>
    __device__ __forceinline__ void ghost_fix()
    {
        if (!a.pvd) return;
        constexpr int o = 2 * S + 2;          // region offset after this sub-step
        constexpr int W = LW - 2 * (A - R + o);
        constexpr int depth = R - o;          // ghost depth still needed
        const int ny = a.ny;
        const bool lo = (y0 - R + o) < 0;
        const bool hi = (y0 - R + LH - o - 1) >= ny;
        if (!(lo || hi)) return;
        constexpr int NR = LH - 2 * o;
        for (int idx = tid; idx < NR * W; idx += NT) {
            const int r = o + idx / W, lx = (A - R + o) + idx % W;
            const int gj = y0 - R + r;
            int gm;
            bool top = false;
            if (gj < 0) {
                if (-gj > depth) continue;
                gm = -1 - gj;
            } else if (gj >= ny) {
                if (gj - ny + 1 > depth) continue;
                gm = 2 * ny - 1 - gj;
                top = true;
            } else {
                continue;
            }
            const int l = r * P + lx, m = (gm - (y0 - R)) * P + lx;
            t.c[l] = t.c[m];
            t.p[l] = t.p[m];
            t.r[l] = top ? a.k.rho_in : t.r[m];
        }
        __syncthreads();
    }

    template <int S>
    __device__ __forceinline__ void substep()
    {
        stage1<S>();
        __syncthreads();
        const bool last = (S == a.nsub - 1);
        stage2<S>(last);
        if constexpr (S + 1 < K) {
            if (!last) substep<S + 1>();
        }
    }
};

template <typename T, int K, int TY>
__global__ __launch_bounds__(256) void step_kernel(StepArgs<T> a)
{
    using G = Geo<T, K, TY>;
    __shared__ Tile<T, G::N> t;
    __shared__ double s_q[64];

    const int tid = threadIdx.x;
    const int b = blockIdx.y;
    const int nx = a.nx, ny = a.ny;
    // Tile order: consecutive workgroup ids go round-robin over the 8 XCDs;
    // give XCD x a contiguous band of tiles so shared halos stay in its L2.
    const int nblk = a.tiles_x * a.tiles_y;
    const int bid = blockIdx.x;
    const int xcd = bid & 7, slot = bid >> 3;
    const int q8 = nblk >> 3, r8 = nblk & 7;
    const int tileid = xcd * q8 + (xcd < r8 ? xcd : r8) + slot;
    const int x0 = (tileid % a.tiles_x) * 64;
    const int y0 = (tileid / a.tiles_x) * TY;

    const Real rl = a.real[b];
    const T vx2h = (T)rl.vx2h, vy2h = (T)rl.vy2h;
    Stepper<T, K, TY> st{a,    t,   s_q,  b,     x0,    y0,    tid,  tid & 63, tid >> 6,
                         vx2h, vy2h, rl.qa, rl.qb, rho_coef(a.k, vx2h, vy2h)};
    st.load();
    const bool top = a.pvd && y0 <= ny - 1 && ny - 1 < y0 + TY;
    if (top && tid < 64 && x0 + tid < nx) s_q[tid] = a.Qcol[(size_t)b * nx + x0 + tid];
    __syncthreads();
    st.template substep<0>();
    if (top) {
        __syncthreads();
        if (tid < 64 && x0 + tid < nx) a.Qcol[(size_t)b * nx + x0 + tid] = s_q[tid];
    }
}

// Tile heights per precision and fused-step count.
template <typename T, int K> struct Shape;
template <> struct Shape<float, 1> { static constexpr int TY = 16; };
template <> struct Shape<float, 2> { static constexpr int TY = 32; };
template <> struct Shape<float, 3> { static constexpr int TY = 32; };
template <> struct Shape<float, 4> { static constexpr int TY = 32; };
template <> struct Shape<double, 1> { static constexpr int TY = 16; };
template <> struct Shape<double, 2> { static constexpr int TY = 16; };

template <typename T, int K>
hipError_t launch_k(StepArgs<T> a, int batch, hipStream_t s)
{
    using G = Geo<T, K, Shape<T, K>::TY>;
    a.fast = (a.nx % G::V == 0) && (a.nx >= 64 + G::A) ? 1 : 0;
    dim3 grid(a.tiles_x * a.tiles_y, batch);
    hipLaunchKernelGGL((step_kernel<T, K, Shape<T, K>::TY>), grid, dim3(256), 0, s, a);
    return hipGetLastError();
}

template <typename T, int K>
hipError_t node_k(hipGraph_t g, hipGraphNode_t* node, hipGraphNode_t dep, StepArgs<T> a, int batch)
{
    using G = Geo<T, K, Shape<T, K>::TY>;
    a.fast = (a.nx % G::V == 0) && (a.nx >= 64 + G::A) ? 1 : 0;
    void* args[] = {&a};
    hipKernelNodeParams kp{};
    kp.func = (void*)step_kernel<T, K, Shape<T, K>::TY>;
    kp.gridDim = dim3(a.tiles_x * a.tiles_y, batch);
    kp.blockDim = dim3(256);
    kp.sharedMemBytes = 0;
    kp.kernelParams = args;
    kp.extra = nullptr;
    return hipGraphAddKernelNode(node, g, dep ? &dep : nullptr, dep ? 1 : 0, &kp);
}

}  // namespace

template <>
hipError_t graph_add_step<float>(hipGraph_t g, hipGraphNode_t* node, hipGraphNode_t dep,
                                 const StepArgs<float>& a, int k, int batch)
{
    switch (k) {
    case 2: return node_k<float, 2>(g, node, dep, a, batch);
    case 3: return node_k<float, 3>(g, node, dep, a, batch);
    case 4: return node_k<float, 4>(g, node, dep, a, batch);
    default: return hipErrorInvalidValue;
    }
}

template <>
hipError_t graph_add_step<double>(hipGraph_t g, hipGraphNode_t* node, hipGraphNode_t dep,
                                  const StepArgs<double>& a, int k, int batch)
{
    switch (k) {
    case 2: return node_k<double, 2>(g, node, dep, a, batch);
    default: return hipErrorInvalidValue;
    }
}

template <>
TileCfg tile_cfg<float>(int k)
{
    switch (k) {
    case 1: return {64, Shape<float, 1>::TY, 1, 256};
    case 2: return {64, Shape<float, 2>::TY, 2, 256};
    case 3: return {64, Shape<float, 3>::TY, 3, 256};
    case 4: return {64, Shape<float, 4>::TY, 4, 256};
    default: return {0, 0, 0, 0};
    }
}

template <>
TileCfg tile_cfg<double>(int k)
{
    switch (k) {
    case 1: return {64, Shape<double, 1>::TY, 1, 256};
    case 2: return {64, Shape<double, 2>::TY, 2, 256};
    default: return {0, 0, 0, 0};
    }
}

template <>
hipError_t launch_step<float>(const StepArgs<float>& a, int k, int batch, hipStream_t s)
{
    switch (k) {
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
    case 2: return launch_k<double, 2>(a, batch, s);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace pfk
