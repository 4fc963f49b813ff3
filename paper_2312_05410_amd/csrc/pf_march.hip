// gfx950 single-step stepper: one wave64 marches down a 64-column strip.
//
// Lane i holds column xs + i of the strip (xs = 60 s - 2) and the wave walks
// the rows of a TY-row chunk from south to north.  North/south neighbours
// are the previous and next rows, kept in registers; east/west neighbours
// are the adjacent lanes, fetched with whole-wave DPP shifts (wave_shl:1,
// wave_shr:1).  Stage 1 (mu_c, mu_phi, M_c) is valid in lanes 1..62 and
// stage 2 (the Euler update) in lanes 2..61, so each strip writes 60
// columns and strips overlap by 4.  There is no LDS and no barrier: each
// wave streams its rows, with the loads of row t issued D rows before they
// are used, and writes every output cell once.  HBM traffic per step is one
// read and one write of c, phi, rho plus the 4-column strip overlap and the
// 4-row chunk halo (mostly L2 hits).
//
// The per-cell arithmetic is the shared code of pf_cell.h, so this kernel is
// bitwise identical to the LDS-tiled kernels.
#include "pf_cell.h"

namespace pfk {
namespace {

using namespace cell;

constexpr int kStripOut = 60;   // output columns per 64-lane strip

// lane i <- lane i+1 (east neighbour) / lane i <- lane i-1 (west).  With
// bound_ctrl set, the lane without a source reads 0 (its results are never
// used) and the move can fold into the consuming instruction as a DPP
// operand.
__device__ __forceinline__ int east_i(int v) { return __builtin_amdgcn_mov_dpp(v, 0x130, 0xf, 0xf, true); }
__device__ __forceinline__ int west_i(int v) { return __builtin_amdgcn_mov_dpp(v, 0x138, 0xf, 0xf, true); }
__device__ __forceinline__ float east(float v) { return __builtin_bit_cast(float, east_i(__builtin_bit_cast(int, v))); }
__device__ __forceinline__ float west(float v) { return __builtin_bit_cast(float, west_i(__builtin_bit_cast(int, v))); }
__device__ __forceinline__ double east(double v)
{
    const int2 w = __builtin_bit_cast(int2, v);
    return __builtin_bit_cast(double, make_int2(east_i(w.x), east_i(w.y)));
}
__device__ __forceinline__ double west(double v)
{
    const int2 w = __builtin_bit_cast(int2, v);
    return __builtin_bit_cast(double, make_int2(west_i(w.x), west_i(w.y)));
}

// Raw buffer loads and stores: the lane's column is a fixed vector offset
// and the row offset is a scalar, so no per-access address arithmetic runs
// on the vector ALU.  A plane must be below 2 GiB (checked on the host).
template <typename T> struct Buf;
template <> struct Buf<float> {
    __device__ static float ld(__amdgpu_buffer_rsrc_t r, int vo, int so)
    {
        return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, vo, so, 0));
    }
    __device__ static void st(float v, __amdgpu_buffer_rsrc_t r, int vo, int so)
    {
        __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, v), r, vo, so, 0);
    }
};
typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));
template <> struct Buf<double> {
    using U = u32x2;
    __device__ static double ld(__amdgpu_buffer_rsrc_t r, int vo, int so)
    {
        return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, vo, so, 0));
    }
    __device__ static void st(double v, __amdgpu_buffer_rsrc_t r, int vo, int so)
    {
        __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(U, v), r, vo, so, 0);
    }
};

// gfx9 raw-buffer descriptor word 3 (32-bit data format, no swizzle)
constexpr int kBufFlags = 0x00020000;

template <typename T>
__device__ __forceinline__ __amdgpu_buffer_rsrc_t plane_rsrc(const T* base, size_t plane)
{
    return __builtin_amdgcn_make_buffer_rsrc((void*)base, (short)0, (int)(plane * sizeof(T)), kBufFlags);
}

// One wave per (strip, chunk).  TY output rows; input rows t = 0..TY+3 are
// global rows y0-2+t; stage 1 runs on t = 1..TY+2, stage 2 on t = 2..TY+1.
// BASE: the update adds to the state at a.cb/pb/rb (the midpoint method's
// second stage) instead of the evaluated state.  NOISE: cells that end on the
// vapour side take the interface composition draw.
template <typename T, int TY, int D, bool BASE, bool NOISE>
__global__ __launch_bounds__(64) void march_kernel(StepArgs<T> a)
{
    constexpr int NR = TY + 4;
    const int lane = threadIdx.x;
    const int b = blockIdx.y;
    const int nx = a.nx, ny = a.ny;
    const int nstrip = a.tiles_x;

    // XCD-aware order: XCD x gets a contiguous band of (chunk, strip) tiles
    const int nblk = a.tiles_x * a.tiles_y;
    const int bid = blockIdx.x;
    const int xcd = bid & 7, slot = bid >> 3;
    const int q8 = nblk >> 3, r8 = nblk & 7;
    const int tileid = xcd * q8 + (xcd < r8 ? xcd : r8) + slot;
    const int strip = tileid % nstrip;
    const int y0 = (tileid / nstrip) * TY;

    int gx = strip * kStripOut - 2 + lane;
    while (gx < 0) gx += nx;
    while (gx >= nx) gx -= nx;
    const int ocol = strip * kStripOut + lane - 2;     // output column of this lane
    const bool out_lane = lane >= 2 && lane < 2 + kStripOut && ocol < nx;

    const size_t plane = (size_t)nx * ny;
    const auto bc = plane_rsrc(a.c + (size_t)b * plane, plane);
    const auto bp = plane_rsrc(a.phi + (size_t)b * plane, plane);
    const auto br = plane_rsrc(a.rho + (size_t)b * plane, plane);
    const auto oc = plane_rsrc(a.c_out + (size_t)b * plane, plane);
    const auto op = plane_rsrc(a.phi_out + (size_t)b * plane, plane);
    const auto orr = plane_rsrc(a.rho_out + (size_t)b * plane, plane);
    const auto bcb = plane_rsrc((BASE ? a.cb : a.c) + (size_t)b * plane, plane);
    const auto bpb = plane_rsrc((BASE ? a.pb : a.phi) + (size_t)b * plane, plane);
    const auto brb = plane_rsrc((BASE ? a.rb : a.rho) + (size_t)b * plane, plane);
    const int vo = gx * (int)sizeof(T);
    const int row_bytes = nx * (int)sizeof(T);
    const Coef<T> k = a.k;
    const Real rl = a.real[b];
    const T vx2h = (T)rl.vx2h, vy2h = (T)rl.vy2h;
    const int pvd = a.pvd;

    T c[NR], p[NR], r[NR];
    T mc[NR], mp[NR], M[NR], pE[NR], pW[NR], FN[NR];
    const RhoCoef<T> rc = rho_coef(k, vx2h, vy2h);

    // row t of the inputs: mirrored (PVD) or wrapped row index, clamped so
    // that rows beyond every dependency cone still address the grid
    auto load_row = [&](int t) {
        const int gj = y0 - 2 + t;
        int jj;
        if (pvd) jj = gj < 0 ? -1 - gj : (gj >= ny ? 2 * ny - 1 - gj : gj);
        else jj = gj < 0 ? gj + ny : (gj >= ny ? gj - ny : gj);
        jj = jj < 0 ? 0 : (jj >= ny ? ny - 1 : jj);
        const int so = jj * row_bytes;
        c[t] = Buf<T>::ld(bc, vo, so);
        p[t] = Buf<T>::ld(bp, vo, so);
        const T rv = Buf<T>::ld(br, vo, so);
        r[t] = (pvd && gj >= ny) ? k.rho_in : rv;
    };

#pragma unroll
    for (int t = 0; t < NR; ++t)
        if (t < 3 + D) load_row(t);

#pragma unroll
    for (int t1 = 1; t1 <= TY + 2; ++t1) {
        if (t1 + 2 + D < NR) load_row(t1 + 2 + D);
        // stage 1 at row t1
        {
            const T cE = east(c[t1]), cW = west(c[t1]);
            pE[t1] = east(p[t1]);
            pW[t1] = west(p[t1]);
            potentials(k, c[t1], cE, cW, c[t1 + 1], c[t1 - 1], p[t1], pE[t1], pW[t1], p[t1 + 1], p[t1 - 1],
                       mc[t1], mp[t1], M[t1]);
        }
        // stage 2 at row t = t1 - 1; each face flux of c is computed once:
        // the west flux is the west lane's east flux, the south flux is the
        // previous row's north flux
        if (t1 >= 3) {
            const int t = t1 - 1;
            const int gj = y0 - 2 + t;
            const bool bottom = pvd && gj == 0;
            if (t == 2) FN[1] = cflux(M[1], mc[1], M[2], mc[2]);
            const T FE = cflux(M[t], mc[t], east(M[t]), east(mc[t]));
            FN[t] = cflux(M[t], mc[t], M[t + 1], mc[t + 1]);
            T nc, np, nr;
            T cb0 = c[t], pb0 = p[t], rb0 = r[t];
            if (BASE && gj < ny) {
                const int so = gj * row_bytes;
                cb0 = Buf<T>::ld(bcb, vo, so);
                pb0 = Buf<T>::ld(bpb, vo, so);
                rb0 = Buf<T>::ld(brb, vo, so);
            }
            update(k, rc, vx2h, vy2h, bottom, c[t],
                   p[t], pE[t], pW[t], p[t + 1], p[t - 1],
                   r[t], east(r[t]), west(r[t]), r[t + 1], r[t - 1],
                   FE, west(FE), FN[t], FN[t - 1],
                   mp[t], east(mp[t]), west(mp[t]), mp[t + 1], mp[t - 1], nc, np, nr, cb0, pb0, rb0);
            if (NOISE && gj < ny && out_lane && np < T(0)) {
                const uint64_t id = (uint64_t)a.step * plane + (uint64_t)gj * nx + ocol;
                nc = interface_draw<T>(rl.nseed, id * 16ull, rl.c0, a.noise);
            }
            if (gj < ny) {
                if (out_lane) {
                    const int so = gj * row_bytes;
                    Buf<T>::st(nc, oc, vo, so);
                    Buf<T>::st(np, op, vo, so);
                    Buf<T>::st(nr, orr, vo, so);
                }
                if (a.Qcol && pvd && gj == ny - 1 && out_lane) {
                    // inflow through the top face: advective + diffusive flux
                    double* q = a.Qcol + (size_t)b * nx + ocol;
                    const double rin = (double)k.rho_in, rr = (double)r[t];
                    *q = *q + (rl.qa * (rr + rin) + rl.qb * (rin - rr));
                }
            }
        }
    }
}

// Two columns per lane (FP32, even nx): lane i holds columns xs + 2i and
// xs + 2i + 1 (xs = 124 s - 2) as one 8-byte load, so a wave covers 128
// columns and writes 124.  Of each cell's east/west neighbours one is the
// lane's other column and one comes from the adjacent lane (a single DPP
// move per field per pair), which halves the neighbour exchanges and the
// scalar work per cell and shrinks the strip overlap from 4/64 to 4/128.
// Same per-cell functions in the same order: bitwise identical results.
constexpr int kStripOut2 = 124;

struct F2 {
    float a, b;
};
__device__ __forceinline__ F2 ld2(__amdgpu_buffer_rsrc_t r, int vo, int so)
{
    // element access on the builtin's own vector type (a bit_cast of it to
    // another two-element vector type compiled to a single-dword load)
    const auto v = __builtin_amdgcn_raw_buffer_load_b64(r, vo, so, 0);
    return {__builtin_bit_cast(float, (unsigned)v[0]), __builtin_bit_cast(float, (unsigned)v[1])};
}
__device__ __forceinline__ void st2(F2 v, __amdgpu_buffer_rsrc_t r, int vo, int so)
{
    u32x2 w;
    w.x = __builtin_bit_cast(unsigned, v.a);
    w.y = __builtin_bit_cast(unsigned, v.b);
    __builtin_amdgcn_raw_buffer_store_b64(w, r, vo, so, 0);
}

template <int TY, int D, bool BASE, bool NOISE>
__global__ __launch_bounds__(64) void march2_kernel(StepArgs<float> a)
{
    using T = float;
    constexpr int NR = TY + 4;
    const int lane = threadIdx.x;
    const int b = blockIdx.y;
    const int nx = a.nx, ny = a.ny;
    const int nstrip = a.tiles_x;

    const int nblk = a.tiles_x * a.tiles_y;
    const int bid = blockIdx.x;
    const int xcd = bid & 7, slot = bid >> 3;
    const int q8 = nblk >> 3, r8 = nblk & 7;
    const int tileid = xcd * q8 + (xcd < r8 ? xcd : r8) + slot;
    const int strip = tileid % nstrip;
    const int y0 = (tileid / nstrip) * TY;

    // nx is even, so the wrapped pair (gx, gx + 1) stays contiguous
    int gx = strip * kStripOut2 - 2 + 2 * lane;
    while (gx < 0) gx += nx;
    while (gx >= nx) gx -= nx;
    const int ocol = strip * kStripOut2 + 2 * lane - 2;  // output column of the pair's first cell
    const bool out_lane = lane >= 1 && lane < 1 + kStripOut2 / 2 && ocol < nx;

    const size_t plane = (size_t)nx * ny;
    const auto bc = plane_rsrc(a.c + (size_t)b * plane, plane);
    const auto bp = plane_rsrc(a.phi + (size_t)b * plane, plane);
    const auto br = plane_rsrc(a.rho + (size_t)b * plane, plane);
    const auto oc = plane_rsrc(a.c_out + (size_t)b * plane, plane);
    const auto op = plane_rsrc(a.phi_out + (size_t)b * plane, plane);
    const auto orr = plane_rsrc(a.rho_out + (size_t)b * plane, plane);
    const auto bcb = plane_rsrc((BASE ? a.cb : a.c) + (size_t)b * plane, plane);
    const auto bpb = plane_rsrc((BASE ? a.pb : a.phi) + (size_t)b * plane, plane);
    const auto brb = plane_rsrc((BASE ? a.rb : a.rho) + (size_t)b * plane, plane);
    const int vo = gx * (int)sizeof(T);
    const int row_bytes = nx * (int)sizeof(T);
    const Coef<T> k = a.k;
    const Real rl = a.real[b];
    const T vx2h = (T)rl.vx2h, vy2h = (T)rl.vy2h;
    const int pvd = a.pvd;

    F2 c[NR], p[NR], r[NR];
    F2 mc[NR], mp[NR], M[NR], pE[NR], pW[NR], FN[NR];
    const RhoCoef<T> rc = rho_coef(k, vx2h, vy2h);

    auto load_row = [&](int t) {
        const int gj = y0 - 2 + t;
        int jj;
        if (pvd) jj = gj < 0 ? -1 - gj : (gj >= ny ? 2 * ny - 1 - gj : gj);
        else jj = gj < 0 ? gj + ny : (gj >= ny ? gj - ny : gj);
        jj = jj < 0 ? 0 : (jj >= ny ? ny - 1 : jj);
        const int so = jj * row_bytes;
        c[t] = ld2(bc, vo, so);
        p[t] = ld2(bp, vo, so);
        const F2 rv = ld2(br, vo, so);
        const bool inlet = pvd && gj >= ny;
        r[t] = {inlet ? k.rho_in : rv.a, inlet ? k.rho_in : rv.b};
    };

#pragma unroll
    for (int t = 0; t < NR; ++t)
        if (t < 3 + D) load_row(t);

#pragma unroll
    for (int t1 = 1; t1 <= TY + 2; ++t1) {
        if (t1 + 2 + D < NR) load_row(t1 + 2 + D);
        // stage 1 at row t1: the first cell's west and the second cell's
        // east neighbours come from the adjacent lanes
        {
            const T cW = west(c[t1].b), cE = east(c[t1].a);
            const T pWv = west(p[t1].b), pEv = east(p[t1].a);
            pE[t1] = {p[t1].b, pEv};
            pW[t1] = {pWv, p[t1].a};
            potentials(k, c[t1].a, c[t1].b, cW, c[t1 + 1].a, c[t1 - 1].a, p[t1].a, pE[t1].a, pW[t1].a,
                       p[t1 + 1].a, p[t1 - 1].a, mc[t1].a, mp[t1].a, M[t1].a);
            potentials(k, c[t1].b, cE, c[t1].a, c[t1 + 1].b, c[t1 - 1].b, p[t1].b, pE[t1].b, pW[t1].b,
                       p[t1 + 1].b, p[t1 - 1].b, mc[t1].b, mp[t1].b, M[t1].b);
        }
        if (t1 >= 3) {
            const int t = t1 - 1;
            const int gj = y0 - 2 + t;
            const bool bottom = pvd && gj == 0;
            if (t == 2) {
                FN[1].a = cflux(M[1].a, mc[1].a, M[2].a, mc[2].a);
                FN[1].b = cflux(M[1].b, mc[1].b, M[2].b, mc[2].b);
            }
            const T FEa = cflux(M[t].a, mc[t].a, M[t].b, mc[t].b);
            const T FEb = cflux(M[t].b, mc[t].b, east(M[t].a), east(mc[t].a));
            const T FWa = west(FEb);
            FN[t].a = cflux(M[t].a, mc[t].a, M[t + 1].a, mc[t + 1].a);
            FN[t].b = cflux(M[t].b, mc[t].b, M[t + 1].b, mc[t + 1].b);
            const T rW = west(r[t].b), rE = east(r[t].a);
            const T qW = west(mp[t].b), qE = east(mp[t].a);
            F2 cb0 = c[t], pb0 = p[t], rb0 = r[t];
            if (BASE && gj < ny) {
                const int so = gj * row_bytes;
                cb0 = ld2(bcb, vo, so);
                pb0 = ld2(bpb, vo, so);
                rb0 = ld2(brb, vo, so);
            }
            F2 nc, np, nr;
            update(k, rc, vx2h, vy2h, bottom, c[t].a, p[t].a, pE[t].a, pW[t].a, p[t + 1].a, p[t - 1].a,
                   r[t].a, r[t].b, rW, r[t + 1].a, r[t - 1].a, FEa, FWa, FN[t].a, FN[t - 1].a,
                   mp[t].a, mp[t].b, qW, mp[t + 1].a, mp[t - 1].a, nc.a, np.a, nr.a, cb0.a, pb0.a, rb0.a);
            update(k, rc, vx2h, vy2h, bottom, c[t].b, p[t].b, pE[t].b, pW[t].b, p[t + 1].b, p[t - 1].b,
                   r[t].b, rE, r[t].a, r[t + 1].b, r[t - 1].b, FEb, FEa, FN[t].b, FN[t - 1].b,
                   mp[t].b, qE, mp[t].a, mp[t + 1].b, mp[t - 1].b, nc.b, np.b, nr.b, cb0.b, pb0.b, rb0.b);
            if (NOISE && gj < ny && out_lane) {
                const uint64_t id = (uint64_t)a.step * plane + (uint64_t)gj * nx + ocol;
                if (np.a < T(0)) nc.a = interface_draw<T>(rl.nseed, id * 16ull, rl.c0, a.noise);
                if (np.b < T(0)) nc.b = interface_draw<T>(rl.nseed, (id + 1ull) * 16ull, rl.c0, a.noise);
            }
            if (gj < ny) {
                if (out_lane) {
                    const int so = gj * row_bytes;
                    st2(nc, oc, vo, so);
                    st2(np, op, vo, so);
                    st2(nr, orr, vo, so);
                }
                if (a.Qcol && pvd && gj == ny - 1 && out_lane) {
                    double* q = a.Qcol + (size_t)b * nx + ocol;
                    const double rin = (double)k.rho_in;
                    const double ra = (double)r[t].a, rb = (double)r[t].b;
                    q[0] = q[0] + (rl.qa * (ra + rin) + rl.qb * (rin - ra));
                    q[1] = q[1] + (rl.qa * (rb + rin) + rl.qb * (rin - rb));
                }
            }
        }
    }
}

// Two fused steps per march (temporal blocking in registers): the strip is
// 64 lanes wide with a radius-4 halo, so it writes 56 columns (lanes 4..59),
// and a TY-row chunk reads TY + 8 rows.  Behind the front of loads the wave
// runs four stages per row, each lagging the previous: stage 1 and 2 of the
// first step (giving the intermediate state u1 in registers), then stage 1
// and 2 of the second step on u1.  The intermediate state obeys the same
// boundary rule as a stored state: in a substrate/inlet run the u1 rows
// beyond the substrate or the top take the mirrored interior u1 rows (and
// the inlet value for rho at the top) before the second step reads them; the
// chunk heights divide ny, so those rows sit at fixed chunk positions.  Each
// cell is evaluated by the same per-cell functions in the same order as in
// two single-step launches, so the result is bitwise identical.  MID also
// stores the intermediate state of the chunk's own rows (c_mid, phi_mid,
// rho_mid): two consecutive states from one launch.
constexpr int kStripOutK2 = 56;

template <typename T, int TY, int D, bool MID>
__global__ __launch_bounds__(64) void march_k2_kernel(StepArgs<T> a)
{
    constexpr int NR = TY + 8;
    const int lane = threadIdx.x;
    const int b = blockIdx.y;
    const int nx = a.nx, ny = a.ny;
    const int nstrip = a.tiles_x;

    const int nblk = a.tiles_x * a.tiles_y;
    const int bid = blockIdx.x;
    const int xcd = bid & 7, slot = bid >> 3;
    const int q8 = nblk >> 3, r8 = nblk & 7;
    const int tileid = xcd * q8 + (xcd < r8 ? xcd : r8) + slot;
    const int strip = tileid % nstrip;
    const int y0 = (tileid / nstrip) * TY;

    int gx = strip * kStripOutK2 - 4 + lane;
    while (gx < 0) gx += nx;
    while (gx >= nx) gx -= nx;
    const int ocol = strip * kStripOutK2 + lane - 4;
    const bool out_lane = lane >= 4 && lane < 4 + kStripOutK2 && ocol < nx;

    const size_t plane = (size_t)nx * ny;
    const auto bc = plane_rsrc(a.c + (size_t)b * plane, plane);
    const auto bp = plane_rsrc(a.phi + (size_t)b * plane, plane);
    const auto br = plane_rsrc(a.rho + (size_t)b * plane, plane);
    const auto oc = plane_rsrc(a.c_out + (size_t)b * plane, plane);
    const auto op = plane_rsrc(a.phi_out + (size_t)b * plane, plane);
    const auto orr = plane_rsrc(a.rho_out + (size_t)b * plane, plane);
    // intermediate-state outputs (MID only; otherwise unused)
    [[maybe_unused]] const auto mc_out = plane_rsrc((MID ? a.c_mid : a.c_out) + (size_t)b * plane, plane);
    [[maybe_unused]] const auto mp_out = plane_rsrc((MID ? a.phi_mid : a.phi_out) + (size_t)b * plane, plane);
    [[maybe_unused]] const auto mr_out = plane_rsrc((MID ? a.rho_mid : a.rho_out) + (size_t)b * plane, plane);
    const int vo = gx * (int)sizeof(T);
    const int row_bytes = nx * (int)sizeof(T);
    const Coef<T> k = a.k;
    const Real rl = a.real[b];
    const T vx2h = (T)rl.vx2h, vy2h = (T)rl.vy2h;
    const int pvd = a.pvd;
    const bool bot = pvd && y0 == 0;         // rows t < 4 are beyond the substrate
    const bool top = pvd && y0 + TY == ny;   // rows t >= TY + 4 are beyond the top

    // first step: input u0, stage-1 values, north fluxes
    T c[NR], p[NR], r[NR];
    T mc[NR], mp[NR], M[NR], pE[NR], pW[NR], FN[NR];
    // second step: the same on u1
    T c1[NR], p1[NR], r1[NR];
    T mc1[NR], mp1[NR], M1[NR], pE1[NR], pW1[NR], FN1[NR];
    const RhoCoef<T> rc = rho_coef(k, vx2h, vy2h);

    auto load_row = [&](int t) {
        const int gj = y0 - 4 + t;
        int jj;
        if (pvd) jj = gj < 0 ? -1 - gj : (gj >= ny ? 2 * ny - 1 - gj : gj);
        else jj = gj < 0 ? gj + ny : (gj >= ny ? gj - ny : gj);
        jj = jj < 0 ? 0 : (jj >= ny ? ny - 1 : jj);
        const int so = jj * row_bytes;
        c[t] = Buf<T>::ld(bc, vo, so);
        p[t] = Buf<T>::ld(bp, vo, so);
        const T rv = Buf<T>::ld(br, vo, so);
        r[t] = (pvd && gj >= ny) ? k.rho_in : rv;
    };
    auto inflow = [&](int gj, T rr) {
        // inflow through the top face in the sub-step that updates row gj
        if (a.Qcol && top && gj == ny - 1 && out_lane) {
            double* q = a.Qcol + (size_t)b * nx + ocol;
            const double rin = (double)k.rho_in, rd = (double)rr;
            *q = *q + (rl.qa * (rd + rin) + rl.qb * (rin - rd));
        }
    };

#pragma unroll
    for (int t = 0; t < NR; ++t)
        if (t < 3 + D) load_row(t);

#pragma unroll
    for (int f = 1; f <= NR; ++f) {
        if (f + 2 + D < NR) load_row(f + 2 + D);
        // step 1, stage 1 at row f
        if (f <= NR - 2) {
            const T cE = east(c[f]), cW = west(c[f]);
            pE[f] = east(p[f]);
            pW[f] = west(p[f]);
            potentials(k, c[f], cE, cW, c[f + 1], c[f - 1], p[f], pE[f], pW[f], p[f + 1], p[f - 1], mc[f], mp[f],
                       M[f]);
        }
        // step 1, stage 2 at row t = f - 1: u1
        if (f - 1 >= 2 && f - 1 <= NR - 3) {
            const int t = f - 1;
            const int gj = y0 - 4 + t;
            const bool bottom = pvd && gj == 0;
            if (t == 2) FN[1] = cflux(M[1], mc[1], M[2], mc[2]);
            const T FE = cflux(M[t], mc[t], east(M[t]), east(mc[t]));
            FN[t] = cflux(M[t], mc[t], M[t + 1], mc[t + 1]);
            update(k, rc, vx2h, vy2h, bottom, c[t], p[t], pE[t], pW[t], p[t + 1], p[t - 1], r[t], east(r[t]),
                   west(r[t]), r[t + 1], r[t - 1], FE, west(FE), FN[t], FN[t - 1], mp[t], east(mp[t]), west(mp[t]),
                   mp[t + 1], mp[t - 1], c1[t], p1[t], r1[t]);
            if (t >= 4 && t < TY + 4) inflow(gj, r[t]);
            if constexpr (MID) {
                if (t >= 4 && t < TY + 4 && out_lane) {
                    const int so = gj * row_bytes;
                    Buf<T>::st(c1[t], mc_out, vo, so);
                    Buf<T>::st(p1[t], mp_out, vo, so);
                    Buf<T>::st(r1[t], mr_out, vo, so);
                }
            }
            // the boundary rule on u1: at the top the rows beyond the grid
            // mirror rows already computed; at the substrate rows 2 and 3
            // mirror rows 5 and 4, complete once row 5 is
            if (t >= TY + 4 && top) {
                c1[t] = c1[2 * TY + 7 - t];
                p1[t] = p1[2 * TY + 7 - t];
                r1[t] = k.rho_in;
            }
            if (t == 5 && bot) {
                c1[3] = c1[4], p1[3] = p1[4], r1[3] = r1[4];
                c1[2] = c1[5], p1[2] = p1[5], r1[2] = r1[5];
            }
        }
        // step 2, stage 1 at row t2 = f - 4 (u1 rows t2 - 1 .. t2 + 1 are final)
        if (f - 4 >= 3 && f - 4 <= NR - 4) {
            const int t = f - 4;
            const T cE = east(c1[t]), cW = west(c1[t]);
            pE1[t] = east(p1[t]);
            pW1[t] = west(p1[t]);
            potentials(k, c1[t], cE, cW, c1[t + 1], c1[t - 1], p1[t], pE1[t], pW1[t], p1[t + 1], p1[t - 1],
                       mc1[t], mp1[t], M1[t]);
        }
        // step 2, stage 2 at row t3 = f - 5: the output row
        if (f - 5 >= 4 && f - 5 <= NR - 5) {
            const int t = f - 5;
            const int gj = y0 - 4 + t;
            const bool bottom = pvd && gj == 0;
            if (t == 4) FN1[3] = cflux(M1[3], mc1[3], M1[4], mc1[4]);
            const T FE = cflux(M1[t], mc1[t], east(M1[t]), east(mc1[t]));
            FN1[t] = cflux(M1[t], mc1[t], M1[t + 1], mc1[t + 1]);
            T nc, np, nr;
            update(k, rc, vx2h, vy2h, bottom, c1[t], p1[t], pE1[t], pW1[t], p1[t + 1], p1[t - 1], r1[t],
                   east(r1[t]), west(r1[t]), r1[t + 1], r1[t - 1], FE, west(FE), FN1[t], FN1[t - 1], mp1[t],
                   east(mp1[t]), west(mp1[t]), mp1[t + 1], mp1[t - 1], nc, np, nr);
            if (out_lane) {
                const int so = gj * row_bytes;
                Buf<T>::st(nc, oc, vo, so);
                Buf<T>::st(np, op, vo, so);
                Buf<T>::st(nr, orr, vo, so);
            }
            inflow(gj, r1[t]);
        }
    }
}

// rows of loads in flight ahead of use: short chunks issue all their loads
// at once, long chunks keep a window of rows in flight
template <int TY> constexpr int lookahead() { return TY <= 8 ? TY + 1 : 4; }

// the kernel instantiation for the arguments' variant
template <typename T, int TY>
void* march_fn(const StepArgs<T>& a)
{
    constexpr int D = lookahead<TY>();
    const bool base = a.cb != nullptr, noise = a.noise > 0;
    if (base && noise) return (void*)march_kernel<T, TY, D, true, true>;
    if (base) return (void*)march_kernel<T, TY, D, true, false>;
    if (noise) return (void*)march_kernel<T, TY, D, false, true>;
    return (void*)march_kernel<T, TY, D, false, false>;
}

template <int TY>
void* march2_fn(const StepArgs<float>& a)
{
    constexpr int D = lookahead<TY>();
    const bool base = a.cb != nullptr, noise = a.noise > 0;
    if (base && noise) return (void*)march2_kernel<TY, D, true, true>;
    if (base) return (void*)march2_kernel<TY, D, true, false>;
    if (noise) return (void*)march2_kernel<TY, D, false, true>;
    return (void*)march2_kernel<TY, D, false, false>;
}

// the launch's kernel and strip width: two columns per lane when asked for
// (FP32, even nx), else one
template <typename T, int TY>
void* pick_march(StepArgs<T>& a, int cols)
{
    if constexpr (sizeof(T) == 4) {
        if (cols == 2 && a.nx % 2 == 0) {
            a.tiles_x = (a.nx + kStripOut2 - 1) / kStripOut2;
            a.tiles_y = (a.ny + TY - 1) / TY;
            return march2_fn<TY>(a);
        }
    }
    a.tiles_x = (a.nx + kStripOut - 1) / kStripOut;
    a.tiles_y = (a.ny + TY - 1) / TY;
    return march_fn<T, TY>(a);
}

template <typename T, int TY>
hipError_t launch_march_ty(StepArgs<T> a, int cols, int batch, hipStream_t s)
{
    void* fn = pick_march<T, TY>(a, cols);
    dim3 grid(a.tiles_x * a.tiles_y, batch);
    void* args[] = {&a};
    return hipLaunchKernel(fn, grid, dim3(64), args, 0, s);
}

template <typename T, int TY>
hipError_t node_march_ty(hipGraph_t g, hipGraphNode_t* node, hipGraphNode_t dep, StepArgs<T> a, int cols,
                         int batch)
{
    void* fn = pick_march<T, TY>(a, cols);
    void* args[] = {&a};
    hipKernelNodeParams kp{};
    kp.func = fn;
    kp.gridDim = dim3(a.tiles_x * a.tiles_y, batch);
    kp.blockDim = dim3(64);
    kp.sharedMemBytes = 0;
    kp.kernelParams = args;
    kp.extra = nullptr;
    return hipGraphAddKernelNode(node, g, dep ? &dep : nullptr, dep ? 1 : 0, &kp);
}

}  // namespace

template <typename T, int TY>
hipError_t k2_node_or_launch(StepArgs<T> a, int batch, hipStream_t s, hipGraph_t g, hipGraphNode_t* node,
                             hipGraphNode_t dep)
{
    void* fn = a.c_mid ? (void*)march_k2_kernel<T, TY, lookahead<TY>(), true>
                       : (void*)march_k2_kernel<T, TY, lookahead<TY>(), false>;
    a.tiles_x = (a.nx + kStripOutK2 - 1) / kStripOutK2;
    a.tiles_y = a.ny / TY;
    void* args[] = {&a};
    if (!g) return hipLaunchKernel(fn, dim3(a.tiles_x * a.tiles_y, batch), dim3(64), args, 0, s);
    hipKernelNodeParams kp{};
    kp.func = fn;
    kp.gridDim = dim3(a.tiles_x * a.tiles_y, batch);
    kp.blockDim = dim3(64);
    kp.sharedMemBytes = 0;
    kp.kernelParams = args;
    kp.extra = nullptr;
    return hipGraphAddKernelNode(node, g, dep ? &dep : nullptr, dep ? 1 : 0, &kp);
}

template <typename T>
hipError_t k2_dispatch(const StepArgs<T>& a, int ty, int batch, hipStream_t s, hipGraph_t g, hipGraphNode_t* node,
                       hipGraphNode_t dep)
{
    if (ty <= 0 || a.ny % ty != 0 || a.ny < 4) return hipErrorInvalidValue;
    switch (ty) {
    case 4: return k2_node_or_launch<T, 4>(a, batch, s, g, node, dep);
    case 8: return k2_node_or_launch<T, 8>(a, batch, s, g, node, dep);
    case 16: return k2_node_or_launch<T, 16>(a, batch, s, g, node, dep);
    default: return hipErrorInvalidValue;
    }
}

template <typename T>
hipError_t launch_march(const StepArgs<T>& a, int ty, int cols, int batch, hipStream_t s)
{
    switch (ty) {
    case 4: return launch_march_ty<T, 4>(a, cols, batch, s);
    case 8: return launch_march_ty<T, 8>(a, cols, batch, s);
    case 16: return launch_march_ty<T, 16>(a, cols, batch, s);
    case 32: return launch_march_ty<T, 32>(a, cols, batch, s);
    default: return hipErrorInvalidValue;
    }
}
template hipError_t launch_march<float>(const StepArgs<float>&, int, int, int, hipStream_t);
template hipError_t launch_march<double>(const StepArgs<double>&, int, int, int, hipStream_t);

template <typename T>
hipError_t graph_add_march(hipGraph_t g, hipGraphNode_t* node, hipGraphNode_t dep, const StepArgs<T>& a,
                           int ty, int cols, int batch)
{
    switch (ty) {
    case 4: return node_march_ty<T, 4>(g, node, dep, a, cols, batch);
    case 8: return node_march_ty<T, 8>(g, node, dep, a, cols, batch);
    case 16: return node_march_ty<T, 16>(g, node, dep, a, cols, batch);
    case 32: return node_march_ty<T, 32>(g, node, dep, a, cols, batch);
    default: return hipErrorInvalidValue;
    }
}
template hipError_t graph_add_march<float>(hipGraph_t, hipGraphNode_t*, hipGraphNode_t, const StepArgs<float>&,
                                           int, int, int);
template hipError_t graph_add_march<double>(hipGraph_t, hipGraphNode_t*, hipGraphNode_t, const StepArgs<double>&,
                                            int, int, int);

template <typename T>
hipError_t launch_march_k2(const StepArgs<T>& a, int ty, int batch, hipStream_t s)
{
    return k2_dispatch<T>(a, ty, batch, s, nullptr, nullptr, nullptr);
}
template <typename T>
hipError_t graph_add_march_k2(hipGraph_t g, hipGraphNode_t* node, hipGraphNode_t dep, const StepArgs<T>& a, int ty,
                              int batch)
{
    return k2_dispatch<T>(a, ty, batch, nullptr, g, node, dep);
}
template hipError_t launch_march_k2<float>(const StepArgs<float>&, int, int, hipStream_t);
template hipError_t launch_march_k2<double>(const StepArgs<double>&, int, int, hipStream_t);
template hipError_t graph_add_march_k2<float>(hipGraph_t, hipGraphNode_t*, hipGraphNode_t, const StepArgs<float>&,
                                              int, int);
template hipError_t graph_add_march_k2<double>(hipGraph_t, hipGraphNode_t*, hipGraphNode_t,
                                               const StepArgs<double>&, int, int);

}  // namespace pfk
