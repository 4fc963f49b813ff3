// gfx950 resident stepper of the explicit PVD phase-field model (Materials
// and Methods, "Phase-field modeling of physical vapor deposition"; second-
// order central differences as stated in "Dataset"; explicit Euler in time).
//
// One launch advances FP32 grids of up to ~1M cells by n explicit
// Euler or midpoint steps with the state held on chip.  Each workgroup owns a 64 x TH tile (TH/4
// waves, 4 rows per wave, lanes = columns) and keeps the tile and a 2-cell
// halo of c, phi, rho in LDS for the whole launch; after every step it
// trades only the 2-cell rim of its tile with its neighbours:
//
//  * step: stage 1 (mu_c, mu_phi, M_c) on the tile plus one cell and stage 2
//    (the conserved updates, deposition source and vapour transport) on the
//    tile, out of LDS, with the same per-cell functions as every other
//    stepper kernel, so the states are bitwise identical to theirs.  A
//    midpoint step is two such passes: the half step u + dt/2 R(u), whose
//    rim is traded like a step's result while each cell keeps u in
//    registers, then u + dt R(u_half).  With interface draws on, the cells
//    that end a step on the vapour side then take their draw (FP32, keyed
//    by global step and cell as in every other stepper kernel);
//  * exchange: every rim cell of the new state is stored as one 8-byte word,
//    the FP32 value in the low half and a 32-bit generation tag in the high
//    half, into one of two rim buffers (by step parity) with device-coherent
//    stores (the first and last two rows straight from registers, the side
//    columns gathered from LDS so that lanes store consecutive words); a
//    neighbour polls the words its halo needs with device-coherent 8-byte
//    loads until each carries the generation it waits for.  Value and tag
//    travel in one single-copy-atomic word, so no flag, fence or grid barrier
//    is needed.  Two buffers suffice: a tile writes generation g + 2 over g
//    only after reading its neighbours' generation g + 1, which each
//    neighbour wrote after reading g;
//  * boundaries: x is periodic; in y the substrate and top ghosts are the
//    mirrored cells (held in the tile's own LDS or on a neighbour's rim) and
//    the vapour above the top is the inlet value; periodic y wraps.
//
// The state is read once at the start and written once at the end, in
// place: a tile writes its result only after generation 2, which it can
// compute only once every neighbour has finished its initial halo read, so
// launches need n >= 2.  Tags are the generation numbers plus an epoch in
// two disjoint spaces: the host's count of generations traded by the
// handle (top bit clear), passed with each launch, or, for a launch
// captured in a graph, whose arguments a replay repeats, a device epoch
// (top bit set) that the last workgroup to finish the launch (counted in a
// completion word) advances, after every workgroup has read it.  Either way
// a launch never meets a stale word carrying a tag it waits for.
//
// The launch is an ordinary dispatch of exactly as many workgroups as the
// device holds at once (checked on the host from the kernel's occupancy),
// on a device that runs nothing else meanwhile.  A wait longer than
// kSpinLimit polls (a grid that did not become co-resident) sets a sticky
// abort word: every tile then stops, writes NaN over its cells, workgroups
// that start later stop at once, and every wave ends; the handle's next
// diagnostic call reports the abort.
#include "pf_cell.h"

namespace pfk {
namespace {

using namespace cell;

constexpr int kTW = 64;                       // tile width: one lane per column
constexpr unsigned kSpinLimit = 1u << 18;     // polls before a wait gives up

template <int TH>
struct RGeo {
    static constexpr int R = 2;                         // halo and rim width
    static constexpr int NW = TH / 4;                   // waves, 4 rows each
    static constexpr int NT = 64 * NW;
    static constexpr int P = kTW + 2 * R;               // LDS row pitch: columns -R .. 63 + R
    static constexpr int LH = TH + 2 * R;               // LDS rows -R .. TH - 1 + R
    static constexpr int N = LH * P;
    static constexpr int RS = 2 * R * kTW + 2 * R * TH; // rim words per field
    static constexpr int NH = 2 * R * P + 2 * R * TH;   // halo cells
    static constexpr int QH = (NH + NT - 1) / NT;       // halo cells per thread
};

template <int N>
struct ResTile {
    float c[N], p[N], r[N], mc[N], mp[N], M[N];
};

// Word offset of rim cell (r, x) of a tile within one field: the first R
// rows, the last R rows, then the first and last R columns of every row
// (rows take precedence, so each rim cell has exactly one word).
template <int TH, int R>
__device__ __forceinline__ int rim_index(int r, int x)
{
    if (r < R) return r * kTW + x;
    if (r >= TH - R) return R * kTW + (r - (TH - R)) * kTW + x;
    if (x < R) return 2 * R * kTW + R * r + x;
    return 2 * R * kTW + R * TH + R * r + (x - (kTW - R));
}

__device__ __forceinline__ uint64_t pack(float v, uint32_t tag)
{
    return (uint64_t)__float_as_uint(v) | ((uint64_t)tag << 32);
}
__device__ __forceinline__ float value_of(uint64_t w) { return __uint_as_float((uint32_t)w); }
__device__ __forceinline__ uint32_t tag_of(uint64_t w) { return (uint32_t)(w >> 32); }

__device__ __forceinline__ void put(uint64_t* p, uint64_t w)
{
    __hip_atomic_store(p, w, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ uint64_t get(const uint64_t* p)
{
    return __hip_atomic_load(const_cast<uint64_t*>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Cells of the ring of width m around the tile (rows -m..-1 and TH..TH-1+m
// over columns -m..63+m, then columns -m..-1 and 64..63+m of rows 0..TH-1).
template <int TH>
__device__ __forceinline__ void ring_cell(int h, int m, int& r, int& x)
{
    const int W = kTW + 2 * m;
    if (h < 2 * m * W) {
        const int rr = h / W;
        r = rr < m ? rr - m : TH + (rr - m);
        x = -m + h % W;
    } else {
        const int s = h - 2 * m * W, k = s % (2 * m);
        r = s / (2 * m);
        x = k < m ? k - m : kTW + (k - m);
    }
}

// Source of halo cell h (ring of width R) of tile (b, tx, ty): *dst its LDS
// index; *src >= 0 the rim word of field 0, parity 0, of the tile holding the
// mirrored or wrapped cell, < 0: -1 - the cell's index in this tile's LDS;
// *above: rho is the inlet value; *nor: outer ring, whose rho no stage reads.
template <int TH>
__device__ __forceinline__ void halo_source(int h, int b, int tx, int ty, int ntx, int nty, int nx, int ny, bool pvd,
                                            int& dst, int& src, bool& above, bool& nor)
{
    using G = RGeo<TH>;
    constexpr int R = G::R, P = G::P;
    int r, x;
    ring_cell<TH>(h, R, r, x);
    dst = (r + R) * P + x + R;
    nor = r == -R || r == TH - 1 + R || x == -R || x == kTW - 1 + R;
    above = false;
    int gi = tx * kTW + x;
    gi = gi < 0 ? gi + nx : (gi >= nx ? gi - nx : gi);
    int gj = ty * TH + r;
    if (pvd) {
        if (gj < 0) {
            gj = -1 - gj;
        } else if (gj >= ny) {
            gj = 2 * ny - 1 - gj;
            above = true;
        }
    } else {
        gj = gj < 0 ? gj + ny : (gj >= ny ? gj - ny : gj);
    }
    const int stx = gi / kTW, sty = gj / TH;
    const int lr = gj - sty * TH, lx = gi - stx * kTW;
    if (stx == tx && sty == ty) src = -1 - ((lr + R) * P + lx + R);
    else src = ((b * nty + sty) * ntx + stx) * 3 * G::RS + rim_index<TH, R>(lr, lx);
}

template <int TH>
struct Resident {
    using G = RGeo<TH>;
    static constexpr int NT = G::NT, P = G::P, R = G::R, RS = G::RS;
    using Tl = ResTile<G::N>;

    const StepArgs<float>& a;
    Tl& t;
    int tid, lane, wv, rb, b, tx, ty, nty, x0, y0;
    bool pvd, qrow;
    float vx2h, vy2h, rin;
    double qa, qb, qacc;
    RhoCoef<float> rc;
    float nc[4], np[4], nr[4];   // the wave's 4 rows after the step (or half step)
    float ubc[4], ubp[4], ubr[4];   // midpoint: the state at the start of the step
    uint64_t nseed;                 // interface draws: the realisation's stream,
    float c0, sigma;                // mean and standard deviation

    __device__ __forceinline__ static int L(int r, int x) { return (r + R) * P + x + R; }

    // The thread index through an empty asm: indexing derived from it is
    // recomputed where it is used instead of being computed ahead of the
    // step loop and held in registers (or spilled) through the stages.
    __device__ __forceinline__ int otid() const
    {
        int x = tid;
        asm volatile("" : "+v"(x));
        return x;
    }

    __device__ __forceinline__ void pot_cell(const Coef<float>& k, int l)
    {
        float mc, mp, M;
        potentials(k, t.c[l], t.c[l + 1], t.c[l - 1], t.c[l + P], t.c[l - P], t.p[l], t.p[l + 1], t.p[l - 1],
                   t.p[l + P], t.p[l - P], mc, mp, M);
        t.mc[l] = mc;
        t.mp[l] = mp;
        t.M[l] = M;
    }

    // stage 1 on the tile plus one cell
    __device__ __forceinline__ void stage1(const Coef<float>& k)
    {
        constexpr int m = 1;
        int l = L(rb, lane);
        float cS = t.c[l - P], cC = t.c[l], pS = t.p[l - P], pC = t.p[l];
#pragma unroll
        for (int i = 0; i < 4; ++i, l += P) {
            const float cN = t.c[l + P], pN = t.p[l + P];
            float mc, mp, M;
            potentials(k, cC, t.c[l + 1], t.c[l - 1], cN, cS, pC, t.p[l + 1], t.p[l - 1], pN, pS, mc, mp, M);
            t.mc[l] = mc;
            t.mp[l] = mp;
            t.M[l] = M;
            cS = cC;
            cC = cN;
            pS = pC;
            pC = pN;
        }
        constexpr int NM = 2 * m * (kTW + 2 * m) + 2 * m * TH;
        for (int h = NT - 1 - otid(); h < NM; h += NT) {
            int r, x;
            ring_cell<TH>(h, m, r, x);
            pot_cell(k, L(r, x));
        }
    }

    // stage 2 on the tile: its updates into nc/np/nr.  MODE 0: explicit
    // Euler; 1: the midpoint method's half step (the cell's own state kept
    // in ubc/ubp/ubr as the step's base, no inflow); 2: its full step on the
    // half-step state, added to that base
    template <int MODE>
    __device__ __forceinline__ void stage2(const Coef<float>& k)
    {
        int l = L(rb, lane);
        float pS = t.p[l - P], pC = t.p[l], rS = t.r[l - P], rC = t.r[l];
        float MS = t.M[l - P], MC = t.M[l], mS = t.mc[l - P], mC = t.mc[l];
        float qS = t.mp[l - P], qC = t.mp[l];
#pragma unroll
        for (int i = 0; i < 4; ++i, l += P) {
            const float pN = t.p[l + P], rN = t.r[l + P], MN = t.M[l + P], mN = t.mc[l + P], qN = t.mp[l + P];
            const bool bottom = pvd && y0 + rb + i == 0;
            const float c0 = t.c[l];
            if constexpr (MODE == 1) {
                ubc[i] = c0;
                ubp[i] = pC;
                ubr[i] = rC;
            }
            update(k, rc, vx2h, vy2h, bottom, c0, pC, t.p[l + 1], t.p[l - 1], pN, pS, rC, t.r[l + 1], t.r[l - 1], rN,
                   rS, cflux(MC, mC, t.M[l + 1], t.mc[l + 1]), cflux(t.M[l - 1], t.mc[l - 1], MC, mC),
                   cflux(MC, mC, MN, mN), cflux(MS, mS, MC, mC), qC, t.mp[l + 1], t.mp[l - 1], qN, qS, nc[i], np[i],
                   nr[i], MODE == 2 ? ubc[i] : c0, MODE == 2 ? ubp[i] : pC, MODE == 2 ? ubr[i] : rC);
            if (MODE != 1 && qrow && i == 3) {
                const double rind = (double)rin, rr = (double)rC;
                qacc += qa * (rr + rind) + qb * (rind - rr);
            }
            pS = pC;
            pC = pN;
            rS = rC;
            rC = rN;
            MS = MC;
            MC = MN;
            mS = mC;
            mC = mN;
            qS = qC;
            qC = qN;
        }
    }

    // interface draws after global step `step`: the wave's cells that end
    // the step on the vapour side take a fresh composition.  The first
    // attempts of two cells at a time are straight-line code (independent
    // work to interleave); the rare rejected ones continue from attempt 1.
    __device__ __forceinline__ void draw(long long step)
    {
        const int xt = otid(), xlane = xt & 63, xrb = 4 * (xt >> 6);
        const uint64_t id = (uint64_t)step * ((uint64_t)a.nx * a.ny) + (uint64_t)(y0 + xrb) * a.nx + x0 + xlane;
#pragma unroll
        for (int i = 0; i < 4; i += 2) {
            const uint64_t k0 = (id + (uint64_t)i * a.nx) * 16ull, k1 = k0 + 16ull * a.nx;
            float x0v, x1v;
            const bool ok0 = gauss_attempt_f32(nseed, k0, 0, c0, sigma, &x0v);
            const bool ok1 = gauss_attempt_f32(nseed, k1, 0, c0, sigma, &x1v);
            if (np[i] < 0.f) nc[i] = ok0 ? x0v : trunc_gauss_f32_from(nseed, k0, 1, c0, sigma);
            if (np[i + 1] < 0.f) nc[i + 1] = ok1 ? x1v : trunc_gauss_f32_from(nseed, k1, 1, c0, sigma);
        }
    }

    // the tile's cells of the final state and the inflow accumulators; the
    // state goes out with device-coherent (write-through) stores, so little
    // of it is left dirty in the L2 caches when the launch ends (measured:
    // 1-2 % per call)
    __device__ __forceinline__ void write_result()
    {
        const int xt = otid(), xlane = xt & 63, xrb = 4 * (xt >> 6);
        const size_t plane = (size_t)a.nx * a.ny, base = (size_t)b * plane;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const size_t g = base + (size_t)(y0 + xrb + i) * a.nx + x0 + xlane;
            __hip_atomic_store(a.c_out + g, nc[i], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __hip_atomic_store(a.phi_out + g, np[i], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __hip_atomic_store(a.rho_out + g, nr[i], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
        if (qrow) a.Qcol[(size_t)b * a.nx + x0 + xlane] = qacc;
    }

    __device__ __forceinline__ void write_tile()
    {
        int l = L(rb, lane);
#pragma unroll
        for (int i = 0; i < 4; ++i, l += P) {
            t.c[l] = nc[i];
            t.p[l] = np[i];
            t.r[l] = nr[i];
        }
    }
};

// At most 128 VGPRs (four waves per SIMD), so that 1024^2 (512 tiles of
// 64 x 32) stays resident at two workgroups per CU.  MID: the midpoint
// method; NZ: interface draws after every step.
template <int TH, bool MID, bool NZ>
__global__ __launch_bounds__(16 * TH) __attribute__((amdgpu_waves_per_eu(4)))
void resident_kernel(ResArgs ra)
{
    using G = RGeo<TH>;
    using St = Resident<TH>;
    constexpr int NT = G::NT, P = G::P, R = G::R, RS = G::RS, QH = G::QH;
    static_assert(NT == 16 * TH, "launch bounds");
    __shared__ typename St::Tl t;
    __shared__ int s_stop;
    __shared__ uint32_t s_e0;

    const StepArgs<float>& a = ra.s;
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    // The dispatcher hands workgroup w to XCD w mod 8; tile (w mod 8)
    // (tiles / 8) + w / 8 gives each XCD a contiguous block of tiles (four
    // tile rows at 1024^2), so most neighbours share an XCD and its L2.
    // Measured at 1024^2: 4.3-4.5 us per step against 4.8-4.9 with tiles in
    // workgroup order (any bijection gives the same results).
    const int tile = gridDim.x % 8 ? (int)blockIdx.x : (int)((blockIdx.x % 8) * (gridDim.x / 8) + blockIdx.x / 8);
    const int per = ra.ntx * ra.nty;
    const int b = tile / per, tr = tile % per;
    const int ty = tr / ra.ntx, tx = tr % ra.ntx;
    const int x0 = tx * kTW, y0 = ty * TH;
    const int nx = a.nx, ny = a.ny;
    const size_t plane = (size_t)nx * ny;
    const float rin = a.k.rho_in;
    const bool pvd = a.pvd != 0;

    // ---- initial state: tile and halo, x wrapped, y mirrored (inlet rho
    // above the top) or wrapped
    // (every load of the thread is issued before the first LDS store, so
    // the tile costs about one memory latency)
    {
        const float* gc = a.c + (size_t)b * plane;
        const float* gp = a.phi + (size_t)b * plane;
        const float* gr = a.rho + (size_t)b * plane;
        constexpr int QL = (G::N + NT - 1) / NT;
        float vc[QL], vp[QL], vr[QL];
#pragma unroll
        for (int q = 0; q < QL; ++q) {
            const int i = tid + q * NT;
            if (i >= G::N) continue;
            const int r = i / P - R, x = i % P - R;
            int gi = x0 + x;
            gi = gi < 0 ? gi + nx : (gi >= nx ? gi - nx : gi);
            int gj = y0 + r;
            bool above = false;
            if (pvd) {
                if (gj < 0) {
                    gj = -1 - gj;
                } else if (gj >= ny) {
                    gj = 2 * ny - 1 - gj;
                    above = true;
                }
            } else {
                gj = gj < 0 ? gj + ny : (gj >= ny ? gj - ny : gj);
            }
            const size_t g = (size_t)gj * nx + gi;
            vc[q] = gc[g];
            vp[q] = gp[g];
            vr[q] = above ? rin : gr[g];
        }
#pragma unroll
        for (int q = 0; q < QL; ++q) {
            const int i = tid + q * NT;
            if (i >= G::N) continue;
            t.c[i] = vc[q];
            t.p[i] = vp[q];
            t.r[i] = vr[q];
        }
    }
    // the epoch and the abort word, read once per workgroup (thread 0's
    // read precedes its completion count at the end of the launch)
    if (tid == 0) {
        s_stop = get(ra.ctl + 1) != 0;
        s_e0 = ra.dev_epoch ? 0x80000000u | ((uint32_t)get(ra.ctl) & 0x3FFFFFFFu) : ra.e0;
    }

    const Real rl = a.real[b];
    St st{a, t, tid, lane, wv, 4 * wv, b, tx, ty, ra.nty, x0, y0, pvd, false, (float)rl.vx2h, (float)rl.vy2h, rin,
          rl.qa, rl.qb, 0.0, rho_coef(a.k, (float)rl.vx2h, (float)rl.vy2h), {}, {}, {}, {}, {}, {},
          rl.nseed, (float)rl.c0, (float)a.noise};
    // inflow through the top face: the last wave of a top tile holds row ny-1
    st.qrow = pvd && a.Qcol && ty == ra.nty - 1 && wv == G::NW - 1;
    if (st.qrow) st.qacc = a.Qcol[(size_t)b * nx + x0 + lane];
    const size_t par_stride = (size_t)gridDim.x * 3 * RS;
    uint64_t* const own_rim = ra.rim + (size_t)tile * 3 * RS;


    // rim generations: one per step; with the midpoint method two, the odd
    // ones holding the half-step state u_half = u + dt/2 R(u) (the step's
    // base u stays in registers) and the even ones u' = u + dt R(u_half)
    const int last = MID ? 2 * ra.n : ra.n;
    __syncthreads();
    const uint32_t e0 = s_e0;
    bool stop = s_stop != 0;
    int g = 0;
    while (!stop) {
        if constexpr (MID) {
            if ((g & 1) == 0) {
                st.stage1(ra.kh);
                __syncthreads();
                st.template stage2<1>(ra.kh);
            } else {
                st.stage1(a.k);
                __syncthreads();
                st.template stage2<2>(a.k);
                if constexpr (NZ) st.draw(a.step + g / 2);
            }
        } else {
            st.stage1(a.k);
            __syncthreads();
            st.template stage2<0>(a.k);
            if constexpr (NZ) st.draw(a.step + g);
        }
        ++g;
        if (g == last) {
            st.write_result();
            break;
        }
        // ---- publish the rim of generation g: the first and last two rows
        // straight from registers (whole rows: full cache lines); the
        // exchange's indexing is recomputed every step (st.otid)
        const int xt = st.otid(), xlane = xt & 63, xrb = 4 * (xt >> 6);
        const uint32_t tag = e0 + (uint32_t)g;
        const size_t poff = (size_t)(g & 1) * par_stride;
        uint64_t* const rim = own_rim + poff;
        if (wv == 0 || wv == G::NW - 1) {
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int r = xrb + i;
                if (r < R || r >= TH - R) {
                    const int k = rim_index<TH, R>(r, xlane);
                    put(rim + k, pack(st.nc[i], tag));
                    put(rim + RS + k, pack(st.np[i], tag));
                    put(rim + 2 * RS + k, pack(st.nr[i], tag));
                }
            }
        }
        __syncthreads();   // every stage-2 read of the old state is done
        st.write_tile();
        __syncthreads();
        // the first and last R columns of every row, gathered from LDS so
        // that consecutive lanes store consecutive words
        for (int j = xt; j < 6 * R * TH; j += NT) {
            const int f = j / (2 * R * TH), rem = j % (2 * R * TH), side = rem / (R * TH), idx = rem % (R * TH);
            const int l = St::L(idx / R, idx % R + (side ? kTW - R : 0));
            const float v = f == 0 ? t.c[l] : (f == 1 ? t.p[l] : t.r[l]);
            put(rim + f * RS + 2 * R * kTW + side * R * TH + idx, pack(v, tag));
        }

        // ---- halo of generation g: own mirror cells from LDS, the rest from
        // the neighbours' rims
        int hdst[QH], hsrc[QH];
        bool habove[QH], hnor[QH];
        uint64_t wc[QH], wp[QH], wr[QH];
#pragma unroll
        for (int q = 0; q < QH; ++q) {
            wc[q] = wp[q] = wr[q] = (uint64_t)tag << 32;
            hdst[q] = -1;
            hsrc[q] = 0;
            habove[q] = false;
            hnor[q] = true;
            const int h = xt + q * NT;
            if (h >= G::NH) continue;
            halo_source<TH>(h, b, tx, ty, ra.ntx, ra.nty, nx, ny, pvd, hdst[q], hsrc[q], habove[q], hnor[q]);
            if (hsrc[q] >= 0) {
                const uint64_t* src = ra.rim + poff + hsrc[q];
                wc[q] = get(src);
                wp[q] = get(src + RS);
                if (!habove[q] && !hnor[q]) wr[q] = get(src + 2 * RS);
            } else {
                const int s = -1 - hsrc[q], d = hdst[q];
                t.c[d] = t.c[s];
                t.p[d] = t.p[s];
                if (!hnor[q]) t.r[d] = habove[q] ? rin : t.r[s];
            }
        }
        bool ok = true;
        for (unsigned it = 0;; ++it) {
            ok = true;
#pragma unroll
            for (int q = 0; q < QH; ++q)
                ok = ok && tag_of(wc[q]) == tag && tag_of(wp[q]) == tag && tag_of(wr[q]) == tag;
            if (ok || it >= kSpinLimit) break;
            if ((it & 255) == 255 && get(ra.ctl + 1) != 0) break;
            __builtin_amdgcn_s_sleep(1);
#pragma unroll
            for (int q = 0; q < QH; ++q) {
                if (hdst[q] < 0 || hsrc[q] < 0) continue;
                const uint64_t* src = ra.rim + poff + hsrc[q];
                if (tag_of(wc[q]) != tag) wc[q] = get(src);
                if (tag_of(wp[q]) != tag) wp[q] = get(src + RS);
                if (tag_of(wr[q]) != tag) wr[q] = get(src + 2 * RS);
            }
        }
        if (!ok) {
            s_stop = 1;
            put(ra.ctl + 1, 1);
        }
#pragma unroll
        for (int q = 0; q < QH; ++q) {
            if (hdst[q] < 0 || hsrc[q] < 0) continue;
            const int d = hdst[q];
            t.c[d] = value_of(wc[q]);
            t.p[d] = value_of(wp[q]);
            if (!hnor[q]) t.r[d] = habove[q] ? rin : value_of(wr[q]);
        }
        __syncthreads();
        stop = s_stop != 0;
    }

    // ---- after an abandoned wait: NaN over the tile
    if (stop) {
#pragma unroll
        for (int i = 0; i < 4; ++i) st.nc[i] = st.np[i] = st.nr[i] = __builtin_nanf("");
        st.write_result();
    }

    // ---- device epoch (captured launches): the last workgroup of the
    // launch advances the epoch by the generations it used (e0 + 1 .. e0 +
    // last) and rearms the count.  Every workgroup read the epoch before its
    // own count (acquire-release on the count orders those reads before the
    // update).
    if (ra.dev_epoch && tid == 0) {
        const uint64_t done = __hip_atomic_fetch_add(ra.ctl + 2, 1ull, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
        if (done + 1 == (uint64_t)gridDim.x) {
            __hip_atomic_store(ra.ctl + 2, 0ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __hip_atomic_fetch_add(ra.ctl, (uint64_t)last, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
    }
}

template <int TH, bool MID, bool NZ>
hipError_t launch_th(const ResArgs& ra, hipStream_t s)
{
    const int ntiles = ra.batch * ra.ntx * ra.nty;
    hipLaunchKernelGGL((resident_kernel<TH, MID, NZ>), dim3(ntiles), dim3(RGeo<TH>::NT), 0, s, ra);
    return hipGetLastError();
}

template <int TH, bool MID, bool NZ>
int blocks_per_cu()
{
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, resident_kernel<TH, MID, NZ>, RGeo<TH>::NT, 0) != hipSuccess)
        return 0;
    return nb;
}

// co-resident tiles of every instantiation at this height
template <int TH>
int capacity_th()
{
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
    int nb = blocks_per_cu<TH, false, false>();
    for (int v : {blocks_per_cu<TH, true, false>(), blocks_per_cu<TH, false, true>(), blocks_per_cu<TH, true, true>()})
        nb = v < nb ? v : nb;
    return nb * cus;
}

template <int TH>
hipError_t launch_h(const ResArgs& ra, hipStream_t s)
{
    const bool nz = ra.s.noise > 0;
    if (ra.mid) return nz ? launch_th<TH, true, true>(ra, s) : launch_th<TH, true, false>(ra, s);
    return nz ? launch_th<TH, false, true>(ra, s) : launch_th<TH, false, false>(ra, s);
}

}  // namespace

size_t resident_rim_words(int th)
{
    return (size_t)(4 * kTW + 4 * th);
}

int resident_capacity(int th)
{
    switch (th) {
    case 8: return capacity_th<8>();
    case 16: return capacity_th<16>();
    case 32: return capacity_th<32>();
    default: return 0;
    }
}

hipError_t launch_resident(const ResArgs& ra, int th, hipStream_t s)
{
    if (ra.n < 2 || ra.s.nx % kTW || ra.ntx * kTW != ra.s.nx || ra.nty * th != ra.s.ny || ra.s.ny < th ||
        (ra.mid ? 2 : 1) * (long)ra.n >= (1L << 31))
        return hipErrorInvalidValue;
    switch (th) {
    case 8: return launch_h<8>(ra, s);
    case 16: return launch_h<16>(ra, s);
    case 32: return launch_h<32>(ra, s);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace pfk
