// C-ABI host code of the MI355X phase-field stepper (declared in pf.h).
//
// Validation happens before anything is enqueued.  The library never
// allocates device memory: the state lives in the caller's buffers and the
// ping-pong copy, inflow accumulators and reduction partials live in the
// caller's workspace.
#include "../../include/pf.h"
#include "pf_kernels.h"

#include <algorithm>
#include <utility>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <mutex>
#include <new>
#include <vector>

namespace {

constexpr size_t kAlign = 256;
constexpr int kGraphLen = 64;   // launches per graph replay (even: parity is preserved)
constexpr long kResAutoMin = 1L << 18;   // resident stepper by default from this many cells

size_t round_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

struct Layout {
    size_t state[3];
    size_t qcol, real, c0, qstage, partials, results, rim, rctl, total;
};

constexpr long kResMaxCells = 1L << 21;   // resident stepper: cells per launch at most

// Tile height of the resident stepper for *p, 0 where it does not run: FP32
// explicit Euler or midpoint, with or without interface draws, asked for or
// left to the library
// (temporal_block 0) from 2^18 cells (measured on MI355X: 512^2 79.9 GLUPS
// against 72.1 for the two-step march, 1024^2 218 against 156 for the LDS
// tile, 4 x 512^2 238 against 154; 256^2 16 against 25), 64-column tiles, a
// height dividing ny: the one asked for, else the largest of 32, 16, 8
// (512^2: 79.9 GLUPS with 32 rows, 73.8 with 16).  Whether the device keeps
// every tile resident is checked when the handle is created.
int resident_th(const pf_params* p)
{
    if (p->precision != PF_F32) return 0;
    if (p->integrator != PF_EULER && p->integrator != PF_MIDPOINT) return 0;
    const long cells = (long)p->nx * p->ny * p->batch;
    if (p->nx % 64 || cells > kResMaxCells) return 0;
    if (p->fused_kernel == PF_FUSED_AUTO) {
        if (p->temporal_block != 0 || cells < kResAutoMin) return 0;
    } else if (p->fused_kernel != PF_FUSED_RESIDENT || p->temporal_block > 1) {
        return 0;
    }
    if (p->tile_rows != 0) {
        // a chunk height asked for: the resident stepper only on request, at
        // a tile height it has
        const bool has = p->tile_rows == 8 || p->tile_rows == 16 || p->tile_rows == 32;
        return p->fused_kernel == PF_FUSED_RESIDENT && has && p->ny % p->tile_rows == 0 ? p->tile_rows : 0;
    }
    for (int t : {32, 16, 8})
        if (p->ny % t == 0) return t;
    return 0;
}

size_t esize(const pf_params* p) { return p->precision == PF_F64 ? 8 : 4; }

Layout layout(const pf_params* p)
{
    Layout L{};
    const size_t B = (size_t)p->batch, cells = (size_t)p->nx * (size_t)p->ny;
    size_t off = 0;
    auto take = [&](size_t bytes) {
        const size_t o = off;
        off += round_up(bytes);
        return o;
    };
    for (int f = 0; f < 3; ++f) L.state[f] = take(B * cells * esize(p));
    L.qcol = take(B * (size_t)p->nx * sizeof(double));
    L.real = take(B * sizeof(pfk::Real));
    L.c0 = take(B * sizeof(double));
    L.qstage = take(B * sizeof(double));
    L.partials = take(B * (size_t)pfk::reduce_geometry(p->nx, p->ny, p->batch, (int)esize(p)).parts() * 4 *
                      sizeof(double));
    L.results = take(B * 5 * sizeof(double));
    const int th = resident_th(p);
    const size_t tiles = th ? B * (size_t)(p->nx / 64) * (size_t)(p->ny / th) : 0;
    L.rim = take(th ? 2 * tiles * 3 * pfk::resident_rim_words(th) * sizeof(uint64_t) : 0);
    L.rctl = take(th ? 3 * sizeof(uint64_t) : 0);   // epoch, abort, completion count
    L.total = off;
    return L;
}

bool finite_all(std::initializer_list<double> v)
{
    for (double x : v)
        if (!std::isfinite(x)) return false;
    return true;
}

int validate(const pf_params* p)
{
    if (!p) return PF_EINVAL;
    if (p->nx < 1 || p->ny < 1 || p->batch < 1 || p->batch > 65535) return PF_EINVAL;

    if (p->precision != PF_F32 && p->precision != PF_F64) return PF_EINVAL;
    // one realisation's field must stay below 2 GiB (32-bit buffer offsets)
    if ((int64_t)p->nx * p->ny * (p->precision == PF_F64 ? 8 : 4) >= ((int64_t)1 << 31)) return PF_EINVAL;
    if (p->bc_mode != PF_BC_PVD && p->bc_mode != PF_BC_PERIODIC) return PF_EINVAL;
    if (p->init_mode != PF_INIT_SEEDED && p->init_mode != PF_INIT_KEEP) return PF_EINVAL;
    if (p->temporal_block < 0 || p->temporal_block > (p->precision == PF_F64 ? 2 : 4)) return PF_EINVAL;
    if (p->graph_mode < 0 || p->graph_mode > 1) return PF_EINVAL;
    if (p->tile_rows != 0 && p->tile_rows != 4 && p->tile_rows != 8 && p->tile_rows != 16 && p->tile_rows != 32)
        return PF_EINVAL;
    if (p->integrator != PF_EULER && p->integrator != PF_MIDPOINT) return PF_EINVAL;
    if (p->lane_cols < 0 || p->lane_cols > 2) return PF_EINVAL;
    if (p->fused_kernel < 0 || p->fused_kernel > PF_FUSED_RESIDENT) return PF_EINVAL;
    // the register strip march fuses exactly two steps
    if (p->fused_kernel == PF_FUSED_MARCH && p->temporal_block > 2) return PF_EINVAL;
    if (!std::isfinite(p->interface_noise) || p->interface_noise < 0 || p->interface_noise > 1) return PF_EINVAL;
    if (p->fused_kernel == PF_FUSED_RESIDENT && resident_th(p) == 0) return PF_EINVAL;
    // the variants run on the single-step kernel
    if ((p->integrator != PF_EULER || p->interface_noise > 0) && p->temporal_block > 1) return PF_EINVAL;
    if (!finite_all({p->h, p->dt, p->dt_factor, p->W_c, p->W_phi, p->kappa_c, p->kappa_phi, p->MA_bulk,
                     p->MB_bulk, p->MA_surf, p->MB_surf, p->sigma_surf, p->M_phi, p->M_scale, p->D_rho,
                     p->v0, p->theta_deg, p->rho_in, p->c0, p->c_noise, p->film_h}))
        return PF_EINVAL;
    if (!(p->h > 0) || !(p->sigma_surf > 0)) return PF_EINVAL;
    if (p->MA_bulk < 0 || p->MB_bulk < 0 || p->MA_surf < 0 || p->MB_surf < 0 || p->M_phi < 0 ||
        p->M_scale < 0 || p->D_rho < 0 || p->kappa_c < 0 || p->kappa_phi < 0)
        return PF_EINVAL;
    if (p->dt <= 0 && !(p->dt_factor > 0)) return PF_EINVAL;
    if (p->init_mode == PF_INIT_SEEDED && !(p->W_phi > 0)) return PF_EINVAL;
    for (int b = 0; b < p->batch; ++b) {
        if (p->v0_per && !std::isfinite(p->v0_per[b])) return PF_EINVAL;
        if (p->c0_per && !std::isfinite(p->c0_per[b])) return PF_EINVAL;
    }
    return PF_OK;
}

double v0_of(const pf_params* p, int b) { return p->v0_per ? p->v0_per[b] : p->v0; }
double c0_of(const pf_params* p, int b) { return p->c0_per ? p->c0_per[b] : p->c0; }

// Frozen-coefficient von Neumann bound of explicit Euler with the 5-point
// operators (symbol at most 8/h^2), taken term by term.
double stability_limit(const pf_params* p)
{
    const double h2 = p->h * p->h, h4 = h2 * h2;
    double lim = INFINITY;
    const double mmax = p->M_scale * (std::max(p->MA_bulk, p->MB_bulk) + std::max(p->MA_surf, p->MB_surf));
    if (mmax > 0) lim = std::min(lim, 2.0 * h4 / (8.0 * mmax * (2.0 * p->W_c * h2 + 8.0 * p->kappa_c)));
    if (p->M_phi > 0)
        lim = std::min(lim, 2.0 * h4 / (8.0 * p->M_phi * ((2.0 * p->W_phi + 3.0 * p->W_c / 32.0) * h2 + 8.0 * p->kappa_phi)));
    if (p->D_rho > 0) lim = std::min(lim, h2 / (4.0 * p->D_rho));
    if (p->flux_on) {
        double vmax = 0;
        for (int b = 0; b < p->batch; ++b) vmax = std::max(vmax, std::fabs(v0_of(p, b)));
        if (vmax > 0) lim = std::min(lim, p->D_rho > 0 ? 2.0 * p->D_rho / (vmax * vmax) : p->h / vmax);
    }
    return lim;
}

bool aligned(const void* ptr, size_t a) { return ((uintptr_t)ptr % a) == 0; }

}  // namespace

struct pf_handle {
    pf_params p{};
    Layout L{};
    void* f[3] = {nullptr, nullptr, nullptr};   // caller's c, phi, rho
    void* w[3] = {nullptr, nullptr, nullptr};   // workspace copies
    char* ws = nullptr;
    hipStream_t stream = nullptr;
    double dt = 0;
    int64_t step = 0;
    int K = 1;
    int march_ty = 16;                   // K == 1: rows per wave of the strip-march kernel
    int march_cols = 1;                  // K == 1: grid columns per lane (2: FP32, even nx)
    int fused = PF_FUSED_TILE;           // K >= 2: LDS tile or register strip march (K == 2)
    int k2_ty = 8;                       // register strip march: rows per wave
    int res_th = 0;                      // resident stepper: tile height (0: not used)
    int res_ntx = 0, res_nty = 0;        // resident stepper: tiles per row / column
    uint32_t res_epoch = 0;              // resident stepper: generations traded by eager launches (mod 2^30)
    int last_hip = 0;
    hipGraph_t graph = nullptr;          // chain of kGraphLen full-K launches
    hipGraphExec_t gexec = nullptr;
    std::vector<pfk::Real> real;
    std::vector<double> c0;
    std::vector<double> host_out;
    std::vector<double> stage;
};

namespace {

int hip_fail(pf_handle* h, hipError_t e)
{
    if (e == hipSuccess) return PF_OK;
    h->last_hip = (int)e;
    return PF_EDEVICE;
}

template <typename T>
pfk::Coef<T> make_coef(const pf_params* p, double dt)
{
    pfk::Coef<T> k{};
    const double h2 = p->h * p->h;
    k.Wc = (T)p->W_c;
    k.Wphi = (T)p->W_phi;
    k.Wc4 = (T)(0.25 * p->W_c);
    k.Wc34 = (T)(0.75 * p->W_c);
    k.kc = (T)(p->kappa_c / h2);
    k.kp = (T)(p->kappa_phi / h2);
    k.MBb = (T)(p->M_scale * p->MB_bulk);
    k.dMb = (T)(p->M_scale * (p->MA_bulk - p->MB_bulk));
    k.MBs = (T)(p->M_scale * p->MB_surf);
    k.dMs = (T)(p->M_scale * (p->MA_surf - p->MB_surf));
    const double inv_s2 = 1.0 / (p->sigma_surf * p->sigma_surf);
    // float: exp(-x) = exp2(-x log2 e)
    k.esurf = sizeof(T) == 4 ? (T)(inv_s2 * 1.4426950408889634074) : (T)inv_s2;
    k.half_ih2 = (T)(0.5 / h2);
    k.mphi_h2 = (T)(p->M_phi / h2);
    k.D_h2 = (T)(p->D_rho / h2);
    k.dt = (T)dt;
    k.rho_in = (T)p->rho_in;
    return k;
}

// Launch plan of n steps with K sub-steps per launch: full launches first,
// then the remainder.  An even number of launches leaves the result in the
// caller's buffers, so when the count is odd one launch is split in two
// (the remainder, or else the last full launch); only runs of single-step
// launches end with a copy.
std::vector<int> launch_plan(int64_t n, int K)
{
    const int64_t q = n / K;
    const int rem = (int)(n % K);
    std::vector<int> plan((size_t)q, K);
    if (rem) plan.push_back(rem);
    if (plan.size() % 2 == 1) {
        if (rem >= 2) {
            plan.back() = rem / 2;
            plan.push_back(rem - rem / 2);
        } else if (K >= 2 && q >= 1) {
            const size_t i = (size_t)q - 1;   // the last full launch
            plan[i] = K / 2;
            plan.insert(plan.begin() + (long)i + 1, K - K / 2);
        }
    }
    return plan;
}

template <typename T>
pfk::StepArgs<T> step_args(pf_handle* h)
{
    const pf_params* p = &h->p;
    const pfk::TileCfg cfg = pfk::tile_cfg<T>(h->K);
    pfk::StepArgs<T> a{};
    a.Qcol = (double*)(h->ws + h->L.qcol);
    a.real = (const pfk::Real*)(h->ws + h->L.real);
    a.k = make_coef<T>(p, h->dt);
    a.nx = p->nx;
    a.ny = p->ny;
    a.tiles_x = (p->nx + cfg.tx - 1) / cfg.tx;
    a.tiles_y = (p->ny + cfg.ty - 1) / cfg.ty;
    a.pvd = p->bc_mode == PF_BC_PVD;
    return a;
}

template <typename T>
void set_parity(pf_handle* h, pfk::StepArgs<T>& a, int parity)
{
    void* const* src = parity == 0 ? h->f : h->w;
    void* const* dst = parity == 0 ? h->w : h->f;
    a.c = (const T*)src[0];
    a.phi = (const T*)src[1];
    a.rho = (const T*)src[2];
    a.c_out = (T*)dst[0];
    a.phi_out = (T*)dst[1];
    a.rho_out = (T*)dst[2];
}

// Arguments of the two launches of one midpoint step: A advances the
// caller's state by dt/2 into the workspace (no inflow), B evaluates the
// rates there and adds dt times them to the caller's state in place.
template <typename T>
void midpoint_args(pf_handle* h, pfk::StepArgs<T>& A, pfk::StepArgs<T>& B)
{
    A = step_args<T>(h);
    B = A;
    set_parity<T>(h, A, 0);
    A.k = make_coef<T>(&h->p, 0.5 * h->dt);
    A.Qcol = nullptr;
    A.noise = 0;
    A.nsub = 1;
    B.c = (const T*)h->w[0];
    B.phi = (const T*)h->w[1];
    B.rho = (const T*)h->w[2];
    B.cb = (const T*)h->f[0];
    B.pb = (const T*)h->f[1];
    B.rb = (const T*)h->f[2];
    B.c_out = (T*)h->f[0];
    B.phi_out = (T*)h->f[1];
    B.rho_out = (T*)h->f[2];
    B.nsub = 1;
}

// A graph of kGraphLen launches (caller -> workspace -> caller ..., or
// kGraphLen / 2 midpoint steps), built once per handle and replayed for
// long runs.  Not used with interface draws (their launches differ).
template <typename T>
int ensure_graph(pf_handle* h)
{
    if (h->gexec) return PF_OK;
    pfk::StepArgs<T> a = step_args<T>(h), A, B;
    const bool mid = h->p.integrator == PF_MIDPOINT;
    if (mid) midpoint_args<T>(h, A, B);
    hipGraph_t g = nullptr;
    hipError_t e = hipGraphCreate(&g, 0);
    hipGraphNode_t prev = nullptr;
    for (int i = 0; i < kGraphLen && e == hipSuccess; ++i) {
        if (mid) {
            a = (i & 1) ? B : A;
        } else {
            set_parity<T>(h, a, i & 1);
            a.nsub = h->K;
        }
        hipGraphNode_t node = nullptr;
        if (h->K == 1) e = pfk::graph_add_march<T>(g, &node, prev, a, h->march_ty, h->march_cols, h->p.batch);
        else if (h->fused == PF_FUSED_MARCH) e = pfk::graph_add_march_k2<T>(g, &node, prev, a, h->k2_ty, h->p.batch);
        else e = pfk::graph_add_step<T>(g, &node, prev, a, h->K, h->p.batch);
        prev = node;
    }
    hipGraphExec_t ex = nullptr;
    if (e == hipSuccess) e = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
    if (e != hipSuccess) {
        if (g) (void)hipGraphDestroy(g);  // the first error is the one reported
        return hip_fail(h, e);
    }
    h->graph = g;
    h->gexec = ex;
    return PF_OK;
}

template <typename T>
int enqueue_midpoint(pf_handle* h, int64_t n)
{
    pfk::StepArgs<T> A, B;
    midpoint_args<T>(h, A, B);
    const bool noise = h->p.interface_noise > 0;
    B.noise = h->p.interface_noise;
    int64_t s = 0;
    int rc;
    if (!noise && h->p.graph_mode == 0 && n >= kGraphLen / 2) {
        if ((rc = ensure_graph<T>(h))) return rc;
        for (; s + kGraphLen / 2 <= n; s += kGraphLen / 2)
            if ((rc = hip_fail(h, hipGraphLaunch(h->gexec, h->stream)))) return rc;
    }
    for (; s < n; ++s) {
        B.step = h->step + s;
        if ((rc = hip_fail(h, pfk::launch_march<T>(A, h->march_ty, h->march_cols, h->p.batch, h->stream)))) return rc;
        if ((rc = hip_fail(h, pfk::launch_march<T>(B, h->march_ty, h->march_cols, h->p.batch, h->stream)))) return rc;
    }
    return PF_OK;
}

// Resident stepper: all n >= 2 steps in one launch, in place on the
// caller's buffers, in chunks of at most 2^29 steps.
int enqueue_resident(pf_handle* h, int64_t n)
{
    pfk::ResArgs ra{};
    ra.s = step_args<float>(h);
    ra.kh = make_coef<float>(&h->p, 0.5 * h->dt);
    ra.mid = h->p.integrator == PF_MIDPOINT;
    ra.s.noise = h->p.interface_noise;
    ra.s.c = (const float*)h->f[0];
    ra.s.phi = (const float*)h->f[1];
    ra.s.rho = (const float*)h->f[2];
    ra.s.c_out = (float*)h->f[0];
    ra.s.phi_out = (float*)h->f[1];
    ra.s.rho_out = (float*)h->f[2];
    ra.s.nsub = 1;
    ra.rim = (uint64_t*)(h->ws + h->L.rim);
    ra.ctl = (uint64_t*)(h->ws + h->L.rctl);
    ra.batch = h->p.batch;
    ra.ntx = h->res_ntx;
    ra.nty = h->res_nty;
    // a launch captured in a graph takes its tags from the device epoch (a
    // replay repeats the arguments); eager launches from the host's count
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(h->stream, &cs) != hipSuccess) (void)hipGetLastError();
    ra.dev_epoch = cs != hipStreamCaptureStatusNone;
    constexpr int64_t kChunk = (int64_t)1 << 29;
    int64_t done = 0;
    while (done < n) {
        // never leave a single step for the last chunk
        ra.n = (int)(n - done > kChunk + 1 ? kChunk : n - done);
        ra.s.step = h->step + done;   // keys the interface draws
        ra.e0 = h->res_epoch;
        const int rc = hip_fail(h, pfk::launch_resident(ra, h->res_th, h->stream));
        if (rc) return rc;
        if (!ra.dev_epoch) h->res_epoch = (h->res_epoch + (uint32_t)(ra.mid ? 2 * ra.n : ra.n)) & 0x3FFFFFFFu;
        done += ra.n;
    }
    return PF_OK;
}

template <typename T>
int enqueue_steps(pf_handle* h, int64_t n)
{
    const pf_params* p = &h->p;
    if (h->res_th && n >= 2) return enqueue_resident(h, n);
    if (p->integrator == PF_MIDPOINT) return enqueue_midpoint<T>(h, n);
    const int K = h->K;
    const bool noise = p->interface_noise > 0;
    pfk::StepArgs<T> a = step_args<T>(h);
    a.noise = p->interface_noise;
    const std::vector<int> plan = launch_plan(n, K);
    size_t full = 0;
    while (full < plan.size() && plan[full] == K) ++full;
    size_t l = 0;
    int rc;
    if (!noise && p->graph_mode == 0 && full >= (size_t)kGraphLen) {
        if ((rc = ensure_graph<T>(h))) return rc;
        for (; l + kGraphLen <= full; l += kGraphLen)
            if ((rc = hip_fail(h, hipGraphLaunch(h->gexec, h->stream)))) return rc;
    }
    int parity = (int)(l & 1);
    for (; l < plan.size(); ++l) {
        set_parity<T>(h, a, parity);
        a.nsub = plan[l];
        a.step = h->step + (int64_t)l;  // one step per launch whenever draws are on (K = 1)
        hipError_t e;
        if (K == 1) e = pfk::launch_march<T>(a, h->march_ty, h->march_cols, p->batch, h->stream);
        else if (h->fused != PF_FUSED_MARCH) e = pfk::launch_step<T>(a, K, p->batch, h->stream);
        else if (a.nsub == 2) e = pfk::launch_march_k2<T>(a, h->k2_ty, p->batch, h->stream);
        else e = pfk::launch_march<T>(a, h->march_ty, h->march_cols, p->batch, h->stream);  // odd step
        if ((rc = hip_fail(h, e))) return rc;
        parity ^= 1;
    }
    if (parity == 1) {
        // odd number of single-step launches: copy the result back
        const size_t bytes = (size_t)p->batch * p->nx * p->ny * sizeof(T);
        for (int f = 0; f < 3; ++f)
            if ((rc = hip_fail(h, hipMemcpyAsync(h->f[f], h->w[f], bytes, hipMemcpyDeviceToDevice, h->stream))))
                return rc;
    }
    return PF_OK;
}

int run_reduce(pf_handle* h)
{
    const pf_params* p = &h->p;
    pfk::RedArgs a{};
    a.nx = p->nx;
    a.ny = p->ny;
    a.pvd = p->bc_mode == PF_BC_PVD;
    a.h2 = p->h * p->h;
    a.Wc = p->W_c;
    a.Wphi = p->W_phi;
    a.half_kc = 0.5 * p->kappa_c;
    a.half_kp = 0.5 * p->kappa_phi;
    double* partials = (double*)(h->ws + h->L.partials);
    double* res = (double*)(h->ws + h->L.results);
    const double* Qcol = (const double*)(h->ws + h->L.qcol);
    const pfk::RedGeo g = pfk::reduce_geometry(p->nx, p->ny, p->batch, (int)esize(p));
    hipError_t e;
    if (p->precision == PF_F64)
        e = pfk::launch_reduce<double>((const double*)h->f[0], (const double*)h->f[1], (const double*)h->f[2],
                                       Qcol, partials, res, a, g, p->batch, h->stream);
    else
        e = pfk::launch_reduce<float>((const float*)h->f[0], (const float*)h->f[1], (const float*)h->f[2],
                                      Qcol, partials, res, a, g, p->batch, h->stream);
    if (e != hipSuccess) return hip_fail(h, e);
    h->host_out.resize((size_t)p->batch * 5);
    e = hipMemcpyAsync(h->host_out.data(), res, h->host_out.size() * sizeof(double), hipMemcpyDeviceToHost,
                       h->stream);
    if (e != hipSuccess) return hip_fail(h, e);
    // the resident stepper's sticky abort word (a wait it gave up)
    uint64_t abort_word = 0;
    if (h->res_th) {
        e = hipMemcpyAsync(&abort_word, h->ws + h->L.rctl + sizeof(uint64_t), sizeof(uint64_t),
                           hipMemcpyDeviceToHost, h->stream);
        if (e != hipSuccess) return hip_fail(h, e);
    }
    e = hipStreamSynchronize(h->stream);
    if (e != hipSuccess) return hip_fail(h, e);
    return abort_word ? PF_EABORTED : PF_OK;
}

}  // namespace

extern "C" {

size_t pf_workspace_bytes(const pf_params* p)
{
    if (validate(p) != PF_OK) return 0;
    return layout(p).total;
}

int pf_dt_limit(const pf_params* p, double* dt_lim)
{
    if (!dt_lim || validate(p) != PF_OK) return PF_EINVAL;
    const double lim = stability_limit(p);
    if (!(lim > 0) || std::isinf(lim)) return PF_EINVAL;
    *dt_lim = lim;
    return PF_OK;
}

int pf_init(pf_handle** out, const pf_params* p, void* c, void* phi, void* rho, void* workspace,
            size_t workspace_bytes, void* stream)
{
    if (!out) return PF_EINVAL;
    *out = nullptr;
    int rc = validate(p);
    if (rc) return rc;
    if (!c || !phi || !rho || !workspace) return PF_EINVAL;
    if (!aligned(c, 16) || !aligned(phi, 16) || !aligned(rho, 16) || !aligned(workspace, kAlign))
        return PF_EINVAL;
    const Layout L = layout(p);
    if (workspace_bytes < L.total) return PF_EINVAL;
    const double lim = stability_limit(p);
    if (!(lim > 0) || std::isinf(lim)) return PF_EINVAL;
    const double dt = p->dt > 0 ? p->dt : p->dt_factor * lim;
    if (dt > lim * (1.0 + 1e-12) && !p->allow_unstable) return PF_EUNSTABLE;

    pf_handle* h = new (std::nothrow) pf_handle;
    if (!h) return PF_EINVAL;
    h->p = *p;
    h->p.v0_per = nullptr;
    h->p.c0_per = nullptr;
    h->L = L;
    h->ws = (char*)workspace;
    h->f[0] = c;
    h->f[1] = phi;
    h->f[2] = rho;
    for (int f = 0; f < 3; ++f) h->w[f] = h->ws + L.state[f];
    h->stream = (hipStream_t)stream;
    h->dt = dt;
    // Launch shape.  Fused steps per launch K: as requested, else by
    // precision, grid size and variant (the rules below, measured on
    // MI355X); the resident stepper, where it runs, replaces them all for
    // calls of two or more steps.  The mirror ghosts of a launch must be real
    // rows, so 2K <= ny.
    const long cells = (long)p->nx * p->ny * p->batch;
    // FP32 Euler runs fuse two steps by default (measured on MI355X) in the
    // register strip march when a chunk height divides ny: 16-row chunks
    // from ~3M cells, 8 for one grid of ~0.75M to ~3M cells, 4 below (512^2:
    // 73 against 59 for single steps; 2048 x 1024: 203 against 178 with 4
    // rows and 162 for the LDS tile; 1000 x 800: 145 against 138 and 121;
    // 2048^2 266, 4096^2 297, 8192^2 343 against 221, 171, 214 for single
    // steps; 32 x 512^2 308 against 250; deeper load look-ahead for 16-row
    // chunks measured slower), else the LDS tile for such a grid (any ny;
    // 1000^2: 152 against 144); the resident stepper takes precedence
    const bool plain_euler = p->integrator == PF_EULER && !(p->interface_noise > 0);
    const bool f32 = p->precision == PF_F32;
    const bool mid_band = f32 && p->batch == 1 && cells >= 786432L && cells < 3000000L;
    const int k2_auto_ty = cells >= 3000000L ? 16 : (mid_band ? 8 : 4);
    int K = p->temporal_block;
    // FP64 fuses two steps only on large grids (4096^2: 146 GLUPS against
    // 102 for single steps; 1024^2: 84 against 82)
    if (K == 0 && plain_euler && f32) K = mid_band || p->ny % 4 == 0 ? 2 : 1;
    if (K == 0 && plain_euler && !f32) K = cells >= 3000000L && p->ny % 4 == 0 ? 2 : 1;
    if (K == 0) K = 1;
    if (p->integrator != PF_EULER || p->interface_noise > 0) K = 1;
    while (K > 1 && 2 * K > p->ny) --K;
    h->K = K;
    if (p->tile_rows > 0) {
        h->march_ty = p->tile_rows;
    } else {
        // strip-march chunk height: 8 rows for one large grid (when that still
        // gives about four waves per SIMD), else 4 (shorter chunks cost more
        // row halo; measured on MI355X, 32 x 512^2 runs at 251 GLUPS with 4
        // rows against 237 with 8)
        const long strips = (p->nx + 59) / 60;
        h->march_ty = p->batch == 1 && strips * ((p->ny + 7) / 8) >= 4096 ? 8 : 4;
    }
    // two grid columns per lane (FP32 with an even row length): on request,
    // and by default from ~8M cells per launch, where the step streams from
    // HBM and the halved neighbour exchange pays (measured on MI355X: +2 % at
    // 4096^2, +7 % at 8192^2; at 2048^2 and below one column is faster),
    // unless the wider strips compute more columns in all (32 x 512^2: 640
    // computed columns per row against 576)
    const bool two_ok = p->precision == PF_F32 && p->nx % 2 == 0;
    const long w1 = (p->nx + 59) / 60 * 64L, w2 = (p->nx + 123) / 124 * 128L;
    const int cols = p->lane_cols ? p->lane_cols : (cells >= 8000000L && w2 <= w1 ? 2 : 1);
    h->march_cols = cols == 2 && two_ok ? 2 : 1;
    // fused steps: the register strip march (two steps, chunk heights
    // dividing ny) as asked for or by default, else the LDS tile
    h->fused = PF_FUSED_TILE;
    const bool march_k2 = p->fused_kernel == PF_FUSED_MARCH ||
                          (p->fused_kernel == PF_FUSED_AUTO && (f32 || p->temporal_block == 0));
    if (K == 2 && march_k2) {
        const int auto_ty = p->fused_kernel == PF_FUSED_MARCH ? 8 : k2_auto_ty;
        const int want = p->tile_rows == 4 || p->tile_rows == 8 || p->tile_rows == 16 ? p->tile_rows : auto_ty;
        for (int ty : {want, 8, 4}) {
            if (p->ny % ty == 0) {
                h->fused = PF_FUSED_MARCH;
                h->k2_ty = ty;
                break;
            }
        }
    }

    // the resident stepper, where the device keeps every tile resident; a
    // single step (n == 1) then runs the single-step kernel
    if (const int rth = resident_th(p)) {
        const int ntx = p->nx / 64, nty = p->ny / rth;
        if ((long)p->batch * ntx * nty <= pfk::resident_capacity(rth)) {
            h->res_th = rth;
            h->res_ntx = ntx;
            h->res_nty = nty;
            h->K = 1;
        } else if (p->fused_kernel == PF_FUSED_RESIDENT) {
            delete h;
            return PF_EINVAL;
        }
    }

    const double th = p->theta_deg * (3.14159265358979323846 / 180.0);
    h->real.resize(p->batch);
    h->c0.resize(p->batch);
    for (int b = 0; b < p->batch; ++b) {
        const double v0 = p->flux_on ? v0_of(p, b) : 0.0;
        const double vx = v0 * std::cos(th), vy = -v0 * std::sin(th);
        h->real[b].vx2h = vx / (2.0 * p->h);
        h->real[b].vy2h = vy / (2.0 * p->h);
        h->real[b].qa = dt * p->h * (-0.5 * vy);
        h->real[b].qb = dt * p->D_rho;
        h->real[b].c0 = c0_of(p, b);
        h->real[b].nseed = (p->seed + (uint64_t)b) ^ 0x2B7E151628AED2A6ull;  // interface-draw stream
        h->c0[b] = c0_of(p, b);
    }
    // pf_params says the per-realisation arrays are read during the call
    hipError_t e = hipMemcpyAsync(h->ws + L.real, h->real.data(), p->batch * sizeof(pfk::Real),
                                  hipMemcpyHostToDevice, h->stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(h->ws + L.c0, h->c0.data(), p->batch * sizeof(double), hipMemcpyHostToDevice,
                           h->stream);
    if (e == hipSuccess) e = pfk::launch_set_inflow((double*)(h->ws + L.qcol), nullptr, p->nx, p->batch, h->stream);
    // rim words start with tag 0, which no generation uses; epoch and abort 0
    if (e == hipSuccess && L.total > L.rim) e = hipMemsetAsync(h->ws + L.rim, 0, L.total - L.rim, h->stream);
    if (e == hipSuccess && p->init_mode == PF_INIT_SEEDED) {
        pfk::InitArgs ia{};
        ia.seed = p->seed;
        ia.nx = p->nx;
        ia.ny = p->ny;
        ia.h = p->h;
        ia.c_noise = p->c_noise;
        ia.H0 = p->film_h > 0 ? p->film_h : p->ny * p->h / 8.0;
        ia.width = std::sqrt(2.0 * p->kappa_phi / p->W_phi);
        ia.rho_in = p->rho_in;
        ia.c0 = (const double*)(h->ws + L.c0);
        if (p->precision == PF_F64)
            e = pfk::launch_init<double>((double*)c, (double*)phi, (double*)rho, ia, p->batch, h->stream);
        else
            e = pfk::launch_init<float>((float*)c, (float*)phi, (float*)rho, ia, p->batch, h->stream);
    }
    if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
    if (e != hipSuccess) {
        h->last_hip = (int)e;
        delete h;
        return PF_EDEVICE;
    }
    *out = h;
    return PF_OK;
}

int pf_step_n(pf_handle* h, int64_t n)
{
    if (!h || n < 0) return PF_EINVAL;
    if (n == 0) return PF_OK;
    if (h->p.interface_noise > 0) {
        // the draws are keyed by the global step the call starts at, passed
        // by value: a captured call would replay the same draws
        hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
        if (hipStreamIsCapturing(h->stream, &cs) != hipSuccess) (void)hipGetLastError();
        if (cs != hipStreamCaptureStatusNone) return PF_EINVAL;
    }
    const int rc = h->p.precision == PF_F64 ? enqueue_steps<double>(h, n) : enqueue_steps<float>(h, n);
    if (rc == PF_OK) h->step += n;
    return rc;
}

int pf_step_out(pf_handle* h, const void* c, const void* phi, const void* rho, void* c_out, void* phi_out,
                void* rho_out)
{
    if (!h) return PF_EINVAL;
    const void* ptrs[6] = {c, phi, rho, c_out, phi_out, rho_out};
    for (const void* q : ptrs)
        if (!q || !aligned(q, 16)) return PF_EINVAL;
    if (c_out == c || phi_out == phi || rho_out == rho) return PF_EINVAL;
    if (h->p.integrator != PF_EULER || h->p.interface_noise > 0) return PF_EINVAL;
    hipError_t e;
    if (h->p.precision == PF_F64) {
        pfk::StepArgs<double> a = step_args<double>(h);
        a.c = (const double*)c, a.phi = (const double*)phi, a.rho = (const double*)rho;
        a.c_out = (double*)c_out, a.phi_out = (double*)phi_out, a.rho_out = (double*)rho_out;
        a.Qcol = nullptr;
        a.nsub = 1;
        a.step = h->step;
        e = pfk::launch_march<double>(a, h->march_ty, h->march_cols, h->p.batch, h->stream);
    } else {
        pfk::StepArgs<float> a = step_args<float>(h);
        a.c = (const float*)c, a.phi = (const float*)phi, a.rho = (const float*)rho;
        a.c_out = (float*)c_out, a.phi_out = (float*)phi_out, a.rho_out = (float*)rho_out;
        a.Qcol = nullptr;
        a.nsub = 1;
        a.step = h->step;
        e = pfk::launch_march<float>(a, h->march_ty, h->march_cols, h->p.batch, h->stream);
    }
    return hip_fail(h, e);
}

int pf_mass(pf_handle* h, double* out)
{
    if (!h || !out) return PF_EINVAL;
    int rc = run_reduce(h);
    if (rc) return rc;
    bool ok = true;
    for (int b = 0; b < h->p.batch; ++b)
        for (int m = 0; m < 4; ++m) {
            out[4 * b + m] = h->host_out[5 * b + m];
            ok = ok && std::isfinite(out[4 * b + m]);
        }
    return ok ? PF_OK : PF_ENONFINITE;
}

int pf_energy(pf_handle* h, double* out)
{
    if (!h || !out) return PF_EINVAL;
    int rc = run_reduce(h);
    if (rc) return rc;
    bool ok = true;
    for (int b = 0; b < h->p.batch; ++b) {
        out[b] = h->host_out[5 * b + 4];
        ok = ok && std::isfinite(out[b]);
    }
    return ok ? PF_OK : PF_ENONFINITE;
}

int pf_get_step(const pf_handle* h, int64_t* step)
{
    if (!h || !step) return PF_EINVAL;
    *step = h->step;
    return PF_OK;
}

int pf_set_step(pf_handle* h, int64_t step)
{
    if (!h || step < 0) return PF_EINVAL;
    h->step = step;
    return PF_OK;
}

int pf_get_dt(const pf_handle* h, double* dt)
{
    if (!h || !dt) return PF_EINVAL;
    *dt = h->dt;
    return PF_OK;
}

int pf_get_inflow(pf_handle* h, double* Q)
{
    if (!h || !Q) return PF_EINVAL;
    int rc = run_reduce(h);
    if (rc) return rc;
    for (int b = 0; b < h->p.batch; ++b) Q[b] = h->host_out[5 * b + 3];
    return PF_OK;
}

int pf_set_inflow(pf_handle* h, const double* Q)
{
    if (!h || !Q) return PF_EINVAL;
    for (int b = 0; b < h->p.batch; ++b)
        if (!std::isfinite(Q[b])) return PF_EINVAL;
    h->stage.assign(Q, Q + h->p.batch);
    double* dq = (double*)(h->ws + h->L.qstage);
    hipError_t e = hipMemcpyAsync(dq, h->stage.data(), h->p.batch * sizeof(double), hipMemcpyHostToDevice,
                                  h->stream);
    if (e == hipSuccess)
        e = pfk::launch_set_inflow((double*)(h->ws + h->L.qcol), dq, h->p.nx, h->p.batch, h->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
    return hip_fail(h, e);
}

void pf_destroy(pf_handle* h)
{
    if (!h) return;
    // teardown: nothing to report to a caller that is discarding the handle
    if (h->gexec) (void)hipGraphExecDestroy(h->gexec);
    if (h->graph) (void)hipGraphDestroy(h->graph);
    delete h;
}

const char* pf_strerror(int code)
{
    switch (code) {
    case PF_OK: return "ok";
    case PF_EINVAL: return "invalid argument";
    case PF_EUNSTABLE: return "time step above the explicit stability limit";
    case PF_ENONFINITE: return "non-finite diagnostic (state diverged or holds NaN/Inf)";
    case PF_EDEVICE: return "HIP device error";
    case PF_EABORTED: return "resident stepper abandoned a wait (tiles not co-resident); state is NaN, re-initialise";
    case PF_ESCRATCH: return "input too large for the static scratch of pf_diagnostics_noalloc";
    default: return "unknown pf status";
    }
}

int pf_last_hip_error(const pf_handle* h) { return h ? h->last_hip : 0; }

}  // extern "C"

namespace {

struct AdjLayout {
    size_t gacc, out, total;
};

AdjLayout adj_layout(const pf_params* p)
{
    AdjLayout L{};
    const size_t cells = (size_t)p->batch * p->nx * p->ny;
    size_t off = 0;
    auto take = [&](size_t bytes) {
        const size_t o = off;
        off += round_up(bytes);
        return o;
    };
    L.gacc = take(2 * cells * sizeof(double));
    L.out = take(2 * (size_t)p->batch * sizeof(double));
    L.total = off;
    return L;
}

template <typename T>
int adjoint_step_t(pf_handle* h, const void* c, const void* phi, const void* rho, const void* lc,
                   const void* lp, const void* lr, void* oc, void* op, void* orr, char* ws)
{
    const pf_params* p = &h->p;
    const AdjLayout L = adj_layout(p);
    pfk::AdjointIO<T> io{};
    io.c = (const T*)c;
    io.phi = (const T*)phi;
    io.rho = (const T*)rho;
    io.lc = (const T*)lc;
    io.lp = (const T*)lp;
    io.lr = (const T*)lr;
    io.oc = (T*)oc;
    io.op = (T*)op;
    io.orr = (T*)orr;
    io.gacc = (double*)(ws + L.gacc);
    const pfk::StepArgs<T> st = step_args<T>(h);
    const double th = p->theta_deg * (3.14159265358979323846 / 180.0);
    const double cx = p->flux_on ? std::cos(th) : 0.0, sy = p->flux_on ? -std::sin(th) : 0.0;
    return hip_fail(h, pfk::launch_adjoint<T>(io, st, p->M_scale, cx, sy, p->h, p->batch, h->stream));
}

// The adjoint is the transpose of one explicit Euler step without
// interface draws; other integrators and the random interface composition
// have no adjoint here.
bool adj_model_ok(const pf_params* p)
{
    return p->integrator == PF_EULER && !(p->interface_noise > 0);
}

bool adj_ws_ok(const pf_handle* h, const void* ws, size_t bytes)
{
    return adj_model_ok(&h->p) && ws && aligned(ws, kAlign) && bytes >= adj_layout(&h->p).total;
}

}  // namespace

extern "C" {

size_t pf_adjoint_workspace_bytes(const pf_params* p)
{
    if (validate(p) != PF_OK || !adj_model_ok(p)) return 0;
    return adj_layout(p).total;
}

int pf_adjoint_step(pf_handle* h, const void* c, const void* phi, const void* rho, const void* lam_c,
                    const void* lam_phi, const void* lam_rho, void* out_c, void* out_phi, void* out_rho,
                    void* adj_workspace, size_t adj_bytes)
{
    if (!h || !adj_ws_ok(h, adj_workspace, adj_bytes)) return PF_EINVAL;
    const void* in[9] = {c, phi, rho, lam_c, lam_phi, lam_rho, out_c, out_phi, out_rho};
    for (const void* q : in)
        if (!q || !aligned(q, 16)) return PF_EINVAL;
    if (out_c == lam_c || out_phi == lam_phi || out_rho == lam_rho) return PF_EINVAL;
    if (!(h->p.M_scale > 0)) return PF_EINVAL;
    char* ws = (char*)adj_workspace;
    return h->p.precision == PF_F64
               ? adjoint_step_t<double>(h, c, phi, rho, lam_c, lam_phi, lam_rho, out_c, out_phi, out_rho, ws)
               : adjoint_step_t<float>(h, c, phi, rho, lam_c, lam_phi, lam_rho, out_c, out_phi, out_rho, ws);
}

int pf_adjoint_reset(pf_handle* h, void* adj_workspace, size_t adj_bytes)
{
    if (!h || !adj_ws_ok(h, adj_workspace, adj_bytes)) return PF_EINVAL;
    const AdjLayout L = adj_layout(&h->p);
    const size_t cells = (size_t)h->p.batch * h->p.nx * h->p.ny;
    return hip_fail(h, pfk::launch_gacc_zero((double*)((char*)adj_workspace + L.gacc), 2 * cells, h->stream));
}

}  // extern "C"

namespace {

// slot t, field k of a ring [len][3][batch][ny][nx]
void* ring_field(const pf_handle* h, void* ring, int64_t t, int k)
{
    const size_t fb = (size_t)h->p.batch * h->p.nx * h->p.ny * (h->p.precision == PF_F64 ? 8 : 4);
    return (char*)ring + (size_t)(3 * t + k) * fb;
}

// two Euler steps out of place in one two-step march launch: q[0..2] the
// input state, q[3..5] the state after one step, q[6..8] after two (no
// inflow accumulation, as pf_step_out)
template <typename T>
int step_pair(pf_handle* h, void* const q[9])
{
    pfk::StepArgs<T> a = step_args<T>(h);
    a.c = (const T*)q[0], a.phi = (const T*)q[1], a.rho = (const T*)q[2];
    a.c_mid = (T*)q[3], a.phi_mid = (T*)q[4], a.rho_mid = (T*)q[5];
    a.c_out = (T*)q[6], a.phi_out = (T*)q[7], a.rho_out = (T*)q[8];
    a.Qcol = nullptr;
    a.nsub = 2;
    a.step = h->step;
    return hip_fail(h, pfk::launch_march_k2<T>(a, h->k2_ty, h->p.batch, h->stream));
}

}  // namespace

extern "C" {

int pf_adjoint_recompute(pf_handle* h, void* ring, int64_t len)
{
    if (!h || !ring || len < 1) return PF_EINVAL;
    // where the handle steps with the two-step register march, one launch
    // writes two slots (the intermediate state and the one after it; bitwise
    // those of two single steps); otherwise, and for a last odd slot,
    // pf_step_out's single-step launch
    const bool pair = h->K == 2 && h->fused == PF_FUSED_MARCH && h->p.integrator == PF_EULER &&
                      !(h->p.interface_noise > 0);
    int64_t t = 1;
    while (t < len) {
        if (pair && t + 1 < len) {
            void* q[9];
            for (int k = 0; k < 3; ++k) {
                q[k] = ring_field(h, ring, t - 1, k);
                q[3 + k] = ring_field(h, ring, t, k);
                q[6 + k] = ring_field(h, ring, t + 1, k);
            }
            for (void* x : q)
                if (!aligned(x, 16)) return PF_EINVAL;
            const int rc = h->p.precision == PF_F64 ? step_pair<double>(h, q) : step_pair<float>(h, q);
            if (rc != PF_OK) return rc;
            t += 2;
        } else {
            const int rc = pf_step_out(h, ring_field(h, ring, t - 1, 0), ring_field(h, ring, t - 1, 1),
                                       ring_field(h, ring, t - 1, 2), ring_field(h, ring, t, 0),
                                       ring_field(h, ring, t, 1), ring_field(h, ring, t, 2));
            if (rc != PF_OK) return rc;
            t += 1;
        }
    }
    return PF_OK;
}

int pf_adjoint_sweep(pf_handle* h, void* ring, int64_t len, void* lam_c, void* lam_phi, void* lam_rho,
                     void* tmp_c, void* tmp_phi, void* tmp_rho, void* adj_workspace, size_t adj_bytes,
                     int32_t* in_tmp)
{
    if (!h || !ring || !in_tmp || len < 1 || !adj_ws_ok(h, adj_workspace, adj_bytes)) return PF_EINVAL;
    // from the last state to the first, the two lambda buffers taking turns
    // as input and output
    void* cur[3] = {lam_c, lam_phi, lam_rho};
    void* nxt[3] = {tmp_c, tmp_phi, tmp_rho};
    for (int64_t t = len - 1; t >= 0; --t) {
        const int rc = pf_adjoint_step(h, ring_field(h, ring, t, 0), ring_field(h, ring, t, 1),
                                       ring_field(h, ring, t, 2), cur[0], cur[1], cur[2], nxt[0], nxt[1], nxt[2],
                                       adj_workspace, adj_bytes);
        if (rc != PF_OK) return rc;
        std::swap(cur, nxt);
    }
    *in_tmp = (int32_t)(len & 1);
    return PF_OK;
}

int pf_adjoint_segment(pf_handle* h, void* ring, int64_t len, void* lam_c, void* lam_phi, void* lam_rho,
                       void* tmp_c, void* tmp_phi, void* tmp_rho, void* adj_workspace, size_t adj_bytes,
                       int32_t* in_tmp)
{
    if (!h || !ring || !in_tmp || len < 1 || !adj_ws_ok(h, adj_workspace, adj_bytes)) return PF_EINVAL;
    const int rc = pf_adjoint_recompute(h, ring, len);
    if (rc != PF_OK) return rc;
    return pf_adjoint_sweep(h, ring, len, lam_c, lam_phi, lam_rho, tmp_c, tmp_phi, tmp_rho, adj_workspace,
                            adj_bytes, in_tmp);
}

int pf_adjoint_grad(pf_handle* h, void* adj_workspace, size_t adj_bytes, double* out)
{
    if (!h || !out || !adj_ws_ok(h, adj_workspace, adj_bytes)) return PF_EINVAL;
    const AdjLayout L = adj_layout(&h->p);
    char* ws = (char*)adj_workspace;
    const size_t per = (size_t)h->p.nx * h->p.ny;
    hipError_t e = pfk::launch_gacc_sum((const double*)(ws + L.gacc), (double*)(ws + L.out), per, h->p.batch,
                                        h->stream);
    h->host_out.resize(2 * (size_t)h->p.batch);
    if (e == hipSuccess)
        e = hipMemcpyAsync(h->host_out.data(), ws + L.out, 2 * h->p.batch * sizeof(double),
                           hipMemcpyDeviceToHost, h->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
    if (e != hipSuccess) return hip_fail(h, e);
    bool ok = true;
    for (int i = 0; i < 2 * h->p.batch; ++i) {
        out[i] = h->host_out[i];
        ok = ok && std::isfinite(out[i]);
    }
    return ok ? PF_OK : PF_ENONFINITE;
}

}  // extern "C"

extern "C" int pf_get_launch(const pf_handle* h, int32_t* temporal_block, int32_t* tile_rows)
{
    if (!h || !temporal_block || !tile_rows) return PF_EINVAL;
    *temporal_block = h->K;
    *tile_rows = h->K == 1 ? h->march_ty : (h->fused == PF_FUSED_MARCH ? h->k2_ty : pfk::tile_cfg<float>(h->K).ty);
    if (h->res_th) *tile_rows = h->res_th;
    if (h->p.precision == PF_F64 && h->K > 1 && h->fused != PF_FUSED_MARCH)
        *tile_rows = pfk::tile_cfg<double>(h->K).ty;
    return PF_OK;
}

extern "C" int pf_get_fused_kernel(const pf_handle* h, int32_t* kind)
{
    if (!h || !kind) return PF_EINVAL;
    *kind = h->res_th ? PF_FUSED_RESIDENT : (h->K == 1 ? 0 : h->fused);
    return PF_OK;
}

extern "C" int pf_get_lane_cols(const pf_handle* h, int32_t* lane_cols)
{
    if (!h || !lane_cols) return PF_EINVAL;
    *lane_cols = h->K == 1 ? h->march_cols : 1;
    return PF_OK;
}

// ------------------------------------------------ allocation-free diagnostics
//
// pf_diagnostics_noalloc keeps its reduction partials in a file-scope device
// array instead of a workspace.  In host code `scratch` names a host-side
// stand-in, not device memory: the device address of each GPU's copy comes
// from hipGetSymbolAddress, looked up once per device on the first call with
// that device current, and only that address is passed to kernels.

namespace {

constexpr size_t kScratchBytes = (size_t)1 << 20;   // per GPU, held until the process ends
constexpr int kMaxDevices = 64;

__device__ __align__(256) double scratch[kScratchBytes / sizeof(double)];

std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// Device address of the current device's scratch array (looked up once per
// device); nullptr with *err set on failure.
void* scratch_address(int dev, hipError_t* err)
{
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !ptr) {
            *err = e != hipSuccess ? e : hipErrorInvalidSymbol;
            return nullptr;
        }
        g_scratch_ptr[dev] = ptr;
    }
    return g_scratch_ptr[dev];
}

}  // namespace

extern "C" size_t pf_diagnostics_noalloc_limit(void) { return kScratchBytes; }

extern "C" int pf_diagnostics_noalloc(const pf_params* p, const void* c, const void* phi, const void* rho,
                                      double* out, void* stream)
{
    if (validate(p) != PF_OK) return PF_EINVAL;
    if (!c || !phi || !rho || !out) return PF_EINVAL;
    if (!aligned(c, 16) || !aligned(phi, 16) || !aligned(rho, 16) || !aligned(out, sizeof(double)))
        return PF_EINVAL;
    const pfk::RedGeo g = pfk::reduce_geometry(p->nx, p->ny, p->batch, (int)esize(p));
    const size_t need = (size_t)p->batch * (size_t)g.parts() * 4 * sizeof(double);
    if (need > kScratchBytes) return PF_ESCRATCH;
    // the stream's device must be the current one (its scratch copy is used)
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return PF_EDEVICE;
    hipStream_t s = (hipStream_t)stream;
    if (s) {
        int sdev = -1;
        if (hipStreamGetDevice(s, &sdev) != hipSuccess) return PF_EDEVICE;
        if (sdev != dev) return PF_EINVAL;
    }
    hipError_t e = hipSuccess;
    double* partials = (double*)scratch_address(dev, &e);
    if (!partials) return PF_EDEVICE;
    pfk::RedArgs a{};
    a.nx = p->nx;
    a.ny = p->ny;
    a.pvd = p->bc_mode == PF_BC_PVD;
    a.h2 = p->h * p->h;
    a.Wc = p->W_c;
    a.Wphi = p->W_phi;
    a.half_kc = 0.5 * p->kappa_c;
    a.half_kp = 0.5 * p->kappa_phi;
    if (p->precision == PF_F64)
        e = pfk::launch_reduce<double>((const double*)c, (const double*)phi, (const double*)rho, nullptr, partials,
                                       out, a, g, p->batch, s);
    else
        e = pfk::launch_reduce<float>((const float*)c, (const float*)phi, (const float*)rho, nullptr, partials, out,
                                      a, g, p->batch, s);
    return e == hipSuccess ? PF_OK : PF_EDEVICE;
}
