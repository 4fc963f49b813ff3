// Internal interface between the C-ABI host code and the gfx950 kernels.
// Not part of the public ABI (that is include/pf.h).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace pfk {

// Model constants in the arithmetic type T of a launch, folded on the host
// in FP64 (e.g. kappa/h^2) and rounded once to T.
template <typename T>
struct Coef {
    T Wc, Wphi;        // double-well heights
    T Wc4, Wc34;       // W_c / 4, 3 W_c / 4
    T kc, kp;          // kappa_c / h^2, kappa_phi / h^2
    T MBb, dMb;        // M_scale*MB_bulk, M_scale*(MA_bulk - MB_bulk)
    T MBs, dMs;        // same for the surface mobilities
    T esurf;           // 1/sigma^2 (double) or log2(e)/sigma^2 (float, exp2 form)
    T half_ih2;        // 0.5 / h^2
    T mphi_h2;         // M_phi / h^2
    T D_h2;            // D_rho / h^2
    T dt;
    T rho_in;
};

// Per-realisation constants (device array, double): vx/(2h), vy/(2h),
// the two inflow weights dt*h*(-vy/2) and dt*D, the mean composition and the
// interface-draw stream.
struct Real {
    double vx2h, vy2h, qa, qb;
    double c0;
    uint64_t nseed;
};

template <typename T>
struct StepArgs {
    const T* c;
    const T* phi;
    const T* rho;
    T* c_out;
    T* phi_out;
    T* rho_out;
    double* Qcol;        // [B][nx] cumulative inflow per column (null: not accumulated)
    const Real* real;    // [B]
    // midpoint second stage: the update adds dt R(c, phi, rho) to these
    // (null: to c, phi, rho themselves)
    const T* cb;
    const T* pb;
    const T* rb;
    double noise;        // interface draw standard deviation (0: off)
    long long step;      // global step index keying the draws
    Coef<T> k;
    int nx, ny;
    int tiles_x, tiles_y;
    int pvd;             // 1: substrate + inlet boundaries; 0: periodic in y
    int nsub;            // sub-steps in this launch (1..K of the kernel)
    int fast;            // set by the launcher: 16-byte vector loads are valid
    // two-step march: the state after the first step is also stored here
    // (null: not stored)
    T* c_mid;
    T* phi_mid;
    T* rho_mid;
};

// Tile configuration of a stepper instantiation.
struct TileCfg {
    int tx, ty, k, nthreads;
};

// Launch one stepper launch of `nsub` sub-steps with fused-step capacity k.
// Returns hipSuccess or the launch error.
template <typename T>
hipError_t launch_step(const StepArgs<T>& a, int k, int batch, hipStream_t s);

template <typename T>
TileCfg tile_cfg(int k);

// Single-step strip-march kernel (K = 1), chunks of ty in {4, 8, 16, 32} rows,
// cols grid columns per lane (2: FP32 with even nx only, else 1 is used).
template <typename T>
hipError_t launch_march(const StepArgs<T>& a, int ty, int cols, int batch, hipStream_t s);
template <typename T>
hipError_t graph_add_march(hipGraph_t g, hipGraphNode_t* node, hipGraphNode_t dep, const StepArgs<T>& a,
                           int ty, int cols, int batch);

// Two fused steps per launch in the register strip march (Euler, no
// variants), chunks of ty in {4, 8, 16} rows with ty dividing ny, one grid
// column per lane; a launch always advances two steps.
template <typename T>
hipError_t launch_march_k2(const StepArgs<T>& a, int ty, int batch, hipStream_t s);
template <typename T>
hipError_t graph_add_march_k2(hipGraph_t g, hipGraphNode_t* node, hipGraphNode_t dep, const StepArgs<T>& a,
                              int ty, int batch);

// Resident stepper: one launch advances FP32 grids by n >= 2 explicit Euler
// or midpoint steps with each 64 x th tile (th in {8, 16, 32}) held in LDS,
// trading 2-cell rims after every step through
// rim[2][tiles][3][resident_rim_words(th)] tagged words.  The tags of a
// launch are e0 + generation: e0 is passed by the host (below 2^30, top bit
// clear), or, for a launch captured in a graph (dev_epoch), read from the
// device epoch ctl[0] with the top bit set, and the launch's last
// workgroup (counted in ctl[2], zero between launches) advances ctl[0].
// ctl[1] is the sticky abort word.  In place: s.c == s.c_out etc.
// nx = 64 ntx, ny = th nty.
struct ResArgs {
    StepArgs<float> s;
    Coef<float> kh;      // midpoint: the half step's constants (dt / 2)
    uint64_t* rim;
    uint64_t* ctl;
    int n;
    int mid;             // 1: explicit midpoint steps (two rim trades per step)
    int batch, ntx, nty;
    uint32_t e0;         // host epoch (dev_epoch == 0)
    int dev_epoch;       // 1: tags from the device epoch (graph capture)
};
size_t resident_rim_words(int th);
// Tiles the device keeps co-resident for tile height th (occupancy of every
// instantiation times the compute units; 0 on a query error).
int resident_capacity(int th);
hipError_t launch_resident(const ResArgs& a, int th, hipStream_t s);

// Append one stepper launch as a kernel node of graph g after node dep
// (dep == nullptr: no dependency).
template <typename T>
hipError_t graph_add_step(hipGraph_t g, hipGraphNode_t* node, hipGraphNode_t dep,
                          const StepArgs<T>& a, int k, int batch);

// Seeded initial condition.
struct InitArgs {
    uint64_t seed;
    int nx, ny;
    double h, c_noise, H0, width, rho_in;
    const double* c0;    // [B] device
};
template <typename T>
hipError_t launch_init(T* c, T* phi, T* rho, const InitArgs& a, int batch, hipStream_t s);

// Qcol[b][i] = (i == 0 ? q[b] : 0)  (q == nullptr: all zero)
hipError_t launch_set_inflow(double* Qcol, const double* q, int nx, int batch, hipStream_t s);

// Diagnostics: out[b*5 + {0..4}] = h^2 sum c, h^2 sum phi, h^2 sum rho, Q, F_h;
// with Qcol == nullptr, out[b*4 + {0..3}] = h^2 sum c, h^2 sum phi, h^2 sum rho, F_h.
// One workgroup per band of rows x chunk of columns; the partition depends on
// the grid's shape and precision only (not on the device), so the FP64 sums
// are taken in one fixed order.
struct RedArgs {
    int nx, ny, pvd;
    double h2, Wc, Wphi, half_kc, half_kp;
};
struct RedGeo {
    int vec;       // elements per 16-byte load (4 FP32, 2 FP64), 1 when nx is not a multiple
    int chunks;    // column chunks of 256 vec columns
    int rows;      // rows per band
    int bands;     // bands per realisation
    int parts() const { return chunks * bands; }
};
RedGeo reduce_geometry(int nx, int ny, int batch, int elem_bytes);
template <typename T>
hipError_t launch_reduce(const T* c, const T* phi, const T* rho, const double* Qcol,
                         double* partials, double* out, const RedArgs& a, const RedGeo& g, int batch,
                         hipStream_t s);

// Discrete adjoint of one step: lambda_out = lambda_in + (dR/du)^T dt lambda_in
// at the state (c, phi, rho); per-cell FP64 parameter gradients accumulate in
// gacc[2][B][ny][nx] (dM_scale, dv0); one launch, no other scratch memory.
template <typename T>
struct AdjointIO {
    const T* c;
    const T* phi;
    const T* rho;
    const T* lc;
    const T* lp;
    const T* lr;
    T* oc;
    T* op;
    T* orr;
    double* gacc;
};
template <typename T>
hipError_t launch_adjoint(const AdjointIO<T>& io, const StepArgs<T>& st, double Mscale, double cos_th,
                          double msin_th, double h, int batch, hipStream_t s);
hipError_t launch_gacc_zero(double* gacc, size_t n, hipStream_t s);
hipError_t launch_gacc_sum(const double* gacc, double* out, size_t cells_per, int batch, hipStream_t s);

}  // namespace pfk
