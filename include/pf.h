/*
 * pf.h - C ABI of the MI355X (gfx950) explicit PVD phase-field stepper.
 *
 * The library advances the phase-field model of physical vapour deposition
 * stated in the paper's Materials and Methods ("Phase-field modeling of
 * physical vapor deposition"): a Cahn-Hilliard equation for the composition
 * c with mobility M_c = M^Bulk + M^Surf, a Cahn-Hilliard equation with the
 * deposition source S = grad(phi).(rho v) for the order parameter phi
 * (solid +1, vapour -1), and convection-diffusion of the vapour density rho
 * with the matching sink -S.  Spatial derivatives are second-order central
 * differences (Materials and Methods, "Dataset"); time stepping is explicit
 * Euler.  The readings where the paper defers to another reference or is
 * garbled (free energy, switching function, surface mobility, boundary
 * conditions, stability limit) are listed with the parameter struct below.
 *
 * Memory: all field buffers are caller-owned device memory (for example
 * torch tensors), contiguous [batch][ny][nx] with x fastest, element type
 * float (PF_F32) or double (PF_F64), 16-byte aligned, one realisation's
 * field below 2 GiB (nx*ny*sizeof < 2^31).  The caller also
 * provides a device workspace of pf_workspace_bytes() bytes, 256-byte
 * aligned.  The library never allocates or frees device memory; a handle
 * owns only host-side metadata.  All host arrays passed in are read during
 * the call and not retained.
 *
 * Streams: every device operation of a handle is enqueued on the stream
 * given to pf_init (a hipStream_t passed as void*; NULL is the default
 * stream).  pf_step_n returns without waiting; pf_mass and pf_energy wait
 * for the stream.  One handle per stream; a handle is not thread-safe.
 *
 * Errors: every int-returning call returns PF_OK (0) or a negative code.
 * Argument errors are detected before anything is enqueued.  No C++
 * exception crosses this interface.
 */
#ifndef PF_H
#define PF_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct pf_handle pf_handle;

enum pf_status {
    PF_OK = 0,
    PF_EINVAL = -1,      /* null/misaligned pointer, bad shape, bad enum, bad n */
    PF_EUNSTABLE = -2,   /* dt above the stability limit and allow_unstable == 0 */
    PF_ENONFINITE = -3,  /* a diagnostic came out NaN or infinite */
    PF_EDEVICE = -4,     /* a HIP call failed; see pf_last_hip_error */
    PF_EABORTED = -5,    /* the resident stepper gave up a wait for its neighbours (its tiles were
                            not all resident at once, e.g. another kernel held part of the device):
                            the state is NaN and the handle stays aborted until pf_init is called
                            again; reported by the next pf_mass, pf_energy or pf_get_inflow */
    PF_ESCRATCH = -6     /* pf_diagnostics_noalloc: the input needs more partial sums than its
                            static scratch holds (see pf_diagnostics_noalloc_limit) */
};

enum pf_precision { PF_F32 = 0, PF_F64 = 1 };
enum pf_bc { PF_BC_PVD = 0, PF_BC_PERIODIC = 1 };
enum pf_init_mode { PF_INIT_SEEDED = 0, PF_INIT_KEEP = 1 };
enum pf_integrator { PF_EULER = 0, PF_MIDPOINT = 1 };

/*
 * Problem definition.  Units are dimensionless, as in the paper's dataset.
 *
 * Model readings (the paper gives no expression for these):
 *   free energy density f = W_c p(phi) g(c) + (W_phi/4)(1 - phi^2)^2 with
 *     p(phi) = (2 - phi)(1 + phi)^2 / 4 and g(c) = c^2 (1 - c)^2, plus
 *     (kappa_c/2)|grad c|^2 + (kappa_phi/2)|grad phi|^2;
 *   M_c = M_scale [ p(phi~)(H MA_bulk + (1-H) MB_bulk)
 *                   + exp(-(phi~/sigma_surf)^2)(H MA_surf + (1-H) MB_surf) ]
 *     with H = x^3 (6x^2 - 15x + 10), x = clamp(c,0,1), phi~ = clamp(phi,-1,1)
 *     (the paper's M^Surf subtracts itself; that trailing term is dropped);
 *   phi mobility M_phi constant; face mobilities are arithmetic means;
 *   v = v0 (cos theta, -sin theta), theta in degrees from the substrate;
 *   PF_BC_PVD: x periodic; mirror ghosts for c and phi at the substrate
 *     (j = 0) and the top (j = ny-1); rho has no flux through the substrate
 *     and the fixed value rho_in above the top row (vapour inlet);
 *   PF_BC_PERIODIC: periodic in x and y, no inlet (a test mode).
 *
 * Model variants (Materials and Methods, "Dataset"; Introduction):
 *   integrator PF_MIDPOINT: the explicit midpoint method of the paper's
 *     solver, u' = u + dt R(u + dt/2 R(u)) (in the resident stepper where it
 *     runs, else two launches per step, the first into the workspace, the
 *     second in place); same stability limit;
 *   interface_noise > 0: the paper's random interface composition, read as:
 *     after every step each cell on the vapour side (phi' < 0) takes a
 *     fresh composition drawn from N(c0_b, interface_noise^2) truncated to
 *     [0, 1].  The draw is Box-Muller on SplitMix64 uniforms of the
 *     stream (seed + b) ^ 0x2B7E151628AED2A6, counters 16 (s nx ny + j nx + i)
 *     + 2a, + 2a + 1 for attempt a = 0..7 at global step s (pf_get_step),
 *     first draw inside [0, 1] kept, else c0_b; evaluated in the run's
 *     precision (FP32 runs: the hardware logarithm, square root and cosine,
 *     within ~3e-7 of the FP64 draw).
 *   Both variants run the resident stepper where it applies (below), else
 *   the single-step kernel (temporal_block 0 or 1); interface_noise then
 *   runs plain launches (no graph replay).
 */
/* Kernel of the launches that fuse several steps: a 64 x TY tile staged in
 * LDS (any K), the register strip march (K = 2: one wave per 64-column
 * strip, radius-4 halo, the intermediate state kept in registers), or the
 * resident stepper: one launch per pf_step_n call (of at least
 * 2 steps; a single step runs the single-step kernel) in which every
 * workgroup keeps a 64 x TY tile of the state in LDS for all the steps and
 * trades its 2-cell rim with its neighbours after each step (and each
 * midpoint half step) through the workspace.  The resident stepper needs
 * FP32, explicit Euler or the midpoint method (with or without interface
 * draws), temporal_block 0 or 1, nx a multiple of 64, a tile height
 * TY in {8, 16, 32} dividing ny (tile_rows, else the library's choice) and
 * a grid of at most 2^21 cells whose tiles the device can keep resident at
 * once (about 1M cells on MI355X); else pf_init returns PF_EINVAL.  Its
 * results are bitwise equal to the other kernels'.  A resident launch takes
 * every workgroup slot of the device for its duration: calls of several
 * handles on one device must not run concurrently on different streams
 * (a launch whose tiles cannot all be resident gives up after a bounded
 * wait and reports PF_EABORTED). */
enum pf_fused { PF_FUSED_AUTO = 0, PF_FUSED_TILE = 1, PF_FUSED_MARCH = 2, PF_FUSED_RESIDENT = 3 };

typedef struct pf_params {
    int32_t nx, ny, batch;        /* grid cells and independent realisations */
    int32_t precision;            /* pf_precision: storage and arithmetic type */
    int32_t bc_mode;              /* pf_bc */
    int32_t flux_on;              /* 0: v = 0 (no deposition, no advection) */
    int32_t init_mode;            /* pf_init_mode */
    int32_t allow_unstable;       /* 1: accept dt above the stability limit */
    int32_t temporal_block;       /* steps fused per launch: 1..4 (FP32), 1..2 (FP64); 0: library's
                                     choice by precision and grid size; lowered so that 2K <= ny */
    int32_t graph_mode;           /* 0: long runs replay a HIP graph of launches; 1: plain launches */
    int32_t tile_rows;            /* single-step kernel: rows per wave (4, 8, 16, 32); resident
                                     stepper: tile height (8, 16, 32; a height asked for with
                                     fused_kernel 0 keeps the strip-march kernels); 0: library's
                                     choice by grid size */
    int32_t integrator;           /* pf_integrator */
    uint64_t seed;                /* seeded initial condition: realisation b uses seed + b */
    double h;                     /* grid spacing */
    double dt;                    /* time step; <= 0 means dt_factor * stability limit */
    double dt_factor;             /* used when dt <= 0 (0.2 in the standard workloads) */
    double W_c, W_phi, kappa_c, kappa_phi;
    double MA_bulk, MB_bulk, MA_surf, MB_surf, sigma_surf, M_phi, M_scale;
    double D_rho, v0, theta_deg, rho_in;
    double c0, c_noise, film_h;   /* initial condition; film_h <= 0 means ny h / 8 */
    const double* v0_per;         /* host [batch] incident speeds, or NULL for v0 */
    const double* c0_per;         /* host [batch] mean compositions, or NULL for c0 */
    double interface_noise;       /* standard deviation of the interface draw, 0..1; 0: off */
    int32_t lane_cols;            /* single-step FP32 kernel: grid columns per lane, 1 or 2 (2 needs
                                     an even nx; else 1 is used); 0: library's choice */
    int32_t fused_kernel;         /* pf_fused: kernel of launches that fuse steps (temporal_block
                                     > 1); PF_FUSED_MARCH fuses exactly 2, with tile_rows (4, 8 or 16,
                                     dividing ny; else 8 or 4) rows per wave; PF_FUSED_RESIDENT: the
                                     resident stepper (conditions above); 0: library's choice */
} pf_params;

/* Bytes of device workspace a handle for *p needs (ping-pong copy of the
 * state, per-column FP64 inflow accumulators, per-realisation constants,
 * FP64 reduction partials and, for grids the resident stepper may run, its
 * rim buffers: 2 x tiles x 3 x (256 + 4 TY) 8-byte words).  Returns 0 if *p
 * is invalid. */
size_t pf_workspace_bytes(const pf_params* p);

/* Explicit-Euler stability limit of *p on the host, in FP64:
 * min(dt_c, dt_phi, dt_rho, dt_adv) of the frozen-coefficient von Neumann
 * bounds with the 5-point symbol at most 8/h^2 (see the model readings).
 * The largest of v0 / v0_per enters dt_adv.  PF_EINVAL on bad input. */
int pf_dt_limit(const pf_params* p, double* dt_lim);

/* Paper: Materials and Methods, "Phase-field modeling of physical vapor
 * deposition" (the three fields c, phi, rho of a film growing from a flat
 * substrate under an incoming vapour flux) and "Dataset" (seeded initial
 * compositions around c0, a uniform 2-D grid).
 * Create a handle that steps the caller's buffers c, phi, rho in place.
 * PF_INIT_SEEDED writes the seeded initial condition (c = c0 + c_noise
 * (2U - 1) from SplitMix64, a flat tanh film of height film_h, rho =
 * rho_in (1 - phi)/2); PF_INIT_KEEP takes the buffers' contents as the
 * initial condition.  The inflow accumulators and the step counter start at
 * zero.  workspace_bytes must be at least pf_workspace_bytes(p).  On
 * success *out receives a handle to release with pf_destroy. */
int pf_init(pf_handle** out, const pf_params* p, void* c, void* phi, void* rho,
            void* workspace, size_t workspace_bytes, void* stream);

/* Paper: Materials and Methods, "Phase-field modeling of physical vapor
 * deposition" (the Cahn-Hilliard equation of c with the mobility
 * M_c = M^Bulk + M^Surf, that of phi with the deposition source S, and the
 * convection-diffusion of rho with the sink -S) discretised as "Dataset"
 * states (second-order central differences; explicit time stepping, the
 * paper's midpoint method as PF_MIDPOINT).
 * Enqueue n >= 0 steps (the handle's integrator) of every realisation.
 * When the stream reaches the end of this work, the new state is in the
 * caller's buffers.  Returns without waiting.  A call may be captured into
 * a HIP graph: each replay advances the state it finds by n steps (the
 * step counter of pf_get_step counts enqueued calls only).  With
 * interface_noise > 0 the draws are keyed by the global step at which the
 * call starts, which a replay would repeat, so a call on a capturing
 * stream returns PF_EINVAL and enqueues nothing. */
int pf_step_n(pf_handle* h, int64_t n);

/* One explicit Euler step (the handle's model and dt) from the state (c,
 * phi, rho) into (c_out, phi_out, rho_out): device buffers with the state's
 * layout and precision, the outputs distinct from the inputs.  The handle's
 * own buffers, inflow accumulators and step counter are untouched (no
 * inflow is accumulated).  For recomputing the states of a checkpointed
 * reverse sweep without copies.  Enqueued; PF_EINVAL for a midpoint or
 * interface-draw handle.  Paper: as pf_step_n. */
int pf_step_out(pf_handle* h, const void* c, const void* phi, const void* rho,
                void* c_out, void* phi_out, void* rho_out);

/* Paper: the conservation form of the c and phi equations in Materials and
 * Methods (masses change only through the deposition flux, which the
 * inflow Q accounts for).
 * Wait for the stream, then write out[4*b + k] for each realisation b:
 * k = 0..2 the masses h^2 sum c, h^2 sum phi, h^2 sum rho, and k = 3 the
 * cumulative vapour inflow Q through the top face.  Sums are accumulated in
 * FP64 in a fixed order (deterministic).  PF_ENONFINITE if any is not
 * finite. */
int pf_mass(pf_handle* h, double* out);

/* Paper: the free-energy functional the chemical potentials derive from
 * (Materials and Methods, "Phase-field modeling of physical vapor
 * deposition"; its double-well and gradient terms as read above).
 * Wait for the stream, then write out[b] = discrete free energy
 * F_h = h^2 sum f(c, phi) + (kappa_c/2) sum_faces (dc)^2
 *       + (kappa_phi/2) sum_faces (dphi)^2 in FP64 (all x faces, interior y
 * faces, plus the wrap faces in PF_BC_PERIODIC).  PF_ENONFINITE if any is
 * not finite. */
int pf_energy(pf_handle* h, double* out);

/* Step counter and time step of a handle (resume support). */
int pf_get_step(const pf_handle* h, int64_t* step);
int pf_set_step(pf_handle* h, int64_t step);
int pf_get_dt(const pf_handle* h, double* dt);

/* Cumulative inflow per realisation: pf_get_inflow waits for the stream and
 * writes Q[b]; pf_set_inflow enqueues Q[b] as the new cumulative value. */
int pf_get_inflow(pf_handle* h, double* Q);
int pf_set_inflow(pf_handle* h, const double* Q);

/* Release a handle (host memory only; the caller's buffers are untouched). */
void pf_destroy(pf_handle* h);

/* Launch shape a handle uses: steps fused per launch (1: single-step
 * strip-march kernel or the resident stepper, which exchanges rims after
 * every step; 2..4: LDS-tiled kernel or register march) and rows per wave /
 * tile. */
int pf_get_launch(const pf_handle* h, int32_t* temporal_block, int32_t* tile_rows);

/* Grid columns per lane of the single-step kernel the handle launches (1 or
 * 2; 1 whenever temporal_block > 1).  PF_EINVAL on a null argument. */
int pf_get_lane_cols(const pf_handle* h, int32_t* lane_cols);

/* pf_fused kind of the handle's fused launches (PF_FUSED_TILE,
 * PF_FUSED_MARCH or PF_FUSED_RESIDENT; 0 when each launch is one step).
 * PF_EINVAL on a null argument. */
int pf_get_fused_kernel(const pf_handle* h, int32_t* kind);

/* ------------------------------------------------------------------ adjoint
 * Discrete adjoint of the explicit step, for gradients of a loss of the
 * final state with respect to the mobility scale M_scale and the deposition
 * rate v0 at fixed dt (the inverse-design use the paper's Discussion names).
 * For one step u' = u + dt R(u; M_scale, v0) started from the state
 * (c, phi, rho), pf_adjoint_step writes lambda = lambda' + (dR/du)^T
 * (dt lambda') into out_* given lambda' = dL/du' in lam_*, and adds
 * dt lambda'.dR/dM_scale and dt lambda'.dR/dv0 per cell into FP64
 * accumulators in the adjoint workspace.  All arrays are device buffers with
 * the state's layout and precision; out_* must not alias lam_*.  The handle
 * supplies the model, dt and the stream (enqueued, returns at once).
 * M_scale must be positive.  A checkpointed reverse sweep calls it once per
 * step, from the last step to the first, on recomputed states.  The adjoint
 * exists for explicit Euler without interface draws only: for a handle with
 * integrator PF_MIDPOINT or interface_noise > 0 the adjoint calls return
 * PF_EINVAL and pf_adjoint_workspace_bytes returns 0. */
size_t pf_adjoint_workspace_bytes(const pf_params* p);
int pf_adjoint_step(pf_handle* h, const void* c, const void* phi, const void* rho,
                    const void* lam_c, const void* lam_phi, const void* lam_rho,
                    void* out_c, void* out_phi, void* out_rho,
                    void* adj_workspace, size_t adj_bytes);
/* One checkpoint segment of that reverse sweep in a single call (the same
 * launches, in the same order, as the per-step calls; no host round trip
 * per step).  ring holds len >= 1 states in the state's precision, laid out
 * [len][3][batch][ny][nx] (slot t = c, phi, rho after t steps of the
 * segment); slot 0 is the caller's checkpoint and slots 1 .. len-1 are
 * written here by pf_step_out.  Then for t = len-1 .. 0 it calls
 * pf_adjoint_step on slot t with the two lambda buffers (lam_*, tmp_*)
 * taking turns as input and output, starting from lam_*.  On return
 * *in_tmp is 1 when the adjoint of the segment's first state is in tmp_*
 * (odd len), else 0 (in lam_*).  The ring belongs to the caller; it must
 * not overlap the lambda buffers.  Errors as pf_step_out and
 * pf_adjoint_step (PF_EINVAL on bad arguments; enqueued, returns at once). */
int pf_adjoint_segment(pf_handle* h, void* ring, int64_t len, void* lam_c, void* lam_phi, void* lam_rho,
                       void* tmp_c, void* tmp_phi, void* tmp_rho, void* adj_workspace, size_t adj_bytes,
                       int32_t* in_tmp);
/* The two halves of pf_adjoint_segment, for callers that overlap the
 * recomputation of one segment with the adjoint steps of another (two
 * handles of the same parameters on two streams, two rings, events between
 * them).  pf_adjoint_recompute writes slots 1 .. len-1 of ring from slot 0
 * by pf_step_out on h's stream.  pf_adjoint_sweep runs the adjoint steps
 * t = len-1 .. 0 over a ring that holds the segment's states, with the
 * lambda buffers and *in_tmp as in pf_adjoint_segment.  Same layouts,
 * ownership and errors as pf_adjoint_segment; both are enqueued and return
 * at once.  pf_adjoint_segment is the recompute followed by the sweep. */
int pf_adjoint_recompute(pf_handle* h, void* ring, int64_t len);
int pf_adjoint_sweep(pf_handle* h, void* ring, int64_t len, void* lam_c, void* lam_phi, void* lam_rho,
                     void* tmp_c, void* tmp_phi, void* tmp_rho, void* adj_workspace, size_t adj_bytes,
                     int32_t* in_tmp);
/* Zero the parameter-gradient accumulators (enqueued). */
int pf_adjoint_reset(pf_handle* h, void* adj_workspace, size_t adj_bytes);
/* Wait for the stream and write out[2*b] = dL/dM_scale, out[2*b+1] = dL/dv0
 * of realisation b, summed in FP64 in a fixed order. */
int pf_adjoint_grad(pf_handle* h, void* adj_workspace, size_t adj_bytes, double* out);

/* ------------------------------------------------ allocation-free variant
 * For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the
 * diagnostics of pf_mass and pf_energy for caller-given fields, with no
 * handle and no workspace.  c, phi, rho: device buffers laid out as for
 * pf_init ([batch][ny][nx], precision per p->precision, 16-byte aligned);
 * out: a device array of batch x 4 doubles that receives, per realisation
 * b, out[4*b + 0..2] = h^2 sum c, h^2 sum phi, h^2 sum rho and out[4*b + 3]
 * = F_h, the same values pf_mass and pf_energy report for these fields
 * (same kernels, same fixed summation order; no inflow, which is handle
 * state).  Enqueued on `stream` (a hipStream_t of the current device, or
 * NULL), returns without waiting; nothing is allocated or freed.  The
 * partial sums live in a static device array of
 * pf_diagnostics_noalloc_limit() bytes (1 MiB) that each GPU the library
 * runs on holds until the process ends, found on the first call on a
 * device.  Every call on a GPU shares that GPU's array (it holds the last
 * call's partials; nothing in it needs clearing): calls that overlap on one
 * GPU (different streams, or host threads) race.  Returns PF_EINVAL on a
 * bad argument or a stream of another device, PF_ESCRATCH when batch x the
 * partial count (about 2048 per launch) needs more than the array, and
 * PF_EDEVICE on a HIP error. */
int pf_diagnostics_noalloc(const pf_params* p, const void* c, const void* phi, const void* rho,
                           double* out, void* stream);
size_t pf_diagnostics_noalloc_limit(void);

/* Text of a pf_status code. */
const char* pf_strerror(int code);

/* Last HIP error code recorded by the handle (0 if none). */
int pf_last_hip_error(const pf_handle* h);

#ifdef __cplusplus
}
#endif
#endif
