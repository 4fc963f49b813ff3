/*
 * CPU FP64 oracle of the explicit step of the PVD phase-field model
 * (Materials and Methods, "Phase-field modeling of physical vapor
 * deposition"; the three evolution equations for c, phi and rho).
 *
 * TEST INFRASTRUCTURE ONLY.  This code exists to check the GPU library.
 * Only the test suite, the smoke check and the CPU-baseline leg of the
 * benchmark may load it; the product path never does.  It shares no code,
 * header, table or constant with the GPU library.
 *
 * Everything is double precision, single realisation at a time, plain
 * loops over cells in the order the equations state them.  Fields are
 * stored [batch][ny][nx], x fastest; x is periodic; j = 0 is next to the
 * substrate and j = ny-1 next to the vapour inlet.
 */
#ifndef PF_ORACLE_H
#define PF_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum { OR_BC_PVD = 0, OR_BC_PERIODIC = 1 };
enum { OR_EULER = 0, OR_MIDPOINT = 1 };

typedef struct or_params {
    int32_t nx, ny, batch;
    int32_t bc_mode;   /* OR_BC_PVD or OR_BC_PERIODIC */
    int32_t flux_on;   /* 0: incident vapour velocity v = 0 */
    int32_t integrator; /* OR_EULER or OR_MIDPOINT */
    uint64_t seed;
    double h, dt;
    /* free energy: double wells and gradient energies */
    double W_c, W_phi, kappa_c, kappa_phi;
    /* composition mobility M_c(phi, c) and order-parameter mobility */
    double MA_bulk, MB_bulk, MA_surf, MB_surf, sigma_surf, M_phi, M_scale;
    /* vapour transport */
    double D_rho, v0, theta_deg, rho_in;
    /* initial condition */
    double c0, c_noise, film_h;
    /* standard deviation of the interface composition draw (0: off) */
    double interface_noise;
} or_params;

/* Frozen-coefficient explicit-Euler stability bound; vmax is the largest
 * incident speed over the batch.  Returns 0, or -1 on bad parameters. */
int or_dt_limit(const or_params* p, double vmax, double* dt_lim);

/* SplitMix64: the (n+1)-th output of the generator started at `seed`. */
uint64_t or_splitmix64(uint64_t seed, uint64_t n);

/* Seeded initial condition for every realisation.  c0_per: [batch] mean
 * compositions, or NULL for p->c0. */
void or_init(const or_params* p, const double* c0_per,
             double* c, double* phi, double* rho);

/* Chemical potentials and composition mobility of one realisation. */
void or_potentials(const or_params* p, const double* c, const double* phi,
                   double* mu_c, double* mu_phi, double* Mc);

/* n steps of every realisation, in place.  v0_per, c0_per: [batch]
 * incident speeds and mean compositions, or NULL for p->v0, p->c0.  step0:
 * global index of the first step (keys the interface composition draws).
 * Q: [batch] cumulative inflow. */
void or_step_n(const or_params* p, const double* v0_per, const double* c0_per, int64_t step0,
               int64_t n, double* c, double* phi, double* rho, double* Q);

/* The interface composition draw (see pf_oracle.c). */
double or_trunc_gauss(uint64_t seed, uint64_t counter0, double mean, double sigma);

/* out[b][4] = h^2 sum c, h^2 sum phi, h^2 sum rho, Q[b]. */
void or_mass(const or_params* p, const double* c, const double* phi,
             const double* rho, const double* Q, double* out);

/* out[b] = discrete free energy F_h of realisation b. */
void or_energy(const or_params* p, const double* c, const double* phi,
               double* out);

/* ------------------------------------------------------------- adjoint
 * Discrete adjoint of one explicit Euler step u' = u + dt R(u; M_scale, v0)
 * of one realisation.  On entry (lc, lphi, lrho) hold lambda' = dL/du'; on
 * exit they hold dL/du = lambda' + (dR/du)^T (dt lambda').  g[0] and g[1]
 * receive += dt lambda'.(dR/dM_scale) and += dt lambda'.(dR/dv0), at fixed
 * dt.  (c, phi, rho) is the state u the step started from. */
void or_adjoint_step(const or_params* p, double v0, const double* c, const double* phi,
                     const double* rho, double* lc, double* lphi, double* lrho, double* g);

/* Loss L = h^2/2 sum over c, phi, rho of (u_n - u*)^2 after n steps of one
 * realisation from (c, phi, rho), and its gradient with respect to M_scale
 * and v0 (fixed dt) by the adjoint with checkpoints every `every` steps and
 * recomputation.  out = {L, dL/dM_scale, dL/dv0}.  The inputs are not
 * modified.  Explicit Euler without interface draws only (else NaN). */
void or_loss_grad(const or_params* p, double v0, int64_t n, int64_t every,
                  const double* c, const double* phi, const double* rho,
                  const double* ct, const double* phit, const double* rhot, double* out);

#ifdef __cplusplus
}
#endif
#endif
