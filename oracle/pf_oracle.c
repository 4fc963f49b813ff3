/*
 * CPU FP64 oracle of the explicit PVD phase-field step.
 *
 * TEST INFRASTRUCTURE ONLY: loaded by the test suite, the smoke check and
 * the CPU-baseline leg of the benchmark, never by the product path.  It
 * shares no code with the GPU library.
 *
 * The model is the one of Materials and Methods, "Phase-field modeling of
 * physical vapor deposition":
 *   dc/dt   = div( M_c(phi,c) grad dF/dc )                     (composition)
 *   dphi/dt = div( M(phi) grad dF/dphi ) + S,  S = grad(phi).(rho v)
 *   drho/dt = div( D grad rho ) - div(rho v) - grad(phi).(rho v)
 * with M_c = M^Bulk + M^Surf as given there, discretised with second-order
 * central differences (Dataset section) on a uniform cell-centred grid.
 * Where the paper defers to another reference or is garbled, the readings
 * used are (each is a choice, not the paper's text):
 *   - free energy density f = W_c p(phi) g(c) + (W_phi/4)(1-phi^2)^2 with
 *     p(phi) = (2-phi)(1+phi)^2/4 (the bulk-mobility prefactor) and
 *     g(c) = c^2 (1-c)^2, plus gradient energies (kappa/2)|grad u|^2;
 *   - switching function h(c) = c^3 (6c^2 - 15c + 10) on c clamped to [0,1];
 *   - the surface mobility drops the self-referential trailing term;
 *   - M(phi) = M_phi constant; face mobilities are arithmetic means;
 *   - time integration: explicit Euler (every right-hand side uses the old
 *     state), or the explicit midpoint method the paper's solver uses
 *     (u' = u + dt R(u + dt/2 R(u)));
 *   - random interface composition (the paper's truncated-Gaussian
 *     boundary condition at the interface), when interface_noise > 0:
 *     after every step each cell on the vapour side (phi' < 0) takes a
 *     fresh composition drawn from N(c0, interface_noise^2) truncated to
 *     [0, 1] (Box-Muller on SplitMix64 uniforms, rejection);
 *   - boundaries: x periodic; at y = 0 and y = top, mirror ghosts for c,
 *     phi and the potentials (no diffusive flux); rho has no flux through
 *     the substrate and a fixed inlet density rho_in as its top ghost;
 *   - v = v0 (cos theta, -sin theta), theta measured from the substrate.
 *
 * Parity with the paper itself is unpinned: the paper prints no worked
 * example of the step.  The test suite pins this file to closed forms,
 * invariants and an independent dense assembly on small grids.
 */
#include "pf_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

/* ---------------------------------------------------------------- helpers */

static int imod(int i, int n)
{
    int r = i % n;
    return r < 0 ? r + n : r;
}

/* Row index of the y-neighbour j (j may be -1 or ny) of a field with
 * mirror ghosts in the PVD mode, or wrapped in the periodic mode. */
static int yrow(const or_params* p, int j)
{
    if (p->bc_mode == OR_BC_PERIODIC) return imod(j, p->ny);
    if (j < 0) return 0;
    if (j >= p->ny) return p->ny - 1;
    return j;
}

static double at(const or_params* p, const double* u, int i, int j)
{
    return u[(size_t)yrow(p, j) * p->nx + imod(i, p->nx)];
}

/* rho with its own boundary rule: mirror at the substrate, rho_in above
 * the top row (PVD); wrapped (periodic). */
static double rho_at(const or_params* p, const double* r, int i, int j)
{
    if (p->bc_mode == OR_BC_PVD && j >= p->ny) return p->rho_in;
    return at(p, r, i, j);
}

/* Five-point Laplacian of u at cell (i, j). */
static double lap5(const or_params* p, const double* u, int i, int j)
{
    double s = at(p, u, i + 1, j) + at(p, u, i - 1, j)
             + at(p, u, i, j + 1) + at(p, u, i, j - 1) - 4.0 * u[(size_t)j * p->nx + i];
    return s / (p->h * p->h);
}

static double clampd(double x, double lo, double hi)
{
    return x < lo ? lo : (x > hi ? hi : x);
}

/* solid indicator p(phi) = (2 - phi)(1 + phi)^2 / 4 and its derivative */
static double pfun(double phi) { return 0.25 * (2.0 - phi) * (1.0 + phi) * (1.0 + phi); }
static double dpfun(double phi) { return 0.75 * (1.0 - phi * phi); }
/* double well in c: g = c^2 (1-c)^2, g' = 2 c (1-c)(1-2c) */
static double gfun(double c) { return c * c * (1.0 - c) * (1.0 - c); }
static double dgfun(double c) { return 2.0 * c * (1.0 - c) * (1.0 - 2.0 * c); }
/* smooth switching function on the clamped composition */
static double hswitch(double c)
{
    double x = clampd(c, 0.0, 1.0);
    return x * x * x * (6.0 * x * x - 15.0 * x + 10.0);
}

/* M_c = M^Bulk + M^Surf, scaled by M_scale (reading: clamped arguments). */
static double mobility_c(const or_params* p, double c, double phi)
{
    double ph = clampd(phi, -1.0, 1.0);
    double H = hswitch(c);
    double bulk = pfun(ph) * (H * p->MA_bulk + (1.0 - H) * p->MB_bulk);
    double q = ph / p->sigma_surf;
    double surf = exp(-q * q) * (H * p->MA_surf + (1.0 - H) * p->MB_surf);
    return p->M_scale * (bulk + surf);
}

static void velocity(const or_params* p, double v0, double* vx, double* vy)
{
    if (!p->flux_on) { *vx = 0.0; *vy = 0.0; return; }
    double th = p->theta_deg * (3.14159265358979323846 / 180.0);
    *vx = v0 * cos(th);
    *vy = -v0 * sin(th);
}

/* ------------------------------------------------------------ public API */

uint64_t or_splitmix64(uint64_t seed, uint64_t n)
{
    /* Steele, Lea & Flood (2014): state advances by the golden gamma and
     * each output is the state passed through the variant-13 finaliser. */
    uint64_t z = seed + (n + 1u) * 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

int or_dt_limit(const or_params* p, double vmax, double* dt_lim)
{
    if (!p || !dt_lim || !(p->h > 0.0)) return -1;
    double h2 = p->h * p->h, h4 = h2 * h2;
    /* largest composition mobility: p <= 1 and exp(.) <= 1 */
    double mmax = p->M_scale * (fmax(p->MA_bulk, p->MB_bulk) + fmax(p->MA_surf, p->MB_surf));
    /* largest curvatures: |g''| <= 2 on [0,1]; |p''| g <= 3/32; the
     * phi double well's curvature is at most 2 W_phi; the 5-point symbol
     * is at most 8/h^2 */
    double lim = INFINITY;
    if (mmax > 0.0) {
        double dtc = 2.0 * h4 / (8.0 * mmax * (2.0 * p->W_c * h2 + 8.0 * p->kappa_c));
        lim = fmin(lim, dtc);
    }
    if (p->M_phi > 0.0) {
        double dtp = 2.0 * h4 / (8.0 * p->M_phi * ((2.0 * p->W_phi + 3.0 * p->W_c / 32.0) * h2
                                                   + 8.0 * p->kappa_phi));
        lim = fmin(lim, dtp);
    }
    if (p->D_rho > 0.0) lim = fmin(lim, h2 / (4.0 * p->D_rho));
    if (p->flux_on && vmax > 0.0) {
        if (p->D_rho > 0.0) lim = fmin(lim, 2.0 * p->D_rho / (vmax * vmax));
        else lim = fmin(lim, p->h / vmax);
    }
    if (!(lim > 0.0) || isinf(lim)) return -1;
    *dt_lim = lim;
    return 0;
}

void or_init(const or_params* p, const double* c0_per,
             double* c, double* phi, double* rho)
{
    int nx = p->nx, ny = p->ny;
    double H0 = p->film_h > 0.0 ? p->film_h : ny * p->h / 8.0;
    double width = sqrt(2.0 * p->kappa_phi / p->W_phi);
    for (int b = 0; b < p->batch; ++b) {
        double cb = c0_per ? c0_per[b] : p->c0;
        for (int j = 0; j < ny; ++j) {
            double y = (j + 0.5) * p->h;
            double ph = tanh((H0 - y) / width);
            for (int i = 0; i < nx; ++i) {
                size_t k = ((size_t)b * ny + j) * nx + i;
                /* realisation b draws from the stream of seed + b, counter
                 * j*nx + i, so it equals a single run with that seed */
                uint64_t u = or_splitmix64(p->seed + (uint64_t)b, (uint64_t)j * nx + i);
                double U = (double)(u >> 11) * 0x1.0p-53;
                c[k] = cb + p->c_noise * (2.0 * U - 1.0);
                phi[k] = ph;
                rho[k] = p->rho_in * (1.0 - ph) / 2.0;
            }
        }
    }
}

void or_potentials(const or_params* p, const double* c, const double* phi,
                   double* mu_c, double* mu_phi, double* Mc)
{
    int nx = p->nx, ny = p->ny;
#pragma omp parallel for schedule(static)
    for (int j = 0; j < ny; ++j) {
        for (int i = 0; i < nx; ++i) {
            size_t k = (size_t)j * nx + i;
            double cc = c[k], pp = phi[k];
            /* mu_c = dF/dc, mu_phi = dF/dphi */
            mu_c[k] = p->W_c * pfun(pp) * dgfun(cc) - p->kappa_c * lap5(p, c, i, j);
            mu_phi[k] = p->W_c * dpfun(pp) * gfun(cc)
                      - p->W_phi * pp * (1.0 - pp * pp)
                      - p->kappa_phi * lap5(p, phi, i, j);
            Mc[k] = mobility_c(p, cc, pp);
        }
    }
}

/* Right-hand side R(u) of one realisation: (Rc, Rp, Rr) per cell and the
 * inflow rate through the top face (per unit time). */
static void rhs(const or_params* p, double v0, const double* c, const double* phi,
                const double* rho, double* mu_c, double* mu_phi, double* Mc,
                double* Rc, double* Rp, double* Rr, double* inflow_rate)
{
    int nx = p->nx, ny = p->ny;
    double h = p->h, h2 = h * h;
    double vx, vy;
    velocity(p, v0, &vx, &vy);
    int pvd = p->bc_mode == OR_BC_PVD;

    or_potentials(p, c, phi, mu_c, mu_phi, Mc);

#pragma omp parallel for schedule(static)
    for (int j = 0; j < ny; ++j) {
        for (int i = 0; i < nx; ++i) {
            size_t k = (size_t)j * nx + i;
            /* composition: flux-form divergence with face-averaged mobility */
            double m0 = Mc[k], u0 = mu_c[k];
            const int di[4] = {1, -1, 0, 0}, dj[4] = {0, 0, 1, -1};
            double div_c = 0.0;
            for (int q = 0; q < 4; ++q) {
                double mn = at(p, Mc, i + di[q], j + dj[q]);
                double un = at(p, mu_c, i + di[q], j + dj[q]);
                div_c += 0.5 * (m0 + mn) * (un - u0);
            }
            div_c /= h2;

            /* order parameter: constant mobility times Laplacian of mu_phi */
            double div_p = p->M_phi * lap5(p, mu_phi, i, j);

            /* deposition source S = grad(phi) . (rho v), central differences */
            double r0 = rho[k];
            double dphx = (at(p, phi, i + 1, j) - at(p, phi, i - 1, j)) / (2.0 * h);
            double dphy = (at(p, phi, i, j + 1) - at(p, phi, i, j - 1)) / (2.0 * h);
            double S = r0 * (vx * dphx + vy * dphy);

            /* vapour: diffusion plus central face fluxes of rho v */
            double rE = rho_at(p, rho, i + 1, j), rW = rho_at(p, rho, i - 1, j);
            double rN = rho_at(p, rho, i, j + 1), rS = rho_at(p, rho, i, j - 1);
            double lap_r = (rE + rW + rN + rS - 4.0 * r0) / h2;
            double Fe = vx * 0.5 * (r0 + rE), Fw = vx * 0.5 * (rW + r0);
            double Gn = vy * 0.5 * (r0 + rN);
            double Gs = (pvd && j == 0) ? 0.0 : vy * 0.5 * (rS + r0);
            double T = p->D_rho * lap_r - ((Fe - Fw) + (Gn - Gs)) / h;

            Rc[k] = div_c;
            Rp[k] = div_p + S;
            Rr[k] = T - S;
        }
    }

    /* inflow through the top face: advective plus diffusive flux of rho
     * per unit length, summed over the top cells (times h: per unit time) */
    *inflow_rate = 0.0;
    if (pvd) {
        int j = ny - 1;
        double acc = 0.0;
        for (int i = 0; i < nx; ++i) {
            double r0 = rho[(size_t)j * nx + i];
            double Gn = vy * 0.5 * (r0 + p->rho_in);
            acc += -Gn + p->D_rho * (p->rho_in - r0) / h;
        }
        *inflow_rate = acc;
    }
}

/* key of the interface-composition stream (first digits of e) */
#define OR_NOISE_KEY 0x2B7E151628AED2A6ull

/* Composition drawn from N(mean, sigma^2) truncated to [0, 1]: Box-Muller
 * on pairs of SplitMix64 uniforms (53 bits; the first in (0, 1], the second
 * in [0, 1)) of the stream `seed`, counters 2a and 2a + 1 of attempt a from
 * `counter0`, the first draw inside [0, 1] taken; after 8 misses, mean. */
double or_trunc_gauss(uint64_t seed, uint64_t counter0, double mean, double sigma)
{
    for (int a = 0; a < 8; ++a) {
        uint64_t x1 = or_splitmix64(seed, counter0 + 2u * (uint64_t)a);
        uint64_t x2 = or_splitmix64(seed, counter0 + 2u * (uint64_t)a + 1u);
        double u1 = (double)((x1 >> 11) + 1u) * 0x1.0p-53;
        double u2 = (double)(x2 >> 11) * 0x1.0p-53;
        double z = sqrt(-2.0 * log(u1)) * cos(2.0 * 3.14159265358979323846 * u2);
        double v = mean + sigma * z;
        if (v >= 0.0 && v <= 1.0) return v;
    }
    return mean;
}

/* One step of one realisation (integrator as p->integrator), then the
 * interface composition draw for global step index `step`. */
static void step_one(const or_params* p, double v0, double c0, int b, int64_t step,
                     double* c, double* phi, double* rho, double* Q, double* w)
{
    int nx = p->nx, ny = p->ny;
    size_t n = (size_t)nx * ny;
    double dt = p->dt;
    double *mu_c = w, *mu_phi = w + n, *Mc = w + 2 * n;
    double *Rc = w + 3 * n, *Rp = w + 4 * n, *Rr = w + 5 * n;
    double *ch = w + 6 * n, *ph = w + 7 * n, *rh = w + 8 * n;
    double rate;

    rhs(p, v0, c, phi, rho, mu_c, mu_phi, Mc, Rc, Rp, Rr, &rate);
    if (p->integrator == OR_MIDPOINT) {
        /* half step to t + dt/2, then the full step with the rates there */
        for (size_t k = 0; k < n; ++k) {
            ch[k] = c[k] + 0.5 * dt * Rc[k];
            ph[k] = phi[k] + 0.5 * dt * Rp[k];
            rh[k] = rho[k] + 0.5 * dt * Rr[k];
        }
        rhs(p, v0, ch, ph, rh, mu_c, mu_phi, Mc, Rc, Rp, Rr, &rate);
    }
    for (size_t k = 0; k < n; ++k) {
        c[k] = c[k] + dt * Rc[k];
        phi[k] = phi[k] + dt * Rp[k];
        rho[k] = rho[k] + dt * Rr[k];
    }
    *Q += dt * p->h * rate;

    if (p->interface_noise > 0.0) {
        uint64_t seed = (p->seed + (uint64_t)b) ^ OR_NOISE_KEY;
        for (size_t k = 0; k < n; ++k)
            if (phi[k] < 0.0)
                c[k] = or_trunc_gauss(seed, ((uint64_t)step * n + k) * 16u, c0, p->interface_noise);
    }
}

void or_step_n(const or_params* p, const double* v0_per, const double* c0_per, int64_t step0,
               int64_t n, double* c, double* phi, double* rho, double* Q)
{
    size_t cells = (size_t)p->nx * p->ny;
    double* buf = (double*)malloc(9 * cells * sizeof(double));
    if (!buf) abort();
    for (int b = 0; b < p->batch; ++b) {
        double v0 = v0_per ? v0_per[b] : p->v0;
        double c0 = c0_per ? c0_per[b] : p->c0;
        double* cb = c + (size_t)b * cells;
        double* pb = phi + (size_t)b * cells;
        double* rb = rho + (size_t)b * cells;
        for (int64_t s = 0; s < n; ++s)
            step_one(p, v0, c0, b, step0 + s, cb, pb, rb, &Q[b], buf);
    }
    free(buf);
}

void or_mass(const or_params* p, const double* c, const double* phi,
             const double* rho, const double* Q, double* out)
{
    size_t cells = (size_t)p->nx * p->ny;
    double h2 = p->h * p->h;
    for (int b = 0; b < p->batch; ++b) {
        double sc = 0.0, sp = 0.0, sr = 0.0;
        for (size_t k = 0; k < cells; ++k) {
            sc += c[b * cells + k];
            sp += phi[b * cells + k];
            sr += rho[b * cells + k];
        }
        out[4 * b + 0] = h2 * sc;
        out[4 * b + 1] = h2 * sp;
        out[4 * b + 2] = h2 * sr;
        out[4 * b + 3] = Q[b];
    }
}

void or_energy(const or_params* p, const double* c, const double* phi,
               double* out)
{
    int nx = p->nx, ny = p->ny;
    size_t cells = (size_t)nx * ny;
    double h2 = p->h * p->h;
    int jfaces = p->bc_mode == OR_BC_PERIODIC ? ny : ny - 1;
    for (int b = 0; b < p->batch; ++b) {
        const double* cb = c + b * cells;
        const double* pb = phi + b * cells;
        double bulk = 0.0, grad_c = 0.0, grad_p = 0.0;
        for (int j = 0; j < ny; ++j)
            for (int i = 0; i < nx; ++i) {
                double cc = cb[(size_t)j * nx + i], pp = pb[(size_t)j * nx + i];
                double w = 1.0 - pp * pp;
                bulk += p->W_c * pfun(pp) * gfun(cc) + 0.25 * p->W_phi * w * w;
            }
        /* x faces, periodic: every cell has an east face */
        for (int j = 0; j < ny; ++j)
            for (int i = 0; i < nx; ++i) {
                size_t k = (size_t)j * nx + i, e = (size_t)j * nx + imod(i + 1, nx);
                grad_c += (cb[e] - cb[k]) * (cb[e] - cb[k]);
                grad_p += (pb[e] - pb[k]) * (pb[e] - pb[k]);
            }
        /* y faces: interior faces (and the wrap face when periodic) */
        for (int j = 0; j < jfaces; ++j)
            for (int i = 0; i < nx; ++i) {
                size_t k = (size_t)j * nx + i, n = (size_t)imod(j + 1, ny) * nx + i;
                grad_c += (cb[n] - cb[k]) * (cb[n] - cb[k]);
                grad_p += (pb[n] - pb[k]) * (pb[n] - pb[k]);
            }
        out[b] = h2 * bulk + 0.5 * p->kappa_c * grad_c + 0.5 * p->kappa_phi * grad_p;
    }
}

/* ============================================================== adjoint
 * Reverse mode of one step, written as a scatter: for every cell, each term
 * of its right-hand side R_i sends its partial derivatives (times the
 * incoming cotangent dt lambda'_i) to the cells whose values it read.  The
 * chain through mu_c, mu_phi and M_c is taken in a second pass.  Mirror
 * ghosts map to the cell itself and the rho inlet ghost is a constant, so
 * the same neighbour rules as the forward step give the transpose.
 */

static int cell(const or_params* p, int i, int j)
{
    return yrow(p, j) * p->nx + imod(i, p->nx);
}

/* index of rho's neighbour, or -1 for the constant inlet value */
static int rho_cell(const or_params* p, int i, int j)
{
    if (p->bc_mode == OR_BC_PVD && j >= p->ny) return -1;
    return cell(p, i, j);
}

static double d2gfun(double c) { return 2.0 * (1.0 - 6.0 * c + 6.0 * c * c); }
static double d2pfun(double phi) { return -1.5 * phi; }

/* m(c, phi) = M_c / M_scale and its partial derivatives (zero where the
 * clamps are active) */
static void mobility_partials(const or_params* p, double c, double phi,
                              double* m, double* dm_dc, double* dm_dphi)
{
    double x = clampd(c, 0.0, 1.0), ph = clampd(phi, -1.0, 1.0);
    double H = hswitch(c);
    double dH = 30.0 * x * x * (1.0 - x) * (1.0 - x);
    double bulk = H * p->MA_bulk + (1.0 - H) * p->MB_bulk;
    double surf = H * p->MA_surf + (1.0 - H) * p->MB_surf;
    double q = ph / p->sigma_surf;
    double e = exp(-q * q);
    double de = -2.0 * ph / (p->sigma_surf * p->sigma_surf) * e;
    *m = pfun(ph) * bulk + e * surf;
    *dm_dc = (c > 0.0 && c < 1.0)
                 ? (pfun(ph) * (p->MA_bulk - p->MB_bulk) + e * (p->MA_surf - p->MB_surf)) * dH : 0.0;
    *dm_dphi = (phi > -1.0 && phi < 1.0) ? dpfun(ph) * bulk + de * surf : 0.0;
}

void or_adjoint_step(const or_params* p, double v0, const double* c, const double* phi,
                     const double* rho, double* lc, double* lphi, double* lrho, double* g)
{
    int nx = p->nx, ny = p->ny;
    size_t n = (size_t)nx * ny;
    double h = p->h, h2 = h * h, dt = p->dt;
    int pvd = p->bc_mode == OR_BC_PVD;
    double vx, vy, dvx = 0.0, dvy = 0.0;
    velocity(p, v0, &vx, &vy);
    if (p->flux_on) {
        double th = p->theta_deg * (3.14159265358979323846 / 180.0);
        dvx = cos(th);
        dvy = -sin(th);
    }
    double* buf = (double*)calloc(9 * n, sizeof(double));
    if (!buf) abort();
    double *mu = buf, *nu = buf + n, *M = buf + 2 * n;
    double *gc = buf + 3 * n, *gp = buf + 4 * n, *gr = buf + 5 * n;
    double *mub = buf + 6 * n, *nub = buf + 7 * n, *Mb = buf + 8 * n;
    or_potentials(p, c, phi, mu, nu, M);

    const int di[4] = {1, -1, 0, 0}, dj[4] = {0, 0, 1, -1};
    for (int j = 0; j < ny; ++j) {
        for (int i = 0; i < nx; ++i) {
            int k = j * nx + i;
            double wc = dt * lc[k], wp = dt * lphi[k], wr = dt * lrho[k];
            /* composition: face terms (M_k + M_n)(mu_n - mu_k) / (2 h^2) */
            for (int q = 0; q < 4; ++q) {
                int kn = cell(p, i + di[q], j + dj[q]);
                double a = wc * 0.5 / h2;
                double dmu = mu[kn] - mu[k], sm = M[k] + M[kn];
                Mb[k] += a * dmu;
                Mb[kn] += a * dmu;
                mub[kn] += a * sm;
                mub[k] -= a * sm;
            }
            /* order parameter: M_phi (nu_n - nu_k) / h^2 */
            for (int q = 0; q < 4; ++q) {
                int kn = cell(p, i + di[q], j + dj[q]);
                nub[kn] += wp * p->M_phi / h2;
                nub[k] -= wp * p->M_phi / h2;
            }
            /* deposition S = rho (vx (phiE - phiW) + vy (phiN - phiS)) / 2h,
             * added to phi and subtracted from rho */
            int kE = cell(p, i + 1, j), kW = cell(p, i - 1, j);
            int kN = cell(p, i, j + 1), kS = cell(p, i, j - 1);
            double sb = wp - wr;
            double gx = phi[kE] - phi[kW], gy = phi[kN] - phi[kS];
            gr[k] += sb * (vx * gx + vy * gy) / (2.0 * h);
            gp[kE] += sb * rho[k] * vx / (2.0 * h);
            gp[kW] -= sb * rho[k] * vx / (2.0 * h);
            gp[kN] += sb * rho[k] * vy / (2.0 * h);
            gp[kS] -= sb * rho[k] * vy / (2.0 * h);
            g[1] += sb * rho[k] * (dvx * gx + dvy * gy) / (2.0 * h);
            /* vapour: D Lap rho - ((Fe - Fw) + (Gn - Gs)) / h */
            int rE = rho_cell(p, i + 1, j), rW = rho_cell(p, i - 1, j);
            int rN = rho_cell(p, i, j + 1), rS = rho_cell(p, i, j - 1);
            int bottom = pvd && j == 0;
            double r0 = rho[k];
            double vE = rE >= 0 ? rho[rE] : p->rho_in, vW = rW >= 0 ? rho[rW] : p->rho_in;
            double vN = rN >= 0 ? rho[rN] : p->rho_in, vS = rS >= 0 ? rho[rS] : p->rho_in;
            double dD = p->D_rho / h2;
            double cE = dD - vx / (2.0 * h), cW = dD + vx / (2.0 * h);
            double cN = dD - vy / (2.0 * h), cS = bottom ? dD : dD + vy / (2.0 * h);
            double c0 = -4.0 * dD + (bottom ? -vy / (2.0 * h) : 0.0);
            if (rE >= 0) gr[rE] += wr * cE;
            if (rW >= 0) gr[rW] += wr * cW;
            if (rN >= 0) gr[rN] += wr * cN;
            if (rS >= 0) gr[rS] += wr * cS;
            gr[k] += wr * c0;
            double dT = -((dvx * 0.5 * (r0 + vE) - dvx * 0.5 * (vW + r0))
                          + (dvy * 0.5 * (r0 + vN) - (bottom ? 0.0 : dvy * 0.5 * (vS + r0)))) / h;
            g[1] += wr * dT;
        }
    }
    /* chain through mu_c, mu_phi and M_c */
    for (int j = 0; j < ny; ++j) {
        for (int i = 0; i < nx; ++i) {
            int k = j * nx + i;
            double cc = c[k], pp = phi[k];
            /* mu_c = W_c p g' - kappa_c Lap c */
            gc[k] += mub[k] * p->W_c * pfun(pp) * d2gfun(cc);
            gp[k] += mub[k] * p->W_c * dpfun(pp) * dgfun(cc);
            /* mu_phi = W_c p' g - W_phi phi (1 - phi^2) - kappa_phi Lap phi */
            gp[k] += nub[k] * (p->W_c * d2pfun(pp) * gfun(cc) - p->W_phi * (1.0 - 3.0 * pp * pp));
            gc[k] += nub[k] * p->W_c * dpfun(pp) * dgfun(cc);
            for (int q = 0; q < 4; ++q) {
                int kn = cell(p, i + di[q], j + dj[q]);
                gc[kn] -= p->kappa_c / h2 * mub[k];
                gc[k] += p->kappa_c / h2 * mub[k];
                gp[kn] -= p->kappa_phi / h2 * nub[k];
                gp[k] += p->kappa_phi / h2 * nub[k];
            }
            /* M_c = M_scale m(c, phi) */
            double m, dmc, dmp;
            mobility_partials(p, cc, pp, &m, &dmc, &dmp);
            gc[k] += Mb[k] * p->M_scale * dmc;
            gp[k] += Mb[k] * p->M_scale * dmp;
            g[0] += Mb[k] * m;
        }
    }
    for (size_t k = 0; k < n; ++k) {
        lc[k] += gc[k];
        lphi[k] += gp[k];
        lrho[k] += gr[k];
    }
    free(buf);
}

void or_loss_grad(const or_params* p, double v0, int64_t n, int64_t every,
                  const double* c, const double* phi, const double* rho,
                  const double* ct, const double* phit, const double* rhot, double* out)
{
    size_t cells = (size_t)p->nx * p->ny;
    if (p->integrator != OR_EULER || p->interface_noise > 0.0) {
        /* the adjoint is that of the explicit Euler step without draws */
        out[0] = out[1] = out[2] = NAN;
        return;
    }
    if (every < 1) every = 1;
    int64_t nseg = (n + every - 1) / every;
    if (nseg < 1) nseg = 1;
    double* ck = (double*)malloc((size_t)nseg * 3 * cells * sizeof(double));
    double* seg = (double*)malloc((size_t)every * 3 * cells * sizeof(double));
    double* w = (double*)malloc(9 * cells * sizeof(double));
    double* u = (double*)malloc(3 * cells * sizeof(double));
    double* lam = (double*)malloc(3 * cells * sizeof(double));
    if (!ck || !seg || !w || !u || !lam) abort();
    memcpy(u, c, cells * sizeof(double));
    memcpy(u + cells, phi, cells * sizeof(double));
    memcpy(u + 2 * cells, rho, cells * sizeof(double));
    double Q = 0.0;
    /* forward, keeping the state at the start of every segment */
    for (int64_t s = 0; s < n; ++s) {
        if (s % every == 0) memcpy(ck + (size_t)(s / every) * 3 * cells, u, 3 * cells * sizeof(double));
        step_one(p, v0, p->c0, 0, s, u, u + cells, u + 2 * cells, &Q, w);
    }
    double L = 0.0, h2 = p->h * p->h;
    const double* tgt[3] = {ct, phit, rhot};
    for (int f = 0; f < 3; ++f)
        for (size_t k = 0; k < cells; ++k) {
            double d = u[f * cells + k] - tgt[f][k];
            L += 0.5 * h2 * d * d;
            lam[f * cells + k] = h2 * d;
        }
    double g[2] = {0.0, 0.0};
    /* reverse: recompute each segment's states from its checkpoint */
    for (int64_t sg = nseg - 1; sg >= 0; --sg) {
        int64_t s0 = sg * every, s1 = s0 + every < n ? s0 + every : n;
        memcpy(seg, ck + (size_t)sg * 3 * cells, 3 * cells * sizeof(double));
        for (int64_t t = 1; t < s1 - s0; ++t) {
            double* dst = seg + (size_t)t * 3 * cells;
            memcpy(dst, dst - 3 * cells, 3 * cells * sizeof(double));
            step_one(p, v0, p->c0, 0, s0 + t - 1, dst, dst + cells, dst + 2 * cells, &Q, w);
        }
        for (int64_t t = s1 - s0 - 1; t >= 0; --t) {
            const double* st = seg + (size_t)t * 3 * cells;
            or_adjoint_step(p, v0, st, st + cells, st + 2 * cells, lam, lam + cells, lam + 2 * cells, g);
        }
    }
    out[0] = L;
    out[1] = g[0];
    out[2] = g[1];
    free(ck);
    free(seg);
    free(w);
    free(u);
    free(lam);
}
