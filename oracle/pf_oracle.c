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
 *   - explicit Euler in time (every right-hand side uses the old state);
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

/* One explicit Euler step of one realisation. */
static void step_one(const or_params* p, double v0, double* c, double* phi,
                     double* rho, double* Q, double* mu_c, double* mu_phi,
                     double* Mc, double* cn, double* pn, double* rn)
{
    int nx = p->nx, ny = p->ny;
    double h = p->h, h2 = h * h, dt = p->dt;
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

            cn[k] = c[k] + dt * div_c;
            pn[k] = phi[k] + dt * (div_p + S);
            rn[k] = r0 + dt * (T - S);
        }
    }

    /* inflow through the top face during this step: advective plus
     * diffusive flux of rho, per unit length, times the face length h */
    if (pvd) {
        int j = ny - 1;
        double acc = 0.0;
        for (int i = 0; i < nx; ++i) {
            double r0 = rho[(size_t)j * nx + i];
            double Gn = vy * 0.5 * (r0 + p->rho_in);
            acc += -Gn + p->D_rho * (p->rho_in - r0) / h;
        }
        *Q += dt * h * acc;
    }

    size_t n = (size_t)nx * ny;
    memcpy(c, cn, n * sizeof(double));
    memcpy(phi, pn, n * sizeof(double));
    memcpy(rho, rn, n * sizeof(double));
}

void or_step_n(const or_params* p, const double* v0_per, int64_t n,
               double* c, double* phi, double* rho, double* Q)
{
    size_t cells = (size_t)p->nx * p->ny;
    double* buf = (double*)malloc(6 * cells * sizeof(double));
    if (!buf) abort();
    for (int b = 0; b < p->batch; ++b) {
        double v0 = v0_per ? v0_per[b] : p->v0;
        double* cb = c + (size_t)b * cells;
        double* pb = phi + (size_t)b * cells;
        double* rb = rho + (size_t)b * cells;
        for (int64_t s = 0; s < n; ++s)
            step_one(p, v0, cb, pb, rb, &Q[b], buf, buf + cells, buf + 2 * cells,
                     buf + 3 * cells, buf + 4 * cells, buf + 5 * cells);
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
