// Per-cell arithmetic of the explicit PVD phase-field step, shared by every
// stepper kernel (Materials and Methods, "Phase-field modeling of physical
// vapor deposition"; second-order central differences as stated in
// "Dataset"; explicit Euler).  Each kernel evaluates every cell through these
// two functions with a fixed expression order (contraction off, explicit
// fma), so all kernels and launch shapes give bitwise-identical states.
#pragma once

#include <hip/hip_runtime.h>
#include <math.h>

#include "pf_kernels.h"

namespace pfk {
namespace cell {

__device__ __forceinline__ float fmaT(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__device__ __forceinline__ double fmaT(double a, double b, double c) { return __builtin_fma(a, b, c); }

// exp(-phi^2/sigma^2): float uses the hardware base-2 exponential with
// log2(e)/sigma^2 folded on the host; double uses the device math library.
__device__ __forceinline__ float surf_exp(float ph2, float e) { return __builtin_amdgcn_exp2f(-(ph2 * e)); }
__device__ __forceinline__ double surf_exp(double ph2, double e) { return exp(-(ph2 * e)); }

__device__ __forceinline__ float clampT(float x, float lo, float hi) { return __builtin_amdgcn_fmed3f(x, lo, hi); }
__device__ __forceinline__ double clampT(double x, double lo, double hi) { return x < lo ? lo : (x > hi ? hi : x); }

// Stage 1 at one cell: chemical potentials and composition mobility.
//   mu_c   = W_c p(phi) g'(c) - kappa_c Lap c
//   mu_phi = W_c p'(phi) g(c) - W_phi phi (1 - phi^2) - kappa_phi Lap phi
//   M_c    = p(phi~)(MB + H dM)_bulk + exp(-(phi~/sigma)^2)(MB + H dM)_surf
// with p(phi) = (2-phi)(1+phi)^2/4, g(c) = c^2(1-c)^2, H the quintic
// switching function of c~ = clamp(c,0,1), phi~ = clamp(phi,-1,1).  The
// constants W_c/4 and 3 W_c/4 are folded on the host.  Neighbour sums are
// (E + W) + (N + S): mirrored ghost rows then reproduce the interior values
// exactly.
template <typename T>
__device__ __forceinline__ void potentials(const Coef<T>& k, T c, T cE, T cW, T cN, T cS,
                                           T p, T pE, T pW, T pN, T pS,
                                           T& mu_c, T& mu_p, T& M)
{
    const T lapc = fmaT(T(-4), c, (cE + cW) + (cN + cS));
    const T lapp = fmaT(T(-4), p, (pE + pW) + (pN + pS));
    const T q1 = T(1) + p;
    const T pf4 = (k.Wc4 * (T(2) - p)) * (q1 * q1);      // W_c p(phi)
    const T w = fmaT(-p, p, T(1));                         // 1 - phi^2
    const T cg = c * (T(1) - c);
    const T g = cg * cg;
    const T dg = cg * fmaT(T(-4), c, T(2));               // g'(c)
    mu_c = fmaT(pf4, dg, -(k.kc * lapc));
    mu_p = fmaT(k.Wc34 * w, g, fmaT(-(k.Wphi * p), w, -(k.kp * lapp)));
    const T x = clampT(c, T(0), T(1));
    const T H = ((x * x) * x) * fmaT(fmaT(T(6), x, T(-15)), x, T(10));
    const T ph = clampT(p, T(-1), T(1));
    const T r1 = T(1) + ph;
    const T pb = (T(0.25) * (T(2) - ph)) * (r1 * r1);
    const T e = surf_exp(ph * ph, k.esurf);
    M = fmaT(pb, fmaT(H, k.dMb, k.MBb), e * fmaT(H, k.dMs, k.MBs));
}

// Composition flux (up to the factor 1/(2h^2)) through the face from a cell
// (M0, m0) to its neighbour (Mn, mn): (Mn + M0)(mn - m0), i.e. the
// face-averaged mobility times the potential difference.  A cell's west
// (south) flux is exactly its west (south) neighbour's east (north) flux,
// so kernels may compute each face once and pass it on.
template <typename T>
__device__ __forceinline__ T cflux(T M0, T m0, T Mn, T mn)
{
    return (Mn + M0) * (mn - m0);
}

// Vapour transport coefficients: D Lap rho - div(rho v) with central face
// fluxes is aE rE + aW rW + aN rN + aS rS + a0 r0.  On the substrate row the
// south neighbour is the mirror ghost (rS = r0) and the south advective flux
// is zero, so aS becomes D/h^2 - vy/(2h) there.
template <typename T>
struct RhoCoef {
    T aE, aW, aN, aS, aS_bottom, a0;
};
template <typename T>
__device__ __forceinline__ RhoCoef<T> rho_coef(const Coef<T>& k, T vx2h, T vy2h)
{
    return {k.D_h2 - vx2h, k.D_h2 + vx2h, k.D_h2 - vy2h, k.D_h2 + vy2h, k.D_h2 - vy2h, T(-4) * k.D_h2};
}

// Stage 2 at one cell: Euler update of (c, phi, rho) from the four face
// fluxes of c (east, west, north, south as defined by cflux), mu_phi at the
// cell and its neighbours, phi's neighbours and rho's 5-point stencil.
//   c'   = c   + dt * (1/2h^2)((FE - FW) + (FN - FS))
//   phi' = phi + dt * (M_phi Lap mu_phi + S),  S = rho v . grad phi
//   rho' = rho + dt * (D Lap rho - div(rho v) - S)
template <typename T>
__device__ __forceinline__ void update(const Coef<T>& k, const RhoCoef<T>& rc, T vx2h, T vy2h, bool bottom,
                                       T c0, T p0, T pE, T pW, T pN, T pS,
                                       T r0, T rE, T rW, T rN, T rS,
                                       T FE, T FW, T FN, T FS,
                                       T q0, T qE, T qW, T qN, T qS,
                                       T& nc, T& np, T& nr)
{
    const T divc = k.half_ih2 * ((FE - FW) + (FN - FS));
    const T divp = k.mphi_h2 * fmaT(T(-4), q0, (qE + qW) + (qN + qS));
    const T src = r0 * fmaT(vx2h, pE - pW, vy2h * (pN - pS));
    const T aS = bottom ? rc.aS_bottom : rc.aS;
    const T Tr = fmaT(rc.aE, rE, fmaT(rc.aW, rW, fmaT(rc.aN, rN, fmaT(aS, rS, rc.a0 * r0))));
    nc = fmaT(k.dt, divc, c0);
    np = fmaT(k.dt, divp + src, p0);
    nr = fmaT(k.dt, Tr - src, r0);
}

}  // namespace cell
}  // namespace pfk
