// Per-cell arithmetic of the explicit PVD phase-field step, shared by every
// stepper kernel (Materials and Methods, "Phase-field modeling of physical
// vapor deposition"; second-order central differences as stated in
// "Dataset"; explicit Euler or the midpoint method).  Each kernel evaluates
// every cell through these functions with a fixed expression order
// (contraction off, explicit fma), so all kernels and launch shapes give
// bitwise-identical states.
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

// Stage 2 at one cell: the rates of (c, phi, rho) from the four face fluxes
// of c (east, west, north, south as defined by cflux), mu_phi at the cell
// and its neighbours, phi's neighbours and rho's 5-point stencil.
//   Rc = (1/2h^2)((FE - FW) + (FN - FS))
//   Rp = M_phi Lap mu_phi + S,  S = rho v . grad phi
//   Rr = D Lap rho - div(rho v) - S
template <typename T>
__device__ __forceinline__ void rates(const Coef<T>& k, const RhoCoef<T>& rc, T vx2h, T vy2h, bool bottom,
                                      T pE, T pW, T pN, T pS,
                                      T r0, T rE, T rW, T rN, T rS,
                                      T FE, T FW, T FN, T FS,
                                      T q0, T qE, T qW, T qN, T qS,
                                      T& Rc, T& Rp, T& Rr)
{
    const T divc = k.half_ih2 * ((FE - FW) + (FN - FS));
    const T divp = k.mphi_h2 * fmaT(T(-4), q0, (qE + qW) + (qN + qS));
    const T src = r0 * fmaT(vx2h, pE - pW, vy2h * (pN - pS));
    const T aS = bottom ? rc.aS_bottom : rc.aS;
    const T Tr = fmaT(rc.aE, rE, fmaT(rc.aW, rW, fmaT(rc.aN, rN, fmaT(aS, rS, rc.a0 * r0))));
    Rc = divc;
    Rp = divp + src;
    Rr = Tr - src;
}

// Euler update from base values (c0, p0, r0): u' = u + dt R.  For explicit
// Euler the base is the cell's own state; the midpoint method's second stage
// passes the state at the start of the step.
template <typename T>
__device__ __forceinline__ void update(const Coef<T>& k, const RhoCoef<T>& rc, T vx2h, T vy2h, bool bottom,
                                       T c0, T p0, T pE, T pW, T pN, T pS,
                                       T r0, T rE, T rW, T rN, T rS,
                                       T FE, T FW, T FN, T FS,
                                       T q0, T qE, T qW, T qN, T qS,
                                       T& nc, T& np, T& nr, T cb, T pb, T rb)
{
    T Rc, Rp, Rr;
    rates(k, rc, vx2h, vy2h, bottom, pE, pW, pN, pS, r0, rE, rW, rN, rS, FE, FW, FN, FS, q0, qE, qW, qN, qS,
          Rc, Rp, Rr);
    nc = fmaT(k.dt, Rc, cb);
    np = fmaT(k.dt, Rp, pb);
    nr = fmaT(k.dt, Rr, rb);
}

template <typename T>
__device__ __forceinline__ void update(const Coef<T>& k, const RhoCoef<T>& rc, T vx2h, T vy2h, bool bottom,
                                       T c0, T p0, T pE, T pW, T pN, T pS,
                                       T r0, T rE, T rW, T rN, T rS,
                                       T FE, T FW, T FN, T FS,
                                       T q0, T qE, T qW, T qN, T qS,
                                       T& nc, T& np, T& nr)
{
    update(k, rc, vx2h, vy2h, bottom, c0, p0, pE, pW, pN, pS, r0, rE, rW, rN, rS, FE, FW, FN, FS, q0, qE, qW, qN,
           qS, nc, np, nr, c0, p0, r0);
}

// SplitMix64 (Steele, Lea & Flood 2014): output n of the stream `seed`.
__device__ __forceinline__ uint64_t mix64(uint64_t seed, uint64_t n)
{
    uint64_t z = seed + (n + 1ull) * 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

// Interface composition: N(mean, sigma^2) truncated to [0, 1] by rejection,
// Box-Muller in FP64 on the uniforms (53 bits; first in (0, 1], second in
// [0, 1)) of counters counter0 + 2a and + 2a + 1, attempts a = 0..7, then
// the mean.
__device__ __noinline__ double trunc_gauss(uint64_t seed, uint64_t counter0, double mean, double sigma)
{
    for (int a = 0; a < 8; ++a) {
        const uint64_t x1 = mix64(seed, counter0 + 2ull * a), x2 = mix64(seed, counter0 + 2ull * a + 1ull);
        const double u1 = (double)((x1 >> 11) + 1ull) * 0x1.0p-53;
        const double u2 = (double)(x2 >> 11) * 0x1.0p-53;
        const double z = sqrt(-2.0 * log(u1)) * cos(2.0 * 3.14159265358979323846 * u2);
        const double v = mean + sigma * z;
        if (v >= 0.0 && v <= 1.0) return v;
    }
    return mean;
}

// The same draw in FP32 arithmetic (FP32 runs): same stream, counters,
// attempts and bounds test, on the hardware base-2 logarithm, square root
// and cosine (whose argument is in revolutions, so cos(2 pi u2) takes u2
// itself).  log2 u1 keeps FP32's relative precision over the whole range:
// up to 1/2 from u1 itself; above from w = 1 - u1 (an integer times 2^-53,
// rounded once) as log2(1 - w) = log2(v) w / (1 - v) with v = 1 - w rounded
// and 1 - v exact (Goldberg's form of log1p), or -w / ln 2 where v rounds
// to 1.
// attempt a of the FP32 draw: true with the value in *x when it lies in [0, 1]
__device__ __forceinline__ bool gauss_attempt_f32(uint64_t seed, uint64_t counter0, int a, float mean, float sigma,
                                                  float* x)
{
    const uint64_t k1 = mix64(seed, counter0 + 2ull * a) >> 11;   // u1 = (k1 + 1) 2^-53
    const uint64_t k2 = mix64(seed, counter0 + 2ull * a + 1ull) >> 11;   // u2 = k2 2^-53
    const bool hi = k1 >= (1ull << 52);
    const float f = (float)(hi ? (1ull << 53) - 1ull - k1 : k1 + 1ull) * 0x1.0p-53f;   // w or u1
    const float v = hi ? 1.f - f : f;
    float l2 = __builtin_amdgcn_logf(v);
    if (hi) l2 = v == 1.f ? -f * 1.4426950408889634f : l2 * (f * __builtin_amdgcn_rcpf(1.f - v));
    const float z = __builtin_amdgcn_sqrtf(-2.f * 0.6931471805599453f * l2) *
                    __builtin_amdgcn_cosf((float)k2 * 0x1.0p-53f);
    *x = mean + sigma * z;
    return *x >= 0.f && *x <= 1.f;
}

// attempts a0 .. 7, then the mean
__device__ __forceinline__ float trunc_gauss_f32_from(uint64_t seed, uint64_t counter0, int a0, float mean,
                                                      float sigma)
{
    for (int a = a0; a < 8; ++a) {
        float x;
        if (gauss_attempt_f32(seed, counter0, a, mean, sigma, &x)) return x;
    }
    return mean;
}

__device__ __forceinline__ float trunc_gauss_f32(uint64_t seed, uint64_t counter0, float mean, float sigma)
{
    return trunc_gauss_f32_from(seed, counter0, 0, mean, sigma);
}

// The interface draw in the precision of the run.
template <typename T>
__device__ __forceinline__ T interface_draw(uint64_t seed, uint64_t counter0, double mean, double sigma);
template <>
__device__ __forceinline__ double interface_draw<double>(uint64_t seed, uint64_t counter0, double mean, double sigma)
{
    return trunc_gauss(seed, counter0, mean, sigma);
}
template <>
__device__ __forceinline__ float interface_draw<float>(uint64_t seed, uint64_t counter0, double mean, double sigma)
{
    return trunc_gauss_f32(seed, counter0, (float)mean, (float)sigma);
}

}  // namespace cell
}  // namespace pfk
