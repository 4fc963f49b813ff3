// gfx950 convolutions of the time-conditioned U-Net (Materials and Methods,
// "U-Net with temporal conditioning": 3x3 convolutions, 2x2 stride-2
// up-sampling, skips concatenated along channels) as implicit GEMMs on BF16
// MFMA with FP32 accumulation.
//
// One kernel computes out[p][o] = sum_k A[p][k] B[o][k] with p a pixel, o an
// output channel and A gathered on the fly from NHWC tensors:
//   kConvFwd    k = (tap, ci), A = in[p + off(tap)][ci] (zero outside),
//               B = W[tap][o][ci];
//   kConvDgrad  the same with off(tap) negated, in = dY, B = W^T[tap][ci][co];
//   kUpFwd      one tap, o = (m, n, co) scattered to output pixel (2y+m, 2x+n);
//   kUpDgrad    k = (m, n, co) gathered from dY at (2y+m, 2x+n).
// A concatenated input in1 (+) in2 is a split of K; the gradient of a
// concatenation is a split of the output channels (out, out2).
//
// A 256-thread block owns 64 pixels x 64 output channels; each wave a 32 x 32
// sub-tile as 2 x 2 v_mfma_f32_16x16x16_bf16.  Lane l supplies row l % 16 and
// k = 4 (l / 16) .. +3 of each 16 x 16 operand, i.e. 8 contiguous bytes of an
// NHWC pixel or of a weight row; the FP32 result of lane l holds rows
// 4 (l / 16) .. +3 of column l % 16.
//
// Weight gradients reduce over pixels: the wgrad kernels form partial
// products over fixed pixel chunks and wsum_kernel adds the chunks in a fixed
// order that depends only on the shapes, so results are deterministic.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>

#include "unet_gelu.h"
#include "unet_kernels.h"

namespace pfu {
namespace {

typedef short bf16x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

// DPP row shifts (within each 16-lane row; a lane whose source lies outside
// the row keeps the old value)
constexpr int kRowShl1 = 0x101, kRowShr1 = 0x111;

// round to nearest even (NaN and infinity keep their class)
__device__ __forceinline__ uint16_t f2bf(float f)
{
    uint32_t u = __builtin_bit_cast(uint32_t, f);
    if ((u & 0x7f800000u) == 0x7f800000u) return (uint16_t)((u >> 16) | ((u & 0xffffu) ? 0x40u : 0u));
    u += 0x7fffu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}

struct Pix {
    int n, y, x;
    bool ok;
};
// coordinates of flat pixel p of an [N][H][W] grid; ok = p < lim
__device__ __forceinline__ Pix pix(int p, int H, int W, int lim)
{
    Pix r;
    r.ok = p < lim;
    const int q = r.ok ? p : 0;
    r.x = q % W;
    const int t = q / W;
    r.y = t % H;
    r.n = t / H;
    return r;
}

// channels c .. c+3 (those below C) of pixel (n, y, x) of an NHWC tensor,
// zero outside the grid
__device__ __forceinline__ bf16x4 ld4(const uint16_t* t, int n, int y, int x, int H, int W, int C, int c, bool ok)
{
    bf16x4 v = {0, 0, 0, 0};
    if (!ok || y < 0 || y >= H || x < 0 || x >= W || c >= C) return v;
    const uint16_t* q = t + (((size_t)n * H + y) * W + x) * C + c;
    if ((C & 3) == 0) return __builtin_bit_cast(bf16x4, *(const uint2*)q);
    for (int j = 0; j < 4; ++j)
        if (c + j < C) v[j] = (short)q[j];
    return v;
}

template <int MODE>
__global__ __launch_bounds__(256) void gemm_kernel(ConvArgs a)
{
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int m0 = blockIdx.x * 64 + (wv & 1) * 32;
    const int o0 = blockIdx.y * 64 + (wv >> 1) * 32;
    const int r = lane & 15, kq = (lane >> 4) * 4;
    const int P = a.N * a.H * a.W;
    const Pix px0 = pix(m0 + r, a.H, a.W, P), px1 = pix(m0 + 16 + r, a.H, a.W, P);
    const int K = a.C1 + a.C2;
    f32x4 acc[2][2] = {};
    constexpr int ntaps = (MODE == kConvFwd || MODE == kConvDgrad) ? 9 : 1;
    for (int tap = 0; tap < ntaps; ++tap) {
        int dy = 0, dx = 0;
        if (ntaps == 9) {
            dy = tap / 3 - 1;
            dx = tap % 3 - 1;
            if (MODE == kConvDgrad) {
                dy = -dy;
                dx = -dx;
            }
        }
        const uint16_t* wt = a.Wt + (size_t)tap * a.ldo * a.ldk;
        const uint16_t* w0 = wt + (size_t)(o0 + r) * a.ldk;
        const uint16_t* w1 = wt + (size_t)(o0 + 16 + r) * a.ldk;
        for (int k0 = 0; k0 < K; k0 += 16) {
            const int kc = k0 + kq;
            bf16x4 A0, A1;
            if (MODE == kUpDgrad) {
                // k = (m, n, co) over the 2H x 2W gradient with C1 / 4 channels
                const int Cd = a.C1 >> 2;
                const int sub = kc / Cd, co = kc - sub * Cd;
                const bool in = kc < K;
                A0 = ld4(a.in1, px0.n, 2 * px0.y + (sub >> 1), 2 * px0.x + (sub & 1), 2 * a.H, 2 * a.W, Cd, co,
                         px0.ok && in);
                A1 = ld4(a.in1, px1.n, 2 * px1.y + (sub >> 1), 2 * px1.x + (sub & 1), 2 * a.H, 2 * a.W, Cd, co,
                         px1.ok && in);
            } else {
                const bool first = kc < a.C1;
                const uint16_t* src = first ? a.in1 : a.in2;
                const int C = first ? a.C1 : a.C2, c = first ? kc : kc - a.C1;
                A0 = ld4(src, px0.n, px0.y + dy, px0.x + dx, a.H, a.W, C, c, px0.ok);
                A1 = ld4(src, px1.n, px1.y + dy, px1.x + dx, a.H, a.W, C, c, px1.ok);
            }
            const bf16x4 B0 = __builtin_bit_cast(bf16x4, *(const uint2*)(w0 + kc));
            const bf16x4 B1 = __builtin_bit_cast(bf16x4, *(const uint2*)(w1 + kc));
            acc[0][0] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(A0, B0, acc[0][0], 0, 0, 0);
            acc[0][1] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(A0, B1, acc[0][1], 0, 0, 0);
            acc[1][0] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(A1, B0, acc[1][0], 0, 0, 0);
            acc[1][1] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(A1, B1, acc[1][1], 0, 0, 0);
        }
    }
    // acc[mi][ni][j]: pixel m0 + 16 mi + kq + j, channel o0 + 16 ni + r
#pragma unroll
    for (int mi = 0; mi < 2; ++mi)
#pragma unroll
        for (int ni = 0; ni < 2; ++ni) {
            const int o = o0 + 16 * ni + r;
            if (o >= a.Nout) continue;
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const int p = m0 + 16 * mi + kq + j;
                if (p >= P) continue;
                const float v = acc[mi][ni][j];
                if (MODE == kUpFwd) {
                    const Pix q = pix(p, a.H, a.W, P);
                    const int Co = a.Nout >> 2, sub = o / Co, co = o - sub * Co;
                    const size_t idx =
                        (((size_t)q.n * 2 * a.H + 2 * q.y + (sub >> 1)) * 2 * a.W + 2 * q.x + (sub & 1)) * Co + co;
                    if (a.out_f32) stwt(a.out_f32, idx, v);
                    if (a.out_bf16) a.out_bf16[idx] = f2bf(v);
                } else if (o < a.O1) {
                    const size_t idx = (size_t)p * a.O1 + o;
                    if (a.out_f32) stwt(a.out_f32, idx, v);
                    if (a.out_bf16) a.out_bf16[idx] = f2bf(v);
                } else {
                    const size_t idx = (size_t)p * (a.Nout - a.O1) + (o - a.O1);
                    if (a.out2_f32) a.out2_f32[idx] = v;
                    if (a.out2_bf16) a.out2_bf16[idx] = f2bf(v);
                }
            }
        }
}

// ---------------------------------------------------------------------------
// Wide-tile variant for channel counts that are multiples of 32 (every layer
// but the 4-channel input and the 3-channel head): v_mfma_f32_16x16x32_bf16,
// each lane loading 16 contiguous bytes (8 channels) per operand tile; a wave
// owns TM x TN 16 x 16 output tiles, a block WGM x WGN waves.  Lane l supplies
// row l % 16, k = 8 (l / 16) .. +7 of each operand; the FP32 result of lane l
// holds rows 4 (l / 16) .. +3 of column l % 16.
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

__device__ __forceinline__ bf16x8 ld8(const uint16_t* p) { return __builtin_bit_cast(bf16x8, *(const uint4*)p); }

template <int MODE, int TM, int TN, int WGM, int WGN>
__global__ __launch_bounds__(256) void gemm32_kernel(ConvArgs a)
{
    static_assert(WGM * WGN == 4, "four waves per block");
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int pm = blockIdx.x * (WGM * TM * 16) + (wv % WGM) * TM * 16;
    const int on = blockIdx.y * (WGN * TN * 16) + (wv / WGM) * TN * 16;
    const int r = lane & 15, kq = (lane >> 4) * 8;
    const int P = a.N * a.H * a.W;
    const int K = MODE == kFirst ? 36 : a.C1 + a.C2;
    Pix px[TM];
#pragma unroll
    for (int i = 0; i < TM; ++i) px[i] = pix(pm + 16 * i + r, a.H, a.W, P);
    f32x4 acc[TM][TN];
#pragma unroll
    for (int i = 0; i < TM; ++i)
#pragma unroll
        for (int j = 0; j < TN; ++j) acc[i][j] = (f32x4){0.f, 0.f, 0.f, 0.f};
    constexpr int ntaps = (MODE == kConvFwd || MODE == kConvDgrad) ? 9 : 1;
    const int nk = (K + 31) / 32;  // K chunks per tap
    const int iters = ntaps * nk;
    const uint16_t* wlane = a.Wt + (size_t)(on + r) * a.ldk + kq;
    // kFirst from the state fields, where a block's BM pixels lie in one row
    // (W a multiple of BM): the three rows y - 1, y, y + 1 over columns
    // x0 - 1 .. x0 + BM are staged once in LDS as the assembled 4-channel
    // BF16 input (each pixel loaded once, coalesced, every load issued before
    // the first is used; indices clamped into the grid, and taps outside it
    // zeroed when the operands are gathered from LDS)
    constexpr int BMr = WGM * TM * 16, kSW = BMr + 2, kStageIt = (3 * kSW + 255) / 256;
    // LDS shared by the input stage (kFirst, dead after the operand loads)
    // and the forward epilogue's output stage (fewer bytes per block: with
    // ~38 KB four blocks fit on a CU)
    constexpr int kStfFloats = (MODE == kFirst || MODE == kConvFwd) ? BMr * (WGN * TN * 16 + 4) : 4;
    constexpr int kXstBytes = MODE == kFirst ? kStageIt * 256 * 8 : 16;
    constexpr int kSmemBytes = kStfFloats * 4 > kXstBytes ? kStfFloats * 4 : kXstBytes;
    __shared__ __align__(16) unsigned char smem[kSmemBytes];
    [[maybe_unused]] const uint2* xs = nullptr;
    [[maybe_unused]] int xs_x0 = 0;
    if constexpr (MODE == kFirst) {
        uint2* xst = (uint2*)smem;
        if (a.raw[0] && a.W % BMr == 0) {
            const int pb = blockIdx.x * BMr, row = pb / a.W, n0 = row / a.H, y0 = row - n0 * a.H;
            xs_x0 = pb - row * a.W;
            const float jv = a.jump[n0];
            float v[kStageIt][3];
#pragma unroll
            for (int u = 0; u < kStageIt; ++u) {
                const int e = threadIdx.x + 256 * u, sr = e / kSW, sc = e - sr * kSW;
                const int yy = min(max(y0 - 1 + sr, 0), a.H - 1), xx = min(max(xs_x0 - 1 + sc, 0), a.W - 1);
                const long q = ((long)n0 * a.H + yy) * a.W + xx;
                v[u][0] = a.raw[0][q];
                v[u][1] = a.raw[1][q];
                v[u][2] = a.raw[2][q];
            }
            const uint32_t jb = (uint32_t)f2bf(jv) << 16;
#pragma unroll
            for (int u = 0; u < kStageIt; ++u) {
                const uint32_t lo = (uint32_t)f2bf(v[u][0] - 0.5f) | ((uint32_t)f2bf(v[u][1]) << 16);
                const uint32_t hi = (uint32_t)f2bf(v[u][2] - 1.0f) | jb;
                xst[threadIdx.x + 256 * u] = make_uint2(lo, hi);
            }
            __syncthreads();
            xs = xst;
        }
    }
    // operands of iteration `it` (tap it / nk, channels 32 (it % nk) ..) in
    // the MFMA lane layout; zero outside the grid
    auto load = [&](int it, bf16x8* A, bf16x8* B) {
        const int tap = it / nk, k0 = (it - tap * nk) * 32;
        int dy = 0, dx = 0;
        if (ntaps == 9) {
            dy = tap / 3 - 1;
            dx = tap % 3 - 1;
            if (MODE == kConvDgrad) {
                dy = -dy;
                dx = -dx;
            }
        }
        const bf16x8 zero = __builtin_bit_cast(bf16x8, make_uint4(0, 0, 0, 0));
        if (MODE == kFirst && xs) {
            // from the staged rows: tap (dy, dx) of column x is row dy + 1,
            // column x - x0 + 1 + dx of the stage
            const int t0 = (k0 + kq) >> 2;
#pragma unroll
            for (int i = 0; i < TM; ++i) {
                uint2 h[2];
#pragma unroll
                for (int u = 0; u < 2; ++u) {
                    const int t = t0 + u, tc = t < 9 ? t : 8;
                    const int dy = tc / 3 - 1, dx = tc % 3 - 1, yy = px[i].y + dy, xx = px[i].x + dx;
                    const bool ok = px[i].ok && t < 9 && yy >= 0 && yy < a.H && xx >= 0 && xx < a.W;
                    const int e = (dy + 1) * kSW + px[i].x - xs_x0 + 1 + dx;
                    const uint2 g = xs[min(max(e, 0), 3 * kSW - 1)];
                    h[u] = ok ? g : make_uint2(0, 0);
                }
                A[i] = __builtin_bit_cast(bf16x8, make_uint4(h[0].x, h[0].y, h[1].x, h[1].y));
            }
        } else if (MODE == kFirst && a.raw[0]) {
            // the same operand assembled from the state fields: indices are
            // clamped into the grid so that every load is issued
            // unconditionally, and taps outside it are zeroed afterwards
            const int t0 = (k0 + kq) >> 2;
#pragma unroll
            for (int i = 0; i < TM; ++i) {
                uint2 h[2];
#pragma unroll
                for (int u = 0; u < 2; ++u) {
                    const int t = t0 + u, tc = t < 9 ? t : 8;
                    const int yy = px[i].y + tc / 3 - 1, xx = px[i].x + tc % 3 - 1;
                    const bool ok = px[i].ok && t < 9 && yy >= 0 && yy < a.H && xx >= 0 && xx < a.W;
                    const long q = ((long)px[i].n * a.H + min(max(yy, 0), a.H - 1)) * a.W + min(max(xx, 0), a.W - 1);
                    const float cv = a.raw[0][q], pv = a.raw[1][q], rv = a.raw[2][q], jv = a.jump[px[i].n];
                    const uint32_t lo = (uint32_t)f2bf(cv - 0.5f) | ((uint32_t)f2bf(pv) << 16);
                    const uint32_t hi = (uint32_t)f2bf(rv - 1.0f) | ((uint32_t)f2bf(jv) << 16);
                    h[u] = ok ? make_uint2(lo, hi) : make_uint2(0, 0);
                }
                A[i] = __builtin_bit_cast(bf16x8, make_uint4(h[0].x, h[0].y, h[1].x, h[1].y));
            }
        } else if (MODE == kFirst && a.C1 < 4) {
            // one to three channels per pixel (the head's output gradient),
            // the missing ones zero: indices clamped into the grid so that
            // the loads are unconditional, taps outside it zeroed afterwards
            const int t0 = (k0 + kq) >> 2;
#pragma unroll
            for (int i = 0; i < TM; ++i) {
                uint2 h[2];
#pragma unroll
                for (int u = 0; u < 2; ++u) {
                    const int t = t0 + u, tc = t < 9 ? t : 8;
                    const int yy = px[i].y + tc / 3 - 1, xx = px[i].x + tc % 3 - 1;
                    const bool ok = px[i].ok && t < 9 && yy >= 0 && yy < a.H && xx >= 0 && xx < a.W;
                    const long q = px[i].ok ? ((long)px[i].n * a.H + min(max(yy, 0), a.H - 1)) * a.W +
                                                  min(max(xx, 0), a.W - 1)
                                            : 0;
                    const uint16_t* e = a.in1 + a.C1 * q;
                    const uint32_t c1 = a.C1 > 1 ? e[1] : 0u, c2 = a.C1 > 2 ? e[2] : 0u;
                    const uint32_t lo = (uint32_t)e[0] | (c1 << 16), hi = c2;
                    h[u] = ok ? make_uint2(lo, hi) : make_uint2(0, 0);
                }
                A[i] = __builtin_bit_cast(bf16x8, make_uint4(h[0].x, h[0].y, h[1].x, h[1].y));
            }
        } else if (MODE == kFirst) {
            // k = 4 tap + c: this lane's 8 values are taps t0 and t0 + 1
            const int t0 = (k0 + kq) >> 2;
#pragma unroll
            for (int i = 0; i < TM; ++i) {
                uint2 h[2];
#pragma unroll
                for (int u = 0; u < 2; ++u) {
                    const int t = t0 + u, yy = px[i].y + t / 3 - 1, xx = px[i].x + t % 3 - 1;
                    const bool ok = px[i].ok && t < 9 && yy >= 0 && yy < a.H && xx >= 0 && xx < a.W;
                    h[u] = ok ? *(const uint2*)(a.in1 + (((long)px[i].n * a.H + yy) * a.W + xx) * 4) : make_uint2(0, 0);
                }
                A[i] = __builtin_bit_cast(bf16x8, make_uint4(h[0].x, h[0].y, h[1].x, h[1].y));
            }
        } else if (MODE == kUpDgrad) {
            // k = (m, n, co): gradient pixel (2y + m, 2x + n), channel co
            const int Cd = a.C1 >> 2, sub = k0 / Cd, co = k0 - sub * Cd + kq;
#pragma unroll
            for (int i = 0; i < TM; ++i) {
                const long src =
                    (((long)px[i].n * 2 * a.H + 2 * px[i].y + (sub >> 1)) * 2 * a.W + 2 * px[i].x + (sub & 1)) * Cd + co;
                A[i] = px[i].ok ? ld8(a.in1 + src) : zero;
            }
        } else if (MODE == kUpFwd) {
            // one tap: the operand row is the flat pixel itself
            const bool first = k0 < a.C1;
            const uint16_t* src = first ? a.in1 : a.in2;
            const int C = first ? a.C1 : a.C2, c = (first ? k0 : k0 - a.C1) + kq;
#pragma unroll
            for (int i = 0; i < TM; ++i)
                A[i] = px[i].ok ? ld8(src + (size_t)(pm + 16 * i + r) * C + c) : zero;
        } else {
            const bool first = k0 < a.C1;
            const uint16_t* src = first ? a.in1 : a.in2;
            const int C = first ? a.C1 : a.C2, c = (first ? k0 : k0 - a.C1) + kq;
#pragma unroll
            for (int i = 0; i < TM; ++i) {
                const int yy = px[i].y + dy, xx = px[i].x + dx;
                const bool ok = px[i].ok && yy >= 0 && yy < a.H && xx >= 0 && xx < a.W;
                A[i] = ok ? ld8(src + (((long)px[i].n * a.H + yy) * a.W + xx) * C + c) : zero;
            }
        }
        const uint16_t* wt = wlane + (size_t)tap * a.ldo * a.ldk + k0;
#pragma unroll
        for (int j = 0; j < TN; ++j) B[j] = ld8(wt + (size_t)(16 * j) * a.ldk);
    };
    if constexpr (MODE == kUpFwd || MODE == kFirst) {
        // few K steps (the up-sampling's 2-8, the first layer's 2): the
        // operands of GI steps are loaded back to back, so a block waits
        // for one memory latency per group instead of one per step
        constexpr int GI = TM + TN <= 4 ? 4 : 2;
        for (int g0 = 0; g0 < iters; g0 += GI) {
            bf16x8 A[GI][TM], B[GI][TN];
#pragma unroll
            for (int u = 0; u < GI; ++u)
                if (g0 + u < iters) load(g0 + u, A[u], B[u]);
#pragma unroll
            for (int u = 0; u < GI; ++u) {
                if (g0 + u >= iters) break;
#pragma unroll
                for (int i = 0; i < TM; ++i)
#pragma unroll
                    for (int j = 0; j < TN; ++j)
                        acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A[u][i], B[u][j], acc[i][j], 0, 0, 0);
            }
        }
    } else {
        // register double buffer: the loads of iteration it + 1 are in flight
        // while the MFMAs of iteration it run
        bf16x8 A[TM], B[TN];
        load(0, A, B);
        for (int it = 0; it < iters; ++it) {
            bf16x8 An[TM], Bn[TN];
            if (it + 1 < iters) load(it + 1, An, Bn);
#pragma unroll
            for (int i = 0; i < TM; ++i)
#pragma unroll
                for (int j = 0; j < TN; ++j)
                    acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A[i], B[j], acc[i][j], 0, 0, 0);
            if (it + 1 < iters) {
#pragma unroll
                for (int i = 0; i < TM; ++i) A[i] = An[i];
#pragma unroll
                for (int j = 0; j < TN; ++j) B[j] = Bn[j];
            }
        }
    }
    // acc[i][j][e]: pixel pm + 16 i + 4 (lane / 16) + e, channel on + 16 j + r
    const int rq = (lane >> 4) * 4;
    if constexpr (MODE == kUpFwd) {
        if (a.out_bf16 && !a.out_f32 && ((a.Nout >> 2) & 7) == 0) {
            // BF16 output staged through LDS as [pixel][output column] and
            // written back as 16-byte runs of 8 channels of one output pixel
            // (consecutive threads take consecutive runs: the two sub-pixels
            // of a row and the next input pixel's are adjacent in memory)
            constexpr int BM = WGM * TM * 16, BN = WGN * TN * 16, LP = BN + 8;
            __shared__ __align__(16) uint16_t stg[BM * LP];
            const int pl = (wv % WGM) * TM * 16, ol = (wv / WGM) * TN * 16;
#pragma unroll
            for (int i = 0; i < TM; ++i)
#pragma unroll
                for (int j = 0; j < TN; ++j)
#pragma unroll
                    for (int e = 0; e < 4; ++e) stg[(pl + 16 * i + rq + e) * LP + ol + 16 * j + r] = f2bf(acc[i][j][e]);
            __syncthreads();
            const unsigned Co = (unsigned)a.Nout >> 2, W2 = 2u * (unsigned)a.W;
            const int pb = blockIdx.x * BM, obase = blockIdx.y * BN;
            for (int idx = threadIdx.x; idx < BM * (BN / 8); idx += 256) {
                const int p = idx / (BN / 8), q = idx - p * (BN / 8);
                const int gp = pb + p, o = obase + 8 * q;
                if (gp >= P || o >= a.Nout) continue;
                const Pix t = pix(gp, a.H, a.W, P);
                const unsigned sub = (unsigned)o / Co, co = (unsigned)o - sub * Co;
                const unsigned dst = ((((unsigned)t.n * 2u * (unsigned)a.H + 2u * (unsigned)t.y + (sub >> 1)) * W2 +
                                       2u * (unsigned)t.x + (sub & 1)) * Co + co);
                st16wt(a.out_bf16, 2 * (size_t)dst, *(const uint4*)(&stg[p * LP + 8 * q]));
            }
            return;
        }
        // sub-pixel scatter: one coordinate decomposition per 4 pixels (the
        // next three step along the row, wrapping where W is not a multiple
        // of 4) and the sub-pixel / channel split once per column tile
        // (32-bit element offsets: the launcher checks the output size)
        const unsigned Co = (unsigned)a.Nout >> 2, W2 = 2u * (unsigned)a.W;
        unsigned offj[TN];
#pragma unroll
        for (int j = 0; j < TN; ++j) {
            const unsigned o = (unsigned)(on + 16 * j + r), sub = o / Co;
            offj[j] = ((sub >> 1) * W2 + (sub & 1)) * Co + (o - sub * Co);
        }
#pragma unroll
        for (int i = 0; i < TM; ++i) {
            const int p0 = pm + 16 * i + rq;
            if (p0 >= P) continue;
            const Pix t0 = pix(p0, a.H, a.W, P);
            int n = t0.n, y = t0.y, x = t0.x;
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                if (e) {
                    ++x;
                    while (x >= a.W) {
                        x -= a.W;
                        if (++y >= a.H) {
                            y = 0;
                            ++n;
                        }
                    }
                }
                if (p0 + e >= P) continue;
                const unsigned row = (((unsigned)n * 2u * (unsigned)a.H + 2u * (unsigned)y) * W2 + 2u * (unsigned)x) * Co;
#pragma unroll
                for (int j = 0; j < TN; ++j) {
                    if (on + 16 * j + r >= a.Nout) continue;
                    const unsigned idx = row + offj[j];
                    const float v = acc[i][j][e];
                    if (a.out_f32) stwt(a.out_f32, idx, v);
                    if (a.out_bf16) a.out_bf16[idx] = f2bf(v);
                }
            }
        }
        return;
    }
    constexpr int BM = WGM * TM * 16, BN = WGN * TN * 16;
    if ((MODE == kFirst || MODE == kConvFwd) && a.out_f32 && !a.out_bf16 && a.O1 == a.Nout && a.Nout == BN) {
        // the block holds every output channel of its BM consecutive pixels,
        // so its FP32 output is one contiguous run: staged through LDS as
        // [pixel][channel] and written back as 16-byte pieces in order
        constexpr int LPF = BN + 4;   // 4 lane groups land 16 banks apart
        static_assert((MODE != kFirst && MODE != kConvFwd) || BM * LPF <= kStfFloats, "output stage fits");
        float* stf = (float*)smem;
        if (MODE == kFirst && xs) __syncthreads();   // every wave is done with the input stage
        const int pl = (wv % WGM) * TM * 16, ol = (wv / WGM) * TN * 16;
#pragma unroll
        for (int i = 0; i < TM; ++i)
#pragma unroll
            for (int j = 0; j < TN; ++j)
#pragma unroll
                for (int e = 0; e < 4; ++e) stf[(pl + 16 * i + rq + e) * LPF + ol + 16 * j + r] = acc[i][j][e];
        __syncthreads();
        const int pb = blockIdx.x * BM;
        for (int idx = threadIdx.x; idx < BM * (BN / 4); idx += 256) {
            const int p = idx / (BN / 4), q = idx - p * (BN / 4);
            if (pb + p >= P) break;
            const f32x4 v = *(const f32x4*)(&stf[p * LPF + 4 * q]);
            st16wt(a.out_f32, 4 * ((size_t)(pb + p) * BN + 4 * q), __builtin_bit_cast(uint4, v));
        }
    } else {
#pragma unroll
        for (int j = 0; j < TN; ++j) {
            const int o = on + 16 * j + r;
            if (o >= a.Nout) continue;
#pragma unroll
            for (int i = 0; i < TM; ++i)
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    const int p = pm + 16 * i + rq + e;
                    if (p >= P) continue;
                    const float v = acc[i][j][e];
                    if (o < a.O1) {
                        const size_t idx = (size_t)p * a.O1 + o;
                        if (a.out_f32) stwt(a.out_f32, idx, v);
                        if (a.out_bf16) a.out_bf16[idx] = f2bf(v);
                    } else {
                        const size_t idx = (size_t)p * (a.Nout - a.O1) + (o - a.O1);
                        if (a.out2_f32) a.out2_f32[idx] = v;
                        if (a.out2_bf16) a.out2_bf16[idx] = f2bf(v);
                    }
                }
        }
    }
    if ((MODE == kConvFwd || MODE == kFirst) && a.gsum) {
        // per-channel sum and sum of squares over the block's pixels (all in
        // one sample): lanes r, r+16, r+32, r+48 share a channel, then the
        // WGM waves of a block column are added in order
        __shared__ float red[WGM][WGN * TN * 16][2];
        const int wm = wv % WGM, col = (wv / WGM) * TN * 16;
#pragma unroll
        for (int j = 0; j < TN; ++j) {
            float s1 = 0.f, s2 = 0.f;
#pragma unroll
            for (int i = 0; i < TM; ++i)
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    s1 += acc[i][j][e];
                    s2 = fmaf(acc[i][j][e], acc[i][j][e], s2);
                }
            s1 += __shfl_xor(s1, 16);
            s2 += __shfl_xor(s2, 16);
            s1 += __shfl_xor(s1, 32);
            s2 += __shfl_xor(s2, 32);
            if (lane < 16) {
                red[wm][col + 16 * j + r][0] = s1;
                red[wm][col + 16 * j + r][1] = s2;
            }
        }
        __syncthreads();
        constexpr int BM = WGM * TM * 16;
        const long Ps = (long)a.H * a.W, b0 = (long)blockIdx.x * BM;
        const int n = (int)(b0 / Ps), tiles = (int)(Ps / BM), t = (int)((b0 - n * Ps) / BM);
        for (int c = threadIdx.x; c < WGN * TN * 16; c += 256) {
            const int o = blockIdx.y * (WGN * TN * 16) + c;
            if (o >= a.Nout) continue;
            float s1 = 0.f, s2 = 0.f;
            for (int w = 0; w < WGM; ++w) {
                s1 += red[w][c][0];
                s2 += red[w][c][1];
            }
            float* g = a.gsum + (((size_t)n * a.Nout + o) * tiles + t) * 2;
            g[0] = s1;
            g[1] = s2;
        }
    }
}

// ---------------------------------------------------------------------------
// Halo-tile variant of the 3x3 convolution (forward and input gradient) for
// channel counts that are multiples of 32.  A block owns a TH x TW pixel
// tile of one sample and TN x 16 output channels; for every 32-channel chunk
// of the input the (TH + 2) x (TW + 2) halo and the chunk's weights of all
// nine taps are staged in LDS once (each 64-byte row padded to 80 so that
// the MFMA-layout 16-byte reads of 8 consecutive rows fall in distinct
// banks) and every tap reads its operands from there; the next chunk is
// loaded into registers while the current one is used.  Wave w takes tile rows TH/4 w .. and their TW/16 16-pixel
// segments (TM = TH/4 * TW/16 operand tiles).
// KC input channels per staged chunk (32, or 64 where every chunk stays
// inside one input: half as many load -> barrier -> multiply rounds, which
// bound the small grids of the deep levels); staged rows of KC + 8 BF16
// elements (80 or 144 bytes: 8 consecutive rows start 16 bytes apart modulo
// 128, so the MFMA-layout reads are conflict-free)
// GNIN: the input is normalised as it is staged (see ConvArgs::gn_y): the
// halo pieces are loaded as FP32, and each becomes 8 BF16 values with the
// arithmetic of the normalisation kernel before it is stored in LDS
template <int MODE, int TN, int TH, int TW, int KC, bool GNIN = false>
__global__ __launch_bounds__(256, (TN == 2 && KC == 32) ? 3 : 2) void conv3_lds_kernel(ConvArgs a)
{
    constexpr int LP = KC + 8;              // BF16 elements per staged row
    constexpr int PPX = KC / 8;             // 16-byte pieces per staged row
    constexpr int HP = TH + 2, WP = TW + 2, NPX = HP * WP;
    constexpr int SEG = TW / 16, TM = (TH / 4) * SEG;
    constexpr int NA = NPX * PPX;           // 16-byte halo pieces per chunk
    constexpr int NB = 9 * TN * 16 * PPX;   // 16-byte weight pieces per chunk
    constexpr int NLD = (NA + NB + 255) / 256;
    // one chunk's halo [NPX][LP] and weights [9][TN 16][LP]
    __shared__ __align__(16) uint16_t lds[(NPX + 9 * TN * 16) * LP];
    uint16_t* const wl = lds + NPX * LP;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, tid = threadIdx.x;
    const int r = lane & 15, kq = (lane >> 4) * 8;
    const int tx = (a.W + TW - 1) / TW, ty = (a.H + TH - 1) / TH;
    const int tpb = tx * ty;
    const int n = blockIdx.x / tpb, t = blockIdx.x - n * tpb;
    const int y0 = (t / tx) * TH, x0 = (t % tx) * TW;
    const int on = blockIdx.y * (TN * 16);
    const int K = a.C1 + a.C2, nk = K / KC;
    // this lane's operand pixel in each of its TM tiles (tile coordinates)
    int ry[TM], cx[TM];
#pragma unroll
    for (int i = 0; i < TM; ++i) {
        ry[i] = wv * (TH / 4) + i / SEG;
        cx[i] = (i % SEG) * 16 + r;
    }
    f32x4 acc[TM][TN];
#pragma unroll
    for (int i = 0; i < TM; ++i)
#pragma unroll
        for (int j = 0; j < TN; ++j) acc[i][j] = (f32x4){0.f, 0.f, 0.f, 0.f};

    // piece e < NA: halo pixel e / PPX, channels 8 (e % PPX) ..; else weight
    // row (tap, o) = (e - NA) / PPX of the chunk, k = 8 ((e - NA) % PPX) ..
    uint4 stage[NLD];
    // Both inputs have the same channel count (or there is one; the launcher
    // checks), so every piece's source differs between chunks only by the
    // chunk's channel offset, which goes into a uniform base pointer: the
    // per-piece byte offsets (~0 for halo pixels outside the image and unused
    // pieces) are computed once, and a chunk's loads take no index arithmetic.
    uint32_t goff[NLD];
#pragma unroll
    for (int u = 0; u < NLD; ++u) {
        const int e = tid + 256 * u;
        goff[u] = ~0u;
        if (e < NA) {
            const int px = e / PPX, q = e % PPX;
            const int gy = y0 - 1 + px / WP, gx = x0 - 1 + px % WP;
            if (gy >= 0 && gy < a.H && gx >= 0 && gx < a.W)
                goff[u] = (GNIN ? 4u : 2u) * (uint32_t)((((n * a.H + gy) * a.W + gx) * a.C1) + 8 * q);
        } else if (e < NA + NB) {
            const int row = (e - NA) / PPX, q = (e - NA) % PPX;
            const int tap = row / (TN * 16), o = row - tap * (TN * 16);
            goff[u] = 2u * (uint32_t)((tap * a.ldo + on + o) * a.ldk + 8 * q);
        }
    }
    // GNIN: the second 16 bytes of each halo piece, and this thread's 8
    // channels' A and B (every piece of a thread has channels 8 (tid % PPX) ..)
    [[maybe_unused]] uint4 stage2[GNIN ? NLD : 1];
    [[maybe_unused]] float gA[GNIN ? 8 : 1], gB[GNIN ? 8 : 1];
    auto gload = [&](int kc) {
        const int k0 = kc * KC;
        const char* hb = GNIN ? (const char*)(a.gn_y + k0)
                              : (const char*)(k0 < a.C1 ? a.in1 + k0 : a.in2 + (k0 - a.C1));
        const char* wb = (const char*)(a.Wt + k0);
        if constexpr (GNIN) {
            const float* cf = a.gn_coef + (size_t)n * a.C1 + k0 + 8 * (tid % PPX);
#pragma unroll
            for (int i = 0; i < 8; ++i) {
                gA[i] = cf[i];
                gB[i] = cf[(size_t)a.N * a.C1 + i];
            }
        }
#pragma unroll
        for (int u = 0; u < NLD; ++u) {
            const int e = tid + 256 * u;
            uint4 v = make_uint4(0, 0, 0, 0);
            if (goff[u] != ~0u) v = *(const uint4*)((e < NA ? hb : wb) + goff[u]);
            stage[u] = v;
            if constexpr (GNIN) {
                uint4 v2 = make_uint4(0, 0, 0, 0);
                if (e < NA && goff[u] != ~0u) v2 = *(const uint4*)(hb + goff[u] + 16);
                stage2[u] = v2;
            }
        }
    };
    // piece e = tid + 256 u lands at row e / PPX, column 8 (e % PPX): 256 is
    // a multiple of PPX, so that is this thread's first slot plus a constant
    const int l0 = (tid / PPX) * LP + 8 * (tid % PPX);
    auto lstore = [&]() {
#pragma unroll
        for (int u = 0; u < NLD; ++u) {
            const int e = tid + 256 * u;
            uint4 v = stage[u];
            if constexpr (GNIN) {
                if (e < NA) {
                    // z = act(A y + B) as the normalisation kernel forms it;
                    // halo pixels outside the image stay zero
                    const float y[8] = {__builtin_bit_cast(float, stage[u].x), __builtin_bit_cast(float, stage[u].y),
                                        __builtin_bit_cast(float, stage[u].z), __builtin_bit_cast(float, stage[u].w),
                                        __builtin_bit_cast(float, stage2[u].x), __builtin_bit_cast(float, stage2[u].y),
                                        __builtin_bit_cast(float, stage2[u].z), __builtin_bit_cast(float, stage2[u].w)};
                    uint32_t h[8];
#pragma unroll
                    for (int i = 0; i < 8; ++i) {
                        const float av = fmaf(gA[i], y[i], gB[i]);
                        h[i] = goff[u] != ~0u ? f2bf(a.gn_gelu ? gelu(av) : av) : 0u;
                    }
                    v = make_uint4(h[0] | (h[1] << 16), h[2] | (h[3] << 16), h[4] | (h[5] << 16), h[6] | (h[7] << 16));
                }
            }
            if (e < NA + NB) *(uint4*)(&lds[l0 + (256 / PPX) * LP * u]) = v;
        }
    };
    gload(0);
    for (int kc = 0; kc < nk; ++kc) {
        if (kc) __syncthreads();   // every wave is done with the previous chunk
        lstore();
        __syncthreads();
        if (kc + 1 < nk) gload(kc + 1);
        // per 32-channel step and tap row: the operands of the row's left
        // and right taps come from LDS; the centre tap's (one pixel over)
        // are the left ones moved one lane down each 16-lane row by a DPP
        // shift, lane 15 taking the right operand of lane 14 (a third fewer
        // LDS reads)
#pragma unroll
        for (int ks = 0; ks < KC / 32; ++ks)
#pragma unroll
            for (int ty = 0; ty < 3; ++ty) {
                const int dy = MODE == kConvDgrad ? 1 - ty : ty - 1;
                bf16x8 L[TM], R[TM], M[TM];
#pragma unroll
                for (int i = 0; i < TM; ++i) {
                    const int row = ((ry[i] + 1 + dy) * WP + cx[i]) * LP + 32 * ks + kq;
                    L[i] = *(const bf16x8*)(&lds[row]);
                    R[i] = *(const bf16x8*)(&lds[row + 2 * LP]);
                }
#pragma unroll
                for (int i = 0; i < TM; ++i) {
                    const u32x4v l = __builtin_bit_cast(u32x4v, L[i]), rr = __builtin_bit_cast(u32x4v, R[i]);
                    u32x4v m;
#pragma unroll
                    for (int d = 0; d < 4; ++d) {
                        const int r15 = __builtin_amdgcn_update_dpp(0, (int)rr[d], kRowShr1, 0xF, 0xF, false);
                        m[d] = (unsigned)__builtin_amdgcn_update_dpp(r15, (int)l[d], kRowShl1, 0xF, 0xF, false);
                    }
                    M[i] = __builtin_bit_cast(bf16x8, m);
                }
#pragma unroll
                for (int tx = 0; tx < 3; ++tx) {
                    const int tap = ty * 3 + tx;
                    // forward: tap columns -1, 0, +1; input gradient mirrored
                    const int side = MODE == kConvDgrad ? 2 - tx : tx;
                    bf16x8 B[TN];
#pragma unroll
                    for (int j = 0; j < TN; ++j)
                        B[j] = *(const bf16x8*)(&wl[(tap * TN * 16 + 16 * j + r) * LP + 32 * ks + kq]);
#pragma unroll
                    for (int i = 0; i < TM; ++i) {
                        const bf16x8 A = side == 0 ? L[i] : side == 1 ? M[i] : R[i];
#pragma unroll
                        for (int j = 0; j < TN; ++j)
                            acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A, B[j], acc[i][j], 0, 0, 0);
                    }
                }
            }
    }
    __syncthreads();   // LDS is reused by the epilogue's reduction
    // acc[i][j][e]: pixel (ry[i], segment base + 4 (lane / 16) + e), channel on + 16 j + r.
    // FP32 outputs are written through (stwt, st16wt): a later kernel reads
    // them
    const int rq = (lane >> 4) * 4;
    float s1[TN], s2[TN];
#pragma unroll
    for (int j = 0; j < TN; ++j) s1[j] = s2[j] = 0.f;
    static_assert(TH * TW * TN * 16 * 4 <= (int)sizeof(lds), "the staged output tile fits in LDS");
    // the output that takes the block's channels, when it is one
    const bool part1 = on + TN * 16 <= a.O1, part2 = on >= a.O1;
    float* const out_f = part1 ? a.out_f32 : part2 ? a.out2_f32 : nullptr;
    uint16_t* const out_b = part1 ? a.out_bf16 : part2 ? a.out2_bf16 : nullptr;
    const int out_cs = part1 ? a.O1 : a.Nout - a.O1, out_co = part1 ? on : on - a.O1;
    const bool stage_out = (part1 || part2) && (out_f != nullptr) != (out_b != nullptr) &&
                           out_cs % (out_f ? 4 : 8) == 0;
    if (MODE == kConvFwd && a.out_f32 && !a.out_bf16 && a.O1 == a.Nout && a.Nout <= TN * 16 && on == 0 &&
        a.W % TW == 0 && (TW * a.Nout) % 4 == 0) {
        // the block holds every output channel of its tile, so each tile row
        // of its FP32 output is one contiguous run of TW Nout values: staged
        // through LDS in memory order and written back as 16-byte pieces
        float* stg = (float*)&lds[0];
#pragma unroll
        for (int j = 0; j < TN; ++j) {
            const int o = 16 * j + r;
#pragma unroll
            for (int i = 0; i < TM; ++i)
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    if (o >= a.Nout || y0 + ry[i] >= a.H) continue;
                    const float v = acc[i][j][e];
                    s1[j] += v;
                    s2[j] = fmaf(v, v, s2[j]);
                    stg[(ry[i] * TW + (i % SEG) * 16 + rq + e) * a.Nout + o] = v;
                }
        }
        __syncthreads();
        const int rows = min(TH, a.H - y0), run4 = TW * a.Nout / 4;
        for (int idx = tid; idx < rows * run4; idx += 256) {
            const int yy = idx / run4, q = idx - yy * run4;
            const f32x4 v = *(const f32x4*)(&stg[yy * TW * a.Nout + 4 * q]);
            st16wt(a.out_f32, 4 * ((((size_t)n * a.H + y0 + yy) * a.W + x0) * a.Nout + 4 * q),
                   __builtin_bit_cast(uint4, v));
        }
        __syncthreads();   // the reduction below reuses LDS
    } else if (stage_out) {
        // the block's channels [on, on + 16 TN) of each pixel are one 16-byte
        // aligned run of one output (the first's O1 channels or the second's
        // Nout - O1, FP32 or BF16): staged through LDS as [pixel][channel]
        // and written back as 16-byte pieces
        constexpr int SP = TN * 16 + 4;   // 4 lane groups land 16 banks apart
        static_assert(TH * TW * SP * 4 <= (int)sizeof(lds), "the staged output tile fits in LDS");
        float* stg = (float*)&lds[0];
#pragma unroll
        for (int j = 0; j < TN; ++j) {
            const int o = on + 16 * j + r;
#pragma unroll
            for (int i = 0; i < TM; ++i)
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    const int y = y0 + ry[i], x = x0 + (i % SEG) * 16 + rq + e;
                    if (o >= a.Nout || y >= a.H || x >= a.W) continue;
                    const float v = acc[i][j][e];
                    s1[j] += v;
                    s2[j] = fmaf(v, v, s2[j]);
                    stg[(ry[i] * TW + (i % SEG) * 16 + rq + e) * SP + 16 * j + r] = v;
                }
        }
        __syncthreads();
        const int pw = out_f ? 4 : 8;                       // channels per 16-byte piece
        const int nq = min(TN * 16, out_cs - out_co) / pw;  // pieces per pixel
        for (int idx = tid; idx < TH * TW * nq; idx += 256) {
            const int pp = idx / nq, q = idx - pp * nq;
            const int y = y0 + pp / TW, x = x0 + pp % TW;
            if (y >= a.H || x >= a.W) continue;
            const size_t e = (((size_t)n * a.H + y) * a.W + x) * out_cs + out_co + pw * q;
            if (out_f) {
                const f32x4 v = *(const f32x4*)(&stg[pp * SP + 4 * q]);
                st16wt(out_f, 4 * e, __builtin_bit_cast(uint4, v));
            } else {
                const f32x4 v0 = *(const f32x4*)(&stg[pp * SP + 8 * q]), v1 = *(const f32x4*)(&stg[pp * SP + 8 * q + 4]);
                const uint32_t w0 = (uint32_t)f2bf(v0[0]) | ((uint32_t)f2bf(v0[1]) << 16);
                const uint32_t w1 = (uint32_t)f2bf(v0[2]) | ((uint32_t)f2bf(v0[3]) << 16);
                const uint32_t w2 = (uint32_t)f2bf(v1[0]) | ((uint32_t)f2bf(v1[1]) << 16);
                const uint32_t w3 = (uint32_t)f2bf(v1[2]) | ((uint32_t)f2bf(v1[3]) << 16);
                st16wt(out_b, 2 * e, make_uint4(w0, w1, w2, w3));
            }
        }
        __syncthreads();   // the reduction below reuses LDS
    } else {
#pragma unroll
        for (int j = 0; j < TN; ++j) {
            const int o = on + 16 * j + r;
#pragma unroll
            for (int i = 0; i < TM; ++i)
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    const int y = y0 + ry[i], x = x0 + (i % SEG) * 16 + rq + e;
                    if (o >= a.Nout || y >= a.H || x >= a.W) continue;
                    const float v = acc[i][j][e];
                    s1[j] += v;
                    s2[j] = fmaf(v, v, s2[j]);
                    const size_t p = ((size_t)n * a.H + y) * a.W + x;
                    if (o < a.O1) {
                        const size_t idx = p * a.O1 + o;
                        if (a.out_f32) stwt(a.out_f32, idx, v);
                        if (a.out_bf16) a.out_bf16[idx] = f2bf(v);
                    } else {
                        const size_t idx = p * (a.Nout - a.O1) + (o - a.O1);
                        if (a.out2_f32) a.out2_f32[idx] = v;
                        if (a.out2_bf16) a.out2_bf16[idx] = f2bf(v);
                    }
                }
        }
    }
    if (MODE == kConvFwd && a.gsum) {
        // per-channel sums over the tile: the 4 lane groups, then the 4 waves
        // in order (LDS reused after the barrier that ended the main loop)
        float* red = (float*)&lds[0];
#pragma unroll
        for (int j = 0; j < TN; ++j) {
            float u1 = s1[j], u2 = s2[j];
            u1 += __shfl_xor(u1, 16);
            u2 += __shfl_xor(u2, 16);
            u1 += __shfl_xor(u1, 32);
            u2 += __shfl_xor(u2, 32);
            if (lane < 16) {
                red[(wv * TN * 16 + 16 * j + r) * 2] = u1;
                red[(wv * TN * 16 + 16 * j + r) * 2 + 1] = u2;
            }
        }
        __syncthreads();
        for (int c = tid; c < TN * 16; c += 256) {
            const int o = on + c;
            if (o >= a.Nout) continue;
            float u1 = 0.f, u2 = 0.f;
            for (int w = 0; w < 4; ++w) {
                u1 += red[(w * TN * 16 + c) * 2];
                u2 += red[(w * TN * 16 + c) * 2 + 1];
            }
            float* g = a.gsum + (((size_t)n * a.Nout + o) * tpb + t) * 2;
            g[0] = u1;
            g[1] = u2;
        }
    }
}

// Partial weight gradient over one pixel chunk: rows o (output channels),
// columns k (input channels), k-dimension = 16 pixels per MFMA.
// blockIdx.z = chunk * taps + tap.
template <int MODE>
__global__ __launch_bounds__(256) void wgrad_kernel(WgradArgs a)
{
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int o0 = blockIdx.x * 64 + (wv & 1) * 32;
    const int k0 = blockIdx.y * 64 + (wv >> 1) * 32;
    constexpr int ntaps = MODE == kConvFwd ? 9 : 1;
    const int tap = (int)(blockIdx.z % ntaps), chunk = (int)(blockIdx.z / ntaps);
    const int dy = ntaps == 9 ? tap / 3 - 1 : 0, dx = ntaps == 9 ? tap % 3 - 1 : 0;
    const int r = lane & 15, pq = (lane >> 4) * 4;
    const int P = a.N * a.H * a.W, K = a.C1 + a.C2;
    const int pb = chunk * a.chunk, pe = min(P, pb + a.chunk);
    f32x4 acc[2][2] = {};
    for (int p0 = pb; p0 < pe; p0 += 16) {
        bf16x4 A[2], B[2];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int p = p0 + pq + j;
            const Pix q = pix(p, a.H, a.W, pe);
            const int yy = q.y + dy, xx = q.x + dx;
            const bool xin = q.ok && yy >= 0 && yy < a.H && xx >= 0 && xx < a.W;
            const size_t xoff = ((size_t)q.n * a.H + yy) * a.W + xx;
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                const int o = o0 + 16 * h + r, k = k0 + 16 * h + r;
                uint16_t va = 0, vb = 0;
                if (q.ok && o < a.Nout) {
                    if (MODE == kUpFwd) {
                        const int Co = a.Nout >> 2, sub = o / Co, co = o - sub * Co;
                        va = a.dy[(((size_t)q.n * 2 * a.H + 2 * q.y + (sub >> 1)) * 2 * a.W + 2 * q.x + (sub & 1)) * Co +
                                  co];
                    } else {
                        va = a.dy[(size_t)p * a.Nout + o];
                    }
                }
                if (xin && k < K) vb = k < a.C1 ? a.x1[xoff * a.C1 + k] : a.x2[xoff * a.C2 + (k - a.C1)];
                A[h][j] = (short)va;
                B[h][j] = (short)vb;
            }
        }
        acc[0][0] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(A[0], B[0], acc[0][0], 0, 0, 0);
        acc[0][1] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(A[0], B[1], acc[0][1], 0, 0, 0);
        acc[1][0] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(A[1], B[0], acc[1][0], 0, 0, 0);
        acc[1][1] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(A[1], B[1], acc[1][1], 0, 0, 0);
    }
    // acc[mi][ni][j]: row o = o0 + 16 mi + pq + j, column k = k0 + 16 ni + r
    float* part = a.partial + ((size_t)chunk * ntaps + tap) * a.Nout * K;
#pragma unroll
    for (int mi = 0; mi < 2; ++mi)
#pragma unroll
        for (int ni = 0; ni < 2; ++ni) {
            const int k = k0 + 16 * ni + r;
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const int o = o0 + 16 * mi + pq + j;
                if (o < a.Nout && k < K) part[(size_t)o * K + k] = acc[mi][ni][j];
            }
        }
}

// Staged weight gradient: per 64-pixel step the block loads dy[64 pixels][64 o]
// and x[64 pixels][64 k] (x at the tap's shifted pixel, zero outside) and
// stores them transposed in LDS ([channel][pixel], rows padded by 8
// elements), so each lane's MFMA operand (8 consecutive pixels of one
// channel) is one 16-byte read; each wave forms a 32 x 32 sub-tile with
// 2 x 2 v_mfma_f32_16x16x32_bf16 per 32 pixels.  A thread stages two
// adjacent pixels of one 8-channel group and writes each channel's pair as
// one 32-bit word: the 32 pairs of a wave land in 32 consecutive banks and
// the wave's second channel group 32 banks further (row pitch 36 words), so
// the transposition is free of bank conflicts.  The next step's operands are
// loaded into registers while the current step is multiplied.  VEC: all
// channel counts are multiples of 8 and rows 16-byte aligned (16-byte loads);
// else 8 guarded 2-byte loads per piece; with FOLD 2, VEC concerns the
// input side; with FOLD 1, dy and the folded 4-channel input, read as 8-byte
// tap pairs.  FOLD (3x3 layers with fewer than 8 channels on one side): 1
// folds the nine taps into the input-channel side (row k' = 9-tap index * K
// + c of x at the tap's shifted pixel), 2 into the output side (row
// o' = tap * Nout + o of dy at the pixel shifted back, which pairs the same
// products); one block then covers all taps.
// blockIdx.z = chunk * taps + tap (taps = 9 unfolded 3x3, else 1).
constexpr int kWgStep = 64;                // pixels per step
constexpr int kWgRow = kWgStep + 8;        // LDS row length (elements)

template <int MODE, bool VEC, int FOLD>
__global__ __launch_bounds__(256) void wgrad32_kernel(WgradArgs a)
{
    __shared__ __align__(16) uint16_t As[64 * kWgRow];
    __shared__ __align__(16) uint16_t Bs[64 * kWgRow];
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int o0 = blockIdx.x * 64, k0 = blockIdx.y * 64;
    constexpr int ntaps = MODE == kConvFwd && FOLD == 0 ? 9 : 1;
    const int tap = (int)(blockIdx.z % ntaps), chunk = (int)(blockIdx.z / ntaps);
    const int dy = ntaps == 9 ? tap / 3 - 1 : 0, dx = ntaps == 9 ? tap % 3 - 1 : 0;
    const int P = a.N * a.H * a.W, K = a.C1 + a.C2;
    const int Ko = FOLD == 1 ? 9 * K : K, No = FOLD == 2 ? 9 * a.Nout : a.Nout;
    const int pb = chunk * a.chunk, pe = min(P, pb + a.chunk);
    // staging: pixels p0 + 2 pp + u (u = 0, 1), channels sg .. sg + 7
    const int pp = tid & 31, sg = (tid >> 5) * 8;
    const int wo = (wv & 1) * 32, wk = (wv >> 1) * 32;
    const int r = lane & 15, kq = (lane >> 4) * 8;
    f32x4 acc[2][2] = {};

    auto piece = [&](const uint16_t* base, int C, int c, bool ok, bool vec) {
        uint4 v = make_uint4(0, 0, 0, 0);
        if (!ok) return v;
        if (vec) return *(const uint4*)(base + c);
        uint16_t* e = (uint16_t*)&v;
        for (int j = 0; j < 8; ++j)
            if (c + j < C) e[j] = base[c + j];
        return v;
    };
    // folded rows: element j of the group is row g + j = t * C + c of the
    // field at pixel (y + sy (t / 3 - 1), x + sy (t % 3 - 1)) of sample n
    auto folded = [&](const uint16_t* f, int C, int g, const Pix& q, int sy) {
        uint4 v = make_uint4(0, 0, 0, 0);
        if (!q.ok) return v;
        if (VEC && FOLD == 1) {
            // C = 4 (the launcher checks): the 8 rows are all channels of
            // taps g / 4 and g / 4 + 1, one 8-byte load each
            uint2 h[2] = {make_uint2(0, 0), make_uint2(0, 0)};
#pragma unroll
            for (int u = 0; u < 2; ++u) {
                const int t = g / 4 + u;
                const int yy = q.y + sy * (t / 3 - 1), xx = q.x + sy * (t % 3 - 1);
                if (t < 9 && yy >= 0 && yy < a.H && xx >= 0 && xx < a.W)
                    h[u] = *(const uint2*)(f + (((size_t)q.n * a.H + yy) * a.W + xx) * 4);
            }
            return make_uint4(h[0].x, h[0].y, h[1].x, h[1].y);
        }
        // element j (static indices: the pieces stay in registers)
        uint32_t w[4] = {0u, 0u, 0u, 0u};
        int t = g / C, c = g - t * C;
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            if (t < 9) {
                const int yy = q.y + sy * (t / 3 - 1), xx = q.x + sy * (t % 3 - 1);
                if (yy >= 0 && yy < a.H && xx >= 0 && xx < a.W)
                    w[j / 2] |= (uint32_t)f[(((size_t)q.n * a.H + yy) * a.W + xx) * C + c] << (16 * (j & 1));
                if (++c == C) {
                    c = 0;
                    ++t;
                }
            }
        }
        return make_uint4(w[0], w[1], w[2], w[3]);
    };
    uint4 va[2], vb[2];
    auto gload = [&](int p0) {
#pragma unroll
        for (int u = 0; u < 2; ++u) {
            const int p = p0 + 2 * pp + u;
            const Pix q = pix(p, a.H, a.W, pe);
            const int o = o0 + sg;
            if (FOLD == 2) {
                va[u] = folded(a.dy, a.Nout, o, q, -1);
            } else if (MODE == kUpFwd) {
                // o = (m, n, co): gradient pixel (2y + m, 2x + n); 8-runs stay in one m, n
                const int Co = a.Nout >> 2, sub = o / Co, co = o - sub * Co;
                const uint16_t* base =
                    a.dy + (((size_t)q.n * 2 * a.H + 2 * q.y + (sub >> 1)) * 2 * a.W + 2 * q.x + (sub & 1)) * Co;
                va[u] = piece(base, Co, co, q.ok && o < a.Nout, VEC);
            } else {
                va[u] = piece(a.dy + (size_t)p * a.Nout, a.Nout, o, q.ok && o < a.Nout, VEC);
            }
            const int k = k0 + sg;
            if (FOLD == 1) {
                vb[u] = folded(a.x1, a.C1, k, q, 1);
            } else {
                const int yy = q.y + dy, xx = q.x + dx;
                const bool xin = q.ok && yy >= 0 && yy < a.H && xx >= 0 && xx < a.W && k < K;
                const size_t xo = ((size_t)q.n * a.H + yy) * a.W + xx;
                if (k < a.C1) vb[u] = piece(a.x1 + xo * a.C1, a.C1, k, xin, VEC);
                else vb[u] = piece(a.x2 + xo * a.C2, a.C2, k - a.C1, xin, VEC);
            }
        }
    };
    gload(pb);
    for (int p0 = pb; p0 < pe; p0 += kWgStep) {
        __syncthreads();  // the previous step's operands have been read
        {
            const uint32_t* a0 = (const uint32_t*)&va[0];
            const uint32_t* a1 = (const uint32_t*)&va[1];
            const uint32_t* b0 = (const uint32_t*)&vb[0];
            const uint32_t* b1 = (const uint32_t*)&vb[1];
            uint32_t* Aw = (uint32_t*)As;
            uint32_t* Bw = (uint32_t*)Bs;
#pragma unroll
            for (int h = 0; h < 4; ++h) {
                // channels sg + 2h (low halves) and sg + 2h + 1 (high halves) of both pixels
                const int w0 = ((sg + 2 * h) * kWgRow) / 2 + pp, w1 = w0 + kWgRow / 2;
                Aw[w0] = (a0[h] & 0xffffu) | (a1[h] << 16);
                Aw[w1] = (a0[h] >> 16) | (a1[h] & 0xffff0000u);
                Bw[w0] = (b0[h] & 0xffffu) | (b1[h] << 16);
                Bw[w1] = (b0[h] >> 16) | (b1[h] & 0xffff0000u);
            }
        }
        __syncthreads();
        if (p0 + kWgStep < pe) gload(p0 + kWgStep);
#pragma unroll
        for (int s = 0; s < kWgStep; s += 32) {
            bf16x8 A[2], B[2];
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                A[h] = *(const bf16x8*)(&As[(wo + 16 * h + r) * kWgRow + s + kq]);
                B[h] = *(const bf16x8*)(&Bs[(wk + 16 * h + r) * kWgRow + s + kq]);
            }
#pragma unroll
            for (int mi = 0; mi < 2; ++mi)
#pragma unroll
                for (int ni = 0; ni < 2; ++ni)
                    acc[mi][ni] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A[mi], B[ni], acc[mi][ni], 0, 0, 0);
        }
    }
    // acc[mi][ni][e]: row o = o0 + wo + 16 mi + 4 (lane / 16) + e, column k = k0 + wk + 16 ni + r;
    // partial layout per chunk [tap][Nout][K] (folded rows o' = t Nout + o map
    // onto it directly; folded columns k' = t K + c are scattered)
    constexpr int chunk_taps = MODE == kConvFwd ? 9 : 1;
    float* part = a.partial + ((size_t)chunk * chunk_taps + tap) * a.Nout * K;
    const int rq = (lane >> 4) * 4;
#pragma unroll
    for (int mi = 0; mi < 2; ++mi)
#pragma unroll
        for (int ni = 0; ni < 2; ++ni) {
            const int kk = k0 + wk + 16 * ni + r;
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int oo = o0 + wo + 16 * mi + rq + e;
                if (oo >= No || kk >= Ko) continue;
                if (FOLD == 1) {
                    const int t = kk / K, c = kk - t * K;
                    part[((size_t)t * a.Nout + oo) * K + c] = acc[mi][ni][e];
                } else {
                    part[(size_t)oo * K + kk] = acc[mi][ni][e];
                }
            }
        }
}

// Halo-tile weight gradient of a 3x3 convolution, all nine taps in one
// block: dW[t][o][k] = sum_p dy[p][o] x[p + d(t)][k].  A block owns 32
// output channels o, 64 input channels k and a run of 4 x 32 pixel tiles of
// one or more samples; per tile it stages dy [128 px][32 o] and the 6 x 34
// halo of x [204 px][64 k] in LDS in their memory layout ([pixel][channel],
// 16-byte pieces) and reads the MFMA operands, whose contraction runs over
// pixels, with the LDS transpose read: in each 16-lane group, lane i gives
// the address of row i / 4, columns 4 (i % 4) .. + 3 of a 4 x 16 block of
// 16-bit values and receives column i, so with rows = 4 consecutive pixels
// and columns = 16 channels lane i gets channel i at those 4 pixels (two
// reads make one 8-pixel operand).  Wave w takes input channels 16 w .. of
// the block's 64, both 16-channel halves of its outputs and all nine taps:
// per 32-pixel row segment the two dy operands serve the nine taps and each
// tap's x operand both halves (22 transpose reads for 18 MFMAs; NARROW,
// fewer than 8 output channels: dy staged by 2-byte loads, one half).  Row
// pitches of 160 (x) and 96 (dy) bytes put the 16 addresses of a read in
// distinct banks.  The next tile is loaded into registers while the current
// one is used.  Pixels outside the image are staged as zeros.
constexpr int kWhTH = 4, kWhTW = 32, kWhO = 32, kWhK = 64;
constexpr int kWhXP = kWhK + 16, kWhDP = kWhO + 16;   // row pitches (elements)
constexpr int kWhBlocks = 512;                        // two blocks per CU
typedef short s16x4 __attribute__((ext_vector_type(4)));
typedef short s16x8 __attribute__((ext_vector_type(8)));

// 8 consecutive pixels (px + 8 q .. + 7 for this lane's group q) of channel
// ch + lane % 16 from a [pixel][channel] LDS array of row pitch `pitch`
__device__ __forceinline__ bf16x8 tr_operand(const uint16_t* base, int pitch, int px, int ch, int lane)
{
    const int gl = lane & 15, q = lane >> 4;
    const uint16_t* p = base + (px + 8 * q + (gl >> 2)) * pitch + ch + 4 * (gl & 3);
    typedef __attribute__((address_space(3))) s16x4 lds_s16x4;
    const s16x4 lo = __builtin_amdgcn_ds_read_tr16_b64_v4i16((lds_s16x4*)p);
    const s16x4 hi = __builtin_amdgcn_ds_read_tr16_b64_v4i16((lds_s16x4*)(p + 4 * pitch));
    return __builtin_bit_cast(bf16x8, (s16x8)__builtin_shufflevector(lo, hi, 0, 1, 2, 3, 4, 5, 6, 7));
}

template <bool NARROW>
__global__ __launch_bounds__(256, 2) void wgrad_halo_kernel(WgradArgs a, int tpc)
{
    constexpr int HP = kWhTH + 2, WP = kWhTW + 2, NX = HP * WP, ND = kWhTH * kWhTW;
    constexpr int PX = kWhK / 8, PD = kWhO / 8;
    constexpr int NA = NX * PX, NB = ND * PD, NLD = (NA + NB + 255) / 256;
    __shared__ __align__(16) uint16_t xs[NX * kWhXP];
    __shared__ __align__(16) uint16_t ds[ND * kWhDP];
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int o0 = blockIdx.x * kWhO, k0 = blockIdx.y * kWhK, chunk = blockIdx.z;
    const int K = a.C1 + a.C2;
    const int tx = (a.W + kWhTW - 1) / kWhTW, tps = tx * ((a.H + kWhTH - 1) / kWhTH);
    const int T = a.N * tps, t0 = chunk * tpc, t1 = min(T, t0 + tpc);
    uint4 st[NLD];
    // piece e = tid + 256 u: x halo pixel e / PX, channels 8 (e % PX) ..;
    // else dy pixel (e - NA) / PD, channels 8 ((e - NA) % PD) ..
    auto gload = [&](int t) {
        const int n = t / tps, tt = t - n * tps, y0 = (tt / tx) * kWhTH, x0 = (tt % tx) * kWhTW;
#pragma unroll
        for (int u = 0; u < NLD; ++u) {
            const int e = tid + 256 * u;
            uint4 v = make_uint4(0, 0, 0, 0);
            if (e < NA) {
                const int px = e / PX, k = k0 + 8 * (e % PX);
                const int gy = y0 - 1 + px / WP, gx = x0 - 1 + px % WP;
                if (gy >= 0 && gy < a.H && gx >= 0 && gx < a.W && k < K) {
                    const size_t pix = ((size_t)n * a.H + gy) * a.W + gx;
                    v = k < a.C1 ? *(const uint4*)(a.x1 + pix * a.C1 + k) : *(const uint4*)(a.x2 + pix * a.C2 + (k - a.C1));
                }
            } else if (e < NA + NB) {
                const int px = (e - NA) / PD, o = o0 + 8 * ((e - NA) % PD);
                const int gy = y0 + px / kWhTW, gx = x0 + px % kWhTW;
                const size_t pix = ((size_t)n * a.H + gy) * a.W + gx;
                if (NARROW) {
                    // fewer than 8 output channels: one piece, 2-byte loads
                    if (gy < a.H && gx < a.W && o == 0) {
                        uint16_t h[8] = {0, 0, 0, 0, 0, 0, 0, 0};
#pragma unroll
                        for (int c = 0; c < 8; ++c)
                            if (c < a.Nout) h[c] = a.dy[pix * a.Nout + c];
                        v = make_uint4(h[0] | ((uint32_t)h[1] << 16), h[2] | ((uint32_t)h[3] << 16),
                                       h[4] | ((uint32_t)h[5] << 16), h[6] | ((uint32_t)h[7] << 16));
                    }
                } else if (gy < a.H && gx < a.W && o < a.Nout) {
                    v = *(const uint4*)(a.dy + pix * a.Nout + o);
                }
            }
            st[u] = v;
        }
    };
    auto lstore = [&]() {
#pragma unroll
        for (int u = 0; u < NLD; ++u) {
            const int e = tid + 256 * u;
            if (e < NA) *(uint4*)(&xs[(e / PX) * kWhXP + 8 * (e % PX)]) = st[u];
            else if (e < NA + NB) *(uint4*)(&ds[((e - NA) / PD) * kWhDP + 8 * ((e - NA) % PD)]) = st[u];
        }
    };
    f32x4 acc[9][2];
#pragma unroll
    for (int t = 0; t < 9; ++t) acc[t][0] = acc[t][1] = (f32x4){0.f, 0.f, 0.f, 0.f};
    if (t0 < t1) gload(t0);
    for (int t = t0; t < t1; ++t) {
        if (t > t0) __syncthreads();   // every wave is done with the previous tile
        lstore();
        __syncthreads();
        if (t + 1 < t1) gload(t + 1);
#pragma unroll
        for (int r = 0; r < kWhTH; ++r) {
            const bf16x8 A0 = tr_operand(ds, kWhDP, r * kWhTW, 0, lane);
            const bf16x8 A1 = NARROW ? A0 : tr_operand(ds, kWhDP, r * kWhTW, 16, lane);
#pragma unroll
            for (int tap = 0; tap < 9; ++tap) {
                const int hy = r + tap / 3, hx = tap % 3;   // halo row r + 1 + dy, column + 1 + dx
                const bf16x8 B = tr_operand(xs, kWhXP, hy * WP + hx, 16 * wv, lane);
                acc[tap][0] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A0, B, acc[tap][0], 0, 0, 0);
                if (!NARROW) acc[tap][1] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A1, B, acc[tap][1], 0, 0, 0);
            }
        }
    }
    // acc[tap][j][e]: o = o0 + 16 j + 4 (lane / 16) + e, k = k0 + 16 wv + lane % 16
    const int k = k0 + 16 * wv + (lane & 15), rq = (lane >> 4) * 4;
    if (k >= K) return;
#pragma unroll
    for (int tap = 0; tap < 9; ++tap) {
        float* part = a.partial + ((size_t)chunk * 9 + tap) * a.Nout * K;
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int o = o0 + 16 * j + rq + e;
                if (o < a.Nout) part[(size_t)o * K + k] = acc[tap][j][e];
            }
    }
}

// Sum of the per-chunk partials: a block owns 64 consecutive outputs
// (coalesced rows) and splits the chunks over blockDim.y lanes (chunk c goes
// to lane c mod blockDim.y), whose sums are combined by a fixed LDS tree, so
// the result depends only on the shapes.
__global__ __launch_bounds__(1024) void wsum_kernel(const float* partial, float* dW, size_t n, int chunks,
                                                    int accumulate)
{
    __shared__ float red[16][64];
    const int x = threadIdx.x, y = threadIdx.y, Y = blockDim.y;
    const size_t i = (size_t)blockIdx.x * 64 + x;
    float s = 0.f;
    if (i < n) {
        int c = y;
        for (; c + 3 * Y < chunks; c += 4 * Y) {
            const float v0 = partial[(size_t)c * n + i], v1 = partial[(size_t)(c + Y) * n + i];
            const float v2 = partial[(size_t)(c + 2 * Y) * n + i], v3 = partial[(size_t)(c + 3 * Y) * n + i];
            s += v0;
            s += v1;
            s += v2;
            s += v3;
        }
        for (; c < chunks; c += Y) s += partial[(size_t)c * n + i];
    }
    red[y][x] = s;
    __syncthreads();
    for (int h = Y >> 1; h > 0; h >>= 1) {
        if (y < h) red[y][x] += red[y + h][x];
        __syncthreads();
    }
    if (y == 0 && i < n) dW[i] = accumulate ? dW[i] + red[0][x] : red[0][x];
}

// launch shape of wsum_kernel: lanes per output grow with the chunk count
static void launch_wsum(const float* partial, float* dW, size_t n, int chunks, int accumulate, hipStream_t s)
{
    int Y = 1;
    while (Y < 16 && Y * 16 < chunks) Y <<= 1;
    hipLaunchKernelGGL(wsum_kernel, dim3((unsigned)((n + 63) / 64)), dim3(64, Y), 0, s, partial, dW, n, chunks,
                       accumulate);
}

// Every item's BF16 operand copies in one launch: element i of the batch
// belongs to the first item whose end lies above it (items in order).
__device__ __forceinline__ void prep_elem(const PrepItem& p, uint32_t i)
{
    // 32-bit index arithmetic: every item holds fewer than 2^31 elements
    if (p.kind == kPrepPlain) {
        const uint32_t nf = p.fwd ? (uint32_t)(p.taps * p.ldo_f * p.ldk_f) : 0u;
        if (i < nf) {
            const uint32_t ro = i / (uint32_t)p.ldk_f, k = i - ro * (uint32_t)p.ldk_f;
            const uint32_t t = ro / (uint32_t)p.ldo_f, o = ro - t * (uint32_t)p.ldo_f;
            p.fwd[i] = ((int)o < p.R && (int)k < p.Kc) ? f2bf(p.W[((size_t)t * p.R + o) * p.Kc + k]) : 0;
        } else {
            const uint32_t j = i - nf;
            const uint32_t ro = j / (uint32_t)p.ldk_t, k = j - ro * (uint32_t)p.ldk_t;
            const uint32_t t = ro / (uint32_t)p.ldo_t, o = ro - t * (uint32_t)p.ldo_t;
            p.tr[j] = ((int)o < p.Kc && (int)k < p.R) ? f2bf(p.W[((size_t)t * p.R + k) * p.Kc + o]) : 0;
        }
        return;
    }
    const int o = (int)(i / 64), k = (int)(i % 64), t = k / 4, c = k % 4;
    if (p.kind == kPrepFirst) {
        p.fwd[i] = (o < p.R && t < 9) ? f2bf(p.W[((size_t)t * p.R + o) * 4 + c]) : 0;
    } else {
        // input gradient: output channel o is the weight's input channel,
        // c its output channel, and the tap is mirrored
        p.tr[i] = (o < p.Kc && t < 9 && c < p.R) ? f2bf(p.W[((size_t)(8 - t) * p.R + c) * p.Kc + o]) : 0;
    }
}

__global__ __launch_bounds__(256) void prep_batch_kernel(PrepBatch b)
{
    const size_t total = b.end[b.n - 1], stride = (size_t)gridDim.x * 256;
    int j = 0;
    for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < total; i += stride) {
        while (i >= b.end[j]) ++j;
        prep_elem(b.it[j], (uint32_t)(i - (j ? b.end[j - 1] : 0)));
    }
}

unsigned grid_for(size_t n)
{
    const size_t b = (n + 255) / 256;
    return (unsigned)(b < 4096 ? (b ? b : 1) : 4096);
}

}  // namespace

namespace {

template <int MODE, int TM, int TN, int WGM, int WGN>
void launch32(const ConvArgs& a, long P, hipStream_t s)
{
    dim3 grid((unsigned)((P + WGM * TM * 16 - 1) / (WGM * TM * 16)),
              (unsigned)((a.Nout + WGN * TN * 16 - 1) / (WGN * TN * 16)));
    hipLaunchKernelGGL((gemm32_kernel<MODE, TM, TN, WGM, WGN>), grid, dim3(256), 0, s, a);
}

// Tile shape for the wide kernel: the largest whose grid still gives about
// two blocks per compute unit, smaller wave tiles for small layers.
// named pixels x channels per block
enum Tile { k128x128, k256x64, k256x32, k256x16, k64x64, k128x32 };

Tile choose_tile(const ConvArgs& a, long P)
{
    auto blocks = [&](long bm, long bn) { return ((P + bm - 1) / bm) * ((a.Nout + bn - 1) / bn); };
    if (a.Nout > 64 && blocks(128, 128) >= 512) return k128x128;
    if (a.Nout > 32 && blocks(256, 64) >= 512) return k256x64;
    if (a.Nout > 16 && blocks(256, 32) >= 512) return k256x32;
    if (a.Nout <= 16) return k256x16;
    return a.Nout > 32 ? k64x64 : k128x32;
}

int tile_rows(Tile t) { return t == k64x64 ? 64 : (t == k128x128 || t == k128x32) ? 128 : 256; }

template <int MODE>
void dispatch32(const ConvArgs& a, long P, hipStream_t s)
{
    switch (choose_tile(a, P)) {
    case k128x128: launch32<MODE, 4, 4, 2, 2>(a, P, s); break;
    case k256x64: launch32<MODE, 4, 4, 4, 1>(a, P, s); break;
    case k256x32: launch32<MODE, 4, 2, 4, 1>(a, P, s); break;
    case k256x16: launch32<MODE, 4, 1, 4, 1>(a, P, s); break;
    case k64x64: launch32<MODE, 2, 2, 2, 2>(a, P, s); break;
    default: launch32<MODE, 2, 2, 4, 1>(a, P, s); break;
    }
}

// Halo-tile kernel: 8 x 32 pixel tiles, 32 output channels per block (16
// for narrower outputs; wider tiles keep one wave per SIMD for their staging
// registers); used when it gives about two blocks per CU.
constexpr int kLdsTH = 8, kLdsTW = 32;
// the normalising-input variant (the 3-channel head) on 4-row tiles: twice
// the blocks for the same work (measured: 19.3 against 21.7 us at 512^2)
constexpr int kLdsTHgn = 4;
int lds_th(const ConvArgs& a) { return a.gn_y ? kLdsTHgn : kLdsTH; }

long lds_tiles(const ConvArgs& a)
{
    return (long)((a.H + lds_th(a) - 1) / lds_th(a)) * ((a.W + kLdsTW - 1) / kLdsTW);
}

// 32 output channels per block while that still gives two blocks per CU,
// else 16 (small grids: the deep levels of one sample)
int lds_tn(const ConvArgs& a)
{
    if (a.Nout <= 16) return 1;
    return lds_tiles(a) * a.N * ((a.Nout + 31) / 32) >= 512 ? 2 : 1;
}

bool lds_ok(const ConvArgs& a, int mode)
{
    if (mode != kConvFwd && mode != kConvDgrad) return false;
    // per-piece offsets shared by both inputs, 32-bit byte offsets
    if ((a.C2 != 0 && a.C2 != a.C1) || (long)a.N * a.H * a.W * a.C1 >= (1l << 30) ||
        (long)9 * a.ldo * a.ldk >= (1l << 30))
        return false;
    const long blocks = lds_tiles(a) * a.N * ((a.Nout + 16 * lds_tn(a) - 1) / (16 * lds_tn(a)));
    return blocks >= 256;
}

template <int MODE>
void launch_lds(const ConvArgs& a, hipStream_t s)
{
    const int tn = lds_tn(a);
    dim3 grid((unsigned)(lds_tiles(a) * a.N), (unsigned)((a.Nout + 16 * tn - 1) / (16 * tn)));
    // 64-channel chunks for the 16-channel blocks of the small grids (every
    // chunk inside one of the concatenated inputs)
    const bool kc64 = tn == 1 && a.C1 % 64 == 0 && a.C2 % 64 == 0 && a.ldk % 64 == 0;
    if constexpr (MODE == kConvFwd) {
        if (a.gn_y) {   // (32-channel chunks: the FP32 halo doubles the staging registers)
            if (tn == 2) hipLaunchKernelGGL((conv3_lds_kernel<MODE, 2, kLdsTHgn, kLdsTW, 32, true>), grid, dim3(256), 0, s, a);
            else hipLaunchKernelGGL((conv3_lds_kernel<MODE, 1, kLdsTHgn, kLdsTW, 32, true>), grid, dim3(256), 0, s, a);
            return;
        }
    }
    if (tn == 2) hipLaunchKernelGGL((conv3_lds_kernel<MODE, 2, kLdsTH, kLdsTW, 32>), grid, dim3(256), 0, s, a);
    else if (kc64) hipLaunchKernelGGL((conv3_lds_kernel<MODE, 1, kLdsTH, kLdsTW, 64>), grid, dim3(256), 0, s, a);
    else hipLaunchKernelGGL((conv3_lds_kernel<MODE, 1, kLdsTH, kLdsTW, 32>), grid, dim3(256), 0, s, a);
}

}  // namespace

bool conv_wide_ok(const ConvArgs& a, int mode)
{
    const auto al = [](const void* p, uintptr_t b) { return ((uintptr_t)p & (b - 1)) == 0; };
    if (mode == kFirst)
        return a.C2 == 0 && a.ldk == 64 && a.ldo % 128 == 0 && al(a.Wt, 16) &&
               (a.raw[0] ? a.C1 == 4 && a.raw[1] && a.raw[2] && a.jump
                         : a.in1 && (a.C1 == 4 ? al(a.in1, 8) : a.C1 >= 1 && a.C1 <= 3 && al(a.in1, 2)));
    const bool chans = mode == kUpDgrad ? (a.C1 % 128 == 0 && a.C2 == 0) : (a.C1 % 32 == 0 && a.C2 % 32 == 0);
    return chans && a.ldk % 32 == 0 && a.ldo % 128 == 0 && al(a.in1, 16) && (!a.in2 || al(a.in2, 16)) &&
           al(a.Wt, 16);
}

bool conv_gn_input_ok(const ConvArgs& a)
{
    return a.C2 == 0 && a.gn_y && a.gn_coef && ((uintptr_t)a.gn_y & 15) == 0 && conv_wide_ok(a, kConvFwd) &&
           lds_ok(a, kConvFwd);
}

int conv_stat_chunks(const ConvArgs& a, int mode)
{
    if ((mode != kConvFwd && mode != kFirst) || !conv_wide_ok(a, mode)) return 0;
    if (mode == kConvFwd && lds_ok(a, mode)) return (int)lds_tiles(a);
    const long Ps = (long)a.H * a.W;
    const int rows = tile_rows(choose_tile(a, (long)a.N * Ps));
    return Ps % rows == 0 ? (int)(Ps / rows) : 0;
}

hipError_t conv_gemm(const ConvArgs& a, int mode, hipStream_t s)
{
    const long P = (long)a.N * a.H * a.W;
    if (P <= 0 || a.Nout <= 0) return hipSuccess;
    if (mode < kConvFwd || mode > kFirst) return hipErrorInvalidValue;
    // outputs are stored with 32-bit byte offsets (below 2^31: 2^29 FP32
    // values); the up-sampling epilogue also forms 32-bit element offsets
    if ((size_t)P * a.Nout >= ((size_t)1 << 29)) return hipErrorInvalidValue;
    if (a.gsum && conv_stat_chunks(a, mode) == 0) return hipErrorInvalidValue;
    if (a.gn_y && (mode != kConvFwd || !conv_gn_input_ok(a))) return hipErrorInvalidValue;
    if (conv_wide_ok(a, mode) && lds_ok(a, mode)) {
        if (mode == kConvFwd) launch_lds<kConvFwd>(a, s);
        else launch_lds<kConvDgrad>(a, s);
        return hipGetLastError();
    }
    if (conv_wide_ok(a, mode)) {
        switch (mode) {
        case kConvFwd: dispatch32<kConvFwd>(a, P, s); break;
        case kConvDgrad: dispatch32<kConvDgrad>(a, P, s); break;
        case kUpFwd: dispatch32<kUpFwd>(a, P, s); break;
        case kUpDgrad: dispatch32<kUpDgrad>(a, P, s); break;
        default: dispatch32<kFirst>(a, P, s); break;
        }
        return hipGetLastError();
    }
    if (mode == kFirst || a.gsum) return hipErrorInvalidValue;
    dim3 grid((unsigned)((P + 63) / 64), (unsigned)((a.Nout + 63) / 64));
    switch (mode) {
    case kConvFwd: hipLaunchKernelGGL(gemm_kernel<kConvFwd>, grid, dim3(256), 0, s, a); break;
    case kConvDgrad: hipLaunchKernelGGL(gemm_kernel<kConvDgrad>, grid, dim3(256), 0, s, a); break;
    case kUpFwd: hipLaunchKernelGGL(gemm_kernel<kUpFwd>, grid, dim3(256), 0, s, a); break;
    default: hipLaunchKernelGGL(gemm_kernel<kUpDgrad>, grid, dim3(256), 0, s, a); break;
    }
    return hipGetLastError();
}

size_t wgrad_partial_floats(const WgradArgs& a, int mode)
{
    const size_t P = (size_t)a.N * a.H * a.W;
    const size_t chunks = (P + a.chunk - 1) / a.chunk;
    return chunks * (mode == kConvFwd ? 9 : 1) * (size_t)a.Nout * (a.C1 + a.C2);
}

// Tap folding of the weight gradient (see wgrad32_kernel): 2 when the
// output side has fewer than 8 channels, 1 when the input side has (single
// input), else 0.
static int wgrad_fold(int mode, int Nout, int C1, int C2)
{
    if (mode != kConvFwd) return 0;
    if (Nout < 8) return 2;
    if (C2 == 0 && C1 < 8) return 1;
    return 0;
}

int wgrad_blocks_per_chunk(int mode, int Nout, int C1, int C2)
{
    const int K = C1 + C2, f = wgrad_fold(mode, Nout, C1, C2);
    const int taps = mode == kConvFwd && f == 0 ? 9 : 1;
    const int No = f == 2 ? 9 * Nout : Nout, Ko = f == 1 ? 9 * K : K;
    return taps * ((No + 63) / 64) * ((Ko + 63) / 64);
}

// The halo-tile kernel's shape conditions and chunking: 8-channel pieces
// (16-byte aligned) that never straddle the two inputs, and about
// kWhBlocks blocks over the (o, k) tile pairs and pixel-tile chunks.
static bool wgrad_halo_shape(int Nout, int C1, int C2)
{
    return Nout >= 1 && (Nout < 8 || Nout % 8 == 0) && C1 % 8 == 0 && C2 % 8 == 0 && C1 + C2 >= 8;
}
static long wgrad_halo_want(int Nout, int C1, int C2)
{
    const long pairs = (long)((Nout + kWhO - 1) / kWhO) * ((C1 + C2 + kWhK - 1) / kWhK);
    return std::max(1L, (kWhBlocks + pairs - 1) / pairs);
}
size_t wgrad_halo_floats(int Nout, int C1, int C2)
{
    if (!wgrad_halo_shape(Nout, C1, C2)) return 0;
    return (size_t)wgrad_halo_want(Nout, C1, C2) * 9 * Nout * (C1 + C2);
}

hipError_t conv_wgrad(const WgradArgs& a, int mode, float* dW, int accumulate, hipStream_t s)
{
    const long P = (long)a.N * a.H * a.W;
    const int ntaps = mode == kConvFwd ? 9 : 1;
    const int K = a.C1 + a.C2;
    const size_t n = (size_t)ntaps * a.Nout * K;
    if (mode != kConvFwd && mode != kUpFwd) return hipErrorInvalidValue;
    if (P <= 0) {
        if (!accumulate) launch_wsum(a.partial, dW, n, 0, 0, s);
        return hipGetLastError();
    }
    const auto al16 = [](const void* q) { return ((uintptr_t)q & 15) == 0; };
    if (mode == kConvFwd && wgrad_halo_shape(a.Nout, a.C1, a.C2) && (a.Nout < 8 || al16(a.dy)) && al16(a.x1) &&
        (!a.x2 || al16(a.x2)) && (a.C2 == 0 || a.x2)) {
        // halo tiles: chunks of whole 4 x 32 pixel tiles, as many as fit the
        // partial buffer (up to the wanted number)
        const long tiles = (long)a.N * ((a.H + kWhTH - 1) / kWhTH) * ((a.W + kWhTW - 1) / kWhTW);
        const size_t per = n;   // floats of one chunk's partial
        long chunks = std::min(wgrad_halo_want(a.Nout, a.C1, a.C2), tiles);
        chunks = std::min<long>(chunks, (long)(a.partial_cap / per));
        if (chunks >= 1) {
            const int tpc = (int)((tiles + chunks - 1) / chunks);
            chunks = (tiles + tpc - 1) / tpc;
            dim3 grid((unsigned)((a.Nout + kWhO - 1) / kWhO), (unsigned)((K + kWhK - 1) / kWhK), (unsigned)chunks);
            if (a.Nout < 8) hipLaunchKernelGGL(wgrad_halo_kernel<true>, grid, dim3(256), 0, s, a, tpc);
            else hipLaunchKernelGGL(wgrad_halo_kernel<false>, grid, dim3(256), 0, s, a, tpc);
            hipError_t e = hipGetLastError();
            if (e != hipSuccess) return e;
            launch_wsum(a.partial, dW, n, (int)chunks, accumulate, s);
            return hipGetLastError();
        }
    }
    const int chunks = (int)((P + a.chunk - 1) / a.chunk);
    const int fold = wgrad_fold(mode, a.Nout, a.C1, a.C2);
    const int No = fold == 2 ? 9 * a.Nout : a.Nout, Ko = fold == 1 ? 9 * K : K;
    const int gz = chunks * (mode == kConvFwd && fold == 0 ? 9 : 1);
    dim3 grid((unsigned)((No + 63) / 64), (unsigned)((Ko + 63) / 64), (unsigned)gz);
    const bool vec = a.Nout % 8 == 0 && (mode == kConvFwd || (a.Nout / 4) % 8 == 0) && a.C1 % 8 == 0 &&
                     a.C2 % 8 == 0 && al16(a.dy) && al16(a.x1) && (!a.x2 || al16(a.x2));
    // 8-channel pieces must not cross a sub-pixel of the up-sampling's dy
    // or the boundary of a concatenated input
    // folded: VEC covers the side that is not folded (16-byte pieces) and,
    // for a folded 4-channel input, its 8-byte tap pairs
    if (fold == 2) {
        const bool vx = a.C1 % 8 == 0 && a.C2 % 8 == 0 && al16(a.x1) && (!a.x2 || al16(a.x2));
        if (vx) hipLaunchKernelGGL((wgrad32_kernel<kConvFwd, true, 2>), grid, dim3(256), 0, s, a);
        else hipLaunchKernelGGL((wgrad32_kernel<kConvFwd, false, 2>), grid, dim3(256), 0, s, a);
    } else if (fold == 1) {
        const bool vd = a.Nout % 8 == 0 && al16(a.dy) && a.C1 == 4 && ((uintptr_t)a.x1 & 7) == 0;
        if (vd) hipLaunchKernelGGL((wgrad32_kernel<kConvFwd, true, 1>), grid, dim3(256), 0, s, a);
        else hipLaunchKernelGGL((wgrad32_kernel<kConvFwd, false, 1>), grid, dim3(256), 0, s, a);
    } else if (!vec && ((mode == kUpFwd && (a.Nout / 4) % 8 != 0) || (a.C2 > 0 && a.C1 % 8 != 0))) {
        if (mode == kConvFwd) hipLaunchKernelGGL(wgrad_kernel<kConvFwd>, grid, dim3(256), 0, s, a);
        else hipLaunchKernelGGL(wgrad_kernel<kUpFwd>, grid, dim3(256), 0, s, a);
    } else if (mode == kConvFwd) {
        if (vec) hipLaunchKernelGGL((wgrad32_kernel<kConvFwd, true, 0>), grid, dim3(256), 0, s, a);
        else hipLaunchKernelGGL((wgrad32_kernel<kConvFwd, false, 0>), grid, dim3(256), 0, s, a);
    } else {
        if (vec) hipLaunchKernelGGL((wgrad32_kernel<kUpFwd, true, 0>), grid, dim3(256), 0, s, a);
        else hipLaunchKernelGGL((wgrad32_kernel<kUpFwd, false, 0>), grid, dim3(256), 0, s, a);
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    launch_wsum(a.partial, dW, n, chunks, accumulate, s);
    return hipGetLastError();
}

size_t prep_item_size(const PrepItem& p)
{
    if (p.kind == kPrepPlain)
        return (p.fwd ? (size_t)p.taps * p.ldo_f * p.ldk_f : 0) + (p.tr ? (size_t)p.taps * p.ldo_t * p.ldk_t : 0);
    return (size_t)(p.kind == kPrepFirst ? p.ldo_f : p.ldo_t) * 64;
}

hipError_t weight_prep_batch(const PrepItem* items, int n, hipStream_t s)
{
    PrepBatch b{};
    size_t total = 0;
    for (int i = 0; i < n; ++i) {
        const size_t m = prep_item_size(items[i]);
        if (!m) continue;
        if (m >= ((size_t)1 << 31)) return hipErrorInvalidValue;
        if (b.n == kMaxPrep) return hipErrorInvalidValue;
        total += m;
        b.it[b.n] = items[i];
        b.end[b.n++] = total;
    }
    if (!b.n) return hipSuccess;
    hipLaunchKernelGGL(prep_batch_kernel, dim3(grid_for(total)), dim3(256), 0, s, b);
    return hipGetLastError();
}

hipError_t weight_prep_folded(const float* W, int R, uint16_t* out, int ldo, hipStream_t s)
{
    PrepItem p{};
    p.kind = kPrepFirst;
    p.W = W;
    p.R = R;
    p.fwd = out;
    p.ldo_f = ldo;
    return weight_prep_batch(&p, 1, s);
}

hipError_t weight_prep(const float* W, int taps, int R, int Kc, uint16_t* fwd, int ldo_f, int ldk_f, uint16_t* tr,
                       int ldo_t, int ldk_t, hipStream_t s)
{
    PrepItem p{};
    p.kind = kPrepPlain;
    p.W = W;
    p.taps = taps;
    p.R = R;
    p.Kc = Kc;
    p.fwd = fwd;
    p.ldo_f = ldo_f;
    p.ldk_f = ldk_f;
    p.tr = tr;
    p.ldo_t = ldo_t;
    p.ldk_t = ldk_t;
    return weight_prep_batch(&p, 1, s);
}

}  // namespace pfu
