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
// Weight gradients reduce over pixels: wgrad_kernel forms partial products
// over fixed pixel chunks with the same MFMA shape (k = 16 pixels) and
// wsum_kernel adds the chunks in index order, so results are deterministic.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "unet_kernels.h"

namespace pfu {
namespace {

typedef short bf16x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

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
                    if (a.out_f32) a.out_f32[idx] = v;
                    if (a.out_bf16) a.out_bf16[idx] = f2bf(v);
                } else if (o < a.O1) {
                    const size_t idx = (size_t)p * a.O1 + o;
                    if (a.out_f32) a.out_f32[idx] = v;
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
        if (MODE == kFirst) {
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
    // acc[i][j][e]: pixel pm + 16 i + 4 (lane / 16) + e, channel on + 16 j + r
    const int rq = (lane >> 4) * 4;
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
                if (MODE == kUpFwd) {
                    const Pix t = pix(p, a.H, a.W, P);
                    const int Co = a.Nout >> 2, sub = o / Co, co = o - sub * Co;
                    const size_t idx =
                        (((size_t)t.n * 2 * a.H + 2 * t.y + (sub >> 1)) * 2 * a.W + 2 * t.x + (sub & 1)) * Co + co;
                    if (a.out_f32) a.out_f32[idx] = v;
                    if (a.out_bf16) a.out_bf16[idx] = f2bf(v);
                } else if (o < a.O1) {
                    const size_t idx = (size_t)p * a.O1 + o;
                    if (a.out_f32) a.out_f32[idx] = v;
                    if (a.out_bf16) a.out_bf16[idx] = f2bf(v);
                } else {
                    const size_t idx = (size_t)p * (a.Nout - a.O1) + (o - a.O1);
                    if (a.out2_f32) a.out2_f32[idx] = v;
                    if (a.out2_bf16) a.out2_bf16[idx] = f2bf(v);
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

__global__ __launch_bounds__(256) void wsum_kernel(const float* partial, float* dW, size_t n, int chunks,
                                                   int accumulate)
{
    for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (size_t)gridDim.x * 256) {
        float s = 0.f;
        for (int c = 0; c < chunks; ++c) s += partial[(size_t)c * n + i];
        dW[i] = accumulate ? dW[i] + s : s;
    }
}

__global__ __launch_bounds__(256) void prep_kernel(const float* W, int taps, int R, int Kc, uint16_t* fwd, int ldo_f,
                                                   int ldk_f, uint16_t* tr, int ldo_t, int ldk_t)
{
    const size_t nf = fwd ? (size_t)taps * ldo_f * ldk_f : 0, nt = tr ? (size_t)taps * ldo_t * ldk_t : 0;
    for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < nf + nt; i += (size_t)gridDim.x * 256) {
        if (i < nf) {
            const int k = (int)(i % ldk_f), o = (int)((i / ldk_f) % ldo_f), t = (int)(i / ((size_t)ldk_f * ldo_f));
            fwd[i] = (o < R && k < Kc) ? f2bf(W[((size_t)t * R + o) * Kc + k]) : 0;
        } else {
            const size_t j = i - nf;
            const int k = (int)(j % ldk_t), o = (int)((j / ldk_t) % ldo_t), t = (int)(j / ((size_t)ldk_t * ldo_t));
            tr[j] = (o < Kc && k < R) ? f2bf(W[((size_t)t * R + k) * Kc + o]) : 0;
        }
    }
}

__global__ __launch_bounds__(256) void fold_kernel(const float* W, int R, uint16_t* out, int ldo)
{
    for (int i = blockIdx.x * 256 + threadIdx.x; i < ldo * 64; i += gridDim.x * 256) {
        const int o = i / 64, k = i % 64, t = k / 4, c = k % 4;
        out[i] = (o < R && t < 9) ? f2bf(W[((size_t)t * R + o) * 4 + c]) : 0;
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

}  // namespace

bool conv_wide_ok(const ConvArgs& a, int mode)
{
    const auto al = [](const void* p, uintptr_t b) { return ((uintptr_t)p & (b - 1)) == 0; };
    if (mode == kFirst)
        return a.C1 == 4 && a.C2 == 0 && a.ldk == 64 && a.ldo % 128 == 0 && al(a.in1, 8) && al(a.Wt, 16);
    const bool chans = mode == kUpDgrad ? (a.C1 % 128 == 0 && a.C2 == 0) : (a.C1 % 32 == 0 && a.C2 % 32 == 0);
    return chans && a.ldk % 32 == 0 && a.ldo % 128 == 0 && al(a.in1, 16) && (!a.in2 || al(a.in2, 16)) &&
           al(a.Wt, 16);
}

int conv_stat_rows(const ConvArgs& a, int mode)
{
    if ((mode != kConvFwd && mode != kFirst) || !conv_wide_ok(a, mode)) return 0;
    return tile_rows(choose_tile(a, (long)a.N * a.H * a.W));
}

hipError_t conv_gemm(const ConvArgs& a, int mode, hipStream_t s)
{
    const long P = (long)a.N * a.H * a.W;
    if (P <= 0 || a.Nout <= 0) return hipSuccess;
    if (mode < kConvFwd || mode > kFirst) return hipErrorInvalidValue;
    if (a.gsum) {
        const int rows = conv_stat_rows(a, mode);
        if (rows == 0 || ((long)a.H * a.W) % rows != 0) return hipErrorInvalidValue;
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

hipError_t conv_wgrad(const WgradArgs& a, int mode, float* dW, int accumulate, hipStream_t s)
{
    const long P = (long)a.N * a.H * a.W;
    const int ntaps = mode == kConvFwd ? 9 : 1;
    const int K = a.C1 + a.C2;
    const size_t n = (size_t)ntaps * a.Nout * K;
    if (mode != kConvFwd && mode != kUpFwd) return hipErrorInvalidValue;
    if (P <= 0) {
        if (!accumulate) hipLaunchKernelGGL(wsum_kernel, dim3(grid_for(n)), dim3(256), 0, s, a.partial, dW, n, 0, 0);
        return hipGetLastError();
    }
    const int chunks = (int)((P + a.chunk - 1) / a.chunk);
    dim3 grid((unsigned)((a.Nout + 63) / 64), (unsigned)((K + 63) / 64), (unsigned)(chunks * ntaps));
    if (mode == kConvFwd) hipLaunchKernelGGL(wgrad_kernel<kConvFwd>, grid, dim3(256), 0, s, a);
    else hipLaunchKernelGGL(wgrad_kernel<kUpFwd>, grid, dim3(256), 0, s, a);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(wsum_kernel, dim3(grid_for(n)), dim3(256), 0, s, a.partial, dW, n, chunks, accumulate);
    return hipGetLastError();
}

hipError_t weight_prep_folded(const float* W, int R, uint16_t* out, int ldo, hipStream_t s)
{
    hipLaunchKernelGGL(fold_kernel, dim3(grid_for((size_t)ldo * 64)), dim3(256), 0, s, W, R, out, ldo);
    return hipGetLastError();
}

hipError_t weight_prep(const float* W, int taps, int R, int Kc, uint16_t* fwd, int ldo_f, int ldk_f, uint16_t* tr,
                       int ldo_t, int ldk_t, hipStream_t s)
{
    const size_t n = (fwd ? (size_t)taps * ldo_f * ldk_f : 0) + (tr ? (size_t)taps * ldo_t * ldk_t : 0);
    if (!n) return hipSuccess;
    hipLaunchKernelGGL(prep_kernel, dim3(grid_for(n)), dim3(256), 0, s, W, taps, R, Kc, fwd, ldo_f, ldk_f, tr, ldo_t,
                       ldk_t);
    return hipGetLastError();
}

}  // namespace pfu
