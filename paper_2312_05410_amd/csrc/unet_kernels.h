// Device kernels of the time-conditioned U-Net (Materials and Methods, "U-Net
// with temporal conditioning" and "Training of the network").  Internal to
// the library; the C ABI is in include/unet.h.
//
// Tensors are NHWC (channels fastest).  MFMA operands are BF16 (stored as
// uint16_t bit patterns), accumulation and every statistic is FP32 or FP64.
#pragma once
#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace pfu {

constexpr int kMaxLevels = 6;

// Stores of large activations that a later kernel reads: buffer stores
// written through to memory at device scope (byte offset below 2^31 from
// base).  Against plain global stores they stream faster, and against
// non-temporal ones they leave no lines whose write-back delays the start of
// the next kernel.
typedef unsigned int u32x4v __attribute__((ext_vector_type(4)));
constexpr int kStoreSc1 = 16;   // cache-policy bit: device scope (write-through)
__device__ __forceinline__ __amdgpu_buffer_rsrc_t wt_rsrc(const void* base)
{
    return __builtin_amdgcn_make_buffer_rsrc((void*)base, (short)0, 0x7FFFFFFF, 0x00020000);
}
__device__ __forceinline__ void st16wt(const void* base, size_t byte_off, uint4 v)
{
    __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(u32x4v, v), wt_rsrc(base), (int)byte_off, 0,
                                           kStoreSc1);
}
__device__ __forceinline__ void stwt(const float* base, size_t idx, float v)
{
    __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, v), wt_rsrc(base), (int)(4 * idx), 0,
                                          kStoreSc1);
}

// Implicit GEMM out[p][o] = sum_k A[p][k] B[o][k]; see unet_conv.hip for
// the four gather/scatter modes.
// kFirst: 3x3 convolution of a 4-channel input (or of 1-3 channels, the
// missing ones zero; not from the state fields) with the taps folded into K
// (k = 4 tap + c, weights [1][ldo][64]).
enum ConvMode { kConvFwd = 0, kConvDgrad = 1, kUpFwd = 2, kUpDgrad = 3, kFirst = 4 };

struct ConvArgs {
    const uint16_t* in1;   // first input (NHWC, C1 channels)
    const uint16_t* in2;   // concatenated second input (C2 channels) or null
    const uint16_t* Wt;    // BF16 operand weights [taps][ldo][ldk], zero padded
    float* out_f32;        // first output, FP32 (or null)
    uint16_t* out_bf16;    // first output, BF16 (or null)
    float* out2_f32;       // channels [O1, Nout) when the output is split
    uint16_t* out2_bf16;
    int N, H, W;           // pixel grid the GEMM rows run over
    int C1, C2;            // input channels (K per tap = C1 + C2)
    int Nout, O1;          // output channels, split point (O1 = Nout: no split)
    int ldk;               // row stride of Wt (K rounded up to 32)
    int ldo;               // rows per tap of Wt (Nout rounded up to 128)
    // optional per-tile channel sums of the FP32 output for group
    // normalisation, [N][Nout][conv_stat_chunks()][2] = (sum, sum of
    // squares); only when conv_stat_chunks() > 0
    float* gsum;
    // kFirst only, or null: gather the network input straight from the state
    // fields, x = BF16 (c - 1/2, phi, rho - 1, jump[n]) (in1 unused)
    const float* raw[3];
    const float* jump;
    // kConvFwd with one input, or null: the input is the normalisation of the
    // FP32 tensor gn_y ([N][H][W][C1]), x = BF16(act(A y + B)) with A, B per
    // (sample, channel) from gn_coef ([2][N][C1]) and act the GELU if gn_gelu
    // (in1 unused)
    const float* gn_y;
    const float* gn_coef;
    int gn_gelu;
};

struct WgradArgs {
    const uint16_t* dy;    // output gradient (NHWC, Nout channels; 2H x 2W for up)
    const uint16_t* x1;    // forward input (C1 channels) at H x W
    const uint16_t* x2;    // concatenated second input or null
    float* partial;        // [chunks][taps][Nout][C1+C2]
    int N, H, W, C1, C2, Nout;
    int chunk;             // pixels per partial product (multiple of 64)
    // floats the partial buffer holds beyond what `chunk` needs (0: only
    // that); the halo-tile 3x3 weight gradient runs when its partials fit
    size_t partial_cap;
};
// Partial floats the halo-tile 3x3 weight gradient asks for (0 when the
// shape does not take it): its chunk count times 9 Nout (C1 + C2).
size_t wgrad_halo_floats(int Nout, int C1, int C2);

hipError_t conv_gemm(const ConvArgs& a, int mode, hipStream_t s);
// True when conv_gemm takes the wide 16x16x32 kernel: channel counts
// multiples of 32 (128 for the up-sampling gradient's 4 sub-pixels),
// ldk % 32 == 0, ldo % 128 == 0 and 16-byte aligned operands.
bool conv_wide_ok(const ConvArgs& a, int mode);
// True when conv_gemm (kConvFwd) can normalise its input as it loads it
// (a.gn_y, a.gn_coef set; one input; the halo-tile kernel).
bool conv_gn_input_ok(const ConvArgs& a);
// Number of per-sample partial sums the kernel conv_gemm picks for
// (a, mode) writes to a.gsum (forward modes of the wide kernels, when its
// pixel blocks do not straddle samples), else 0.
int conv_stat_chunks(const ConvArgs& a, int mode);
// dW[taps][Nout][C1+C2] = (accumulate ? dW : 0) + sum over pixels; mode
// kConvFwd (3x3) or kUpFwd (2x2 stride 2).  a.partial must hold
// wgrad_partial_floats() floats.
hipError_t conv_wgrad(const WgradArgs& a, int mode, float* dW, int accumulate, hipStream_t s);
size_t wgrad_partial_floats(const WgradArgs& a, int mode);
// Blocks conv_wgrad launches per pixel chunk (taps and 64 x 64 output tiles).
int wgrad_blocks_per_chunk(int mode, int Nout, int C1, int C2);
// BF16 operand copies of an FP32 weight [taps][R][Kc]: fwd[t][o][k] = W[t][o][k]
// (ldo_f x ldk_f, zero padded) and tr[t][o][k] = W[t][k][o] (ldo_t x ldk_t);
// either may be null.
hipError_t weight_prep(const float* W, int taps, int R, int Kc, uint16_t* fwd, int ldo_f, int ldk_f, uint16_t* tr,
                       int ldo_t, int ldk_t, hipStream_t s);
// kFirst operand of a [9][R][4] weight: out[o][4 t + c] = W[t][o][c],
// [ldo][64] zero padded.
hipError_t weight_prep_folded(const float* W, int R, uint16_t* out, int ldo, hipStream_t s);
// Several weights' operand copies in one launch.  kPrepPlain: fwd and tr as
// weight_prep; kPrepFirst: fwd as weight_prep_folded (ldo_f); kPrepFirstGrad:
// the kFirst operand of the input gradient of a [9][R][Kc] weight with
// R <= 4 output channels, tr[o][4 t + c] = W[8 - t][c][o] ([ldo_t][64], zero
// padded; tap 8 - t is tap t mirrored through the centre).
enum PrepKind { kPrepPlain = 0, kPrepFirst = 1, kPrepFirstGrad = 2 };
struct PrepItem {
    const float* W;
    uint16_t* fwd;
    uint16_t* tr;
    int kind, taps, R, Kc, ldo_f, ldk_f, ldo_t, ldk_t;
};
constexpr int kMaxPrep = 24;
struct PrepBatch {
    PrepItem it[kMaxPrep];
    size_t end[kMaxPrep];   // running element counts
    int n;
};
hipError_t weight_prep_batch(const PrepItem* items, int n, hipStream_t s);

// ---------------------------------------------------------------- elementwise
// Per-channel partial sums over pixel chunks, then finished per sample.
struct GNArgs {
    const float* y;        // pre-normalisation input [N][P][C] (FP32)
    const float* gamma;    // [C]
    const float* beta;     // [C]
    const float* scale;    // FiLM scale [N][C] or null
    float* stats;          // [N][G][2]: mean, 1/sqrt(var + eps)
    float* csum;           // partial sums (workspace): forward [N][C][chunks][2],
                           // backward [N][chunks][C][3]
    double* cacc;          // [N][C][3] finished per-channel sums (workspace)
    // forward outputs (any may be null): z = act(GN(y)), zs = z * scale
    float* z_f32;
    uint16_t* z_bf16;
    float* zs_f32;
    uint16_t* zs_bf16;
    // backward: dz = dA + dB * scale (dA, dB may be null), outputs dy
    const float* dA;
    const float* dB;
    float* dy_f32;
    uint16_t* dy_bf16;
    float* dgamma;         // [C] (=, summed over samples)
    float* dbeta;          // [C] (=)
    float* dscale;         // [N][C] (=), when scale and dB are given
    uint16_t* pool_bf16;   // forward: 2x2 max pool of z (BF16) or null
    // backward, in place of dA: the gradient of that pool, routed to the
    // first maximum of each window of pool_z (BF16 z [N][H][W][C]) from
    // pool_dq ([N][H/2][W/2][C]); pool_tmp ([N][H][W][C] FP32) holds it
    // where the kernels cannot form it themselves
    const uint16_t* pool_z;
    const float* pool_dq;
    float* pool_tmp;
    int H, W;              // pixel grid of one sample when pooling (H W = P)
    int N, P, C, G;
    int gelu;
    float eps;
    int chunks;            // partial sums per sample
    int sums_ready;        // forward: csum already holds `chunks` partials
    float* coef;           // forward workspace [2][N][C] (16-byte aligned) or null: the
                           // normalisation as A y + B per channel, A = gamma rstd,
                           // B = beta - A mean
    // forward: the statistics and coefficients need not be written out
    // (inference), so a batch-1 launch may finish them inside the
    // normalisation blocks
    int stats_internal;
    // forward, C = 3, or null: instead of z, write the prediction
    // res_out[f][n][p] = res_in[f][n][p] + res_jump[n] z[n][p][f] (the head)
    const float* res_jump;
    const float* res_in[3];
    float* res_out[3];
};
// mlp (or null): the same launch also evaluates the time basis and every
// level's FiLM scales (mlp_fused_ok must hold) and copies the jumps to
// jump_copy (or not, if null).  With no output requested (z, zs, pool and
// res_jump null) only the statistics and coefficients are computed.
hipError_t gn_forward(const GNArgs& a, hipStream_t s, const struct MLPArgs* mlp = nullptr, float* jump_copy = nullptr);
hipError_t gn_backward(const GNArgs& a, hipStream_t s);
size_t gn_csum_floats(int N, int P, int C);
int gn_chunks(int P);

// 2x2 stride-2 max pool of BF16 NHWC; backward writes the full-resolution
// FP32 gradient (the first maximum in (0,0), (0,1), (1,0), (1,1) order
// receives it, the others zero).
hipError_t maxpool_fwd(const uint16_t* x, uint16_t* y, int N, int H, int W, int C, hipStream_t s);
hipError_t maxpool_bwd(const uint16_t* x, const float* dy, float* dx, int N, int H, int W, int C, hipStream_t s);

// Time basis f(jump) (two sin layers of width Hd) and the per-level FiLM
// scales s_l = w_l f.
struct MLPArgs {
    const float* jump;     // [N]
    const float* W0;       // [Hd]
    const float* b0;       // [Hd]
    const float* W1;       // [Hd][Hd]
    const float* b1;
    const float* W2;       // [F][Hd]
    const float* b2;       // [F]
    const float* Wl[kMaxLevels];    // [C_l][F]
    float* h0;             // [N][Hd] pre-activations (saved)
    float* h1;             // [N][Hd]
    float* f;              // [N][F]
    float* sc[kMaxLevels];          // [N][C_l]
    const float* dsc[kMaxLevels];   // backward: [N][C_l]
    float* df;             // backward workspace [N][F]
    float* dh1;            // [N][Hd]
    float* dh0;            // [N][Hd]
    float* gW0; float* gb0; float* gW1; float* gb1; float* gW2; float* gb2;
    float* gWl[kMaxLevels];
    int N, Hd, F, L;
    int C[kMaxLevels];
    // forward memo, or null: [N][L][2] (jump bits, gen) of the last
    // computation of sc[l][n] (and, for l = 0, h0, h1, f of sample n); a block
    // whose entry matches jump[n] and gen leaves them as they are
    uint32_t* cache;
    uint32_t gen;
};
// Forward prologue in one launch: the network input x[n][p] = BF16 (c - 1/2,
// phi, rho - 1, jump[n]), the time basis f(jump) and every level's FiLM
// scales (a.jump the caller's jumps; jump_copy, or null, receives them)
hipError_t prologue_forward(const MLPArgs& a, const float* c, const float* phi, const float* rho, uint16_t* x, int P,
                            float* jump_copy, hipStream_t s);
hipError_t mlp_backward(const MLPArgs& a, hipStream_t s);
// True when gn_forward can take the MLP (widths up to 128, FiLM rows up to
// 256 per level).
bool mlp_fused_ok(const MLPArgs& a);

// Relative MSE per field: L = sum_f sum (pred - tgt)^2 / sum tgt^2.
// Writes dL/dhead = jump[n] dL/dpred as [N][P][3] (NHWC, the head's layout)
// and L (FP64).
hipError_t rel_mse(const float* pc, const float* pphi, const float* prho, const float* tc, const float* tphi,
                   const float* trho, const float* jump, float* grad, double* part, double* loss, int N, int P,
                   hipStream_t s);
size_t rel_mse_partial_doubles();

// Adam on FP32 master parameters.
hipError_t adam_update(float* w, const float* g, float* m, float* v, size_t n, float lr, float b1, float b2,
                       float eps, float bc1, float bc2, hipStream_t s);

hipError_t fill_f32(float* p, size_t n, float v, hipStream_t s);

}  // namespace pfu
