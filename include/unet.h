/*
 * unet.h - C ABI of the gfx950 time-conditioned U-Net surrogate.
 *
 * The network is the one of the paper's Materials and Methods ("U-Net with
 * temporal conditioning"): convolution blocks GELU(GN(conv3x3(u))) with the
 * tanh form of GELU, 2x2 max pooling down, 2x2 stride-2 transposed
 * convolutions up, skips concatenated along channels, and every encoder
 * level's latent multiplied channel by channel with w_l f(dt), where f is a
 * two-layer sin MLP of the time step.  The output head is GN(conv(block)).
 * Training follows "Training of the network" (Adam) with the relative
 * squared error of "Error metrics".  Readings where the paper is silent:
 *   - input channels (c - 1/2, phi, rho - 1, jump length dt), centred so
 *     that BF16 keeps the small composition and vapour-density fluctuations;
 *     the head gives the three
 *     fields' mean rate over the leap: u(t+dt) = u(t) + dt head (the
 *     head's normalisation fixes its overall scale, the increment grows
 *     with dt);
 *   - 3x3 convolutions with zero "same" padding and no bias; transposed
 *     convolutions without bias; GN with `groups` groups (eps gn_eps) in the
 *     blocks and `head_groups` in the head;
 *   - decoder: the bottom block keeps the deepest width, each transposed
 *     convolution halves the width to that of the next level up;
 *   - loss: sum over the three fields of sum (pred - true)^2 / sum true^2
 *     over the batch (the per-element quotient of the paper's formula is
 *     undefined where a field is zero, as rho is inside the film).
 *
 * Numbers: MFMA operands (activations, BF16 weight copies) are BF16 with
 * FP32 accumulation; convolution outputs, normalisation statistics and all
 * gradients reaching the parameters are FP32 (statistics summed in FP64);
 * master parameters and Adam moments are FP32.
 *
 * Layouts: fields are SoA float [n][height][width] (the phase-field
 * library's layout); internal activations are NHWC.  Parameters are one
 * flat float array described by unet_param_entry(): conv3x3 weights
 * [9][Cout][Cin] with tap = 3 ky + kx (offsets ky - 1, kx - 1), transposed
 * convolutions [4][Cout][Cin] with sub-pixel 2 m + n (output pixel
 * (2y + m, 2x + n)), MLP matrices [out][in], projections w_l [C_l][basis].
 *
 * Memory: parameters, gradients and the workspace (unet_workspace_bytes(),
 * 256-byte aligned) are caller-owned device memory; the library never
 * allocates device memory.  Device pointers to BF16 data must be 8-byte
 * aligned, to float data 4-byte aligned.  Errors are the pf_status codes of
 * pf.h.  Every call enqueues on the handle's stream; unet_backward waits for
 * it when asked for the loss on the host.  A handle is not thread-safe.
 */
#ifndef UNET_H
#define UNET_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct unet_handle unet_handle;

typedef struct unet_config {
    int32_t height, width;  /* grid (ny, nx); divisible by 2^(levels-1) */
    int32_t in_ch;          /* must be 4: c, phi, rho, jump-length map */
    int32_t out_ch;         /* must be 3: increments of c, phi, rho */
    int32_t base;           /* channels of the first level, a multiple of 8; level l has base*2^l */
    int32_t levels;         /* encoder levels, 2..6 */
    int32_t groups;         /* GN groups of the convolution blocks */
    int32_t head_groups;    /* GN groups of the output head (divides out_ch) */
    int32_t mlp_hidden;     /* width of both sin layers, <= 256 */
    int32_t basis;          /* length of f(dt), <= 256 */
    int32_t max_batch;      /* largest batch the workspace is sized for */
    float gn_eps;           /* GN epsilon */
} unet_config;

typedef struct unet_param_desc {
    char name[32];          /* e.g. "enc0.w", "up3.w", "mlp.b1", "film2.w" */
    int64_t offset;         /* first float of the tensor in the flat array */
    int64_t count;          /* floats */
    int32_t ndim;
    int32_t dims[4];
} unet_param_desc;

/* Floats in the flat parameter (and gradient) array; -1 if cfg is invalid. */
int64_t unet_param_count(const unet_config* cfg);

/* Description of parameter tensor `index` (0-based); PF_EINVAL past the end. */
int unet_param_entry(const unet_config* cfg, int index, unet_param_desc* out);

/* Workspace bytes for cfg (activations and their gradients at max_batch,
 * BF16 weight copies, reduction scratch); 0 if cfg is invalid. */
size_t unet_workspace_bytes(const unet_config* cfg);

/* Create a handle over caller-owned params/grads (unet_param_count floats
 * each) and workspace; stream is a hipStream_t (NULL: default stream).
 * Enqueues the BF16 weight copies of the current parameters. */
int unet_create(unet_handle** out, const unet_config* cfg, float* params, float* grads, void* workspace,
                size_t workspace_bytes, void* stream);

/* Refresh the BF16 weight copies after the caller changed `params`.  It
 * also voids the forward's memo of the time basis: the time basis and FiLM
 * scales of a sample are kept between forward calls while its jump and the
 * parameters stay the same, so a caller that changes `params` must call
 * this (unet_adam does) before the next forward. */
int unet_prepare(unet_handle* h);

/* Forward pass of n <= max_batch samples: jump[n] (device floats) is the
 * time step of each sample in units of the training jump; (c, phi, rho) the
 * state; (oc, ophi, orho) receive the prediction (they may alias the
 * inputs).  Activations are kept for unet_backward. */
int unet_forward(unet_handle* h, int n, const float* jump, const float* c, const float* phi, const float* rho,
                 float* oc, float* ophi, float* orho);

/* The same prediction without keeping what unet_backward needs (inference:
 * less memory traffic); a following unet_backward returns PF_EINVAL. */
int unet_forward_infer(unet_handle* h, int n, const float* jump, const float* c, const float* phi, const float* rho,
                       float* oc, float* ophi, float* orho);

/* Loss of the last forward's prediction (pc, pphi, prho) against the truth
 * (tc, tphi, trho), and its gradient with respect to every parameter,
 * written (not added) to grads.  loss (host, may be NULL) receives the loss
 * after the stream has drained. */
int unet_backward(unet_handle* h, const float* pc, const float* pphi, const float* prho, const float* tc,
                  const float* tphi, const float* trho, double* loss);

/* One Adam step (t >= 1 counts steps) on params with moments m, v (device,
 * unet_param_count floats each, zero before the first step), then the BF16
 * weight copies are refreshed. */
int unet_adam(unet_handle* h, float* m, float* v, int64_t t, float lr, float beta1, float beta2, float eps);

void unet_destroy(unet_handle* h);

/* ----------------------------------------------------------- single ops
 * The kernels of the network one at a time, for tests and benchmarks.
 * Tensors are NHWC; BF16 as uint16_t bit patterns; all other data float.
 * `workspace` holds at least unet_op_workspace_bytes(n, H, W, Cmax) bytes
 * where Cmax bounds every channel count of the call.  Outputs of the
 * convolutions and normalisations are limited to 2^29 values (PF_EINVAL
 * beyond). */
size_t unet_op_workspace_bytes(int n, int H, int W, int Cmax);

/* y[n][H][W][Cout] = conv3x3(x1 (+) x2), w [9][Cout][C1+C2] (x2 may be
 * NULL with C2 = 0); zero padding. */
int unet_conv3x3_fwd(int n, int H, int W, const uint16_t* x1, int C1, const uint16_t* x2, int C2, const float* w,
                     int Cout, float* y, void* workspace, size_t workspace_bytes, void* stream);
/* The same in two parts, for callers that apply one weight many times
 * (inference, benchmarks): unet_conv3x3_prepare writes w's BF16 MFMA operand
 * into the caller's wprep (256-byte aligned, at least
 * unet_conv3x3_prep_bytes(C1, C2, Cout) bytes; 0 means invalid sizes), and
 * unet_conv3x3_fwd_prepared runs the convolution from it, launching the
 * convolution kernel alone.  wprep belongs to the caller and stays valid
 * until it changes w or frees it; PF_EINVAL on bad sizes or alignment. */
size_t unet_conv3x3_prep_bytes(int C1, int C2, int Cout);
int unet_conv3x3_prepare(const float* w, int C1, int C2, int Cout, void* wprep, size_t bytes, void* stream);
int unet_conv3x3_fwd_prepared(int n, int H, int W, const uint16_t* x1, int C1, const uint16_t* x2, int C2,
                              const void* wprep, int Cout, float* y, void* stream);
/* Input gradient: dx1 [n][H][W][C1], dx2 [n][H][W][C2] (or NULL) from
 * dy [n][H][W][Cout]. */
int unet_conv3x3_dgrad(int n, int H, int W, const uint16_t* dy, int Cout, const float* w, int C1, int C2, float* dx1,
                       float* dx2, void* workspace, size_t workspace_bytes, void* stream);
/* Weight gradient dw [9][Cout][C1+C2] (overwritten). */
int unet_conv3x3_wgrad(int n, int H, int W, const uint16_t* dy, int Cout, const uint16_t* x1, int C1,
                       const uint16_t* x2, int C2, float* dw, void* workspace, size_t workspace_bytes, void* stream);
/* 2x2 stride-2 transposed convolution x [n][H][W][Cin] -> y [n][2H][2W][Cout],
 * w [4][Cout][Cin]; dgrad gives dx [n][H][W][Cin]; wgrad dw [4][Cout][Cin]. */
int unet_up_fwd(int n, int H, int W, const uint16_t* x, int Cin, const float* w, int Cout, float* y, void* workspace,
                size_t workspace_bytes, void* stream);
int unet_up_dgrad(int n, int H, int W, const uint16_t* dy, int Cout, const float* w, int Cin, float* dx,
                  void* workspace, size_t workspace_bytes, void* stream);
int unet_up_wgrad(int n, int H, int W, const uint16_t* dy, int Cout, const uint16_t* x, int Cin, float* dw,
                  void* workspace, size_t workspace_bytes, void* stream);
/* z = act(GN(y)), zs = z * scale[n][C] (scale, zs may be NULL); act = GELU if
 * gelu else identity; stats [n][G][2] = mean, 1/sqrt(var + eps).  y is
 * [n][P][C] with P pixels, C <= 256. */
int unet_groupnorm_fwd(int n, int P, int C, int G, float eps, int gelu, const float* y, const float* gamma,
                       const float* beta, const float* scale, float* z, float* zs, float* stats, void* workspace,
                       size_t workspace_bytes, void* stream);
/* Backward of the above from dz = dA + dB * scale (dA or dB may be NULL):
 * dy [n][P][C], dgamma and dbeta [C], dscale [n][C] (when dB and scale). */
int unet_groupnorm_bwd(int n, int P, int C, int G, float eps, int gelu, const float* y, const float* gamma,
                       const float* beta, const float* scale, const float* stats, const float* dA, const float* dB,
                       float* dy, float* dgamma, float* dbeta, float* dscale, void* workspace,
                       size_t workspace_bytes, void* stream);
/* 2x2 stride-2 max pool of BF16 x [n][H][W][C] -> y [n][H/2][W/2][C]; the
 * backward sends dy [n][H/2][W/2][C] to the first maximal input of each
 * window (row-major order) and zero elsewhere, dx [n][H][W][C]. */
int unet_maxpool_fwd(int n, int H, int W, int C, const uint16_t* x, uint16_t* y, void* stream);
int unet_maxpool_bwd(int n, int H, int W, int C, const uint16_t* x, const float* dy, float* dx, void* stream);

#ifdef __cplusplus
}
#endif
#endif
