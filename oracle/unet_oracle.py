"""Plain PyTorch CPU FP64 oracle of the time-conditioned U-Net.

TEST INFRASTRUCTURE ONLY: imported by the test suite, the smoke check and
the CPU-baseline leg of the benchmark.  The product path never imports it,
and it imports nothing from the GPU package.

Every function follows one passage of the paper's Materials and Methods
("U-Net with temporal conditioning", "Error metrics"), written out with
plain tensor operations on NCHW float64 tensors.  Gradients are those of
torch.autograd on this forward.  Readings where the paper is silent (they
match the GPU library's documented interface):
  * input channels (c - 1/2, phi, rho - 1, jump map); the head gives the fields' mean
    rate over the leap: prediction = state + jump * head;
  * 3x3 convolutions, zero padding, no bias; transposed convolutions
    without bias;
  * decoder widths: the bottom block keeps the deepest width, each
    up-sampling halves it;
  * loss = sum over fields of sum (pred - true)^2 / sum true^2.
Parameters come as a dict of arrays named and laid out as the library's
flat parameter array: conv weights [9][Cout][Cin] (tap 3 ky + kx), up
weights [4][Cout][Cin] (sub-pixel 2 m + n), MLP matrices [out][in].

`bf16=True` rounds to BF16 where the GPU stores BF16 (network input,
convolution and up-sampling weights, block outputs, pooled and conditioned
latents, up-sampled maps); arithmetic stays FP64.  Its gradients pass those
roundings unchanged and are rounded to BF16 where the GPU stores gradients
in BF16 instead: the gradient of each block's convolution output (the
normalisation's backward result, the convolution gradients' operand) and of
each up-sampled map (the up-sampling gradients' operand); weight gradients
and the other activation gradients stay unrounded, as the GPU keeps them in
FP32.  `Net(..., dtype=float32)` evaluates the same definitions in FP32;
tests use the gap between the two to measure how strongly the BF16
roundings amplify accumulation error.
"""
from __future__ import annotations

import math

import numpy as np
import torch

GELU_S = math.sqrt(2.0 / math.pi)


def _t(a, dtype=torch.float64):
    return torch.as_tensor(np.asarray(a), dtype=dtype)


def round_bf16(u: torch.Tensor) -> torch.Tensor:
    """Nearest BF16 value (ties to even), in u's dtype."""
    return u.to(torch.float32).to(torch.bfloat16).to(u.dtype)


class _RoundValue(torch.autograd.Function):
    """BF16 rounding of a stored value; its gradient passes unchanged."""

    @staticmethod
    def forward(ctx, u):
        return round_bf16(u)

    @staticmethod
    def backward(ctx, g):
        return g


class _RoundGrad(torch.autograd.Function):
    """Identity on the value; its gradient rounded to BF16 (a gradient the
    GPU stores in BF16)."""

    @staticmethod
    def forward(ctx, u):
        return u.clone()

    @staticmethod
    def backward(ctx, g):
        return round_bf16(g)


def conv3x3(u: torch.Tensor, w: torch.Tensor) -> torch.Tensor:
    """conv(u)_{k',i,j} = sum_k sum_{m,n} u_{k, i+m-1, j+n-1} w_{k,k',m,n}
    over a 3x3 window centred on (i, j), zero outside the grid.  u [n][C][H][W],
    w [9][C'][C] with tap 3 m + n."""
    n, C, H, W = u.shape
    up = torch.nn.functional.pad(u, (1, 1, 1, 1))
    out = torch.zeros(n, w.shape[1], H, W, dtype=u.dtype)
    for m in range(3):
        for q in range(3):
            out = out + torch.einsum("oc,nchw->nohw", w[3 * m + q], up[:, :, m:m + H, q:q + W])
    return out


def group_norm(u: torch.Tensor, G: int, gamma: torch.Tensor, beta: torch.Tensor, eps: float) -> torch.Tensor:
    """Group normalisation: per sample, the C channels split into G groups of
    C/G; each group's mean and (biased) variance over its channels and
    pixels normalise it; then the per-channel affine gamma, beta."""
    n, C, H, W = u.shape
    g = u.reshape(n, G, C // G, H, W)
    mu = g.mean(dim=(2, 3, 4), keepdim=True)
    var = ((g - mu) ** 2).mean(dim=(2, 3, 4), keepdim=True)
    uh = ((g - mu) / torch.sqrt(var + eps)).reshape(n, C, H, W)
    return gamma.view(1, C, 1, 1) * uh + beta.view(1, C, 1, 1)


def gelu(u: torch.Tensor) -> torch.Tensor:
    """GELU in its tanh form."""
    return 0.5 * u * (1.0 + torch.tanh(GELU_S * (u + 0.044715 * u ** 3)))


def down(u: torch.Tensor) -> torch.Tensor:
    """2x2 max pooling with stride 2."""
    return torch.maximum(torch.maximum(u[:, :, 0::2, 0::2], u[:, :, 0::2, 1::2]),
                         torch.maximum(u[:, :, 1::2, 0::2], u[:, :, 1::2, 1::2]))


def up(u: torch.Tensor, w: torch.Tensor) -> torch.Tensor:
    """2x2 stride-2 transposed convolution: input pixel (i, j) spreads to
    output pixels (2i + m, 2j + n) with weight w[2m + n] (channel mixing
    [C'][C])."""
    n, C, H, W = u.shape
    out = torch.zeros(n, w.shape[1], 2 * H, 2 * W, dtype=u.dtype)
    for m in range(2):
        for q in range(2):
            out[:, :, m::2, q::2] = torch.einsum("oc,nchw->nohw", w[2 * m + q], u)
    return out


def time_basis(jump: torch.Tensor, p: dict) -> torch.Tensor:
    """f(dt) = w2 sin(w1 sin(w0 dt + b0) + b1) + b2; jump [n] -> [n][F]."""
    a0 = torch.sin(jump[:, None] * p["mlp.w0"][:, 0][None, :] + p["mlp.b0"][None, :])
    a1 = torch.sin(a0 @ p["mlp.w1"].T + p["mlp.b1"][None, :])
    return a1 @ p["mlp.w2"].T + p["mlp.b2"][None, :]


def rel_mse(pred, true) -> torch.Tensor:
    """sum over fields of sum (pred - true)^2 / sum true^2 (whole batch)."""
    return sum(((a - b) ** 2).sum() / (b ** 2).sum() for a, b in zip(pred, true))


class Net:
    """The network for a config (attributes levels, base, groups,
    head_groups, gn_eps) and a parameter dict."""

    def __init__(self, cfg, params: dict, requires_grad: bool = False, dtype=torch.float64):
        self.L = int(cfg.levels)
        self.base = int(cfg.base)
        self.G = int(cfg.groups)
        self.Gh = int(cfg.head_groups)
        self.eps = float(cfg.gn_eps)
        self.dtype = dtype
        self.p = {k: _t(v, dtype).clone().requires_grad_(requires_grad) for k, v in params.items()}
        self.R = self.Rg = lambda u: u

    def block(self, u, name, G=None, act=True):
        y = group_norm(self.Rg(conv3x3(u, self.W(name + ".w"))), G or self.G, self.p[name + ".gamma"],
                       self.p[name + ".beta"], self.eps)
        return gelu(y) if act else y

    def W(self, name):
        return self.R(self.p[name])

    def forward(self, c, phi, rho, jump, bf16: bool = False):
        """Prediction (c', phi', rho') for states [n][H][W] and jumps [n]."""
        self.R = _RoundValue.apply if bf16 else (lambda u: u)
        self.Rg = _RoundGrad.apply if bf16 else (lambda u: u)
        R = self.R
        c, phi, rho, jump = (_t(a, self.dtype) for a in (c, phi, rho, jump))
        n, H, W = c.shape
        x = R(torch.stack([c - 0.5, phi, rho - 1.0, jump.view(n, 1, 1).expand(n, H, W)], dim=1))
        f = time_basis(jump, self.p)
        zs = []
        h = x
        for l in range(self.L):
            z = self.block(h, f"enc{l}")
            s = f @ self.p[f"film{l}.w"].T                    # w_l f(dt), [n][C_l]
            zs.append(R(z * s[:, :, None, None]))
            if l < self.L - 1:
                h = down(R(z))
        a = R(self.block(zs[-1], "mid"))
        for l in range(self.L - 2, -1, -1):
            d = self.Rg(R(up(a, self.W(f"up{l + 1}.w"))))
            a = R(self.block(torch.cat([zs[l], d], dim=1), f"dec{l}"))
        head = self.block(a, "head", G=self.Gh, act=False)
        dt = jump.view(n, 1, 1)
        return c + dt * head[:, 0], phi + dt * head[:, 1], rho + dt * head[:, 2]

    def loss_and_grads(self, state, jump, target, bf16: bool = False):
        """Loss of the prediction from `state` against `target` and its
        gradient for every parameter (FP64; with bf16, values and gradients
        are rounded as described above)."""
        for v in self.p.values():
            if v.grad is not None:
                v.grad = None
            v.requires_grad_(True)
        pred = self.forward(*state, jump, bf16=bf16)
        L = rel_mse(pred, [_t(t, self.dtype) for t in target])
        L.backward()
        return float(L.detach()), {k: v.grad.detach().numpy().copy() for k, v in self.p.items()}


def adam(w, g, m, v, t: int, lr: float, b1: float, b2: float, eps: float):
    """One step of Adam (Kingma and Ba, the optimiser the paper trains with):
    biased moment estimates, bias correction by 1 - beta^t, then
    w - lr m_hat / (sqrt(v_hat) + eps).  Returns (w, m, v) as float64."""
    w, g, m, v = (np.asarray(a, dtype=np.float64) for a in (w, g, m, v))
    m = b1 * m + (1 - b1) * g
    v = b2 * v + (1 - b2) * g * g
    mh = m / (1 - b1 ** t)
    vh = v / (1 - b2 ** t)
    return w - lr * mh / (np.sqrt(vh) + eps), m, v
