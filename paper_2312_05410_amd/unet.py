"""ctypes binding of the U-Net half of libpf.so (C ABI in include/unet.h).

Argument marshalling only: torch supplies device memory and the current HIP
stream; every layer, the loss and Adam run in the library's gfx950 kernels.
There is no fallback: without libpf.so, `_lib.load()` raises.
"""
from __future__ import annotations

import ctypes
from dataclasses import asdict, dataclass
from typing import Optional

import numpy as np

from . import _lib
from .unet_inputs import init_params

_H = ctypes.c_void_p
_I = ctypes.c_int

UNET_EXPORTS = (
    "unet_param_count", "unet_param_entry", "unet_workspace_bytes", "unet_create", "unet_prepare",
    "unet_forward", "unet_forward_infer", "unet_backward", "unet_adam", "unet_destroy", "unet_op_workspace_bytes",
    "unet_conv3x3_fwd", "unet_conv3x3_prep_bytes", "unet_conv3x3_prepare", "unet_conv3x3_fwd_prepared",
    "unet_conv3x3_dgrad", "unet_conv3x3_wgrad", "unet_up_fwd", "unet_up_dgrad",
    "unet_up_wgrad", "unet_groupnorm_fwd", "unet_groupnorm_bwd", "unet_maxpool_fwd", "unet_maxpool_bwd",
)


class UNetConfigC(ctypes.Structure):
    """Mirror of `unet_config`."""

    _fields_ = [(n, ctypes.c_int32) for n in ("height", "width", "in_ch", "out_ch", "base", "levels", "groups",
                                              "head_groups", "mlp_hidden", "basis", "max_batch")] + [
        ("gn_eps", ctypes.c_float)]


class ParamDescC(ctypes.Structure):
    """Mirror of `unet_param_desc`."""

    _fields_ = [("name", ctypes.c_char * 32), ("offset", ctypes.c_int64), ("count", ctypes.c_int64),
                ("ndim", ctypes.c_int32), ("dims", ctypes.c_int32 * 4)]


@dataclass
class UNetConfig:
    """Network shape (defaults: 4 levels of 32/64/128/256 channels, sin-MLP
    of width 128, basis of 128, batch 5 as in the paper's training)."""

    height: int = 512
    width: int = 512
    in_ch: int = 4
    out_ch: int = 3
    base: int = 32
    levels: int = 4
    groups: int = 8
    head_groups: int = 1
    mlp_hidden: int = 128
    basis: int = 128
    max_batch: int = 5
    gn_eps: float = 1e-5

    def c(self) -> UNetConfigC:
        return UNetConfigC(**asdict(self))


_ready = False


def lib():
    """libpf.so with the U-Net signatures declared."""
    global _ready
    L = _lib.load()
    if not _ready:
        C = ctypes.POINTER(UNetConfigC)
        sz, f32, i64 = ctypes.c_size_t, ctypes.c_float, ctypes.c_int64
        L.unet_param_count.argtypes = [C]
        L.unet_param_count.restype = i64
        L.unet_param_entry.argtypes = [C, _I, ctypes.POINTER(ParamDescC)]
        L.unet_workspace_bytes.argtypes = [C]
        L.unet_workspace_bytes.restype = sz
        L.unet_create.argtypes = [ctypes.POINTER(_H), C, _H, _H, _H, sz, _H]
        L.unet_prepare.argtypes = [_H]
        L.unet_forward.argtypes = [_H, _I] + [_H] * 7
        L.unet_forward_infer.argtypes = [_H, _I] + [_H] * 7
        L.unet_backward.argtypes = [_H] * 7 + [ctypes.POINTER(ctypes.c_double)]
        L.unet_adam.argtypes = [_H, _H, _H, i64, f32, f32, f32, f32]
        L.unet_destroy.argtypes = [_H]
        L.unet_destroy.restype = None
        L.unet_op_workspace_bytes.argtypes = [_I] * 4
        L.unet_op_workspace_bytes.restype = sz
        L.unet_conv3x3_fwd.argtypes = [_I, _I, _I, _H, _I, _H, _I, _H, _I, _H, _H, sz, _H]
        L.unet_conv3x3_prep_bytes.argtypes = [_I, _I, _I]
        L.unet_conv3x3_prep_bytes.restype = sz
        L.unet_conv3x3_prepare.argtypes = [_H, _I, _I, _I, _H, sz, _H]
        L.unet_conv3x3_fwd_prepared.argtypes = [_I, _I, _I, _H, _I, _H, _I, _H, _I, _H, _H]
        L.unet_conv3x3_dgrad.argtypes = [_I, _I, _I, _H, _I, _H, _I, _I, _H, _H, _H, sz, _H]
        L.unet_conv3x3_wgrad.argtypes = [_I, _I, _I, _H, _I, _H, _I, _H, _I, _H, _H, sz, _H]
        L.unet_up_fwd.argtypes = [_I, _I, _I, _H, _I, _H, _I, _H, _H, sz, _H]
        L.unet_up_dgrad.argtypes = [_I, _I, _I, _H, _I, _H, _I, _H, _H, sz, _H]
        L.unet_up_wgrad.argtypes = [_I, _I, _I, _H, _I, _H, _I, _H, _H, sz, _H]
        L.unet_groupnorm_fwd.argtypes = [_I, _I, _I, _I, f32, _I] + [_H] * 7 + [_H, sz, _H]
        L.unet_groupnorm_bwd.argtypes = [_I, _I, _I, _I, f32, _I] + [_H] * 11 + [_H, sz, _H]
        L.unet_maxpool_fwd.argtypes = [_I] * 4 + [_H, _H, _H]
        L.unet_maxpool_bwd.argtypes = [_I] * 4 + [_H, _H, _H, _H]
        for name in UNET_EXPORTS:
            if name not in ("unet_param_count", "unet_workspace_bytes", "unet_destroy", "unet_op_workspace_bytes",
                            "unet_conv3x3_prep_bytes"):
                getattr(L, name).restype = _I
        _ready = True
    return L


def _check(rc: int, what: str):
    if rc != _lib.PF_OK:
        raise _lib.PFError(rc, what)


def param_entries(cfg: UNetConfig):
    """[(name, offset, dims)] of the flat parameter array."""
    L = lib()
    cc = cfg.c()
    n = L.unet_param_count(ctypes.byref(cc))
    if n < 0:
        raise ValueError(f"invalid U-Net config {cfg}")
    out, i = [], 0
    d = ParamDescC()
    while L.unet_param_entry(ctypes.byref(cc), i, ctypes.byref(d)) == _lib.PF_OK:
        out.append((d.name.decode(), int(d.offset), tuple(int(x) for x in d.dims[:d.ndim])))
        i += 1
    assert sum(int(np.prod(e[2])) for e in out) == n
    return out


def _ptr(t) -> Optional[int]:
    return None if t is None else t.data_ptr()


def _stream():
    import torch

    return torch.cuda.current_stream().cuda_stream


class UNet:
    """The network on one GPU: FP32 master parameters, gradients and Adam
    moments, and the library workspace, all torch tensors."""

    def __init__(self, cfg: UNetConfig, params: Optional[dict] = None, seed: int = 0, device: str = "cuda"):
        import torch

        self.cfg = cfg
        self.entries = param_entries(cfg)
        L = lib()
        cc = cfg.c()
        n = L.unet_param_count(ctypes.byref(cc))
        self.params = torch.zeros(n, dtype=torch.float32, device=device)
        self.grads = torch.zeros(n, dtype=torch.float32, device=device)
        self.m = torch.zeros(n, dtype=torch.float32, device=device)
        self.v = torch.zeros(n, dtype=torch.float32, device=device)
        self.t = 0
        self.set_params(params if params is not None else init_params([(e[0], e[2]) for e in self.entries], seed))
        ws = L.unet_workspace_bytes(ctypes.byref(cc))
        if ws == 0:
            raise ValueError("invalid U-Net config")
        self.workspace = torch.empty(ws, dtype=torch.uint8, device=device)
        h = _H()
        _check(L.unet_create(ctypes.byref(h), ctypes.byref(cc), self.params.data_ptr(), self.grads.data_ptr(),
                             self.workspace.data_ptr(), ws, _stream()), "unet_create")
        self._h = h

    # -- parameters
    def set_params(self, params: dict):
        import torch

        flat = np.zeros(self.params.numel(), dtype=np.float32)
        for name, off, dims in self.entries:
            a = np.asarray(params[name], dtype=np.float32)
            assert a.shape == tuple(dims), (name, a.shape, dims)
            flat[off:off + a.size] = a.ravel()
        self.params.copy_(torch.from_numpy(flat))
        if getattr(self, "_h", None):
            _check(lib().unet_prepare(self._h), "unet_prepare")

    def _split(self, flat) -> dict:
        a = flat.detach().cpu().numpy()
        return {name: a[off:off + int(np.prod(d))].reshape(d).copy() for name, off, d in self.entries}

    def param_dict(self) -> dict:
        return self._split(self.params)

    def grad_dict(self) -> dict:
        return self._split(self.grads)

    # -- passes
    def forward(self, c, phi, rho, jump, out=None, train: bool = True):
        """Prediction for states [n][H][W] (float32, device) and jumps [n];
        train=False skips what the backward pass needs."""
        import torch

        n = c.shape[0]
        if out is None:
            out = tuple(torch.empty_like(c) for _ in range(3))
        jump = torch.as_tensor(jump, dtype=torch.float32, device=c.device).reshape(n).contiguous()
        self._jump = jump  # the library copies it, but keep the tensor alive until enqueued
        fn = lib().unet_forward if train else lib().unet_forward_infer
        _check(fn(self._h, n, jump.data_ptr(), c.data_ptr(), phi.data_ptr(), rho.data_ptr(),
                  *(o.data_ptr() for o in out)), "unet_forward")
        return out

    def backward(self, pred, target, want_loss: bool = True) -> Optional[float]:
        loss = ctypes.c_double(float("nan"))
        _check(lib().unet_backward(self._h, *(p.data_ptr() for p in pred), *(t.data_ptr() for t in target),
                                   ctypes.byref(loss) if want_loss else None), "unet_backward")
        return loss.value if want_loss else None

    def adam_step(self, lr: float = 1e-4, beta1: float = 0.9, beta2: float = 0.999, eps: float = 1e-8):
        self.t += 1
        _check(lib().unet_adam(self._h, self.m.data_ptr(), self.v.data_ptr(), self.t, lr, beta1, beta2, eps),
               "unet_adam")

    def close(self):
        if getattr(self, "_h", None):
            lib().unet_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ---------------------------------------------------------------- single ops
def _ws(n, H, W, cmax, device):
    import torch

    b = lib().unet_op_workspace_bytes(n, H, W, cmax)
    return torch.empty(max(b, 256), dtype=torch.uint8, device=device)


def conv3x3_fwd(x1, w, x2=None):
    """x1 [n][H][W][C1] bf16 (+ x2 [n][H][W][C2]), w [9][Cout][C1+C2] f32 ->
    y [n][H][W][Cout] f32."""
    import torch

    n, H, W, C1 = x1.shape
    C2 = 0 if x2 is None else x2.shape[3]
    Cout = w.shape[1]
    y = torch.empty(n, H, W, Cout, dtype=torch.float32, device=x1.device)
    ws = _ws(n, H, W, max(C1 + C2, Cout), x1.device)
    _check(lib().unet_conv3x3_fwd(n, H, W, x1.data_ptr(), C1, _ptr(x2), C2, w.data_ptr(), Cout, y.data_ptr(),
                                  ws.data_ptr(), ws.numel(), _stream()), "unet_conv3x3_fwd")
    return y


def conv3x3_prepare(w, C1, C2=0):
    """BF16 MFMA operand of w [9][Cout][C1+C2] (a device byte tensor)."""
    import torch

    Cout = w.shape[1]
    nb = lib().unet_conv3x3_prep_bytes(C1, C2, Cout)
    if nb == 0:
        raise ValueError("invalid convolution sizes")
    wp = torch.empty(nb, dtype=torch.uint8, device=w.device)
    _check(lib().unet_conv3x3_prepare(w.data_ptr(), C1, C2, Cout, wp.data_ptr(), nb, _stream()),
           "unet_conv3x3_prepare")
    return wp


def conv3x3_fwd_prepared(x1, wp, Cout, x2=None, out=None):
    """conv3x3_fwd from a prepared operand (the convolution kernel alone)."""
    import torch

    n, H, W, C1 = x1.shape
    C2 = 0 if x2 is None else x2.shape[3]
    y = out if out is not None else torch.empty(n, H, W, Cout, dtype=torch.float32, device=x1.device)
    _check(lib().unet_conv3x3_fwd_prepared(n, H, W, x1.data_ptr(), C1, _ptr(x2), C2, wp.data_ptr(), Cout,
                                           y.data_ptr(), _stream()), "unet_conv3x3_fwd_prepared")
    return y


def conv3x3_dgrad(dy, w, C1, C2=0):
    import torch

    n, H, W, Cout = dy.shape
    dx1 = torch.empty(n, H, W, C1, dtype=torch.float32, device=dy.device)
    dx2 = torch.empty(n, H, W, C2, dtype=torch.float32, device=dy.device) if C2 else None
    ws = _ws(n, H, W, max(C1 + C2, Cout), dy.device)
    _check(lib().unet_conv3x3_dgrad(n, H, W, dy.data_ptr(), Cout, w.data_ptr(), C1, C2, dx1.data_ptr(), _ptr(dx2),
                                    ws.data_ptr(), ws.numel(), _stream()), "unet_conv3x3_dgrad")
    return dx1, dx2


def conv3x3_wgrad(dy, x1, x2=None):
    import torch

    n, H, W, Cout = dy.shape
    C1 = x1.shape[3]
    C2 = 0 if x2 is None else x2.shape[3]
    dw = torch.empty(9, Cout, C1 + C2, dtype=torch.float32, device=dy.device)
    ws = _ws(n, H, W, max(C1 + C2, Cout), dy.device)
    _check(lib().unet_conv3x3_wgrad(n, H, W, dy.data_ptr(), Cout, x1.data_ptr(), C1, _ptr(x2), C2, dw.data_ptr(),
                                    ws.data_ptr(), ws.numel(), _stream()), "unet_conv3x3_wgrad")
    return dw


def up_fwd(x, w):
    """x [n][H][W][Cin] bf16, w [4][Cout][Cin] -> y [n][2H][2W][Cout] f32."""
    import torch

    n, H, W, Cin = x.shape
    Cout = w.shape[1]
    y = torch.empty(n, 2 * H, 2 * W, Cout, dtype=torch.float32, device=x.device)
    ws = _ws(n, H, W, max(Cin, Cout), x.device)
    _check(lib().unet_up_fwd(n, H, W, x.data_ptr(), Cin, w.data_ptr(), Cout, y.data_ptr(), ws.data_ptr(),
                             ws.numel(), _stream()), "unet_up_fwd")
    return y


def up_dgrad(dy, w):
    import torch

    n, H2, W2, Cout = dy.shape
    Cin = w.shape[2]
    dx = torch.empty(n, H2 // 2, W2 // 2, Cin, dtype=torch.float32, device=dy.device)
    ws = _ws(n, H2 // 2, W2 // 2, max(Cin, Cout), dy.device)
    _check(lib().unet_up_dgrad(n, H2 // 2, W2 // 2, dy.data_ptr(), Cout, w.data_ptr(), Cin, dx.data_ptr(),
                               ws.data_ptr(), ws.numel(), _stream()), "unet_up_dgrad")
    return dx


def up_wgrad(dy, x):
    import torch

    n, H, W, Cin = x.shape
    Cout = dy.shape[3]
    dw = torch.empty(4, Cout, Cin, dtype=torch.float32, device=x.device)
    ws = _ws(n, H, W, max(Cin, Cout), x.device)
    _check(lib().unet_up_wgrad(n, H, W, dy.data_ptr(), Cout, x.data_ptr(), Cin, dw.data_ptr(), ws.data_ptr(),
                               ws.numel(), _stream()), "unet_up_wgrad")
    return dw


def groupnorm_fwd(y, G, gamma, beta, eps=1e-5, gelu=True, scale=None):
    """y [n][P][C] f32 -> (z, zs or None, stats [n][G][2])."""
    import torch

    n, P, C = y.shape
    z = torch.empty_like(y)
    zs = torch.empty_like(y) if scale is not None else None
    st = torch.empty(n, G, 2, dtype=torch.float32, device=y.device)
    ws = _ws(n, P, 1, C, y.device)
    _check(lib().unet_groupnorm_fwd(n, P, C, G, eps, int(gelu), y.data_ptr(), gamma.data_ptr(), beta.data_ptr(),
                                    _ptr(scale), z.data_ptr(), _ptr(zs), st.data_ptr(), ws.data_ptr(), ws.numel(),
                                    _stream()), "unet_groupnorm_fwd")
    return z, zs, st


def groupnorm_bwd(y, G, gamma, beta, stats, dA=None, dB=None, eps=1e-5, gelu=True, scale=None):
    """-> (dy, dgamma, dbeta, dscale or None)."""
    import torch

    n, P, C = y.shape
    dy = torch.empty_like(y)
    dg = torch.empty(C, dtype=torch.float32, device=y.device)
    db = torch.empty(C, dtype=torch.float32, device=y.device)
    ds = torch.empty(n, C, dtype=torch.float32, device=y.device) if (scale is not None and dB is not None) else None
    ws = _ws(n, P, 1, C, y.device)
    _check(lib().unet_groupnorm_bwd(n, P, C, G, eps, int(gelu), y.data_ptr(), gamma.data_ptr(), beta.data_ptr(),
                                    _ptr(scale), stats.data_ptr(), _ptr(dA), _ptr(dB), dy.data_ptr(), dg.data_ptr(),
                                    db.data_ptr(), _ptr(ds), ws.data_ptr(), ws.numel(), _stream()),
           "unet_groupnorm_bwd")
    return dy, dg, db, ds


def maxpool_fwd(x):
    import torch

    n, H, W, C = x.shape
    y = torch.empty(n, H // 2, W // 2, C, dtype=x.dtype, device=x.device)
    _check(lib().unet_maxpool_fwd(n, H, W, C, x.data_ptr(), y.data_ptr(), _stream()), "unet_maxpool_fwd")
    return y


def maxpool_bwd(x, dy):
    import torch

    n, H, W, C = x.shape
    dx = torch.empty(n, H, W, C, dtype=torch.float32, device=x.device)
    _check(lib().unet_maxpool_bwd(n, H, W, C, x.data_ptr(), dy.data_ptr(), dx.data_ptr(), _stream()),
           "unet_maxpool_bwd")
    return dx
