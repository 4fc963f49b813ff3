"""ctypes binding of libpf.so (the C ABI in include/pf.h).

Argument marshalling only: torch provides device memory (tensors) and the
stream (torch's current HIP stream); every step of the phase-field path
runs in the library's gfx950 kernels.  There is no fallback: if libpf.so is
missing, `load()` raises.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional

import numpy as np

from .inputs import PFParams

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libpf.so")

PF_OK, PF_EINVAL, PF_EUNSTABLE, PF_ENONFINITE, PF_EDEVICE, PF_EABORTED, PF_ESCRATCH = 0, -1, -2, -3, -4, -5, -6
PF_F32, PF_F64 = 0, 1
PF_BC_PVD, PF_BC_PERIODIC = 0, 1
PF_INIT_SEEDED, PF_INIT_KEEP = 0, 1
PF_INTEGRATOR = {"euler": 0, "midpoint": 1}
PF_FUSED_TILE, PF_FUSED_MARCH, PF_FUSED_RESIDENT = 1, 2, 3

EXPORTS = (
    "pf_workspace_bytes", "pf_dt_limit", "pf_init", "pf_step_n", "pf_mass", "pf_energy",
    "pf_get_step", "pf_set_step", "pf_get_dt", "pf_get_inflow", "pf_set_inflow", "pf_step_out",
    "pf_destroy", "pf_strerror", "pf_last_hip_error", "pf_get_launch", "pf_get_lane_cols", "pf_get_fused_kernel",
    "pf_adjoint_workspace_bytes", "pf_adjoint_step", "pf_adjoint_segment", "pf_adjoint_recompute",
    "pf_adjoint_sweep", "pf_adjoint_reset", "pf_adjoint_grad",
    "pf_diagnostics_noalloc", "pf_diagnostics_noalloc_limit",
)


class PFParamsC(ctypes.Structure):
    """Mirror of `pf_params` in include/pf.h (same field order and types)."""

    _fields_ = [
        ("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("batch", ctypes.c_int32),
        ("precision", ctypes.c_int32), ("bc_mode", ctypes.c_int32), ("flux_on", ctypes.c_int32),
        ("init_mode", ctypes.c_int32), ("allow_unstable", ctypes.c_int32),
        ("temporal_block", ctypes.c_int32), ("graph_mode", ctypes.c_int32),
        ("tile_rows", ctypes.c_int32), ("integrator", ctypes.c_int32),
        ("seed", ctypes.c_uint64),
        ("h", ctypes.c_double), ("dt", ctypes.c_double), ("dt_factor", ctypes.c_double),
        ("W_c", ctypes.c_double), ("W_phi", ctypes.c_double),
        ("kappa_c", ctypes.c_double), ("kappa_phi", ctypes.c_double),
        ("MA_bulk", ctypes.c_double), ("MB_bulk", ctypes.c_double),
        ("MA_surf", ctypes.c_double), ("MB_surf", ctypes.c_double),
        ("sigma_surf", ctypes.c_double), ("M_phi", ctypes.c_double), ("M_scale", ctypes.c_double),
        ("D_rho", ctypes.c_double), ("v0", ctypes.c_double), ("theta_deg", ctypes.c_double),
        ("rho_in", ctypes.c_double),
        ("c0", ctypes.c_double), ("c_noise", ctypes.c_double), ("film_h", ctypes.c_double),
        ("v0_per", ctypes.c_void_p), ("c0_per", ctypes.c_void_p),
        ("interface_noise", ctypes.c_double),
        ("lane_cols", ctypes.c_int32), ("fused_kernel", ctypes.c_int32),
    ]


class PFError(RuntimeError):
    def __init__(self, code: int, what: str, hip: int = 0):
        self.code = code
        self.hip = hip
        msg = f"{what}: {_strerror(code)} ({code})"
        if hip:
            msg += f", HIP error {hip}"
        super().__init__(msg)


_lib = None


def load():
    """Load libpf.so once; raise if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(
                f"{LIB_PATH} is not built; run `python -c 'import __graft_entry__ as g; g.build()'`"
                " (or `python paper_2312_05410_amd/build.py`) first")
        L = ctypes.CDLL(LIB_PATH)
        P = ctypes.POINTER(PFParamsC)
        H = ctypes.c_void_p
        dp = ctypes.POINTER(ctypes.c_double)
        L.pf_workspace_bytes.argtypes = [P]
        L.pf_workspace_bytes.restype = ctypes.c_size_t
        L.pf_dt_limit.argtypes = [P, dp]
        L.pf_init.argtypes = [ctypes.POINTER(H), P, H, H, H, H, ctypes.c_size_t, H]
        L.pf_step_n.argtypes = [H, ctypes.c_int64]
        L.pf_step_out.argtypes = [H] * 7
        L.pf_step_out.restype = ctypes.c_int
        L.pf_mass.argtypes = [H, dp]
        L.pf_energy.argtypes = [H, dp]
        L.pf_get_step.argtypes = [H, ctypes.POINTER(ctypes.c_int64)]
        L.pf_set_step.argtypes = [H, ctypes.c_int64]
        L.pf_get_dt.argtypes = [H, dp]
        L.pf_get_inflow.argtypes = [H, dp]
        L.pf_set_inflow.argtypes = [H, dp]
        for f in (L.pf_dt_limit, L.pf_init, L.pf_step_n, L.pf_mass, L.pf_energy, L.pf_get_step,
                  L.pf_set_step, L.pf_get_dt, L.pf_get_inflow, L.pf_set_inflow):
            f.restype = ctypes.c_int
        L.pf_destroy.argtypes = [H]
        L.pf_destroy.restype = None
        L.pf_strerror.argtypes = [ctypes.c_int]
        L.pf_strerror.restype = ctypes.c_char_p
        L.pf_last_hip_error.argtypes = [H]
        L.pf_last_hip_error.restype = ctypes.c_int
        L.pf_get_launch.argtypes = [H, ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int32)]
        L.pf_get_launch.restype = ctypes.c_int
        L.pf_get_lane_cols.argtypes = [H, ctypes.POINTER(ctypes.c_int32)]
        L.pf_get_lane_cols.restype = ctypes.c_int
        L.pf_get_fused_kernel.argtypes = [H, ctypes.POINTER(ctypes.c_int32)]
        L.pf_get_fused_kernel.restype = ctypes.c_int
        L.pf_adjoint_workspace_bytes.argtypes = [P]
        L.pf_adjoint_workspace_bytes.restype = ctypes.c_size_t
        L.pf_adjoint_step.argtypes = [H] * 11 + [ctypes.c_size_t]
        L.pf_adjoint_step.restype = ctypes.c_int
        L.pf_adjoint_segment.argtypes = [H, H, ctypes.c_int64] + [H] * 7 + [ctypes.c_size_t,
                                                                            ctypes.POINTER(ctypes.c_int32)]
        L.pf_adjoint_segment.restype = ctypes.c_int
        L.pf_adjoint_recompute.argtypes = [H, H, ctypes.c_int64]
        L.pf_adjoint_recompute.restype = ctypes.c_int
        L.pf_adjoint_sweep.argtypes = [H, H, ctypes.c_int64] + [H] * 7 + [ctypes.c_size_t,
                                                                          ctypes.POINTER(ctypes.c_int32)]
        L.pf_adjoint_sweep.restype = ctypes.c_int
        L.pf_adjoint_reset.argtypes = [H, H, ctypes.c_size_t]
        L.pf_adjoint_reset.restype = ctypes.c_int
        L.pf_adjoint_grad.argtypes = [H, H, ctypes.c_size_t, dp]
        L.pf_adjoint_grad.restype = ctypes.c_int
        L.pf_diagnostics_noalloc.argtypes = [P, H, H, H, H, H]
        L.pf_diagnostics_noalloc.restype = ctypes.c_int
        L.pf_diagnostics_noalloc_limit.argtypes = []
        L.pf_diagnostics_noalloc_limit.restype = ctypes.c_size_t
        _lib = L
    return _lib


def _strerror(code: int) -> str:
    try:
        return load().pf_strerror(code).decode()
    except Exception:
        return "?"


_PREC = {"f32": PF_F32, "f64": PF_F64}
_BC = {"pvd": PF_BC_PVD, "periodic": PF_BC_PERIODIC}


def to_c(p: PFParams, init_mode: int = PF_INIT_SEEDED, temporal_block: int = 0,
         allow_unstable: bool = False, graph_mode: int = 0, tile_rows: int = 0, lane_cols: int = 0,
         fused_kernel: int = 0):
    """Build the C struct; returns (struct, keep-alive arrays)."""
    keep = []

    def arr(a: Optional[np.ndarray]):
        if a is None:
            return None
        a = np.ascontiguousarray(a, dtype=np.float64)
        if a.shape != (p.batch,):
            raise ValueError("per-realisation arrays must have shape (batch,)")
        keep.append(a)
        return a.ctypes.data

    s = PFParamsC(
        nx=p.nx, ny=p.ny, batch=p.batch, precision=_PREC[p.precision], bc_mode=_BC[p.bc_mode],
        flux_on=int(bool(p.flux_on)), init_mode=init_mode, allow_unstable=int(bool(allow_unstable)),
        temporal_block=temporal_block, graph_mode=graph_mode, tile_rows=tile_rows,
        integrator=PF_INTEGRATOR[p.integrator], seed=p.seed & 0xFFFFFFFFFFFFFFFF,
        h=p.h, dt=p.dt, dt_factor=p.dt_factor,
        W_c=p.W_c, W_phi=p.W_phi, kappa_c=p.kappa_c, kappa_phi=p.kappa_phi,
        MA_bulk=p.MA_bulk, MB_bulk=p.MB_bulk, MA_surf=p.MA_surf, MB_surf=p.MB_surf,
        sigma_surf=p.sigma_surf, M_phi=p.M_phi, M_scale=p.M_scale,
        D_rho=p.D_rho, v0=p.v0, theta_deg=p.theta_deg, rho_in=p.rho_in,
        c0=p.c0, c_noise=p.c_noise, film_h=p.film_h,
        v0_per=arr(p.v0_per), c0_per=arr(p.c0_per), interface_noise=float(p.interface_noise),
        lane_cols=lane_cols, fused_kernel=fused_kernel)
    return s, keep


def workspace_bytes(p: PFParams) -> int:
    s, _keep = to_c(p)
    n = load().pf_workspace_bytes(ctypes.byref(s))
    if n == 0:
        raise PFError(PF_EINVAL, "pf_workspace_bytes")
    return int(n)


def diagnostics_noalloc(p: PFParams, c, phi, rho, out, stream=None) -> None:
    """Enqueue pf_diagnostics_noalloc: out (a float64 device tensor of
    batch x 4) receives h^2 sum c, h^2 sum phi, h^2 sum rho and F_h per
    realisation of the device tensors c, phi, rho; no allocation, no wait."""
    import torch

    s, _keep = to_c(p)
    if stream is None:
        stream = torch.cuda.current_stream(c.device)
    rc = load().pf_diagnostics_noalloc(ctypes.byref(s), c.data_ptr(), phi.data_ptr(), rho.data_ptr(),
                                       out.data_ptr(), stream.cuda_stream)
    if rc:
        raise PFError(rc, "pf_diagnostics_noalloc")


def dt_limit(p: PFParams) -> float:
    s, _keep = to_c(p)
    out = ctypes.c_double()
    rc = load().pf_dt_limit(ctypes.byref(s), ctypes.byref(out))
    if rc:
        raise PFError(rc, "pf_dt_limit")
    return out.value


class Simulator:
    """Owns torch tensors c, phi, rho [batch, ny, nx] and a workspace, and a
    pf_handle that steps them on the current stream of `device`."""

    def __init__(self, p: PFParams, state=None, temporal_block: int = 0, device: str = "cuda",
                 allow_unstable: bool = False, graph_mode: int = 0, tile_rows: int = 0, tensors=None,
                 lane_cols: int = 0, fused_kernel: int = 0):
        """state: host arrays copied to the device as the initial condition;
        tensors: (c, phi, rho) device tensors stepped in place (no copy);
        neither: the seeded initial condition."""
        import torch

        L = load()
        self.p = p
        self.device = torch.device(device)
        dtype = torch.float64 if p.precision == "f64" else torch.float32
        shape = (p.batch, p.ny, p.nx)
        if tensors is not None:
            for u in tensors:
                if u.dtype != dtype or tuple(u.shape) != shape or not u.is_contiguous() or u.device.type != "cuda":
                    raise ValueError("tensors must be contiguous device tensors of shape (batch, ny, nx) "
                                     "and the handle's precision")
            self.c, self.phi, self.rho = tensors
            self.device = tensors[0].device
            mode = PF_INIT_KEEP
        elif state is None:
            self.c, self.phi, self.rho = (torch.empty(shape, dtype=dtype, device=self.device) for _ in range(3))
            mode = PF_INIT_SEEDED
        else:
            self.c, self.phi, self.rho = (
                torch.as_tensor(np.asarray(u), dtype=dtype).reshape(shape).to(self.device).contiguous()
                for u in state)
            mode = PF_INIT_KEEP
        s, keep = to_c(p, init_mode=mode, temporal_block=temporal_block, allow_unstable=allow_unstable,
                       graph_mode=graph_mode, tile_rows=tile_rows, lane_cols=lane_cols,
                       fused_kernel=fused_kernel)
        nbytes = L.pf_workspace_bytes(ctypes.byref(s))
        if nbytes == 0:
            raise PFError(PF_EINVAL, "pf_workspace_bytes")
        self.workspace = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        self.stream = torch.cuda.current_stream(self.device)
        h = ctypes.c_void_p()
        rc = L.pf_init(ctypes.byref(h), ctypes.byref(s), self.c.data_ptr(), self.phi.data_ptr(),
                       self.rho.data_ptr(), self.workspace.data_ptr(), nbytes, self.stream.cuda_stream)
        del keep
        if rc:
            raise PFError(rc, "pf_init")
        self._h = h

    # -- stepping and diagnostics -------------------------------------------------
    def _check(self, rc: int, what: str):
        if rc:
            raise PFError(rc, what, load().pf_last_hip_error(self._h))

    def step(self, n: int) -> "Simulator":
        self._check(load().pf_step_n(self._h, int(n)), "pf_step_n")
        return self

    def step_out(self, src, dst) -> "Simulator":
        """One Euler step from the (c, phi, rho) tensors `src` into `dst`
        (pf_step_out: no inflow, the handle's own state untouched)."""
        self._check(load().pf_step_out(self._h, *(u.data_ptr() for u in src), *(u.data_ptr() for u in dst)),
                    "pf_step_out")
        return self

    def mass(self) -> np.ndarray:
        out = np.empty((self.p.batch, 4))
        self._check(load().pf_mass(self._h, out.ctypes.data_as(ctypes.POINTER(ctypes.c_double))), "pf_mass")
        return out

    def energy(self) -> np.ndarray:
        out = np.empty(self.p.batch)
        self._check(load().pf_energy(self._h, out.ctypes.data_as(ctypes.POINTER(ctypes.c_double))), "pf_energy")
        return out

    def inflow(self) -> np.ndarray:
        out = np.empty(self.p.batch)
        self._check(load().pf_get_inflow(self._h, out.ctypes.data_as(ctypes.POINTER(ctypes.c_double))),
                    "pf_get_inflow")
        return out

    def set_inflow(self, Q) -> None:
        q = np.ascontiguousarray(Q, dtype=np.float64).reshape(self.p.batch)
        self._check(load().pf_set_inflow(self._h, q.ctypes.data_as(ctypes.POINTER(ctypes.c_double))),
                    "pf_set_inflow")

    @property
    def dt(self) -> float:
        out = ctypes.c_double()
        self._check(load().pf_get_dt(self._h, ctypes.byref(out)), "pf_get_dt")
        return out.value

    @property
    def launch(self):
        """(steps fused per launch, rows per wave or tile) this handle uses."""
        k, r = ctypes.c_int32(), ctypes.c_int32()
        self._check(load().pf_get_launch(self._h, ctypes.byref(k), ctypes.byref(r)), "pf_get_launch")
        return k.value, r.value

    @property
    def lane_cols(self) -> int:
        """Grid columns per lane of the single-step kernel (1 or 2)."""
        c = ctypes.c_int32()
        self._check(load().pf_get_lane_cols(self._h, ctypes.byref(c)), "pf_get_lane_cols")
        return c.value

    @property
    def fused_kernel(self) -> int:
        """Kernel of the fused launches: 1 LDS tile, 2 register strip march,
        3 resident stepper (one launch per call), 0 when each launch is one
        step."""
        c = ctypes.c_int32()
        self._check(load().pf_get_fused_kernel(self._h, ctypes.byref(c)), "pf_get_fused_kernel")
        return c.value

    @property
    def step_count(self) -> int:
        out = ctypes.c_int64()
        self._check(load().pf_get_step(self._h, ctypes.byref(out)), "pf_get_step")
        return out.value

    # -- adjoint -------------------------------------------------------------------
    def adjoint_workspace(self):
        """A zeroed device workspace for the adjoint calls of this handle."""
        import torch

        s, _keep = to_c(self.p)
        n = load().pf_adjoint_workspace_bytes(ctypes.byref(s))
        if n == 0:
            raise PFError(PF_EINVAL, "pf_adjoint_workspace_bytes")
        ws = torch.empty(n, dtype=torch.uint8, device=self.device)
        self._check(load().pf_adjoint_reset(self._h, ws.data_ptr(), n), "pf_adjoint_reset")
        return ws

    def adjoint_step(self, state, lam, out, ws) -> None:
        """out = lam + (dR/du)^T dt lam at `state`; (c, phi, rho) tensors each."""
        args = [u.data_ptr() for u in (*state, *lam, *out)]
        self._check(load().pf_adjoint_step(self._h, *args, ws.data_ptr(), ws.numel()), "pf_adjoint_step")

    def adjoint_segment(self, ring, length: int, lam, tmp, ws) -> bool:
        """One checkpoint segment of the reverse sweep (pf_adjoint_segment):
        ring [>= length][3][...] holds the checkpoint in slot 0; returns True
        when the result is in `tmp` (odd length), else it is in `lam`."""
        self._check_ring(ring, length)
        flag = ctypes.c_int32(0)
        args = [u.data_ptr() for u in (*lam, *tmp)]
        self._check(load().pf_adjoint_segment(self._h, ring.data_ptr(), int(length), *args, ws.data_ptr(), ws.numel(),
                                              ctypes.byref(flag)), "pf_adjoint_segment")
        return bool(flag.value)

    def adjoint_recompute(self, ring, length: int) -> None:
        """Slots 1 .. length-1 of `ring` stepped from slot 0 (pf_adjoint_recompute)."""
        self._check_ring(ring, length)
        self._check(load().pf_adjoint_recompute(self._h, ring.data_ptr(), int(length)), "pf_adjoint_recompute")

    def adjoint_sweep(self, ring, length: int, lam, tmp, ws) -> bool:
        """The adjoint steps over a recomputed ring (pf_adjoint_sweep); the
        return value as for adjoint_segment."""
        self._check_ring(ring, length)
        flag = ctypes.c_int32(0)
        args = [u.data_ptr() for u in (*lam, *tmp)]
        self._check(load().pf_adjoint_sweep(self._h, ring.data_ptr(), int(length), *args, ws.data_ptr(), ws.numel(),
                                            ctypes.byref(flag)), "pf_adjoint_sweep")
        return bool(flag.value)

    def _check_ring(self, ring, length: int) -> None:
        want = (3, self.p.batch, self.p.ny, self.p.nx) if self.p.batch > 1 else (3, self.p.ny, self.p.nx)
        esize = 8 if self.p.precision == "f64" else 4
        if not ring.is_contiguous() or ring.element_size() != esize or ring.shape[0] < length or tuple(
                ring.shape[1:]) not in (
                want, (3, self.p.batch, self.p.ny, self.p.nx)):
            raise PFError(PF_EINVAL, f"ring of shape {tuple(ring.shape)} for {length} states")

    def adjoint_grad(self, ws) -> np.ndarray:
        """[batch, 2] accumulated (dL/dM_scale, dL/dv0)."""
        out = np.empty((self.p.batch, 2))
        self._check(load().pf_adjoint_grad(self._h, ws.data_ptr(), ws.numel(),
                                           out.ctypes.data_as(ctypes.POINTER(ctypes.c_double))), "pf_adjoint_grad")
        return out

    def state(self):
        """Host float64 copies of (c, phi, rho), after the stream finishes."""
        self.stream.synchronize()
        return tuple(u.detach().to("cpu", torch_dtype_f64()).numpy() for u in (self.c, self.phi, self.rho))

    def close(self) -> None:
        if getattr(self, "_h", None):
            self.stream.synchronize()
            load().pf_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def torch_dtype_f64():
    import torch

    return torch.float64
