"""CPU FP64 oracle of the explicit PVD phase-field step (ctypes wrapper).

TEST INFRASTRUCTURE ONLY: imported by the test suite, the smoke check and
the CPU-baseline leg of the benchmark.  The product path never imports it.

The arithmetic lives in `pf_oracle.c` (plain C, double precision, plain
loops); this module compiles it with gcc on first use and marshals numpy
arrays.  It shares no code with the GPU library.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "pf_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

_BC = {"pvd": 0, "periodic": 1}
_INTEGRATOR = {"euler": 0, "midpoint": 1}


class _OrParams(ctypes.Structure):
    _fields_ = [
        ("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("batch", ctypes.c_int32),
        ("bc_mode", ctypes.c_int32), ("flux_on", ctypes.c_int32), ("integrator", ctypes.c_int32),
        ("seed", ctypes.c_uint64),
        ("h", ctypes.c_double), ("dt", ctypes.c_double),
        ("W_c", ctypes.c_double), ("W_phi", ctypes.c_double),
        ("kappa_c", ctypes.c_double), ("kappa_phi", ctypes.c_double),
        ("MA_bulk", ctypes.c_double), ("MB_bulk", ctypes.c_double),
        ("MA_surf", ctypes.c_double), ("MB_surf", ctypes.c_double),
        ("sigma_surf", ctypes.c_double), ("M_phi", ctypes.c_double),
        ("M_scale", ctypes.c_double),
        ("D_rho", ctypes.c_double), ("v0", ctypes.c_double),
        ("theta_deg", ctypes.c_double), ("rho_in", ctypes.c_double),
        ("c0", ctypes.c_double), ("c_noise", ctypes.c_double), ("film_h", ctypes.c_double),
        ("interface_noise", ctypes.c_double),
    ]


def build(force: bool = False) -> str:
    """Compile liboracle.so (gcc, -O2, OpenMP, no FP contraction)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call([
            "gcc", "-std=c11", "-O2", "-fopenmp", "-ffp-contract=off", "-fno-fast-math",
            "-fPIC", "-shared", _SRC, "-o", tmp, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        build()
        L = ctypes.CDLL(_LIB)
        P = ctypes.POINTER(_OrParams)
        dp = ctypes.POINTER(ctypes.c_double)
        L.or_dt_limit.argtypes = [P, ctypes.c_double, dp]
        L.or_dt_limit.restype = ctypes.c_int
        L.or_splitmix64.argtypes = [ctypes.c_uint64, ctypes.c_uint64]
        L.or_splitmix64.restype = ctypes.c_uint64
        L.or_init.argtypes = [P, ctypes.c_void_p, dp, dp, dp]
        L.or_potentials.argtypes = [P, dp, dp, dp, dp, dp]
        L.or_step_n.argtypes = [P, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64, ctypes.c_int64,
                                dp, dp, dp, dp]
        L.or_trunc_gauss.argtypes = [ctypes.c_uint64, ctypes.c_uint64, ctypes.c_double, ctypes.c_double]
        L.or_trunc_gauss.restype = ctypes.c_double
        L.or_mass.argtypes = [P, dp, dp, dp, dp, dp]
        L.or_energy.argtypes = [P, dp, dp, dp]
        L.or_adjoint_step.argtypes = [P, ctypes.c_double, dp, dp, dp, dp, dp, dp, dp]
        L.or_loss_grad.argtypes = [P, ctypes.c_double, ctypes.c_int64, ctypes.c_int64,
                                   dp, dp, dp, dp, dp, dp, dp]
        for f in (L.or_init, L.or_potentials, L.or_step_n, L.or_mass, L.or_energy,
                  L.or_adjoint_step, L.or_loss_grad):
            f.restype = None
        _lib = L
    return _lib


def _ptr(a: np.ndarray):
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _opt(a):
    if a is None:
        return None
    a = np.ascontiguousarray(a, dtype=np.float64)
    return a


def to_c(p, dt: float | None = None) -> _OrParams:
    """Convert a parameter object (attributes as in PFParams) to the C struct."""
    return _OrParams(
        nx=p.nx, ny=p.ny, batch=p.batch, bc_mode=_BC[p.bc_mode], flux_on=int(bool(p.flux_on)),
        integrator=_INTEGRATOR[getattr(p, "integrator", "euler")], seed=p.seed & 0xFFFFFFFFFFFFFFFF,
        h=p.h, dt=p.dt if dt is None else dt,
        W_c=p.W_c, W_phi=p.W_phi, kappa_c=p.kappa_c, kappa_phi=p.kappa_phi,
        MA_bulk=p.MA_bulk, MB_bulk=p.MB_bulk, MA_surf=p.MA_surf, MB_surf=p.MB_surf,
        sigma_surf=p.sigma_surf, M_phi=p.M_phi, M_scale=p.M_scale,
        D_rho=p.D_rho, v0=p.v0, theta_deg=p.theta_deg, rho_in=p.rho_in,
        c0=p.c0, c_noise=p.c_noise, film_h=p.film_h,
        interface_noise=float(getattr(p, "interface_noise", 0.0)))


def _vmax(p) -> float:
    v = getattr(p, "v0_per", None)
    return float(np.max(np.abs(v))) if v is not None else abs(float(p.v0))


def dt_limit(p) -> float:
    out = ctypes.c_double()
    if lib().or_dt_limit(ctypes.byref(to_c(p)), _vmax(p), ctypes.byref(out)) != 0:
        raise ValueError("oracle: bad parameters for the stability limit")
    return out.value


def resolve_dt(p) -> float:
    """The time step the oracle uses: p.dt if positive, else dt_factor * limit."""
    return p.dt if p.dt > 0 else p.dt_factor * dt_limit(p)


def splitmix64(seed: int, n: int) -> int:
    return int(lib().or_splitmix64(seed & 0xFFFFFFFFFFFFFFFF, n))


def init(p):
    """Seeded initial condition, float64 arrays [batch, ny, nx]."""
    shape = (p.batch, p.ny, p.nx)
    c, phi, rho = (np.empty(shape) for _ in range(3))
    c0 = _opt(getattr(p, "c0_per", None))
    lib().or_init(ctypes.byref(to_c(p)), None if c0 is None else c0.ctypes.data, _ptr(c), _ptr(phi), _ptr(rho))
    return c, phi, rho


def potentials(p, c, phi):
    """mu_c, mu_phi, M_c of one realisation [ny, nx]."""
    c = np.ascontiguousarray(c, dtype=np.float64)
    phi = np.ascontiguousarray(phi, dtype=np.float64)
    mc, mp, M = (np.empty_like(c) for _ in range(3))
    lib().or_potentials(ctypes.byref(to_c(p)), _ptr(c), _ptr(phi), _ptr(mc), _ptr(mp), _ptr(M))
    return mc, mp, M


def trunc_gauss(seed: int, counter0: int, mean: float, sigma: float) -> float:
    """The interface composition draw (see pf_oracle.c)."""
    return float(lib().or_trunc_gauss(seed & 0xFFFFFFFFFFFFFFFF, counter0, mean, sigma))


class State:
    """Oracle state: c, phi, rho [batch, ny, nx], cumulative inflow Q[batch]
    and the global step count (it keys the interface composition draws)."""

    def __init__(self, p, c, phi, rho, Q=None, dt: float | None = None, nstep: int = 0):
        self.p = p
        self.dt = resolve_dt(p) if dt is None else dt
        shape = (p.batch, p.ny, p.nx)
        self.c = np.array(c, dtype=np.float64).reshape(shape)
        self.phi = np.array(phi, dtype=np.float64).reshape(shape)
        self.rho = np.array(rho, dtype=np.float64).reshape(shape)
        self.Q = np.zeros(p.batch) if Q is None else np.array(Q, dtype=np.float64)
        self._v0 = _opt(getattr(p, "v0_per", None))
        self._c0 = _opt(getattr(p, "c0_per", None))
        self.nstep = int(nstep)

    @classmethod
    def seeded(cls, p, dt: float | None = None):
        return cls(p, *init(p), dt=dt)

    def step(self, n: int):
        cp = to_c(self.p, self.dt)
        lib().or_step_n(ctypes.byref(cp), None if self._v0 is None else self._v0.ctypes.data,
                        None if self._c0 is None else self._c0.ctypes.data, self.nstep, int(n),
                        _ptr(self.c), _ptr(self.phi), _ptr(self.rho), _ptr(self.Q))
        self.nstep += int(n)
        return self

    def mass(self) -> np.ndarray:
        out = np.empty((self.p.batch, 4))
        lib().or_mass(ctypes.byref(to_c(self.p, self.dt)), _ptr(self.c), _ptr(self.phi), _ptr(self.rho),
                      _ptr(self.Q), _ptr(out))
        return out

    def energy(self) -> np.ndarray:
        out = np.empty(self.p.batch)
        lib().or_energy(ctypes.byref(to_c(self.p, self.dt)), _ptr(self.c), _ptr(self.phi), _ptr(out))
        return out


# ------------------------------------------------------------------ adjoint

def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def adjoint_step(p, v0: float, dt: float, state, lam):
    """(lambda_prev, g) for one step of one realisation from `state` =
    (c, phi, rho) [ny, nx], given lam = dL/du' as three [ny, nx] arrays.
    g = (dL/dM_scale, dL/dv0) contributions of this step (fixed dt)."""
    c, phi, rho = (_f64(u) for u in state)
    lc, lp, lr = (np.array(u, dtype=np.float64) for u in lam)
    g = np.zeros(2)
    cp = to_c(p.replace(batch=1) if hasattr(p, "replace") else p, dt)
    lib().or_adjoint_step(ctypes.byref(cp), float(v0), _ptr(c), _ptr(phi), _ptr(rho),
                          _ptr(lc), _ptr(lp), _ptr(lr), _ptr(g))
    return (lc, lp, lr), g


def loss_grad(p, v0: float, dt: float, n: int, every: int, state, target):
    """(L, dL/dM_scale, dL/dv0) of L = h^2/2 sum (u_n - u*)^2 after n steps of
    one realisation from `state`, by the checkpointed adjoint."""
    c, phi, rho = (_f64(u) for u in state)
    ct, pt, rt = (_f64(u) for u in target)
    out = np.zeros(3)
    cp = to_c(p.replace(batch=1) if hasattr(p, "replace") else p, dt)
    lib().or_loss_grad(ctypes.byref(cp), float(v0), int(n), int(every), _ptr(c), _ptr(phi), _ptr(rho),
                       _ptr(ct), _ptr(pt), _ptr(rt), _ptr(out))
    return out


def run(p, v0: float, dt: float, n: int, state):
    """Final (c, phi, rho) [ny, nx] after n steps of one realisation."""
    q = p.replace(batch=1, v0=float(v0), v0_per=None, c0_per=None)
    s = State(q, *(np.asarray(u)[None] for u in state), dt=dt).step(n)
    return s.c[0], s.phi[0], s.rho[0]


def loss(p, v0, dt, n, state, target):
    u = run(p, v0, dt, n, state)
    return 0.5 * p.h ** 2 * sum(float(np.sum((a - b) ** 2)) for a, b in zip(u, target))
