"""Dense-matrix assembly of the discrete PVD phase-field step on tiny grids.

An independent second formulation used to pin the oracle: every operator
is built as an explicit matrix over the cells (a graph form, faces times
cells) instead of the oracle's neighbour loops, so a wrong index, a
transposed axis, a wrong boundary rule or a dropped term in either one
shows up as a mismatch.  It follows the same model readings (free energy,
switching function, mobility, Euler, boundaries) stated in the oracle's
header; it does not import the oracle.
"""
from __future__ import annotations

import numpy as np


class Grid:
    def __init__(self, nx: int, ny: int, h: float, periodic_y: bool):
        self.nx, self.ny, self.h = nx, ny, h
        self.N = nx * ny
        self.periodic_y = periodic_y
        k = lambda i, j: (j % ny) * nx + (i % nx)
        self.k = k
        # face incidence: one row per face, -1 on the tail cell, +1 on the head
        xf = [(k(i, j), k(i + 1, j)) for j in range(ny) for i in range(nx)]
        ylim = ny if periodic_y else ny - 1
        yf = [(k(i, j), k(i, j + 1)) for j in range(ylim) for i in range(nx)]
        self.Dx = self._incidence(xf)
        self.Dy = self._incidence(yf)
        self.Ax = self._average(xf)
        self.Ay = self._average(yf)
        D = np.vstack([self.Dx, self.Dy])
        # graph Laplacian: no flux through faces that are not listed
        self.L = -(D.T @ D) / h**2
        # central first differences; at a mirror boundary the missing
        # neighbour takes the cell's own value
        self.Gx = np.zeros((self.N, self.N))
        self.Gy = np.zeros((self.N, self.N))
        for j in range(ny):
            for i in range(nx):
                r = k(i, j)
                self.Gx[r, k(i + 1, j)] += 1 / (2 * h)
                self.Gx[r, k(i - 1, j)] -= 1 / (2 * h)
                jn = j + 1 if (periodic_y or j + 1 < ny) else j
                js = j - 1 if (periodic_y or j - 1 >= 0) else j
                self.Gy[r, k(i, jn)] += 1 / (2 * h)
                self.Gy[r, k(i, js)] -= 1 / (2 * h)
        self.top = np.zeros(self.N)
        if not periodic_y:
            self.top[[k(i, ny - 1) for i in range(nx)]] = 1.0

    def _incidence(self, faces):
        M = np.zeros((len(faces), self.N))
        for f, (a, b) in enumerate(faces):
            M[f, a] -= 1.0
            M[f, b] += 1.0
        return M

    def _average(self, faces):
        M = np.zeros((len(faces), self.N))
        for f, (a, b) in enumerate(faces):
            M[f, a] += 0.5
            M[f, b] += 0.5
        return M


def _switch(c):
    x = np.clip(c, 0.0, 1.0)
    return x**3 * (6 * x**2 - 15 * x + 10)


def mobility(p, c, phi):
    ph = np.clip(phi, -1.0, 1.0)
    H = _switch(c)
    bulk = (2 - ph) * (1 + ph) ** 2 / 4 * (H * p.MA_bulk + (1 - H) * p.MB_bulk)
    surf = np.exp(-(ph / p.sigma_surf) ** 2) * (H * p.MA_surf + (1 - H) * p.MB_surf)
    return p.M_scale * (bulk + surf)


def potentials(p, g: Grid, c, phi):
    pf = (2 - phi) * (1 + phi) ** 2 / 4
    dpf = 3 * (1 - phi**2) / 4
    gw = c**2 * (1 - c) ** 2
    dgw = 2 * c * (1 - c) * (1 - 2 * c)
    mu_c = p.W_c * pf * dgw - p.kappa_c * (g.L @ c)
    mu_p = p.W_c * dpf * gw - p.W_phi * phi * (1 - phi**2) - p.kappa_phi * (g.L @ phi)
    return mu_c, mu_p, mobility(p, c, phi)


def step(p, g: Grid, dt, v0, c, phi, rho, Q):
    """One explicit Euler step on flattened fields; returns new (c, phi, rho, Q)."""
    h = g.h
    if p.flux_on:
        th = np.deg2rad(p.theta_deg)
        vx, vy = v0 * np.cos(th), -v0 * np.sin(th)
    else:
        vx = vy = 0.0
    mu_c, mu_p, M = potentials(p, g, c, phi)
    D = np.vstack([g.Dx, g.Dy])
    A = np.vstack([g.Ax, g.Ay])
    div_c = -(D.T @ ((A @ M) * (D @ mu_c))) / h**2
    div_p = p.M_phi * (g.L @ mu_p)
    S = rho * (vx * (g.Gx @ phi) + vy * (g.Gy @ phi))
    pvd = not g.periodic_y
    rin = p.rho_in if pvd else 0.0
    diff = p.D_rho * (g.L @ rho + g.top * (rin - rho) / h**2)
    F = vx * (g.Ax @ rho)
    G = vy * (g.Ay @ rho)
    Gtop = vy * (rho + rin) / 2 * g.top
    adv = -(-(g.Dx.T @ F) - (g.Dy.T @ G) + Gtop) / h
    T = diff + adv
    dQ = 0.0
    if pvd:
        dQ = dt * h * np.sum(g.top * (-vy * (rho + rin) / 2 + p.D_rho * (rin - rho) / h))
    return c + dt * div_c, phi + dt * (div_p + S), rho + dt * (T - S), Q + dQ


def energy(p, g: Grid, c, phi):
    f = p.W_c * (2 - phi) * (1 + phi) ** 2 / 4 * c**2 * (1 - c) ** 2 + p.W_phi / 4 * (1 - phi**2) ** 2
    D = np.vstack([g.Dx, g.Dy])
    return g.h**2 * f.sum() + p.kappa_c / 2 * np.sum((D @ c) ** 2) + p.kappa_phi / 2 * np.sum((D @ phi) ** 2)
