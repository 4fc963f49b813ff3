"""Brute-force definitions of the blended run's microstructure statistics.

TEST INFRASTRUCTURE ONLY (imported by the test suite).  Plain loops over
small grids, following the paper's description (Results, "autocorrelations
of the microstructure"): S2^(A,A)(r) is the probability that x and x + r
both lie in phase A, here over the pairs inside the domain (x periodic, y
bounded), and its radial average over annuli |r| in [k, k + 1).
"""
from __future__ import annotations

import math

import numpy as np


def indicator(c, phi):
    """1 where solid (phi > 0) and A-rich (c > 1/2)."""
    return ((np.asarray(phi) > 0) & (np.asarray(c) > 0.5)).astype(np.float64)


def s2(ind):
    """[2 ny - 1][nx]: row ry + ny - 1, column rx (periodic in x)."""
    ind = np.asarray(ind, dtype=np.float64)
    ny, nx = ind.shape
    out = np.zeros((2 * ny - 1, nx))
    for ry in range(-(ny - 1), ny):
        for rx in range(nx):
            s = 0.0
            n = 0
            for y in range(ny):
                y2 = y + ry
                if not 0 <= y2 < ny:
                    continue
                for x in range(nx):
                    s += ind[y, x] * ind[y2, (x + rx) % nx]
                    n += 1
            out[ry + ny - 1, rx] = s / n
    return out


def radial_average(s, rmax):
    n2, nx = s.shape
    ny = (n2 + 1) // 2
    tot = np.zeros(rmax)
    cnt = np.zeros(rmax)
    for i in range(n2):
        ry = i - (ny - 1)
        for rx in range(nx):
            rxi = min(rx, nx - rx)
            k = int(math.floor(math.sqrt(ry * ry + rxi * rxi)))
            if k < rmax:
                tot[k] += s[i, rx]
                cnt[k] += 1
    return tot / np.maximum(cnt, 1)
