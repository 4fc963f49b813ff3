"""The GPU metrics (torch, run here on the CPU) against brute-force
definitions, and the brute force against closed forms."""
from __future__ import annotations

import numpy as np
import torch

from oracle import metrics_oracle as mo
from paper_2312_05410_amd import metrics
from paper_2312_05410_amd.inputs import uniform01


def test_bruteforce_closed_forms():
    ny, nx = 6, 8
    y, x = np.mgrid[0:ny, 0:nx]
    checker = ((x + y) % 2).astype(float)
    s = mo.s2(checker)
    for ry in range(-(ny - 1), ny):
        for rx in range(nx):
            assert s[ry + ny - 1, rx] == (0.5 if (rx + ry) % 2 == 0 else 0.0)
    ind = (uniform01(5, np.arange(ny * nx)).reshape(ny, nx) > 0.6).astype(float)
    assert mo.s2(ind)[ny - 1, 0] == ind.mean()            # S2(0) = volume fraction
    full = np.ones((ny, nx))
    assert np.all(mo.s2(full) == 1.0)
    ra = mo.radial_average(mo.s2(full), 4)
    assert np.allclose(ra, 1.0)


def test_indicator_needs_solid_and_a_rich():
    c = np.array([[0.6, 0.4], [0.6, 0.4]])
    phi = np.array([[0.5, 0.5], [-0.5, -0.5]])
    assert mo.indicator(c, phi).tolist() == [[1.0, 0.0], [0.0, 0.0]]
    assert metrics.phase_indicator(torch.tensor(c), torch.tensor(phi)).tolist() == [[1.0, 0.0], [0.0, 0.0]]


def test_fft_s2_matches_bruteforce():
    ny, nx = 9, 12
    c = uniform01(11, np.arange(ny * nx)).reshape(ny, nx)
    phi = 2 * uniform01(12, np.arange(ny * nx)).reshape(ny, nx) - 0.6
    ref = mo.s2(mo.indicator(c, phi))
    got = metrics.s2(metrics.phase_indicator(torch.tensor(c), torch.tensor(phi))).numpy()
    np.testing.assert_allclose(got, ref, rtol=0, atol=1e-12)
    np.testing.assert_allclose(metrics.radial_average(torch.tensor(ref), 6).numpy(), mo.radial_average(ref, 6),
                               rtol=0, atol=1e-12)


def test_radial_average_hand_binned_annuli():
    """Annulus membership written out by hand for ny = 3, nx = 5 (rows
    ry = -2..2, columns rx = 0..4, x displacements folded to the nearest
    periodic image min(rx, 5 - rx)).  |r| = sqrt(ry^2 + rx_folded^2):
    k = 0: (0, 0); k = 1: (0, 1), (0, 4) and rx in {0, 1, 4} at ry = +-1;
    k = 2: (0, 2), (0, 3), rx in {2, 3} at ry = +-1, every rx at ry = +-2
    (sqrt 8 = 2.83 floors to 2); k = 3: empty.  Without the fold, rx = 3, 4
    land in k = 3 or beyond; with rounding instead of floor, sqrt 2 and
    sqrt 8 move to k = 1 -> 1 and 2 -> 3; either mistake changes these means."""
    ny, nx = 3, 5
    s = uniform01(31, np.arange((2 * ny - 1) * nx)).reshape(2 * ny - 1, nx)

    def at(ry, rx):
        return s[ry + ny - 1, rx]

    k0 = [at(0, 0)]
    k1 = [at(0, 1), at(0, 4)] + [at(ry, rx) for ry in (-1, 1) for rx in (0, 1, 4)]
    k2 = [at(0, 2), at(0, 3)] + [at(ry, rx) for ry in (-1, 1) for rx in (2, 3)] + \
         [at(ry, rx) for ry in (-2, 2) for rx in range(5)]
    assert len(k0) + len(k1) + len(k2) == s.size
    want = np.array([np.mean(k0), np.mean(k1), np.mean(k2), 0.0])
    np.testing.assert_allclose(mo.radial_average(s, 4), want, rtol=0, atol=1e-15)
    np.testing.assert_allclose(metrics.radial_average(torch.tensor(s), 4).numpy(), want, rtol=0, atol=1e-15)
