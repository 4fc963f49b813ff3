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
