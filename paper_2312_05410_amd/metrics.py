"""Error metrics of the blended run (Results, "autocorrelations of the
microstructure"; Materials and Methods, "Error metrics"), evaluated on the
GPU with torch tensor operations.

* relative L2 error of a field;
* the two-point autocorrelation S2^(A,A)(r) of phase A in the solid film:
  the fraction of point pairs (x, x + r) that are both solid (phi > 0) and
  A-rich (c > 1/2), over the pairs that lie inside the domain (x periodic,
  y bounded by the substrate and the top), and its relative L2 error;
* the radial average of S2 over annuli |r| in [k, k + 1).
"""
from __future__ import annotations

import torch


def rel_l2(pred: torch.Tensor, true: torch.Tensor) -> float:
    d = (pred.double() - true.double()).norm()
    return float(d / true.double().norm().clamp_min(1e-300))


def phase_indicator(c: torch.Tensor, phi: torch.Tensor) -> torch.Tensor:
    """1 where the cell is solid and A-rich, else 0 (float64) [..., ny, nx]."""
    return ((phi > 0) & (c > 0.5)).double()


def s2(ind: torch.Tensor) -> torch.Tensor:
    """S2(r) for an indicator [ny, nx]: entry [ry + ny - 1, rx] holds the
    displacement (ry, rx), ry in (-ny, ny), rx in [0, nx) periodic.  FFT with
    zero padding in y, divided by the number of pairs inside the domain."""
    ny, nx = ind.shape
    f = torch.fft.rfft2(torch.nn.functional.pad(ind, (0, 0, 0, ny)))
    corr = torch.fft.irfft2(f.conj() * f, s=(2 * ny, nx))          # sum_x I(x) I(x + r), ry mod 2ny
    corr = torch.cat([corr[ny + 1:], corr[:ny]], dim=0)              # ry = -(ny-1) .. ny-1
    ry = torch.arange(-(ny - 1), ny, device=ind.device, dtype=torch.float64)
    pairs = nx * (ny - ry.abs())
    return corr / pairs[:, None]


def s2_rel_l2(c_pred, phi_pred, c_true, phi_true) -> float:
    return rel_l2(s2(phase_indicator(c_pred, phi_pred)), s2(phase_indicator(c_true, phi_true)))


def radial_average(s: torch.Tensor, rmax: int) -> torch.Tensor:
    """Mean of S2 over |r| in [k, k + 1) for k < rmax (x displacements taken
    as the nearest periodic image)."""
    n2, nx = s.shape
    ny = (n2 + 1) // 2
    ry = torch.arange(-(ny - 1), ny, device=s.device, dtype=torch.float64)[:, None]
    rx = torch.arange(nx, device=s.device, dtype=torch.float64)[None, :]
    rx = torch.minimum(rx, nx - rx)
    k = torch.sqrt(ry ** 2 + rx ** 2).floor().long()
    keep = k < rmax
    tot = torch.zeros(rmax, dtype=torch.float64, device=s.device).index_add_(0, k[keep], s[keep])
    cnt = torch.zeros(rmax, dtype=torch.float64, device=s.device).index_add_(0, k[keep], torch.ones_like(s[keep]))
    return tot / cnt.clamp_min(1)
