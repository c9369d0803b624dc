"""Despeckling quality indexes (Sec. 4), on the device of their inputs.

These evaluate results; they are not part of the filter's hot path.  They take
torch tensors [H][W] (or [N][H][W], averaged over images) on any device and
compute in FP64 there:

  psnr(u, ref, peak)         10 log10(peak^2 / MSE)
  mssim(u, ref, D)           mean SSIM (Wang et al. 2004): 11 x 11 Gaussian window,
                             sigma 1.5, C1 = (0.01 D)^2, C2 = (0.03 D)^2, 'valid' positions
  edge_correlation(u, ref)   correlation of the mean-removed 3 x 3 Laplacians (interior)
  ratio_image_stats(f, u)    (mean, population variance) of RI = f / u
  coeff_variation(u)         std(u) / mean(u)

For an L-look speckle field the ratio image of a perfect despeckler is the
noise itself: RI_M = 1 and RI_V = 1/L for intensity speckle (Gamma(L, 1/L)),
and RI_V = L Gamma(L)^2 / Gamma(L + 1/2)^2 - 1 (about (4/pi - 1)/L) for
amplitude speckle normalised to unit mean.
"""
from __future__ import annotations

import math

import torch
import torch.nn.functional as F


def _batch(a: torch.Tensor) -> torch.Tensor:
    a = a.to(torch.float64)
    return a[None] if a.dim() == 2 else a


def psnr(u: torch.Tensor, ref: torch.Tensor, peak: float = 255.0) -> float:
    u, ref = _batch(u), _batch(ref)
    mse = ((u - ref) ** 2).mean(dim=(1, 2))
    return float((10.0 * torch.log10(peak * peak / mse)).mean())


def _gauss(size: int, sigma: float, device) -> torch.Tensor:
    c = (size - 1) / 2.0
    g = torch.exp(-((torch.arange(size, dtype=torch.float64, device=device) - c) ** 2) / (2 * sigma * sigma))
    return g / g.sum()


def ssim_map(u: torch.Tensor, ref: torch.Tensor, dynamic_range: float = 255.0, size: int = 11,
             sigma: float = 1.5, k1: float = 0.01, k2: float = 0.03) -> torch.Tensor:
    """[N][H-size+1][W-size+1] SSIM at every window position inside the image."""
    x, y = _batch(ref)[:, None], _batch(u)[:, None]
    g = _gauss(size, sigma, x.device)
    gr, gc = g.view(1, 1, size, 1), g.view(1, 1, 1, size)

    def blur(a):  # separable window: rows, then columns
        return F.conv2d(F.conv2d(a, gr), gc)

    mx, my = blur(x), blur(y)
    vx = blur(x * x) - mx * mx
    vy = blur(y * y) - my * my
    cxy = blur(x * y) - mx * my
    c1, c2 = (k1 * dynamic_range) ** 2, (k2 * dynamic_range) ** 2
    s = ((2 * mx * my + c1) * (2 * cxy + c2)) / ((mx * mx + my * my + c1) * (vx + vy + c2))
    return s[:, 0]


def mssim(u: torch.Tensor, ref: torch.Tensor, dynamic_range: float = 255.0) -> float:
    return float(ssim_map(u, ref, dynamic_range).mean(dim=(1, 2)).mean())


def _laplacian(a: torch.Tensor) -> torch.Tensor:
    return a[:, :-2, 1:-1] + a[:, 2:, 1:-1] + a[:, 1:-1, :-2] + a[:, 1:-1, 2:] - 4.0 * a[:, 1:-1, 1:-1]


def edge_correlation(u: torch.Tensor, ref: torch.Tensor) -> float:
    p, q = _laplacian(_batch(ref)), _laplacian(_batch(u))
    p = p - p.mean(dim=(1, 2), keepdim=True)
    q = q - q.mean(dim=(1, 2), keepdim=True)
    ec = (p * q).sum(dim=(1, 2)) / torch.sqrt((p * p).sum(dim=(1, 2)) * (q * q).sum(dim=(1, 2)))
    return float(ec.mean())


def ratio_image_stats(f: torch.Tensor, u: torch.Tensor):
    """(RI_M, RI_V): mean and population variance of RI = f / u, averaged over images."""
    ri = _batch(f) / _batch(u)
    m = ri.mean(dim=(1, 2))
    v = ((ri - m[:, None, None]) ** 2).mean(dim=(1, 2))
    return float(m.mean()), float(v.mean())


def coeff_variation(u: torch.Tensor) -> float:
    u = _batch(u)
    m = u.mean(dim=(1, 2))
    s = torch.sqrt(((u - m[:, None, None]) ** 2).mean(dim=(1, 2)))
    return float((s / m).mean())


def ideal_ratio_variance(L: int, amplitude: bool = False) -> float:
    """RI_V of a perfect despeckler: the variance of unit-mean L-look speckle."""
    if not amplitude:
        return 1.0 / L
    # n = sqrt(G)/E[sqrt(G)], G ~ Gamma(L, 1/L): E[G] = 1, E[sqrt(G)] = Gamma(L+1/2)/(Gamma(L) sqrt(L))
    e = math.exp(math.lgamma(L + 0.5) - math.lgamma(L)) / math.sqrt(L)
    return 1.0 / (e * e) - 1.0
