"""Shared helpers for the GPU parity tests (no filter arithmetic here)."""
import numpy as np

import oracle


def rel_inf(a, b) -> float:
    """||a - b||_inf / ||b||_inf, the per-tensor relative error used as the bar."""
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    den = np.abs(b).max()
    return float(np.abs(a - b).max() / (den if den > 0 else 1.0))


def crop_window(p, n, radius):
    """[lo, hi) of a crop around index p in [0, n) that reproduces the full
    image's values at p: either at least `radius` away from the crop edge, or
    flush with the image border (same reflection there)."""
    lo = max(0, p - radius)
    hi = min(n, p + radius + 1)
    return lo, hi


def oracle_uT_at(f, model, points, radius):
    """u_T at the given (y, x) pixels of a single image f, each computed by the
    oracle on a crop whose edges are either image borders or outside the
    receptive field (radius = T * (ksize - 1))."""
    H, W = f.shape
    out = []
    for (y, x) in points:
        y0, y1 = crop_window(y, H, radius)
        x0, x1 = crop_window(x, W, radius)
        uT = oracle.forward(f[y0:y1, x0:x1], model)
        out.append(uT[y - y0, x - x0])
    return np.array(out)
