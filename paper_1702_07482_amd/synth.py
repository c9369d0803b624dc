"""Seeded synthetic inputs shared by the oracle tests, the GPU tests and the bench.

This module draws numbers only; it contains none of the filter's arithmetic.

* Clean images stand in for the paper's 8-bit optical test images (intensities
  between 1 and 255; Sec. 4): a smooth background (plane + one sinusoid) with
  16 painted shapes, half axis-aligned rectangles and half ellipses, each with
  a constant level and a small internal linear ramp, clipped to [1, 255].
* Speckle follows the multiplicative model f = u * n (Sec. 2.1, eq. mul), with
  n ~ Gamma(shape L, scale 1/L) (unit mean).  ``amplitude=True`` instead draws
  n = sqrt(Gamma(L, 1/L)), the Nakagami amplitude law the paper states.
* Models: zero-mean unit-norm Gaussian filters, N(0, 0.1^2) RBF weights,
  lambda = 1 per stage, 63 centres on [-310, 310] with spacing and width 10.
"""
from __future__ import annotations

import numpy as np

SEED_ROOT = (1702, 7482)


def rng_for(config_id: int, stream: int, index: int = 0) -> np.random.Generator:
    """Generator for (config, stream, index); streams: 0 clean, 1 speckle,
    2 model, 3 misc (loss targets, probes)."""
    return np.random.default_rng(np.random.SeedSequence(
        [SEED_ROOT[0], SEED_ROOT[1], int(config_id), int(stream), int(index)]))


def make_clean(H: int, W: int, rng: np.random.Generator, n_shapes: int = 16) -> np.ndarray:
    y, x = np.mgrid[0:H, 0:W].astype(np.float64)
    a0 = rng.uniform(40.0, 200.0)
    a1, a2 = rng.uniform(-40.0, 40.0, size=2)
    a3 = rng.uniform(5.0, 30.0)
    fx, fy = rng.uniform(0.5, 2.0, size=2)
    ph = rng.uniform(0.0, 2.0 * np.pi)
    img = a0 + a1 * x / W + a2 * y / H + a3 * np.sin(2.0 * np.pi * (fx * x / W + fy * y / H) + ph)
    for s in range(n_shapes):
        h = rng.uniform(0.05, 0.40) * H
        w = rng.uniform(0.05, 0.40) * W
        cy = rng.uniform(0.0, H)
        cx = rng.uniform(0.0, W)
        level = rng.uniform(1.0, 255.0)
        gy, gx = rng.uniform(-20.0, 20.0, size=2)
        if s % 2 == 0:
            mask = (np.abs(y - cy) <= h / 2) & (np.abs(x - cx) <= w / 2)
        else:
            mask = ((y - cy) / (h / 2)) ** 2 + ((x - cx) / (w / 2)) ** 2 <= 1.0
        ramp = level + gy * (y - cy) / max(h, 1.0) + gx * (x - cx) / max(w, 1.0)
        img = np.where(mask, ramp, img)
    return np.clip(img, 1.0, 255.0).astype(np.float32)


def speckle(u: np.ndarray, L: int, rng: np.random.Generator, amplitude: bool = False) -> np.ndarray:
    n = rng.gamma(shape=float(L), scale=1.0 / float(L), size=u.shape)
    if amplitude:
        n = np.sqrt(n)
    f = u.astype(np.float64) * n
    # Gamma draws are strictly positive; keep f representable and > 0 in FP32.
    return np.maximum(f, np.finfo(np.float32).tiny).astype(np.float32)


def make_model(T: int, Nk: int, ks: int, rng: np.random.Generator, Nrbf: int = 63,
               mu0: float = -310.0, step: float = 10.0, sigma: float = 10.0,
               lam: float = 1.0, w_std: float = 0.1) -> dict:
    g = rng.standard_normal((T, Nk, ks, ks))
    g = g - g.mean(axis=(2, 3), keepdims=True)
    g = g / np.sqrt((g * g).sum(axis=(2, 3), keepdims=True))
    w = rng.normal(0.0, w_std, size=(T, Nk, Nrbf))
    return {
        "filters": g.astype(np.float32),
        "rbf_w": w.astype(np.float32),
        "lam": np.full((T,), lam, dtype=np.float32),
        "mu0": float(mu0), "step": float(step), "sigma": float(sigma),
        "T": T, "Nk": Nk, "ks": ks, "Nrbf": Nrbf,
    }


def make_gaussian_pair(H: int, W: int, sigma: float, config_id: int, index: int = 0):
    """(clean u_gt, noisy f = u_gt + N(0, sigma^2)) for one image, both FP32 H x W
    (f may leave [0, 255] and take either sign)."""
    u = make_clean(H, W, rng_for(config_id, 0, index))
    n = rng_for(config_id, 1, index).normal(0.0, sigma, size=u.shape)
    return u, (u.astype(np.float64) + n).astype(np.float32)


def make_pair(H: int, W: int, L: int, config_id: int, index: int = 0, amplitude: bool = False,
              peak: float | None = None):
    """(clean u_gt, speckled f) for one image, both FP32 H x W.  With ``peak``
    the clean image is divided by max(u)/peak first (the low-peak images of the
    paper's comparison of the projected model, peaks 0.5 to 255)."""
    u = make_clean(H, W, rng_for(config_id, 0, index))
    if peak is not None:
        u = (u.astype(np.float64) * (peak / float(u.max()))).astype(np.float32)
    f = speckle(u, L, rng_for(config_id, 1, index), amplitude=amplitude)
    return u, f


# The five workloads (shapes and model sizes).  ``sizes`` lists H x W per image.
CONFIGS = {
    1: dict(name="c1 plain forward 1x128x128, L=1, 5 stages x 24 5x5", T=5, Nk=24, ks=5,
            sizes=[(128, 128)], looks=[1]),
    2: dict(name="c2 plain forward 1x512x512, L=1 (and 4), 8 stages x 48 7x7", T=8, Nk=48, ks=7,
            sizes=[(512, 512)], looks=[1]),
    3: dict(name="c3 forward+backward 16x180x180, L=1, 8 stages x 48 7x7", T=8, Nk=48, ks=7,
            sizes=[(180, 180)] * 16, looks=[1] * 16),
    4: dict(name="c4 batched uneven forward, 64 images, 8 stages x 48 7x7", T=8, Nk=48, ks=7,
            sizes=None, looks=None),
    5: dict(name="c5 mixed precision 8x2048x2048, L=1, 8 stages x 48 7x7", T=8, Nk=48, ks=7,
            sizes=[(2048, 2048)] * 8, looks=[1] * 8),
    # the paper's comparison of the projected model: 5 stages of 5x5 filters, L = 1
    6: dict(name="projected variant 1x128x128, L=1, 5 stages x 24 5x5, c = 1", T=5, Nk=24, ks=5,
            sizes=[(128, 128)], looks=[1], reaction="projected"),
    # the framework's Gaussian-denoising reaction: 5 stages of 48 7x7 filters, noise sigma 25
    7: dict(name="quadratic data term (Gaussian denoising), 5 stages x 48 7x7, lambda = 0.1", T=5,
            Nk=48, ks=7, sizes=[(512, 512)], looks=[1], reaction="l2", lam=0.1),
}

C4_SIZES = [(256, 256), (384, 512), (512, 512), (1024, 768)]
C4_LOOKS = [1, 2, 4, 8]


def c4_batch(n_images: int = 64):
    """Sizes and look numbers for the uneven batch, drawn uniformly."""
    rng = rng_for(4, 3, 0)
    si = rng.integers(0, len(C4_SIZES), size=n_images)
    li = rng.integers(0, len(C4_LOOKS), size=n_images)
    return [C4_SIZES[i] for i in si], [C4_LOOKS[i] for i in li]


def config_model(config_id: int, look: int = 0) -> dict:
    c = CONFIGS[config_id]
    m = make_model(c["T"], c["Nk"], c["ks"], rng_for(config_id, 2, look), lam=c.get("lam", 1.0))
    if c.get("reaction", "prox") != "prox":
        m["reaction"] = c["reaction"]
        m["proj_c"] = 1.0
    return m
