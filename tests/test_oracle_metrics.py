"""Pins of the FP64 quality indexes in oracle/metrics.py (Sec. 4) against closed
forms, an independent window implementation (scipy) and exact identities."""
import math

import numpy as np
import pytest
from scipy import ndimage, signal

from oracle import metrics as om


def _img(seed, H=40, W=33, lo=1.0, hi=255.0):
    return np.random.default_rng(seed).uniform(lo, hi, size=(H, W))


def test_psnr_closed_form():
    ref = _img(1)
    assert om.psnr(ref + 3.0, ref) == pytest.approx(10 * math.log10(255.0 ** 2 / 9.0), rel=1e-12)


def test_gaussian_window_is_the_standard_one():
    w = om.gaussian_window(11, 1.5)
    g = signal.windows.gaussian(11, 1.5)
    assert w.sum() == pytest.approx(1.0, abs=1e-15)
    np.testing.assert_allclose(w, np.outer(g, g) / np.outer(g, g).sum(), rtol=1e-12)


def test_ssim_identity_and_constants():
    x = _img(2)
    np.testing.assert_allclose(om.ssim_map(x, x), 1.0, rtol=1e-12)
    a, b = np.full((20, 20), 80.0), np.full((20, 20), 120.0)
    c1 = (0.01 * 255) ** 2
    np.testing.assert_allclose(om.ssim_map(a, b), (2 * 80 * 120 + c1) / (80 ** 2 + 120 ** 2 + c1),
                               rtol=1e-12)


def test_ssim_shifted_image_against_scipy_local_means():
    """y = x + c: the structure term is 1 and the luminance term follows from the
    local means, computed here with scipy's correlate (an independent window sum)."""
    x = _img(3)
    c = 17.0
    w = om.gaussian_window()
    mx = ndimage.correlate(x, w, mode="constant")[5:-5, 5:-5]
    c1 = (0.01 * 255) ** 2
    want = (2 * mx * (mx + c) + c1) / (mx * mx + (mx + c) ** 2 + c1)
    np.testing.assert_allclose(om.ssim_map(x + c, x), want, rtol=1e-10)


def test_laplacian_of_a_quadratic():
    y, x = np.mgrid[0:12, 0:9].astype(np.float64)
    np.testing.assert_allclose(om.laplacian(x * x + 3 * y * y + 2 * x - y), 8.0, rtol=1e-12)


def test_edge_correlation_identities():
    x = _img(4)
    assert om.edge_correlation(x, x) == pytest.approx(1.0, abs=1e-12)
    assert om.edge_correlation(-x, x) == pytest.approx(-1.0, abs=1e-12)
    assert om.edge_correlation(2.5 * x + 40.0, x) == pytest.approx(1.0, abs=1e-12)


def test_ratio_image_is_the_noise_for_a_perfect_despeckler():
    rng = np.random.default_rng(5)
    u = _img(6, 300, 300)
    for L in (1, 4):
        n = rng.gamma(L, 1.0 / L, size=u.shape)
        m, v = om.ratio_image_stats(u * n, u)
        assert m == pytest.approx(n.mean(), rel=1e-12)
        assert v == pytest.approx(n.var(), rel=1e-10)
        # and the noise law: mean 1, variance 1/L (90 000 samples)
        assert m == pytest.approx(1.0, abs=0.02)
        assert v == pytest.approx(1.0 / L, rel=0.05)


def test_coefficient_of_variation_closed_forms():
    assert om.coeff_variation(np.full((8, 8), 7.0)) == 0.0
    a = np.where(np.arange(64).reshape(8, 8) % 2 == 0, 10.0, 30.0)
    assert om.coeff_variation(a) == pytest.approx(20.0 / 40.0, rel=1e-12)


def test_package_metrics_match_oracle_on_cpu_tensors():
    """The package's torch implementation (any device) against the FP64 definitions."""
    torch = pytest.importorskip("torch")
    from paper_1702_07482_amd import metrics as pm
    x, y = _img(7, 50, 45), _img(8, 50, 45)
    tx, ty = torch.from_numpy(x), torch.from_numpy(y)
    assert pm.psnr(tx, ty) == pytest.approx(om.psnr(x, y), rel=1e-12)
    assert pm.mssim(tx, ty) == pytest.approx(om.mssim(x, y), rel=1e-10)
    assert pm.edge_correlation(tx, ty) == pytest.approx(om.edge_correlation(x, y), rel=1e-10)
    assert pm.ratio_image_stats(tx, ty)[0] == pytest.approx(om.ratio_image_stats(x, y)[0], rel=1e-12)
    assert pm.ratio_image_stats(tx, ty)[1] == pytest.approx(om.ratio_image_stats(x, y)[1], rel=1e-10)
    assert pm.coeff_variation(tx) == pytest.approx(om.coeff_variation(x), rel=1e-12)


def test_ideal_ratio_variance_amplitude():
    """Unit-mean amplitude speckle: (4/pi - 1) at L = 1; sampled variance at L = 3."""
    from paper_1702_07482_amd import metrics as pm
    assert pm.ideal_ratio_variance(1, amplitude=True) == pytest.approx(4 / math.pi - 1, rel=1e-12)
    g = np.sqrt(np.random.default_rng(9).gamma(3, 1 / 3, size=400_000))
    assert pm.ideal_ratio_variance(3, amplitude=True) == pytest.approx((g / g.mean()).var(), rel=0.02)
