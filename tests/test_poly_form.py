"""Error bound of the forward's polynomial influence form.

The fused forward replaces phi on each unit interval of the RBF grid by its
degree-7 interpolant at the Chebyshev points of the interval; the interpolant is
linear in the weights.  These checks restate that construction in numpy (FP64)
and pin the bound the library states: summed over all centres, below 8e-7 of the
largest weight for every rho = (step/sigma)^2 the automatic window of 5 admits
([0.914, 1.365)), and below 3e-7 at rho = 1.
"""
import numpy as np
import pytest

DEG = 7
MW = 6          # centres on each side of the interval centre that enter the fit
W = 5           # window of the automatic rule for step = sigma


def chebyshev_nodes():
    n = DEG + 1
    return 0.5 * np.cos((2 * np.arange(n) + 1) * np.pi / (2 * n))


def gauss_coeffs(rho):
    """M[k][m]: monomial coefficients of the interpolant of exp(-rho (d - m)^2 / 2)."""
    x = chebyshev_nodes()
    V = np.vander(x, DEG + 1, increasing=True)
    M = np.zeros((DEG + 1, MW + 1))
    for m in range(MW + 1):
        M[:, m] = np.linalg.solve(V, np.exp(-rho * (x - m) ** 2 / 2))
    return M


def summed_bound(rho, samples=4001):
    """max over d of sum over all centres of |G_m(d) - p_m(d)| (unit weights, worst signs)."""
    M = gauss_coeffs(rho)
    d = np.linspace(-0.5, 0.5, samples)
    tot = np.zeros_like(d)
    for m in range(-40, 41):
        g = np.exp(-rho * (d - m) ** 2 / 2)
        if abs(m) <= MW:
            c = M[:, abs(m)] * ((-1.0) ** np.arange(DEG + 1) if m < 0 else 1.0)
            p = np.polynomial.polynomial.polyval(d, c)
        else:
            p = 0.0
        tot += np.abs(g - p)
    return tot.max()


def automatic_window(rho):
    # smallest w with exp(-rho (w + 1/2)^2 / 2) < 1e-6
    return int(np.ceil(np.sqrt(2.0 * 13.82 / rho) - 0.5))


@pytest.mark.parametrize("rho", [0.915, 1.0, 1.2, 1.364])
def test_bound_over_the_automatic_window_range(rho):
    assert automatic_window(rho) == W
    assert summed_bound(rho) < 8e-7


def test_bound_at_unit_ratio():
    assert summed_bound(1.0) < 3e-7


def test_window_range_edges():
    # the range of rho for which the automatic window is 5
    assert automatic_window(0.913) == 6 and automatic_window(0.915) == 5
    assert automatic_window(1.364) == 5 and automatic_window(1.366) == 4


def test_linear_form_matches_full_rbf_sum():
    """phi on an interval from the weights through M equals the full 63-term sum
    within the bound (random weights, every interval the form covers)."""
    rng = np.random.default_rng(1702)
    nrbf, rho = 63, 1.0
    M = gauss_coeffs(rho)
    w = rng.normal(0.0, 0.1, nrbf)
    wp = np.zeros(nrbf + 2 * (W + MW))
    wp[W + MW:W + MW + nrbf] = w
    d = np.linspace(-0.5, 0.5, 101)
    j = np.arange(nrbf)
    worst = 0.0
    for j0 in range(-W, nrbf + W):
        wc = lambda m: wp[j0 + m + W + MW]
        c = np.zeros(DEG + 1)
        for k in range(DEG + 1):
            c[k] = M[k, 0] * wc(0) if k % 2 == 0 else 0.0
            for m in range(1, MW + 1):
                c[k] += M[k, m] * (wc(m) + (-1) ** k * wc(-m))
        approx = np.polynomial.polynomial.polyval(d, c)
        exact = (w[None, :] * np.exp(-rho * ((j0 + d)[:, None] - j[None, :]) ** 2 / 2)).sum(1)
        worst = max(worst, np.abs(approx - exact).max() / np.abs(w).max())
    assert worst < 3e-7


def test_odd_coefficients_vanish_at_the_centre():
    # the Gaussian centred on the interval is even in d
    M = gauss_coeffs(1.0)
    assert np.all(np.abs(M[1::2, 0]) < 1e-12)


def deriv_coeffs(rho):
    """Md[k][m]: monomial coefficients of the interpolant of -rho (d - m) exp(-rho (d - m)^2 / 2)."""
    x = chebyshev_nodes()
    V = np.vander(x, DEG + 1, increasing=True)
    M = np.zeros((DEG + 1, MW + 1))
    for m in range(MW + 1):
        M[:, m] = np.linalg.solve(V, -rho * (x - m) * np.exp(-rho * (x - m) ** 2 / 2))
    return M


@pytest.mark.parametrize("rho", [0.915, 1.0, 1.2, 1.364])
def test_derivative_form_bound(rho):
    """The input-gradient mode's interpolant of d phi / ds: summed error over all
    centres below 1e-6 of the largest weight over the automatic-window range
    (and below 2e-7 at rho = 1)."""
    M = deriv_coeffs(rho)
    d = np.linspace(-0.5, 0.5, 4001)
    tot = np.zeros_like(d)
    for m in range(-40, 41):
        h = -rho * (d - m) * np.exp(-rho * (d - m) ** 2 / 2)
        if abs(m) <= MW:
            c = M[:, abs(m)] * ((-1.0) ** (np.arange(DEG + 1) + 1) if m < 0 else 1.0)
            p = np.polynomial.polynomial.polyval(d, c)
        else:
            p = 0.0
        tot += np.abs(h - p)
    assert tot.max() < (2e-7 if rho == 1.0 else 1e-6)


def test_derivative_form_matches_full_sum():
    """d phi / ds on an interval from the weights (odd part as sums, even part as
    differences) equals the full sum's derivative within the bound."""
    rng = np.random.default_rng(7482)
    nrbf, rho = 63, 1.0
    M = deriv_coeffs(rho)
    assert np.all(np.abs(M[0::2, 0]) < 1e-12)  # the centred term is odd in d
    w = rng.normal(0.0, 0.1, nrbf)
    wp = np.zeros(nrbf + 2 * (W + MW))
    wp[W + MW:W + MW + nrbf] = w
    d = np.linspace(-0.5, 0.5, 101)
    j = np.arange(nrbf)
    worst = 0.0
    for j0 in range(-W, nrbf + W):
        wc = lambda m: wp[j0 + m + W + MW]
        c = np.zeros(DEG + 1)
        for k in range(DEG + 1):
            c[k] = M[k, 0] * wc(0) if k % 2 == 1 else 0.0
            for m in range(1, MW + 1):
                c[k] += M[k, m] * (wc(m) - (-1) ** k * wc(-m))
        approx = np.polynomial.polynomial.polyval(d, c)
        s = (j0 + d)[:, None] - j[None, :]
        exact = (w[None, :] * (-rho * s) * np.exp(-rho * s ** 2 / 2)).sum(1)
        worst = max(worst, np.abs(approx - exact).max() / np.abs(w).max())
    assert worst < 2e-7
