"""Pins of the oracle's projected variant (Sec. 3.1, eq. diffusion_backP) and
of the full input gradient dl/df.

The projected stage is ut = u - (sum_i K_i^T phi_i(K_i u) + psi(u)),
u_next = max(ut, c), with psi(u) = (lambda/u)(1 - f^2/u^2) as printed in
eq. diffusion_backP.  Nothing here re-types the oracle's formulas: psi is
checked against the gradient of the data term it descends (eq. dataterm1,
see below), the stage against an energy built from scipy convolutions and erf,
the special cases against closed forms, and every gradient against central
differences of the oracle's own forward (with a Richardson check).

psi is the derivative of (lambda/2) <2 log u + f^2/u^2, 1>, i.e. of the data
term of eq. dataterm1 with lambda halved: eq. diffusion_backP prints the
reaction with that factor, and the oracle follows the equation as printed.
"""
import math

import numpy as np
import pytest
import scipy.ndimage as ndi
from scipy.special import erf

import oracle
from paper_1702_07482_amd import synth


def _rng(i=0):
    return np.random.default_rng(2000 + i)


def _proj(m, c=1.0):
    m = {k: (np.array(v, dtype=np.float64) if isinstance(v, np.ndarray) else v) for k, v in m.items()}
    m["reaction"] = "projected"
    m["proj_c"] = c
    return m


def _tiny(T=2, Nk=2, ks=3, seed=0, w_std=0.1, lam=(0.5, 2.0)):
    g = _rng(50 + seed)
    m = synth.make_model(T, Nk, ks, g, w_std=w_std)
    m["lam"] = g.uniform(*lam, T)
    return m


def _rho(z, w, mu0, step, sigma):
    """Penalty with rho' = phi: sum_j w_j sigma sqrt(pi/2) erf((z - mu_j)/(sigma sqrt 2))."""
    mu = mu0 + step * np.arange(w.size)
    zz = np.asarray(z, dtype=np.float64)[..., None]
    return (w * sigma * math.sqrt(math.pi / 2) * erf((zz - mu) / (sigma * math.sqrt(2)))).sum(-1)


# ---------------------------------------------------------------- reaction
@pytest.mark.parametrize("lam", [0.3, 1.0, 4.0])
def test_psi_is_gradient_of_the_data_term(lam):
    """psi(u) = d/du (lam/2)(2 log u + f^2/u^2), by central differences of that term."""
    g = _rng(1)
    u = g.uniform(0.4, 300.0, 200)
    f = g.uniform(0.4, 300.0, 200)
    h = 1e-6 * u

    def D(uu):
        return 0.5 * lam * (2.0 * np.log(uu) + f ** 2 / uu ** 2)

    fd = (D(u + h) - D(u - h)) / (2 * h)
    np.testing.assert_allclose(oracle.psi(u, f, lam), fd, rtol=1e-6, atol=1e-12)
    # psi vanishes at u = f: the data term's minimiser
    np.testing.assert_allclose(oracle.psi(f, f, lam), 0.0, atol=1e-14)


def test_psi_partials_match_finite_differences():
    g = _rng(2)
    for _ in range(20):
        u, f, lam = g.uniform(0.5, 50), g.uniform(0.5, 50), g.uniform(0.1, 3)
        du, dlam, df = oracle.psi_partials(u, f, lam)
        h = 1e-6
        fu = (oracle.psi(u * (1 + h), f, lam) - oracle.psi(u * (1 - h), f, lam)) / (2 * u * h)
        fl = (oracle.psi(u, f, lam * (1 + h)) - oracle.psi(u, f, lam * (1 - h))) / (2 * lam * h)
        ff = (oracle.psi(u, f * (1 + h), lam) - oracle.psi(u, f * (1 - h), lam)) / (2 * f * h)
        assert du == pytest.approx(float(fu), rel=1e-6, abs=1e-12)
        assert dlam == pytest.approx(float(fl), rel=1e-6, abs=1e-12)
        assert df == pytest.approx(float(ff), rel=1e-6, abs=1e-12)


def test_prox_df_matches_finite_differences():
    """d prox / df at fixed ut (the prox's explicit dependence on f)."""
    g = _rng(3)
    for _ in range(20):
        ut, f, lam = g.uniform(-50, 200), g.uniform(0.5, 200), g.uniform(0.05, 5)
        h = 1e-6 * f
        fd = (oracle.prox(ut, f + h, lam) - oracle.prox(ut, f - h, lam)) / (2 * h)
        assert oracle.prox_df(ut, f, lam) == pytest.approx(float(fd), rel=1e-6, abs=1e-12)


# ---------------------------------------------------------------- stage
def test_projected_stage_is_energy_gradient_step_then_max():
    """ut_1 = f - grad E_filters(f) - psi(f) with E from scipy convolutions and
    erf (eq. foemodel), psi(f) = 0 at u = f; u_1 = max(ut_1, c)."""
    g = _rng(4)
    H, W = 8, 9
    m = _proj(_tiny(T=1, Nk=2, ks=5, seed=1, w_std=3.0), c=1.0)
    f = g.uniform(0.3, 40, (H, W))
    u1, states, utilde = oracle.forward(f, m, want_states=True, want_utilde=True)
    K, Wt = m["filters"][0], m["rbf_w"][0]

    def energy(uu):
        return sum(_rho(ndi.convolve(uu, K[i], mode="reflect"), Wt[i], -310, 10, 10).sum()
                   for i in range(K.shape[0]))

    h = 1e-3
    grad = np.empty_like(f)
    for idx in np.ndindex(H, W):
        up, um = f.copy(), f.copy()
        up[idx] += h
        um[idx] -= h
        grad[idx] = (energy(up) - energy(um)) / (2 * h)
    np.testing.assert_allclose(utilde[0], f - grad, rtol=0, atol=1e-7)
    np.testing.assert_array_equal(u1, np.maximum(utilde[0], 1.0))
    assert (utilde[0] < 1.0).any() and (utilde[0] > 1.0).any()  # both branches taken


def test_projected_second_stage_from_pieces():
    """Stage 2 from u_1 uses psi at u_1 (not f): built from the separately
    pinned K, phi, K^T and psi."""
    g = _rng(5)
    f = g.uniform(0.5, 60, (9, 10))
    m = _proj(_tiny(T=2, Nk=2, ks=3, seed=2, w_std=2.0), c=1.0)
    uT, states = oracle.forward(f, m, want_states=True)
    u = states[1]
    xs = sum(oracle.conv_adj(oracle.phi(oracle.conv(u, m["filters"][1, i]), m["rbf_w"][1, i],
                                        -310, 10, 10), m["filters"][1, i]) for i in range(2))
    ut = u - (xs + oracle.psi(u, f, float(m["lam"][1])))
    np.testing.assert_allclose(uT, np.maximum(ut, 1.0), rtol=1e-13, atol=1e-12)


def test_projected_zero_weights_closed_form():
    """Zero RBF weights: psi(f) = 0, so u_1 = max(f, c); below c, psi(c) > 0
    pushes ut under c and the projection holds the pixel at c: u_t = max(f, c)
    for every t >= 1."""
    g = _rng(6)
    f = g.uniform(0.2, 30, (2, 12, 11))
    m = _proj(_tiny(T=4, Nk=2, ks=5, seed=3), c=1.0)
    m["rbf_w"][:] = 0
    _, states = oracle.forward(f, m, want_states=True)
    np.testing.assert_array_equal(states[0], f)
    for t in range(1, 5):
        np.testing.assert_allclose(states[t], np.maximum(f, 1.0), rtol=1e-15, atol=0)


# ---------------------------------------------------------------- gradients
def _loss(f, m, gT):
    return float((oracle.forward(f, m) * gT).sum())


def _fd_param(f, m, gT, which, idx, h):
    mp = {k: (v.copy() if isinstance(v, np.ndarray) else v) for k, v in m.items()}
    mn = {k: (v.copy() if isinstance(v, np.ndarray) else v) for k, v in m.items()}
    mp[which][idx] += h
    mn[which][idx] -= h
    return (_loss(f, mp, gT) - _loss(f, mn, gT)) / (2 * h)


def _kink_margin(f, m):
    """Smallest |ut - c| over all stages and pixels (FD must not cross the kink)."""
    _, ut = oracle.forward(f, m, want_utilde=True)
    return float(np.abs(ut - m["proj_c"]).min())


def test_projected_backward_matches_finite_differences():
    """dK, dW, dlambda of the projected model against central differences,
    error falling ~100x per decade of h, on low-peak inputs where some pixels
    are projected (and none lies within the FD step of the kink)."""
    g = _rng(21)  # a draw whose ut stays >= 0.05 from c at every pixel and stage
    u_gt = g.uniform(0.2, 6.0, (2, 7, 8))
    f = u_gt * g.gamma(1.0, 1.0, u_gt.shape)
    m = _proj(_tiny(T=2, Nk=2, ks=3, seed=5, w_std=2.0), c=1.0)
    f = np.maximum(f, 0.05)
    assert _kink_margin(f, m) > 4e-2
    _, ut = oracle.forward(f, m, want_utilde=True)
    assert (ut < 1.0).any() and (ut > 1.0).any()
    gT = g.standard_normal(f.shape)
    _, states = oracle.forward(f, m, want_states=True)
    dK, dW, dl, _ = oracle.backward(f, m, states, gT)
    picks = [("filters", (0, 1, 0, 2), dK), ("filters", (1, 0, 1, 1), dK),
             ("rbf_w", (0, 0, 31), dW), ("rbf_w", (1, 1, 30), dW), ("rbf_w", (1, 0, 32), dW),
             ("lam", (0,), dl), ("lam", (1,), dl)]
    for which, idx, grad in picks:
        an = grad[idx]
        e1 = abs(_fd_param(f, m, gT, which, idx, 1e-3) - an)
        e2 = abs(_fd_param(f, m, gT, which, idx, 1e-4) - an)
        tol = 1e-7 * max(1.0, abs(an))
        assert e2 <= max(tol, 2e-2 * e1 + 1e-9), (which, idx, an, e1, e2)
        assert e2 <= 1e-5 * max(1.0, abs(an)), (which, idx, an, e2)


def test_projected_zero_weight_gradients_closed_form():
    """Zero weights, f > c: u_t = f, m = 1, so dK = 0, dlambda = 0 (psi_lambda(f) = 0)
    and g_{t-1} = g_t (1 - psi_u(f)) with psi_u(f) = 2 lambda / f^2."""
    g = _rng(8)
    f = g.uniform(2.0, 40, (1, 9, 10))
    m = _proj(_tiny(T=3, Nk=2, ks=5, seed=7), c=1.0)
    m["rbf_w"][:] = 0
    gT = g.standard_normal(f.shape)
    _, states = oracle.forward(f, m, want_states=True)
    dK, dW, dl, g0 = oracle.backward(f, m, states, gT)
    assert np.abs(dK).max() <= 1e-12 and np.abs(dl).max() <= 1e-12
    ref = gT[0].copy()
    for t in range(2, -1, -1):
        ref = ref * (1 - 2 * m["lam"][t] / f[0] ** 2)
    np.testing.assert_allclose(g0[0], ref, rtol=1e-12)


@pytest.mark.parametrize("reaction", ["prox", "projected"])
def test_full_input_gradient_matches_finite_differences(reaction):
    """dl/df in full (u_0 = f plus every stage's explicit f) against central
    differences of <gT, u_T(f)> in a random direction, h = 1e-3 and 1e-4."""
    g = _rng(10)  # (projected) a draw whose ut stays >= 0.06 from c
    if reaction == "prox":
        f = g.uniform(5, 250, (2, 7, 6))
        m = _tiny(T=2, Nk=2, ks=3, seed=6, w_std=2.0)
        m = {k: (np.array(v, dtype=np.float64) if isinstance(v, np.ndarray) else v) for k, v in m.items()}
    else:
        f = np.maximum(g.uniform(0.2, 6.0, (2, 7, 6)) * g.gamma(1.0, 1.0, (2, 7, 6)), 0.05)
        m = _proj(_tiny(T=2, Nk=2, ks=3, seed=6, w_std=2.0), c=1.0)
        assert _kink_margin(f, m) > 4e-2
    gT = g.standard_normal(f.shape)
    d = g.standard_normal(f.shape)
    _, states = oracle.forward(f, m, want_states=True)
    _, _, _, g0, gf = oracle.backward(f, m, states, gT, want_df=True)
    an = float((gf * d).sum())
    errs = []
    for h in (1e-3, 1e-4):
        fd = (_loss(f + h * d, m, gT) - _loss(f - h * d, m, gT)) / (2 * h)
        errs.append(abs(fd - an))
    assert errs[1] <= max(1e-8 * max(1.0, abs(an)), 2e-2 * errs[0] + 1e-9), (an, errs)
    assert errs[1] <= 1e-5 * max(1.0, abs(an)), (an, errs)
    # the full gradient differs from the diffusion-chain-only g0 by the explicit terms
    assert np.abs(gf - g0).max() > 1e-6 * np.abs(gf).max()


def test_full_input_gradient_zero_weights_prox_closed_form():
    """Zero weights, prox model: u_t = f for all t, so u_T(f) = f and dl/df = gT."""
    g = _rng(10)
    f = g.uniform(1, 255, (1, 8, 9))
    m = _tiny(T=3, Nk=2, ks=5, seed=8)
    m = {k: (np.array(v, dtype=np.float64) if isinstance(v, np.ndarray) else v) for k, v in m.items()}
    m["rbf_w"][:] = 0
    gT = g.standard_normal(f.shape)
    _, states = oracle.forward(f, m, want_states=True)
    *_, gf = oracle.backward(f, m, states, gT, want_df=True)
    np.testing.assert_allclose(gf, gT, rtol=1e-12, atol=1e-14)


# ---------------------------------------------------------------- quadratic data term
# The TNRD framework's Gaussian-denoising reaction (Sec. 2.2.1, eq. diffusion with
# G = 0, D = (lambda/2) ||u - f||^2, psi = lambda (u - f)).
def _l2(m):
    m = {k: (np.array(v, dtype=np.float64) if isinstance(v, np.ndarray) else v) for k, v in m.items()}
    m["reaction"] = "l2"
    return m


def test_l2_stage_is_gradient_step_on_full_energy():
    """Stage 2 (from u_1, where the data term's gradient is not zero) is
    u_1 - grad [E_filters + (lam/2)||u - f||^2](u_1), the gradient by central
    differences of an energy built from scipy convolutions and erf."""
    g = _rng(11)
    H, W = 8, 7
    m = _l2(_tiny(T=2, Nk=2, ks=5, seed=9, w_std=3.0))
    f = g.uniform(0, 255, (H, W))
    lam = float(m["lam"][1])
    K, Wt = m["filters"][1], m["rbf_w"][1]

    def energy(uu):
        return (sum(_rho(ndi.convolve(uu, K[i], mode="reflect"), Wt[i], -310, 10, 10).sum()
                    for i in range(K.shape[0])) + 0.5 * lam * ((uu - f) ** 2).sum())

    uT, states = oracle.forward(f, m, want_states=True)
    u1 = states[1]
    assert np.abs(u1 - f).max() > 1e-3  # stage 1 moved away from f
    h = 1e-3
    grad = np.empty_like(f)
    for idx in np.ndindex(H, W):
        up, um = u1.copy(), u1.copy()
        up[idx] += h
        um[idx] -= h
        grad[idx] = (energy(up) - energy(um)) / (2 * h)
    np.testing.assert_allclose(uT, u1 - grad, rtol=0, atol=1e-6)


def test_l2_zero_weights_closed_form():
    """Zero weights from u_0 = f: psi(f) = 0, so u_t = f; the backward gives
    dlambda = 0, g_{t-1} = (1 - lam_t) g_t and dl/df = g_0 + sum_t lam_t g_t."""
    g = _rng(12)
    f = g.uniform(0, 255, (1, 9, 8))
    m = _l2(_tiny(T=3, Nk=2, ks=3, seed=10, lam=(0.05, 0.4)))
    m["rbf_w"][:] = 0
    gT = g.standard_normal(f.shape)
    _, states = oracle.forward(f, m, want_states=True)
    for t in range(4):
        np.testing.assert_array_equal(states[t], f)
    dK, dW, dl, g0, gf = oracle.backward(f, m, states, gT, want_df=True)
    assert np.abs(dl).max() == 0.0 and np.abs(dK).max() == 0.0
    gt, acc = gT[0].copy(), np.zeros_like(gT[0])
    for t in range(2, -1, -1):
        acc += m["lam"][t] * gt
        gt = (1 - m["lam"][t]) * gt
    np.testing.assert_allclose(g0[0], gt, rtol=1e-13)
    np.testing.assert_allclose(gf[0], gt + acc, rtol=1e-13)


def test_l2_backward_matches_finite_differences():
    g = _rng(13)
    f = g.uniform(0, 255, (2, 7, 8))
    m = _l2(_tiny(T=2, Nk=2, ks=3, seed=11, w_std=2.0, lam=(0.05, 0.5)))
    gT = g.standard_normal(f.shape)
    d = g.standard_normal(f.shape)
    _, states = oracle.forward(f, m, want_states=True)
    dK, dW, dl, _, gf = oracle.backward(f, m, states, gT, want_df=True)
    for which, idx, grad in [("filters", (0, 1, 0, 2), dK), ("rbf_w", (1, 1, 30), dW),
                             ("lam", (0,), dl), ("lam", (1,), dl)]:
        an = grad[idx]
        e1 = abs(_fd_param(f, m, gT, which, idx, 1e-3) - an)
        e2 = abs(_fd_param(f, m, gT, which, idx, 1e-4) - an)
        assert e2 <= max(1e-7 * max(1.0, abs(an)), 2e-2 * e1 + 1e-9), (which, idx, an, e1, e2)
    an = float((gf * d).sum())
    fd = (_loss(f + 1e-4 * d, m, gT) - _loss(f - 1e-4 * d, m, gT)) / 2e-4
    assert abs(fd - an) <= 1e-6 * max(1.0, abs(an))
