"""Training-side pins on the FP64 oracle: the loss of eq. learning and the
beta = log(lambda) reparametrisation of eq. derv5 (dl/dbeta = lambda dl/dlambda),
checked by central differences in beta."""
import numpy as np
import pytest

import oracle
from paper_1702_07482_amd import synth


def _setup():
    g = np.random.default_rng(77)
    m = synth.make_model(2, 6, 5, g, w_std=0.05)
    m["lam"] = np.array([0.7, 1.6])
    u, f = synth.make_pair(18, 16, 2, config_id=1, index=3)
    return m, u, f


def _loss(m, f, u):
    uT = oracle.forward(f, m)
    return 0.5 * float(np.sum((uT - u) ** 2))


@pytest.mark.parametrize("t", [0, 1])
def test_beta_gradient_is_lambda_times_lambda_gradient(t):
    m, u, f = _setup()
    uT, st = oracle.forward(f, m, want_states=True)
    _, _, dlam, _ = oracle.backward(f, m, st, uT - u)
    h = 1e-4  # the loss is O(1e4): smaller steps drown in its rounding
    beta = np.log(m["lam"])
    lp, lm = dict(m), dict(m)
    bp, bm = beta.copy(), beta.copy()
    bp[t] += h
    bm[t] -= h
    lp["lam"], lm["lam"] = np.exp(bp), np.exp(bm)
    fd = (_loss(lp, f, u) - _loss(lm, f, u)) / (2 * h)
    assert m["lam"][t] * dlam[t] == pytest.approx(fd, rel=1e-6)
