"""The oracle still reproduces its stored tiny-case output (regression guard)."""
import json
import os

import numpy as np

import oracle
from tests.golden.make_golden import case

GOLD = os.path.join(os.path.dirname(__file__), "golden", "oracle_tiny.json")


def test_oracle_matches_stored_tiny_case():
    with open(GOLD) as fh:
        ref = json.load(fh)
    u, f, m = case()
    uT, states = oracle.forward(f, m, want_states=True)
    dK, dW, dl, g0 = oracle.backward(f, m, states, uT - u)
    for name, got in [("uT", uT), ("dK", dK), ("dW", dW), ("dlam", dl), ("g0", g0)]:
        np.testing.assert_allclose(got, np.array(ref[name]), rtol=1e-12, atol=1e-12, err_msg=name)
