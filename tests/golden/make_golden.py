"""Write oracle_tiny.json: a small seeded forward/backward run of the FP64 oracle.

The paper prints no worked example of the filter (its tables need trained
weights and image sets that are not available), so these values are not the
paper's: they are the oracle's own output on a tiny seeded case, kept as a
regression guard so that any later change to the oracle's arithmetic shows up.
Inputs come from the shared seeded generators; outputs only from ``oracle``.

Run:  python tests/golden/make_golden.py
"""
import json
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_1702_07482_amd import synth  # noqa: E402


def case():
    u, f = synth.make_pair(9, 10, 1, config_id=91)
    m = synth.make_model(2, 3, 5, synth.rng_for(91, 2), w_std=1.0)
    m["lam"] = np.array([0.75, 1.5], dtype=np.float32)
    return u, f, m


def main():
    u, f, m = case()
    uT, states = oracle.forward(f, m, want_states=True)
    gT = uT - u
    dK, dW, dl, g0 = oracle.backward(f, m, states, gT)
    out = {
        "source": "FP64 oracle (oracle/tnrd_oracle.c) on synth case config_id=91; not paper values",
        "uT": uT.tolist(), "dK": dK.tolist(), "dW": dW.tolist(), "dlam": dl.tolist(),
        "g0": g0.tolist(),
    }
    with open(os.path.join(os.path.dirname(__file__), "oracle_tiny.json"), "w") as fh:
        json.dump(out, fh)


if __name__ == "__main__":
    main()
