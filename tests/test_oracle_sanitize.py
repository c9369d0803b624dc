"""The FP64 oracle built with AddressSanitizer and UndefinedBehaviorSanitizer
(tests/oracle_sanitize.c drives it): forward with every state, backward with
dl/df, K and K^T, for the three reactions, filter sizes 3, 5 and 7, images as
small as the filter (where the reflection covers all but the centre) and
uneven shapes.  Every run must end without a sanitizer report, and its
outputs must equal those of the regular oracle build on the same case."""
import os
import shutil
import subprocess

import numpy as np
import pytest

import oracle

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
DRIVER = os.path.join(ROOT, "tests", "oracle_sanitize.c")
SRC = os.path.join(ROOT, "oracle", "tnrd_oracle.c")

pytestmark = pytest.mark.skipif(shutil.which("gcc") is None, reason="needs gcc")


@pytest.fixture(scope="module")
def driver(tmp_path_factory):
    exe = str(tmp_path_factory.mktemp("san") / "oracle_sanitize")
    subprocess.check_call(["gcc", "-std=c99", "-O1", "-g", "-fno-omit-frame-pointer",
                           "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
                           DRIVER, SRC, "-o", exe, "-lm"])
    return exe


# (reaction, ks, N, H, W, T, Nk, Nrbf)
CASES = [("prox", 3, 2, 3, 3, 2, 4, 7), ("prox", 5, 1, 9, 13, 3, 6, 11), ("prox", 7, 2, 7, 10, 2, 5, 9),
         ("projected", 5, 2, 11, 6, 2, 4, 8), ("l2", 7, 1, 8, 7, 3, 3, 10), ("l2", 3, 1, 17, 4, 2, 8, 5)]


def _model(rng, reaction, ks, T, Nk, Nrbf):
    filt = rng.standard_normal((T, Nk, ks, ks))
    filt -= filt.mean(axis=(2, 3), keepdims=True)
    filt /= np.linalg.norm(filt.reshape(T, Nk, -1), axis=2)[:, :, None, None]
    return {"filters": filt, "rbf_w": 0.1 * rng.standard_normal((T, Nk, Nrbf)),
            "lam": rng.uniform(0.5, 2.0, T), "mu0": -1.0, "step": 2.0 / (Nrbf - 1), "sigma": 0.15,
            "reaction": reaction, "proj_c": 0.2}


@pytest.mark.parametrize("case", CASES, ids=[f"{c[0]}-k{c[1]}-{c[3]}x{c[4]}" for c in CASES])
def test_oracle_under_sanitizers(driver, tmp_path, case):
    reaction, ks, N, H, W, T, Nk, Nrbf = case
    rng = np.random.default_rng(ks * 1000 + H * 10 + W)
    m = _model(rng, reaction, ks, T, Nk, Nrbf)
    f = rng.uniform(0.5, 1.5, (N, H, W))
    gT = rng.standard_normal((N, H, W))
    cin, cout = tmp_path / "case.bin", tmp_path / "out.bin"
    with open(cin, "wb") as fp:
        fp.write(np.array([oracle.REACTIONS[reaction], ks, N, H, W, T, Nk, Nrbf], np.int32).tobytes())
        fp.write(np.array([m["mu0"], m["step"], m["sigma"], m["proj_c"]], np.float64).tobytes())
        for a in (f, m["filters"], m["rbf_w"], m["lam"], gT):
            fp.write(np.ascontiguousarray(a, np.float64).tobytes())
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0:exitcode=66",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1:exitcode=67")
    r = subprocess.run([driver, str(cin), str(cout)], capture_output=True, text=True, timeout=120, env=env)
    assert r.returncode == 0 and "runtime error" not in r.stderr, r.stderr[-4000:]
    got = np.fromfile(cout, np.float64)

    uT, states, utilde = oracle.forward(f, m, want_states=True, want_utilde=True, nthreads=1)
    dK, dW, dlam, g0, gf = oracle.backward(f, m, states, gT, nthreads=1, want_df=True)
    want = [uT, states, utilde, dK, dW, dlam, g0, gf]
    sizes = [a.size for a in want]
    parts = np.split(got[:sum(sizes)], np.cumsum(sizes)[:-1])
    for name, a, b in zip(["uT", "states", "utilde", "dK", "dW", "dlam", "g0", "gf"], parts, want):
        np.testing.assert_allclose(a, b.ravel(), rtol=1e-13, atol=1e-13, err_msg=name)
    rest = got[sum(sizes):]
    assert rest.size == 2 * H * W
    np.testing.assert_allclose(rest[:H * W], oracle.conv(f[0], m["filters"][0, 0]).ravel(),
                               rtol=1e-13, atol=1e-13)
    np.testing.assert_allclose(rest[H * W:], oracle.conv_adj(gT[0], m["filters"][0, 0]).ravel(),
                               rtol=1e-13, atol=1e-13)
    # K^T is the adjoint of K on this image: <K u, v> = <u, K^T v>
    lhs = float(rest[:H * W] @ gT[0].ravel())
    rhs = float(f[0].ravel() @ rest[H * W:])
    assert abs(lhs - rhs) <= 1e-12 * max(1.0, abs(lhs))
