"""Write c3_backward.npz: the FP64 oracle's gradients on the full
forward + backward workload (16 crops of 180 x 180, L = 1, 8 stages of 48 7x7
filters, loss mean((u_T - u_gt)^2), so dl/du_T = 2 (u_T - u_gt) / n).

The oracle's backward on this workload takes minutes of CPU time, too long to
repeat inside a GPU test, so its outputs are stored: dK, dW, dlambda (FP64) and
dl/du_0 (rounded to FP32, 2 MB).  Inputs come from the shared seeded
generators; the loss gradient and every stored value come only from
``oracle``.  The GPU test recomputes the oracle's forward (seconds) and checks
the digests stored here before it uses the file, so a change of the inputs or
of the oracle's forward invalidates it loudly.

The images are independent, so the oracle runs one image per worker thread
(one OpenMP thread each) and the gradients are summed in image order.

Run:  python tests/golden/make_c3_reference.py
"""
import hashlib
import os
import sys
from concurrent.futures import ThreadPoolExecutor

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_1702_07482_amd import synth  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "c3_backward.npz")
N, H, W = 16, 180, 180


def case():
    """(model, u_gt [N][H][W], f [N][H][W]) of the workload."""
    m = synth.config_model(3)
    pairs = [synth.make_pair(H, W, 1, config_id=3, index=60 + n) for n in range(N)]
    return m, np.stack([p[0] for p in pairs]), np.stack([p[1] for p in pairs])


def digest(*arrays) -> str:
    h = hashlib.sha256()
    for a in arrays:
        h.update(np.ascontiguousarray(a).tobytes())
    return h.hexdigest()


def model_digest(m) -> str:
    return digest(m["filters"], m["rbf_w"], m["lam"],
                  np.array([m["mu0"], m["step"], m["sigma"]], dtype=np.float64))


def oracle_forward(f, m, workers):
    """u_T and the states u_0..u_T of every image, one image per worker."""
    with ThreadPoolExecutor(workers) as ex:
        res = list(ex.map(lambda n: oracle.forward(f[n], m, want_states=True, nthreads=1),
                          range(f.shape[0])))
    uT = np.stack([r[0] for r in res])
    states = np.stack([r[1] for r in res], axis=1)
    return uT, states


def loss_gradient(uT, u):
    """dl/du_T of mean((u_T - u_gt)^2), rounded to FP32 (the GPU receives FP32)."""
    return ((uT - u) * (2.0 / u.size)).astype(np.float32).astype(np.float64)


def main():
    workers = min(16, os.cpu_count() or 1)
    m, u, f = case()
    uT, states = oracle_forward(f, m, workers)
    gT = loss_gradient(uT, u)

    def one(n):
        return oracle.backward(f[n], m, states[:, n], gT[n], nthreads=1)

    with ThreadPoolExecutor(workers) as ex:
        res = list(ex.map(one, range(N)))
    dK = np.zeros_like(res[0][0])
    dW = np.zeros_like(res[0][1])
    dl = np.zeros_like(res[0][2])
    for r in res:  # image order
        dK += r[0]
        dW += r[1]
        dl += r[2]
    g0 = np.stack([r[3] for r in res]).astype(np.float32)
    np.savez_compressed(OUT, dK=dK, dW=dW, dlam=dl, g0=g0,
                        digest_f=digest(f), digest_u=digest(u), digest_model=model_digest(m),
                        digest_uT=digest(uT),
                        source="FP64 oracle (oracle/tnrd_oracle.c) on the seeded 16 x 180 x 180 "
                               "workload; not paper values")
    print("wrote", OUT)


if __name__ == "__main__":
    main()
