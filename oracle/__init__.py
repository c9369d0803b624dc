"""FP64 CPU oracle for the trained reaction-diffusion despeckling filter.

TEST INFRASTRUCTURE ONLY: the tests, the smoke check and the benchmark's
CPU-baseline leg may import this package; the product path never does.

The arithmetic lives in ``tnrd_oracle.c`` (plain C, double precision, OpenMP),
built into ``liboracle.so`` next to this file by :func:`build`.  This module
only marshals numpy arrays into it.  It shares no code with the HIP library.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "tnrd_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None

_D = ctypes.POINTER(ctypes.c_double)


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (FP64, no fast-math, OpenMP)."""
    if force or not os.path.exists(_LIB):
        cmd = ["gcc", "-O2", "-std=c99", "-fopenmp", "-fPIC", "-shared",
               "-o", _LIB + ".tmp", _SRC, "-lm"]
        subprocess.check_call(cmd)
        os.replace(_LIB + ".tmp", _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        lib = ctypes.CDLL(_LIB)
        i, d = ctypes.c_int, ctypes.c_double
        lib.oracle_reflect.argtypes = [i, i]
        lib.oracle_reflect.restype = i
        lib.oracle_max_threads.restype = i
        lib.oracle_conv.argtypes = [_D, i, i, _D, i, _D]
        lib.oracle_conv_adj.argtypes = [_D, i, i, _D, i, _D]
        lib.oracle_rbf.argtypes = [d, i, d, d, d]
        lib.oracle_rbf.restype = d
        lib.oracle_phi.argtypes = [d, _D, i, d, d, d]
        lib.oracle_phi.restype = d
        lib.oracle_dphi.argtypes = [d, _D, i, d, d, d]
        lib.oracle_dphi.restype = d
        lib.oracle_prox.argtypes = [d, d, d]
        lib.oracle_prox.restype = d
        lib.oracle_prox_grad.argtypes = [d, d, d, _D, _D]
        lib.oracle_prox_df.argtypes = [d, d, d]
        lib.oracle_prox_df.restype = d
        lib.oracle_psi.argtypes = [d, d, d]
        lib.oracle_psi.restype = d
        lib.oracle_psi_du.argtypes = [d, d, d]
        lib.oracle_psi_du.restype = d
        lib.oracle_psi_dlam.argtypes = [d, d]
        lib.oracle_psi_dlam.restype = d
        lib.oracle_psi_df.argtypes = [d, d, d]
        lib.oracle_psi_df.restype = d
        lib.oracle_forward.argtypes = [_D, i, i, i, i, i, i, i, d, d, d, _D, _D, _D,
                                       _D, _D, _D, i]
        lib.oracle_forward_ex.argtypes = [_D, i, i, i, i, i, i, i, d, d, d, _D, _D, _D, i, d,
                                          _D, _D, _D, i]
        lib.oracle_stage_ex.argtypes = [_D, _D, i, i, i, i, i, i, i, d, d, d, _D, _D, _D, i, d,
                                        _D, _D, i]
        lib.oracle_backward.argtypes = [_D, i, i, i, i, i, i, i, d, d, d, _D, _D, _D,
                                        _D, _D, _D, _D, _D, _D, i]
        lib.oracle_backward_ex.argtypes = [_D, i, i, i, i, i, i, i, d, d, d, _D, _D, _D, i, d,
                                           _D, _D, _D, _D, _D, _D, _D, i]
        _lib = lib
    return _lib


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(a, dtype=np.float64))


def _p(a: np.ndarray | None):
    if a is None:
        return ctypes.cast(None, _D)
    return a.ctypes.data_as(_D)


def max_threads() -> int:
    return int(_load().oracle_max_threads())


def reflect(q: int, n: int) -> int:
    return int(_load().oracle_reflect(int(q), int(n)))


def conv(u, k) -> np.ndarray:
    """z = K u for one H x W image and one odd ks x ks kernel (true convolution,
    half-sample symmetric extension)."""
    u, k = _f64(u), _f64(k)
    H, W = u.shape
    z = np.empty_like(u)
    _load().oracle_conv(_p(u), H, W, _p(k), k.shape[0], _p(z))
    return z


def conv_adj(v, k) -> np.ndarray:
    """x = K^T v, the exact adjoint of :func:`conv`."""
    v, k = _f64(v), _f64(k)
    H, W = v.shape
    x = np.empty_like(v)
    _load().oracle_conv_adj(_p(v), H, W, _p(k), k.shape[0], _p(x))
    return x


def rbf(z: float, j: int, mu0: float, step: float, sigma: float) -> float:
    return float(_load().oracle_rbf(float(z), int(j), mu0, step, sigma))


def phi(z, w, mu0: float, step: float, sigma: float) -> np.ndarray:
    """Influence function phi(z) = sum_j w_j exp(-(z-mu_j)^2/(2 sigma^2)), elementwise."""
    w = _f64(w)
    lib = _load()
    zz = np.asarray(z, dtype=np.float64)
    out = np.array([lib.oracle_phi(float(x), _p(w), w.size, mu0, step, sigma)
                    for x in zz.ravel()])
    return out.reshape(zz.shape)


def dphi(z, w, mu0: float, step: float, sigma: float) -> np.ndarray:
    w = _f64(w)
    lib = _load()
    zz = np.asarray(z, dtype=np.float64)
    out = np.array([lib.oracle_dphi(float(x), _p(w), w.size, mu0, step, sigma)
                    for x in zz.ravel()])
    return out.reshape(zz.shape)


def prox(ut, f, lam: float) -> np.ndarray:
    lib = _load()
    ut = np.asarray(ut, dtype=np.float64)
    f = np.broadcast_to(np.asarray(f, dtype=np.float64), ut.shape)
    out = np.array([lib.oracle_prox(float(a), float(b), float(lam))
                    for a, b in zip(ut.ravel(), f.ravel())])
    return out.reshape(ut.shape)


def prox_grad(ut: float, f: float, lam: float):
    """(du/dut, du/dlambda) of the prox at one point."""
    y, xl = ctypes.c_double(), ctypes.c_double()
    _load().oracle_prox_grad(float(ut), float(f), float(lam), ctypes.byref(y), ctypes.byref(xl))
    return y.value, xl.value


def psi(u, f, lam: float) -> np.ndarray:
    """Reaction (lambda/u)(1 - f^2/u^2) of the projected variant, elementwise."""
    lib = _load()
    u = np.asarray(u, dtype=np.float64)
    f = np.broadcast_to(np.asarray(f, dtype=np.float64), u.shape)
    out = np.array([lib.oracle_psi(float(a), float(b), float(lam)) for a, b in zip(u.ravel(), f.ravel())])
    return out.reshape(u.shape)


def psi_partials(u: float, f: float, lam: float):
    """(d psi/du, d psi/dlambda, d psi/df) at one point."""
    lib = _load()
    return (lib.oracle_psi_du(float(u), float(f), float(lam)),
            lib.oracle_psi_dlam(float(u), float(f)),
            lib.oracle_psi_df(float(u), float(f), float(lam)))


def prox_df(ut: float, f: float, lam: float) -> float:
    """d prox / d f at fixed ut."""
    return float(_load().oracle_prox_df(float(ut), float(f), float(lam)))


REACTIONS = {"prox": 0, "projected": 1, "l2": 2}


def _reaction(model):
    """(reaction code, projection threshold c) of a model dict: reaction
    "prox" (default, eq. diffusionprocessfinal), "projected" (eq. diffusion_backP)
    or "l2" (gradient step on (lambda/2)||u - f||^2, eq. diffusion with G = 0)."""
    return REACTIONS[model.get("reaction", "prox")], float(model.get("proj_c", 1.0))


def _model_args(m):
    filters = _f64(m["filters"])
    rbf_w = _f64(m["rbf_w"])
    lam = _f64(m["lam"])
    T, Nk, ks, _ = filters.shape
    Nrbf = rbf_w.shape[-1]
    assert rbf_w.shape == (T, Nk, Nrbf) and lam.shape == (T,)
    return filters, rbf_w, lam, T, Nk, ks, Nrbf


def forward(f, model, want_states: bool = False, want_utilde: bool = False,
            nthreads: int = 0):
    """T-stage forward on f [N][H][W] (or [H][W]).  ``model`` is a dict with
    filters [T][Nk][ks][ks], rbf_w [T][Nk][Nrbf], lam [T], mu0, step, sigma.
    Returns u_T, and optionally states [T+1][N][H][W] and utilde [T][N][H][W]."""
    f = _f64(f)
    squeeze = f.ndim == 2
    if squeeze:
        f = f[None]
    N, H, W = f.shape
    filters, rbf_w, lam, T, Nk, ks, Nrbf = _model_args(model)
    uT = np.empty_like(f)
    states = np.empty((T + 1, N, H, W)) if want_states else None
    utilde = np.empty((T, N, H, W)) if want_utilde else None
    react, cproj = _reaction(model)
    _load().oracle_forward_ex(_p(f), N, H, W, T, Nk, ks, Nrbf,
                              float(model["mu0"]), float(model["step"]), float(model["sigma"]),
                              _p(filters), _p(rbf_w), _p(lam), react, cproj,
                              _p(uT), _p(states), _p(utilde), int(nthreads))
    out = [uT[0] if squeeze else uT]
    if want_states:
        out.append(states[:, 0] if squeeze else states)
    if want_utilde:
        out.append(utilde[:, 0] if squeeze else utilde)
    return out[0] if len(out) == 1 else tuple(out)


def stage(u_prev, f, model, t: int, nthreads: int = 0):
    """Stage t (0-based) alone: u_t from u_prev [N][H][W] (or [H][W]) with data
    f.  Returns (u_t, ut_t)."""
    u_prev, f = _f64(u_prev), _f64(f)
    squeeze = f.ndim == 2
    if squeeze:
        f, u_prev = f[None], u_prev[None]
    assert u_prev.shape == f.shape
    N, H, W = f.shape
    filters, rbf_w, lam, T, Nk, ks, Nrbf = _model_args(model)
    assert 0 <= t < T
    ut = np.empty_like(f)
    un = np.empty_like(f)
    react, cproj = _reaction(model)
    _load().oracle_stage_ex(_p(u_prev), _p(f), N, H, W, int(t), Nk, ks, Nrbf,
                            float(model["mu0"]), float(model["step"]), float(model["sigma"]),
                            _p(filters), _p(rbf_w), _p(lam), react, cproj, _p(ut), _p(un),
                            int(nthreads))
    return (un[0], ut[0]) if squeeze else (un, ut)


def backward(f, model, states, gT, nthreads: int = 0, want_df: bool = False):
    """Gradients (dK, dW, dlam, g0) of a loss with dl/du_T = gT, given the
    forward states u_0..u_T.  Sums over images.  With want_df, also dl/df in
    full (g0 plus the explicit f-dependence of every stage)."""
    f = _f64(f)
    squeeze = f.ndim == 2
    if squeeze:
        f = f[None]
        states = np.asarray(states)[:, None]
        gT = np.asarray(gT)[None]
    N, H, W = f.shape
    states, gT = _f64(states), _f64(gT)
    filters, rbf_w, lam, T, Nk, ks, Nrbf = _model_args(model)
    assert states.shape == (T + 1, N, H, W)
    dK = np.empty_like(filters)
    dW = np.empty_like(rbf_w)
    dlam = np.empty_like(lam)
    g0 = np.empty_like(f)
    gf = np.empty_like(f) if want_df else None
    react, cproj = _reaction(model)
    _load().oracle_backward_ex(_p(f), N, H, W, T, Nk, ks, Nrbf,
                               float(model["mu0"]), float(model["step"]), float(model["sigma"]),
                               _p(filters), _p(rbf_w), _p(lam), react, cproj, _p(states), _p(gT),
                               _p(dK), _p(dW), _p(dlam), _p(g0), _p(gf), int(nthreads))
    out = (dK, dW, dlam, (g0[0] if squeeze else g0))
    if want_df:
        out = out + ((gf[0] if squeeze else gf),)
    return out
