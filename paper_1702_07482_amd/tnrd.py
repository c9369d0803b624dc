"""ctypes binding of libtnrd.so (include/tnrd.h).

The functions named like the C entry points (``tnrd_forward``,
``tnrd_backward``, ``tnrd_forward_batched``, ``tnrd_workspace_bytes``, ...)
only marshal arguments: torch CUDA tensors become device pointers, the current
torch stream becomes the ``stream`` argument.  Every step of the filter runs in
the HIP kernels of the library.  There is no fallback: if the library is not
built, or a call returns an error, a RuntimeError is raised.

``forward``, ``backward`` and ``forward_batched`` are conveniences that
allocate outputs and the workspace with torch and call the entry points.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libtnrd.so")

TNRD_OK = 0
TNRD_ERR_ARG = -1
TNRD_ERR_DOMAIN = -2
TNRD_ERR_WORKSPACE = -3
TNRD_ERR_HIP = -4
TNRD_ERR_UNSUPPORTED = -5
TNRD_ERR_CAPACITY = -6
TNRD_ERR_TIMEOUT = -7
NOALLOC_SCRATCH_BYTES = 64 << 20

PREC_FP32, PREC_BF16, PREC_FP16 = 0, 1, 2
REACT_PROX, REACT_PROJECTED, REACT_L2 = 0, 1, 2
REACTIONS = {"prox": REACT_PROX, "projected": REACT_PROJECTED, "l2": REACT_L2}
IMPL_AUTO, IMPL_FUSED, IMPL_SPLIT = 0, 1, 2


class TnrdModel(ctypes.Structure):
    _fields_ = [
        ("T", ctypes.c_int32), ("Nk", ctypes.c_int32), ("ksize", ctypes.c_int32),
        ("Nrbf", ctypes.c_int32), ("L", ctypes.c_int32),
        ("rbf_mu0", ctypes.c_float), ("rbf_step", ctypes.c_float), ("rbf_sigma", ctypes.c_float),
        ("filters", ctypes.c_void_p), ("rbf_w", ctypes.c_void_p), ("lambda_", ctypes.c_void_p),
        ("reaction", ctypes.c_int32), ("proj_c", ctypes.c_float),
    ]


class TnrdOpts(ctypes.Structure):
    _fields_ = [
        ("prec", ctypes.c_int32), ("impl", ctypes.c_int32), ("rbf_window", ctypes.c_int32),
        ("recompute_every", ctypes.c_int32), ("validate", ctypes.c_int32),
        ("tile_h", ctypes.c_int32), ("tile_w", ctypes.c_int32), ("wg_waves", ctypes.c_int32),
        ("use_graph", ctypes.c_int32), ("persistent", ctypes.c_int32),
    ]


class TnrdPeaks(ctypes.Structure):
    _fields_ = [(n, ctypes.c_double) for n in (
        "copy_gbs", "mfma_f32_tflops", "mfma_bf16_k16_tflops", "mfma_bf16_k32_tflops",
        "valu_f32_tflops", "exp_per_s")]


class TnrdImage(ctypes.Structure):
    _fields_ = [
        ("f", ctypes.c_void_p), ("u_out", ctypes.c_void_p),
        ("H", ctypes.c_int32), ("W", ctypes.c_int32), ("L", ctypes.c_int32),
    ]


_lib = None

_P = ctypes.c_void_p
_I = ctypes.c_int
_SZ = ctypes.c_size_t

# (name, restype, argtypes) of every entry point in include/tnrd.h
SIGNATURES = [
    ("tnrd_default_opts", None, [ctypes.POINTER(TnrdOpts)]),
    ("tnrd_workspace_bytes", _SZ, [_I, _I, _I, ctypes.POINTER(TnrdModel), ctypes.POINTER(TnrdOpts), _I]),
    ("tnrd_num_checkpoints", _I, [_I, _I]),
    ("tnrd_forward", _I, [_P, _I, _I, _I, _I, ctypes.POINTER(TnrdModel), _P, _P,
                          ctypes.POINTER(TnrdOpts), _P, _SZ, _P]),
    ("tnrd_backward", _I, [_P, _I, _I, _I, _I, ctypes.POINTER(TnrdModel), _P, _P, _P, _P, _P, _P,
                           _P, ctypes.POINTER(TnrdOpts), _P, _SZ, _P]),
    ("tnrd_batched_workspace_bytes", _SZ, [_I, ctypes.POINTER(TnrdImage), _I,
                                           ctypes.POINTER(TnrdModel), ctypes.POINTER(TnrdOpts)]),
    ("tnrd_forward_batched", _I, [_I, ctypes.POINTER(TnrdImage), _I, ctypes.POINTER(TnrdModel),
                                  ctypes.POINTER(TnrdOpts), _P, _SZ, _P]),
    ("tnrd_forward_noalloc", _I, [_P, _I, _I, _I, _I, ctypes.POINTER(TnrdModel), _P, _P,
                                  ctypes.POINTER(TnrdOpts), _P]),
    ("tnrd_status_str", ctypes.c_char_p, [_I]),
    ("tnrd_selected_impl", _I, [ctypes.POINTER(TnrdModel), ctypes.POINTER(TnrdOpts)]),
    ("tnrd_peaks_sink_floats", _SZ, []),
    ("tnrd_measure_peaks", _I, [_P, _P, _SZ, _P, ctypes.POINTER(TnrdPeaks), _P]),
]


def load():
    """Load libtnrd.so (raises if it is not built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is not built; run __graft_entry__.build() "
                               "(the HIP library is required, there is no fallback)")
        lib = ctypes.CDLL(LIB_PATH)
        for name, res, args in SIGNATURES:
            fn = getattr(lib, name)
            fn.restype = res
            fn.argtypes = args
        _lib = lib
    return _lib


def status_str(st: int) -> str:
    return load().tnrd_status_str(int(st)).decode()


def _check(st: int, what: str):
    if st != TNRD_OK:
        raise RuntimeError(f"{what} failed: {status_str(st)} ({st})")


def default_opts(**kw) -> TnrdOpts:
    o = TnrdOpts()
    load().tnrd_default_opts(ctypes.byref(o))
    for k, v in kw.items():
        if not hasattr(o, k):
            raise KeyError(k)
        setattr(o, k, int(v))
    return o


def _ptr(t):
    if t is None:
        return None
    return ctypes.c_void_p(t.data_ptr())


def _stream(stream=None):
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


# ------------------------------------------------------------------ raw entry points
def tnrd_workspace_bytes(N, H, W, model: "TnrdModel", opts: TnrdOpts, which: int) -> int:
    return int(load().tnrd_workspace_bytes(N, H, W, ctypes.byref(model), ctypes.byref(opts), which))


def tnrd_num_checkpoints(T: int, recompute_every: int) -> int:
    return int(load().tnrd_num_checkpoints(T, recompute_every))


def tnrd_forward(f, N, H, W, L, model: TnrdModel, u_out, states, opts: TnrdOpts, ws, ws_bytes,
                 stream=None) -> int:
    return int(load().tnrd_forward(_ptr(f), N, H, W, L, ctypes.byref(model), _ptr(u_out),
                                   _ptr(states), ctypes.byref(opts), _ptr(ws), ws_bytes,
                                   _stream(stream)))


def tnrd_forward_noalloc(f, N, H, W, L, model: TnrdModel, u_out, states, opts: TnrdOpts,
                         stream=None) -> int:
    return int(load().tnrd_forward_noalloc(_ptr(f), N, H, W, L, ctypes.byref(model), _ptr(u_out),
                                           _ptr(states), ctypes.byref(opts), _stream(stream)))


def tnrd_backward(f, N, H, W, L, model: TnrdModel, states, grad_uT, grad_filters, grad_rbf_w,
                  grad_lambda, grad_u0, grad_f, opts: TnrdOpts, ws, ws_bytes, stream=None) -> int:
    return int(load().tnrd_backward(_ptr(f), N, H, W, L, ctypes.byref(model), _ptr(states),
                                    _ptr(grad_uT), _ptr(grad_filters), _ptr(grad_rbf_w),
                                    _ptr(grad_lambda), _ptr(grad_u0), _ptr(grad_f),
                                    ctypes.byref(opts), _ptr(ws), ws_bytes, _stream(stream)))


def tnrd_batched_workspace_bytes(B, imgs, n_models, models, opts: TnrdOpts) -> int:
    return int(load().tnrd_batched_workspace_bytes(B, imgs, n_models, models, ctypes.byref(opts)))


def tnrd_forward_batched(B, imgs, n_models, models, opts: TnrdOpts, ws, ws_bytes, stream=None) -> int:
    return int(load().tnrd_forward_batched(B, imgs, n_models, models, ctypes.byref(opts),
                                           _ptr(ws), ws_bytes, _stream(stream)))


def tnrd_peaks_sink_floats() -> int:
    return int(load().tnrd_peaks_sink_floats())


def tnrd_measure_peaks(copy_src, copy_dst, copy_bytes, sink, stream=None) -> dict:
    """Measured throughput of the units the kernels run on (a measurement aid)."""
    out = TnrdPeaks()
    _check(load().tnrd_measure_peaks(_ptr(copy_src), _ptr(copy_dst), copy_bytes, _ptr(sink),
                                     ctypes.byref(out), _stream(stream)), "tnrd_measure_peaks")
    return {n: getattr(out, n) for n, _ in TnrdPeaks._fields_}


# ------------------------------------------------------------------ conveniences
@dataclass
class DeviceModel:
    """Model parameters resident on the GPU plus the ABI struct pointing at them."""
    filters: torch.Tensor   # [T][Nk][k][k] fp32
    rbf_w: torch.Tensor     # [T][Nk][Nrbf] fp32
    lam: torch.Tensor       # [T] fp32
    mu0: float
    step: float
    sigma: float
    L: int = 0
    reaction: int = REACT_PROX
    proj_c: float = 1.0

    @classmethod
    def from_numpy(cls, m: dict, device="cuda", L: int = 0) -> "DeviceModel":
        """From a model dict (filters, rbf_w, lam, mu0, step, sigma; optional
        reaction "prox" or "projected" and proj_c)."""
        t = lambda a: torch.as_tensor(a, dtype=torch.float32).contiguous().to(device)
        return cls(t(m["filters"]), t(m["rbf_w"]), t(m["lam"]), float(m["mu0"]),
                   float(m["step"]), float(m["sigma"]), L,
                   REACTIONS[m.get("reaction", "prox")], float(m.get("proj_c", 1.0)))

    @property
    def T(self):
        return self.filters.shape[0]

    def abi(self, filters=None, rbf_w=None, lam=None) -> TnrdModel:
        fi = self.filters if filters is None else filters
        rw = self.rbf_w if rbf_w is None else rbf_w
        la = self.lam if lam is None else lam
        for t in (fi, rw, la):
            if not (t.is_cuda and t.dtype == torch.float32 and t.is_contiguous()):
                raise ValueError("model tensors must be contiguous float32 CUDA tensors")
        T, Nk, k, k2 = fi.shape
        assert k == k2 and rw.shape[:2] == (T, Nk) and la.shape == (T,)
        return TnrdModel(T, Nk, k, rw.shape[2], self.L, self.mu0, self.step, self.sigma,
                         fi.data_ptr(), rw.data_ptr(), la.data_ptr(), self.reaction, self.proj_c)


def _img3(f):
    if f.dim() == 2:
        f = f[None]
    if not (f.is_cuda and f.dtype == torch.float32 and f.is_contiguous()):
        raise ValueError("images must be contiguous float32 CUDA tensors [N][H][W]")
    return f


def _workspace(nbytes, device):
    return torch.empty(max(int(nbytes), 1), dtype=torch.uint8, device=device)


def forward(f, model: DeviceModel, L: int = 1, want_states: bool = False, opts: TnrdOpts = None,
            filters=None, rbf_w=None, lam=None):
    """u_T (and the checkpoint states if asked) for f [N][H][W]."""
    f = _img3(f)
    N, H, W = f.shape
    o = opts if opts is not None else default_opts()
    m = model.abi(filters, rbf_w, lam)
    nb = tnrd_workspace_bytes(N, H, W, m, o, 0)
    if nb == 0:
        raise RuntimeError("tnrd_workspace_bytes: invalid or unsupported configuration")
    ws = _workspace(nb, f.device)
    u = torch.empty_like(f)
    states = None
    if want_states:
        ns = tnrd_num_checkpoints(m.T, o.recompute_every)
        states = torch.empty((ns, N, H, W), dtype=torch.float32, device=f.device)
    _check(tnrd_forward(f, N, H, W, L, m, u, states, o, ws, nb), "tnrd_forward")
    return (u, states) if want_states else u


def backward(f, model: DeviceModel, states, grad_uT, L: int = 1, opts: TnrdOpts = None,
             want_u0: bool = False, filters=None, rbf_w=None, lam=None, want_f: bool = False):
    """(dK, dW, dlambda[, g0][, gf]) for dl/du_T = grad_uT (g0 = dl/du_0 through the
    diffusion chain, gf = dl/df in full)."""
    f = _img3(f)
    grad_uT = _img3(grad_uT)
    N, H, W = f.shape
    o = opts if opts is not None else default_opts()
    m = model.abi(filters, rbf_w, lam)
    nb = tnrd_workspace_bytes(N, H, W, m, o, 1)
    if nb == 0:
        raise RuntimeError("tnrd_workspace_bytes(backward): invalid or unsupported configuration")
    ws = _workspace(nb, f.device)
    fi = model.filters if filters is None else filters
    rw = model.rbf_w if rbf_w is None else rbf_w
    la = model.lam if lam is None else lam
    dK = torch.empty_like(fi)
    dW = torch.empty_like(rw)
    dl = torch.empty_like(la)
    g0 = torch.empty_like(f) if want_u0 else None
    gf = torch.empty_like(f) if want_f else None
    _check(tnrd_backward(f, N, H, W, L, m, states, grad_uT, dK, dW, dl, g0, gf, o, ws, nb),
           "tnrd_backward")
    out = (dK, dW, dl) + ((g0,) if want_u0 else ()) + ((gf,) if want_f else ())
    return out


def forward_batched(fs, looks, models, opts: TnrdOpts = None, outs=None, ws=None):
    """Uneven batch: fs is a list of [H][W] CUDA tensors, looks their L values,
    models a list of DeviceModel whose .L select them (0 = any).  Returns the
    list of u_T tensors (and keeps using `outs`/`ws` if given, so repeated
    calls with the same buffers replay the recorded HIP graph)."""
    B = len(fs)
    o = opts if opts is not None else default_opts()
    if outs is None:
        outs = [torch.empty_like(f) for f in fs]
    imgs = (TnrdImage * B)()
    for b, (f, L, u) in enumerate(zip(fs, looks, outs)):
        if not (f.is_cuda and f.dtype == torch.float32 and f.is_contiguous() and f.dim() == 2):
            raise ValueError("batched images must be contiguous 2-D float32 CUDA tensors")
        imgs[b] = TnrdImage(f.data_ptr(), u.data_ptr(), f.shape[0], f.shape[1], int(L))
    mods = (TnrdModel * len(models))()
    for k, m in enumerate(models):
        mods[k] = m.abi()
    nb = tnrd_batched_workspace_bytes(B, imgs, len(models), mods, o)
    if nb == 0:
        raise RuntimeError("tnrd_batched_workspace_bytes: invalid or unsupported batch")
    if ws is None or ws.numel() < nb:
        ws = _workspace(nb, fs[0].device)
    _check(tnrd_forward_batched(B, imgs, len(models), mods, o, ws, nb), "tnrd_forward_batched")
    return outs, ws
