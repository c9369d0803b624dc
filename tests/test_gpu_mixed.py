"""Mixed precision: the filter-bank contractions (K u and the K^T GEMM of the
forward and of the input-gradient pass; K e and the dK contraction of the
parameter-gradient pass) with BF16 or FP16 operands and FP32 accumulation; the
influence function and the prox stay FP32.  The parameter gradients take z = K u
on FP32 operands with FP16, and with BF16 the input-gradient pass's BF16 z, kept
as BF16 words (with BF16 operands the influence comes from cubics on half intervals,
whose interpolation error, below 2.6e-4 of the largest RBF weight for phi and
6.7e-4 for d phi / ds, is a tenth of the BF16 rounding its values get for the
K^T GEMM).  Errors against the FP64 oracle are bounded per output, and the
despeckling quality (PSNR against the clean image) moves by at most 1e-2 dB.

Forward bound: an operand rounded to BF16 carries a relative error of at most
u_p = 2^-8 (FP16: 2^-11).  The diffusion update x = sum_i K_i^T phi_i(K_i u) is
a small correction of u (|x| ~ 1 against u ~ 1e2 for these models), so one
stage changes u by about u_p |x| in BF16; eight stages and the conditioning of
phi stay far below 1e-3 of ||u||_inf.  The tests use 1e-3 (BF16) and 2e-4
(FP16) relative to ||u_T||_inf.

Backward bound (per tensor, derived from the oracle alone): the mixed path
perturbs every operand a contraction reads by a relative error of at most
u_p.  Those operands are the filters and quantities computed from the states
and dl/du_T, so the bound is the oracle's own sensitivity to perturbations of
that size: D_k, the change of each gradient when the oracle runs with its
filters rounded to the format, plus D_s, the change when every state u_t and
dl/du_T is multiplied pixel by pixel by 1 + u_p xi, xi uniform in [-1, 1]
(the larger of two seeded draws).  The test requires error <= D_k + D_s.
"""
import numpy as np
import pytest
import torch

import oracle
from paper_1702_07482_amd import synth, tnrd
from tests.helpers import crop_window, oracle_uT_at, rel_inf

pytestmark = pytest.mark.gpu

BOUND = {tnrd.PREC_BF16: 1e-3, tnrd.PREC_FP16: 2e-4}
PRECS = [tnrd.PREC_BF16, tnrd.PREC_FP16]


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).cuda()


def psnr(u, ref, peak=255.0):
    mse = float(np.mean((np.asarray(u, np.float64) - np.asarray(ref, np.float64)) ** 2))
    return 10.0 * np.log10(peak * peak / mse)


@pytest.mark.parametrize("prec", PRECS)
def test_mixed_forward_against_oracle(prec):
    m = synth.config_model(5)
    u, f = synth.make_pair(96, 88, 1, config_id=5, index=1)
    ref = oracle.forward(f, m)
    dm = tnrd.DeviceModel.from_numpy(m)
    got = tnrd.forward(_dev(f), dm, opts=tnrd.default_opts(prec=prec)).cpu().numpy()[0]
    err = rel_inf(got, ref)
    d = np.abs(got.astype(np.float64) - ref)
    dpsnr = abs(psnr(got, u) - psnr(ref, u))
    print(f"prec={prec} rel_inf={err:.2e} max_abs={d.max():.3e} mean_abs={d.mean():.3e} "
          f"dPSNR={dpsnr:.2e} dB", flush=True)
    assert err <= BOUND[prec]
    assert dpsnr <= 1e-2


@pytest.mark.parametrize("tile", [(32, 32, 4), (64, 32, 8), (32, 48, 4), (128, 32, 4)])
def test_bf16_forward_tiles(tile):
    """The BF16 forward on requested tiles and wave counts (4 and 8 waves, 2 and 3
    sixteen-pixel blocks per row), ragged at both edges, against the oracle
    within the BF16 bound."""
    th, tw, nw = tile
    print(f"[bf16 forward tile {tile}]", flush=True)
    m = synth.config_model(5)
    u, f = synth.make_pair(150, 137, 1, config_id=5, index=7)
    ref = oracle.forward(f, m)
    dm = tnrd.DeviceModel.from_numpy(m)
    o = tnrd.default_opts(prec=tnrd.PREC_BF16)
    o.tile_h, o.tile_w, o.wg_waves = th, tw, nw
    got = tnrd.forward(_dev(f), dm, opts=o).cpu().numpy()[0]
    err = rel_inf(got, ref)
    print(f"rel_inf={err:.2e}", flush=True)
    assert err <= BOUND[tnrd.PREC_BF16]


@pytest.mark.parametrize("prec", PRECS)
def test_mixed_full_size_sampled(prec):
    """8 x 2048 x 2048 (the mixed workload): sampled pixels against the oracle on
    receptive-field crops; whole-batch PSNR against the FP32 path."""
    m = synth.config_model(5)
    pairs = [synth.make_pair(2048, 2048, 1, config_id=5, index=n) for n in range(8)]
    f = np.stack([p[1] for p in pairs])
    u = np.stack([p[0] for p in pairs])
    dm = tnrd.DeviceModel.from_numpy(m)
    fd = _dev(f)
    got = tnrd.forward(fd, dm, opts=tnrd.default_opts(prec=prec)).cpu().numpy()
    g32 = tnrd.forward(fd, dm, opts=tnrd.default_opts()).cpu().numpy()
    dpsnr = abs(psnr(got, u) - psnr(g32, u))
    print(f"prec={prec} full-size dPSNR vs FP32 path = {dpsnr:.2e} dB", flush=True)
    assert dpsnr <= 1e-2
    radius = m["T"] * (m["ks"] - 1)
    for n, pts in [(0, [(0, 0), (1024, 2047)]), (7, [(2047, 5), (700, 1300)])]:
        ref = oracle_uT_at(f[n], m, pts, radius)
        g = np.array([got[n][p] for p in pts])
        # normalised by the oracle's sampled u_T values (not by max|f|, which for
        # L = 1 speckle is many times max|u_T|)
        assert np.abs(g - ref).max() <= BOUND[prec] * np.abs(ref).max(), (n, g, ref)


UNIT_ROUNDOFF = {tnrd.PREC_BF16: 2.0 ** -8, tnrd.PREC_FP16: 2.0 ** -11}


def _round_to(x, prec):
    """x rounded to nearest (even) in the operand format (FP64 values back)."""
    x = np.asarray(x, np.float32)
    if prec == tnrd.PREC_FP16:
        return x.astype(np.float16).astype(np.float64)
    b = x.view(np.uint32).astype(np.uint64)
    b = ((b + 0x7FFF + ((b >> 16) & 1)) >> 16) << 16
    return b.astype(np.uint32).view(np.float32).astype(np.float64)


def _backward_bound(f, u, m, prec):
    """D_k + D_s of the module docstring, per output (dK, dW, dlam, g0)."""
    uT, st = oracle.forward(f, m, want_states=True)
    gT = (uT - u) * (2.0 / u.size)
    ref = oracle.backward(f, m, st, gT)
    mk = dict(m)
    mk["filters"] = _round_to(m["filters"], prec)
    uTk, stk = oracle.forward(f, mk, want_states=True)
    outk = oracle.backward(f, mk, stk, (uTk - u) * (2.0 / u.size))
    dk = [rel_inf(a, b) for a, b in zip(outk, ref)]
    up = UNIT_ROUNDOFF[prec]
    rng = np.random.default_rng(1702)
    ds = [0.0] * 4
    for _ in range(2):
        sts = st * (1.0 + up * rng.uniform(-1.0, 1.0, size=st.shape))
        sts[0] = st[0]  # u_0 = f is an input, not a computed operand
        gs = gT * (1.0 + up * rng.uniform(-1.0, 1.0, size=gT.shape))
        outs = oracle.backward(f, m, sts, gs)
        ds = [max(d, rel_inf(a, b)) for d, a, b in zip(ds, outs, ref)]
    return ref, gT, [a + b for a, b in zip(dk, ds)]


def _bound_given_g(f, m, gT, prec):
    """The oracle's gradients for dl/du_T = gT and the derived bound D_k + D_s
    (as _backward_bound, with gT given)."""
    _, st = oracle.forward(f, m, want_states=True)
    ref = oracle.backward(f, m, st, gT)
    mk = dict(m)
    mk["filters"] = _round_to(m["filters"], prec)
    _, stk = oracle.forward(f, mk, want_states=True)
    dk = [rel_inf(a, b) for a, b in zip(oracle.backward(f, mk, stk, gT), ref)]
    up = UNIT_ROUNDOFF[prec]
    rng = np.random.default_rng(1703)
    ds = [0.0] * 4
    for _ in range(2):
        sts = st * (1.0 + up * rng.uniform(-1.0, 1.0, size=st.shape))
        sts[0] = st[0]
        gs = gT * (1.0 + up * rng.uniform(-1.0, 1.0, size=gT.shape))
        ds = [max(d, rel_inf(a, b)) for d, a, b in zip(ds, oracle.backward(f, m, sts, gs), ref)]
    return ref, [a + b for a, b in zip(dk, ds)]


@pytest.mark.parametrize("prec", PRECS)
def test_mixed_backward_full_size_localized(prec):
    """8 x 2048 x 2048 (the mixed workload) with the loss gradient on one pixel:
    every gradient comes from that pixel's receptive field, which the oracle
    covers with a crop of radius T (k - 1); dK, dW, dlambda and dl/du_0 on the
    crop within the derived bound computed there, and dl/du_0 exactly zero
    outside it."""
    m = synth.config_model(5)
    pairs = [synth.make_pair(2048, 2048, 1, config_id=5, index=n) for n in range(8)]
    f = np.stack([p[1] for p in pairs])
    del pairs
    n, y, x = 5, 1500, 700
    print(f"[mixed full-size localized prec {prec} n={n} y={y} x={x}]", flush=True)
    gT = np.zeros(f.shape, dtype=np.float32)
    gT[n, y, x] = 1.0
    dm = tnrd.DeviceModel.from_numpy(m)
    o = tnrd.default_opts(prec=prec)
    fd = _dev(f)
    _, states = tnrd.forward(fd, dm, want_states=True, opts=o)
    dK, dW, dl, g0 = tnrd.backward(fd, dm, states, _dev(gT), opts=o, want_u0=True)
    g0 = g0.cpu().numpy()
    radius = m["T"] * (m["ks"] - 1)
    y0, y1 = crop_window(y, 2048, radius)
    x0, x1 = crop_window(x, 2048, radius)
    (rK, rW, rl, rg), bound = _bound_given_g(f[n, y0:y1, x0:x1], m, gT[n, y0:y1, x0:x1], prec)
    names = ["dK", "dW", "dlam", "g0"]
    got = [dK.cpu().numpy(), dW.cpu().numpy(), dl.cpu().numpy(), g0[n, y0:y1, x0:x1]]
    errs = {k: rel_inf(a, b) for k, a, b in zip(names, got, (rK, rW, rl, rg))}
    bounds = dict(zip(names, bound))
    print(f"rel errors {errs} bounds {bounds}", flush=True)
    outside = g0.copy()
    outside[n, y0:y1, x0:x1] = 0.0
    assert not outside.any()
    for k in names:
        assert errs[k] <= bounds[k], (k, errs, bounds)


@pytest.mark.parametrize("want_u0", [True, False])
@pytest.mark.parametrize("prec", PRECS)
def test_mixed_backward_input_gradient(prec, want_u0):
    """The backward with the mixed filter bank (input gradient and parameter
    gradients): each gradient within the derived bound D_k + D_s of the FP64
    oracle (relative to each tensor's max).  Without dl/du_0 the first stage's
    parameter gradients come from the variant that computes z and a itself
    (the input-gradient kernel does not run there)."""
    m = synth.config_model(5)
    u, f = synth.make_pair(48, 56, 1, config_id=5, index=2)
    (rK, rW, rl, rg), gT, bound = _backward_bound(f, u, m, prec)
    dm = tnrd.DeviceModel.from_numpy(m)
    o = tnrd.default_opts(prec=prec)
    fd = _dev(f)
    _, states = tnrd.forward(fd, dm, want_states=True, opts=o)
    out = tnrd.backward(fd, dm, states, _dev(gT), opts=o, want_u0=want_u0)
    names = ["dK", "dW", "dlam", "g0"][:len(out)]
    errs = {n: rel_inf(a.cpu().numpy(), b) for n, a, b in
            zip(names, out, (rK, rW, rl, rg))}
    bounds = dict(zip(names, bound))
    print(f"prec={prec} want_u0={want_u0} backward rel errors {errs} bounds {bounds}", flush=True)
    for n in names:
        assert errs[n] <= bounds[n], (n, errs, bounds)


@pytest.mark.parametrize("nk", [13, 40])
@pytest.mark.parametrize("prec", PRECS)
def test_mixed_backward_uneven_filter_counts(prec, nk):
    """Filter counts that fill neither a 16-filter block nor the last 4-filter
    quad of the z/a export (BF16 words with BF16 operands), within the derived
    bound of the FP64 oracle."""
    print(f"[mixed bwd prec {prec} nk {nk}]", flush=True)
    g = np.random.default_rng(4400 + nk)
    m = synth.make_model(3, nk, 7, g)
    u, f = synth.make_pair(37, 45, 1, config_id=5, index=nk)
    (rK, rW, rl, rg), gT, bound = _backward_bound(f, u, m, prec)
    dm = tnrd.DeviceModel.from_numpy(m)
    o = tnrd.default_opts(prec=prec)
    fd = _dev(f)
    _, states = tnrd.forward(fd, dm, want_states=True, opts=o)
    out = tnrd.backward(fd, dm, states, _dev(gT), opts=o, want_u0=True)
    names = ["dK", "dW", "dlam", "g0"]
    errs = {n: rel_inf(a.cpu().numpy(), b) for n, a, b in zip(names, out, (rK, rW, rl, rg))}
    bounds = dict(zip(names, bound))
    print(f"rel errors {errs} bounds {bounds}", flush=True)
    for n in names:
        assert errs[n] <= bounds[n], (n, errs, bounds)


def _reaction_case(reaction):
    """(model, clean, noisy) of the projected (Sec. 3.1, c = 1) or quadratic
    (Sec. 2.2.1) reaction with 7x7 filters, the size the mixed kernels take."""
    if reaction == "l2":
        m = synth.config_model(7)  # 5 stages x 48 7x7, lambda 0.1
        u, f = synth.make_gaussian_pair(44, 52, 25.0, config_id=7, index=61)
        return m, u, f
    g = np.random.default_rng(6210)
    m = synth.make_model(3, 24, 7, g)
    m["reaction"], m["proj_c"] = "projected", 1.0
    u, f = synth.make_pair(44, 52, 1, config_id=2, index=62, peak=12.0)
    return m, u, f


@pytest.mark.parametrize("reaction", ["projected", "l2"])
@pytest.mark.parametrize("prec", PRECS)
def test_mixed_other_reactions(prec, reaction):
    """The projected and quadratic reactions with BF16/FP16 filter-bank operands:
    the forward within the forward bound, and dK, dW, dlambda and dl/du_0 within
    the derived bound D_k + D_s of the FP64 oracle."""
    print(f"[mixed {reaction} prec {prec}]", flush=True)
    m, u, f = _reaction_case(reaction)
    ref = oracle.forward(f, m)
    dm = tnrd.DeviceModel.from_numpy(m)
    o = tnrd.default_opts(prec=prec)
    fd = _dev(f)
    got, states = tnrd.forward(fd, dm, want_states=True, opts=o)
    ferr = rel_inf(got.cpu().numpy()[0], ref)
    (rK, rW, rl, rg), gT, bound = _backward_bound(f, u, m, prec)
    out = tnrd.backward(fd, dm, states, _dev(gT), opts=o, want_u0=True)
    names = ["dK", "dW", "dlam", "g0"]
    errs = {n: rel_inf(a.cpu().numpy(), b) for n, a, b in zip(names, out, (rK, rW, rl, rg))}
    bounds = dict(zip(names, bound))
    print(f"forward rel_inf={ferr:.2e}; backward rel errors {errs} bounds {bounds}", flush=True)
    assert ferr <= BOUND[prec]
    for n in names:
        assert errs[n] <= bounds[n], (n, errs, bounds)


def test_fp16_validate_rejects_values_beyond_its_range():
    """FP16 operands hold the states unscaled; validate refuses f >= 2^15 for
    them (TNRD_ERR_UNSUPPORTED), and accepts the same image in BF16 and FP32,
    whose exponent range covers it."""
    m = synth.config_model(5)
    f = synth.make_pair(40, 40, 1, config_id=5, index=3)[1].astype(np.float64)
    f = f / f.max() * 1.0e5
    dm = tnrd.DeviceModel.from_numpy(m)
    with pytest.raises(RuntimeError, match="unsupported"):
        tnrd.forward(_dev(f), dm, opts=tnrd.default_opts(prec=tnrd.PREC_FP16, validate=1))
    for prec in (tnrd.PREC_BF16, tnrd.PREC_FP32):
        out = tnrd.forward(_dev(f), dm, opts=tnrd.default_opts(prec=prec, validate=1)).cpu().numpy()
        assert np.isfinite(out).all()
