"""Benchmark of the trained reaction-diffusion despeckling filter on one MI355X.

Default workload (the headline figure): one 512 x 512 speckled image (L = 1),
8 stages of 48 7x7 filters, 63 Gaussian RBFs per filter, FP32.  A step is one
forward pass of all stages over that image through the C ABI (tnrd_forward),
inputs resident in HBM.  Metric: megapixel-stages per second
(H * W * T / 1e6 / seconds).

Extra legs reported on the same JSON line (each its own workload):
  fwd_bwd  16 x 180 x 180, forward with saved states + hand-written backward
  batched  64 uneven images, one launch per stage over all tiles, replayed from a HIP graph
           (and the single persistent launch over every (stage, tile), timed beside it)
  mixed    8 x 2048 x 2048 with BF16/FP16 filter-bank operands
  projected  the paper's comparison model (projection onto u >= 1), 8 x 512 x 512,
           5 stages of 24 5x5 filters, forward and forward + backward with dl/df
  denoise  the framework's Gaussian-denoising reaction (quadratic data term),
           8 x 512 x 512, 5 stages of 48 7x7 filters
  train    joint L-BFGS training (train.py) on the fwd_bwd workload: loss evaluations
           (forward + backward) per second, and the quality indexes (PSNR, MSSIM, EC,
           ratio image, coefficient of variation) of the model before and after
  peaks    measured copy, matrix, vector-FMA and exp2 throughput; the legs' rates
           against them ("fractions")
  fused_vs_split  (not a default leg) the 8 x 2048 x 2048 FP32 forward with the fused
           stage kernel and with the split path

The CPU baseline times the FP64 oracle (tests' reference, not a product path)
on a bounded strip of the same workload.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--legs fwd,fwd_bwd,...]
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_FP32_MFMA_TFLOPS = 157.3     # MI355X dense FP32 matrix
PEAK_FP32_VECTOR_TFLOPS = 157.3   # MI355X FP32 vector (published; packed FP32)
PEAK_BF16_TFLOPS = 2500.0
PEAK_HBM_GBS = 8000.0

FLOP_PER_PX_STAGE_FWD = 2 * 2 * 48 * 49   # K and K^T, 48 filters of 7x7 (multiply-add = 2 flop)
# forward + backward: the forward's K and K^T, then the backward's K u (z, not stored by the
# forward), K e, K^T (phi' a) and the two dK correlations: 5 more contractions of 4704 flop
FLOP_PER_PX_STAGE_FWD_BWD = FLOP_PER_PX_STAGE_FWD + 5 * 4704


def roofline_entry(mpst, flop_per_pxst, peak_tflops, note):
    """Convolution work of a whole form (every kernel of a call) against a published
    peak: achieved = algorithmic flop per pixel-stage x pixel-stages per second."""
    achieved = mpst * 1e6 * flop_per_pxst / 1e12
    return {"bound": "mfma", "achieved": achieved, "peak": peak_tflops, "unit": "TFLOP/s",
            "frac": achieved / peak_tflops, "flop_per_pixel_stage": flop_per_pxst, "basis": note}


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--impl", default="auto", choices=["auto", "fused", "split"])
    ap.add_argument("--legs", default="fwd,fwd_bwd,batched,mixed,projected,denoise,train,peaks")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--calib-copy-mib", type=int, default=0,
                    help="run one device-to-device copy of this many MiB first (a kernel of known "
                         "traffic, to scale HBM counters)")
    ap.add_argument("--cpu-rows", type=int, default=512,
                    help="rows of the 512-wide strip the oracle baseline runs on")
    return ap.parse_args()


FUSED_SOURCES = ["paper_1702_07482_amd/csrc/tnrd_fused_tile.hpp",
                 "paper_1702_07482_amd/csrc/tnrd_fused.hip",
                 "paper_1702_07482_amd/csrc/tnrd_fused_common.hpp",
                 "paper_1702_07482_amd/csrc/tnrd_device.hpp",
                 "paper_1702_07482_amd/csrc/tnrd_prep.hip"]
FUSED_PROFILE = "profiles/fused_stage_fwd_512x512_48x7x7.md"


def profiled_traffic():
    """HBM bytes per fused-stage launch from the committed FETCH_SIZE/WRITE_SIZE
    profile, or None if the kernel sources changed since it was taken."""
    import hashlib
    import re
    try:
        text = open(os.path.join(ROOT, FUSED_PROFILE)).read()
        rec = json.loads(re.search(r"```json\n(.*?)\n```", text, re.S).group(1))
    except (OSError, AttributeError, ValueError):
        return None
    h = hashlib.sha256()
    for src in FUSED_SOURCES:
        with open(os.path.join(ROOT, src), "rb") as fh:
            h.update(fh.read())
    return rec["traffic_bytes_per_launch"] if h.hexdigest() == rec["source_sha256"] else None


def _events():
    import torch
    return torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)


def leg_forward(args, impl_code):
    import torch
    from paper_1702_07482_amd import synth, tnrd

    H = W = 512
    T = 8
    m = synth.config_model(2)
    _, f = synth.make_pair(H, W, 1, config_id=2)
    dm = tnrd.DeviceModel.from_numpy(m)
    fd = torch.from_numpy(f).cuda()[None].contiguous()
    o = tnrd.default_opts(impl=impl_code)
    mm = dm.abi()
    nb = tnrd.tnrd_workspace_bytes(1, H, W, mm, o, 0)
    if nb == 0:
        raise RuntimeError("unsupported configuration")
    ws = torch.empty(nb, dtype=torch.uint8, device="cuda")
    u = torch.empty_like(fd)

    def step():
        st = tnrd.tnrd_forward(fd, 1, H, W, 1, mm, u, None, o, ws, nb)
        if st != 0:
            raise RuntimeError(tnrd.status_str(st))

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    evs = [_events() for _ in range(args.steps)]
    t0 = time.perf_counter()
    for a, b in evs:
        a.record()
        step()
        b.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    per_call_ms = [a.elapsed_time(b) for a, b in evs]
    ms = float(np.mean(per_call_ms))
    mpst = H * W * T / 1e6 / (ms / 1e3)
    per_launch_s = ms / 1e3 / T  # T stage launches per call
    flop = H * W * FLOP_PER_PX_STAGE_FWD
    achieved_tflops = flop / per_launch_s / 1e12
    impl_name = "split" if impl_code == tnrd.IMPL_SPLIT else "fused"
    peak = PEAK_FP32_VECTOR_TFLOPS if impl_name == "split" else PEAK_FP32_MFMA_TFLOPS
    return {
        "value": mpst, "ms_per_step": ms, "wall_s": wall, "impl": impl_name,
        "min_ms": float(np.min(per_call_ms)),
        "roofline": {
            "bound": "alu" if impl_name == "split" else "mfma",
            "achieved": achieved_tflops, "peak": peak, "unit": "TFLOP/s",
            "frac": achieved_tflops / peak,
            "traffic": profiled_traffic() if impl_name == "fused" else None,
            "traffic_unit": "bytes per launch (rocprofv3 FETCH_SIZE + WRITE_SIZE, copy-calibrated)",
            "algorithmic_bytes_per_launch": H * W * 12,
            "kernel": "tnrd stage kernel (k_split_* pair)" if impl_name == "split"
                      else "tnrd::k_fused_stage",
            "per_launch_us": per_launch_s * 1e6,
            "flop_per_launch": flop,
        },
        "f": f, "m": m,
    }


def leg_fwd_bwd(args):
    """16 x 180 x 180: forward (checkpoints every 4 stages; the backward recomputes the
    states between them) + hand-written backward, and the same with every state stored."""
    import torch
    from paper_1702_07482_amd import synth, tnrd

    N, H, W, T = 16, 180, 180, 8
    m = synth.config_model(3)
    pairs = [synth.make_pair(H, W, 1, config_id=3, index=i) for i in range(N)]
    f = np.stack([p[1] for p in pairs])
    ugt = np.stack([p[0] for p in pairs])
    dm = tnrd.DeviceModel.from_numpy(m)
    fd = torch.from_numpy(f).cuda().contiguous()
    ud = torch.from_numpy(ugt).cuda().contiguous()
    mm = dm.abi()
    u = torch.empty_like(fd)
    g = torch.empty_like(fd)
    dK = torch.empty_like(dm.filters)
    dW = torch.empty_like(dm.rbf_w)
    dl = torch.empty_like(dm.lam)
    res = {}
    for every in (4, 1):
        o = tnrd.default_opts(recompute_every=every)
        nbf = tnrd.tnrd_workspace_bytes(N, H, W, mm, o, 0)
        nbb = tnrd.tnrd_workspace_bytes(N, H, W, mm, o, 1)
        if nbf == 0 or nbb == 0:
            raise RuntimeError("unsupported configuration")
        wsf = torch.empty(nbf, dtype=torch.uint8, device="cuda")
        wsb = torch.empty(nbb, dtype=torch.uint8, device="cuda")
        ns = tnrd.tnrd_num_checkpoints(T, every)
        states = torch.empty((ns, N, H, W), dtype=torch.float32, device="cuda")

        def step():
            st = tnrd.tnrd_forward(fd, N, H, W, 1, mm, u, states, o, wsf, nbf)
            if st != 0:
                raise RuntimeError(tnrd.status_str(st))
            torch.sub(u, ud, out=g)
            g.mul_(2.0 / g.numel())
            st = tnrd.tnrd_backward(fd, N, H, W, 1, mm, states, g, dK, dW, dl, None, None, o, wsb, nbb)
            if st != 0:
                raise RuntimeError(tnrd.status_str(st))

        steps = max(3, args.steps // 5)
        for _ in range(max(2, args.warmup // 5)):
            step()
        torch.cuda.synchronize()
        a, b = _events()
        a.record()
        for _ in range(steps):
            step()
        b.record()
        torch.cuda.synchronize()
        ms = a.elapsed_time(b) / steps
        mpst = N * H * W * T / 1e6 / (ms / 1e3)
        res[every] = {"value": mpst, "ms_per_step": ms, "steps": steps, "checkpoints": ns,
                      "state_bytes": ns * N * H * W * 4}
        del wsf, wsb, states
    out = dict(res[4])
    out.update({
        "unit": "megapixel-stages/s", "recompute_every": 4,
        "roofline": roofline_entry(out["value"], FLOP_PER_PX_STAGE_FWD_BWD, PEAK_FP32_MFMA_TFLOPS,
                                   "FP32 matrix peak; 32928 flop per pixel-stage (forward K, K^T; "
                                   "backward K u, K e, K^T, two dK correlations); the recomputed "
                                   "forward stages are not counted"),
        "store_all": dict(res[1], recompute_every=1),
        "workload": "forward (states checkpointed every 4 stages, recomputed in the backward) + "
                    "backward, 16 x 180 x 180 FP32, L=1, 8 stages x 48 7x7 filters, loss "
                    "mean((u_T - u_gt)^2); gradients for all filters, RBF weights and lambda"})
    out["store_all"]["roofline"] = roofline_entry(res[1]["value"], FLOP_PER_PX_STAGE_FWD_BWD,
                                                  PEAK_FP32_MFMA_TFLOPS, "as above")
    return out


def leg_train(args):
    """Joint L-BFGS training on 16 x 180 x 180 pairs (8 stages x 48 7x7): evaluation rate
    and the quality indexes of u_T before and after."""
    import torch
    from paper_1702_07482_amd import metrics, synth
    from paper_1702_07482_amd.train import TrainableModel, train_joint

    N, H, W = 16, 180, 180
    m = synth.config_model(3)
    pairs = [synth.make_pair(H, W, 1, config_id=3, index=i) for i in range(N)]
    fd = torch.from_numpy(np.stack([p[1] for p in pairs])).cuda().contiguous()
    ud = torch.from_numpy(np.stack([p[0] for p in pairs])).cuda().contiguous()
    model = TrainableModel.from_dict(m)

    def quality():
        with torch.no_grad():
            u = model(fd)
        ri = metrics.ratio_image_stats(fd, torch.clamp(u, min=1e-3))
        return {"psnr_db": metrics.psnr(u, ud), "mssim": metrics.mssim(u, ud),
                "ec": metrics.edge_correlation(u, ud), "ri_mean": ri[0], "ri_var": ri[1],
                "cv": metrics.coeff_variation(u), "cv_clean": metrics.coeff_variation(ud)}

    q0 = quality()
    # warm-up on a copy: the first backward call and the optimiser's first use of
    # each torch operation load their GPU code (a few hundred ms, once per process)
    warm = TrainableModel.from_dict(m)
    train_joint(warm, fd, ud, iters=2)
    del warm
    torch.cuda.synchronize()
    a, b = _events()
    a.record()
    log = train_joint(model, fd, ud, iters=max(2, args.steps // 10))
    b.record()
    torch.cuda.synchronize()
    ms = a.elapsed_time(b)
    ev = len(log.losses)
    return {"evals_per_s": ev / (ms / 1e3), "mpst_s": ev * N * H * W * m["T"] / 1e6 / (ms / 1e3),
            "unit": "megapixel-stages/s of forward + backward inside L-BFGS",
            "evaluations": ev, "ms": ms, "loss_first": log.losses[0], "loss_last": log.losses[-1],
            "quality_before": q0, "quality_after": quality(),
            "workload": "joint L-BFGS (strong Wolfe) over all filters, RBF weights and "
                        "beta = log lambda, loss 1/2 sum ||u_T - u_gt||^2, 16 x 180 x 180 FP32, "
                        "L=1, 8 stages x 48 7x7"}


def leg_batched(args):
    """64 uneven images, L in {1,2,4,8}, one launch per stage over all tiles, from a HIP
    graph; the single persistent launch over every (stage, tile) timed beside it."""
    import torch
    from paper_1702_07482_amd import autotune, synth, tnrd

    sizes, looks = synth.c4_batch(64)
    T = 8
    models = {L: synth.config_model(4, look=L) for L in sorted(set(looks))}
    dms = [tnrd.DeviceModel.from_numpy(models[L], L=L) for L in sorted(models)]
    fs = [torch.from_numpy(synth.make_pair(h, w, L, config_id=4, index=100 + i)[1]).cuda()
          for i, ((h, w), L) in enumerate(zip(sizes, looks))]
    th, tw, nw = autotune.tune_batched(fs, looks, dms)
    mp = sum(h * w for h, w in sizes) / 1e6
    steps = max(3, args.steps // 5)

    def timed(persistent):
        o = tnrd.default_opts(tile_h=th, tile_w=tw, wg_waves=nw, use_graph=1, persistent=persistent)
        stream = torch.cuda.Stream()
        with torch.cuda.stream(stream):
            outs, ws = tnrd.forward_batched(fs, looks, dms, opts=o)  # records the graph
            for _ in range(2):
                tnrd.forward_batched(fs, looks, dms, opts=o, outs=outs, ws=ws)
            stream.synchronize()
            a, b = _events()
            a.record(stream)
            for _ in range(steps):
                tnrd.forward_batched(fs, looks, dms, opts=o, outs=outs, ws=ws)
            b.record(stream)
            stream.synchronize()
        return a.elapsed_time(b) / steps

    ms = timed(0)
    ms_p = timed(1)
    mpst = mp * T / (ms / 1e3)
    return {"value": mpst, "unit": "megapixel-stages/s", "ms_per_step": ms,
            "steps": steps, "megapixels": mp, "tile": [th, tw, nw],
            "persistent": {"value": mp * T / (ms_p / 1e3), "ms_per_step": ms_p,
                           "form": "one persistent launch over every (stage, tile), graph replay"},
            "roofline": roofline_entry(mpst, FLOP_PER_PX_STAGE_FWD, PEAK_FP32_MFMA_TFLOPS,
                                       "FP32 matrix peak; 9408 flop per pixel-stage (K and K^T)"),
            "workload": "batched forward, 64 images of 256x256/384x512/512x512/1024x768, "
                        "L in {1,2,4,8} (one model per L), 8 stages x 48 7x7, FP32, one "
                        "launch per stage over all tiles, replayed from a HIP graph"}


def leg_mixed(args):
    """8 x 2048 x 2048: forward and forward+backward with FP32, BF16 and FP16
    filter-bank operands (FP32 accumulation, influence function and prox)."""
    import torch
    from paper_1702_07482_amd import synth, tnrd

    N, H, W, T = 8, 2048, 2048, 8
    m = synth.config_model(5)
    pairs = [synth.make_pair(H, W, 1, config_id=5, index=n) for n in range(N)]
    f = np.stack([p[1] for p in pairs])
    ugt = np.stack([p[0] for p in pairs])
    del pairs
    dm = tnrd.DeviceModel.from_numpy(m)
    mm = dm.abi()
    fd = torch.from_numpy(f).cuda()
    ud = torch.from_numpy(ugt).cuda()
    u = torch.empty_like(fd)
    states = torch.empty((T + 1, N, H, W), dtype=torch.float32, device="cuda")
    g = torch.empty_like(fd)
    dK = torch.empty_like(dm.filters)
    dW = torch.empty_like(dm.rbf_w)
    dl = torch.empty_like(dm.lam)
    res = {}
    outs = {}
    for name, prec in [("fp32", tnrd.PREC_FP32), ("bf16", tnrd.PREC_BF16), ("fp16", tnrd.PREC_FP16)]:
        o = tnrd.default_opts(prec=prec)
        nbf = tnrd.tnrd_workspace_bytes(N, H, W, mm, o, 0)
        nbb = tnrd.tnrd_workspace_bytes(N, H, W, mm, o, 1)
        wsf = torch.empty(nbf, dtype=torch.uint8, device="cuda")
        wsb = torch.empty(nbb, dtype=torch.uint8, device="cuda")

        def fwd():
            st = tnrd.tnrd_forward(fd, N, H, W, 1, mm, u, None, o, wsf, nbf)
            if st != 0:
                raise RuntimeError(tnrd.status_str(st))

        def fwd_bwd():
            st = tnrd.tnrd_forward(fd, N, H, W, 1, mm, u, states, o, wsf, nbf)
            if st != 0:
                raise RuntimeError(tnrd.status_str(st))
            torch.sub(u, ud, out=g)
            g.mul_(2.0 / g.numel())
            st = tnrd.tnrd_backward(fd, N, H, W, 1, mm, states, g, dK, dW, dl, None, None, o, wsb, nbb)
            if st != 0:
                raise RuntimeError(tnrd.status_str(st))

        fwd()
        torch.cuda.synchronize()
        outs[name] = u.clone()
        a, b = _events()
        a.record()
        for _ in range(3):
            fwd()
        b.record()
        torch.cuda.synchronize()
        ms_f = a.elapsed_time(b) / 3
        fwd_bwd()
        torch.cuda.synchronize()
        a.record()
        for _ in range(2):
            fwd_bwd()
        b.record()
        torch.cuda.synchronize()
        ms_fb = a.elapsed_time(b) / 2
        mpst = N * H * W * T / 1e6
        peak = PEAK_FP32_MFMA_TFLOPS if name == "fp32" else PEAK_BF16_TFLOPS
        pname = "FP32 matrix" if name == "fp32" else f"dense {name.upper()} matrix (2.5 PFLOP/s)"
        res[name] = {"fwd_mpst_s": mpst / (ms_f / 1e3), "fwd_ms": ms_f,
                     "fwd_bwd_mpst_s": mpst / (ms_fb / 1e3), "fwd_bwd_ms": ms_fb,
                     "roofline_fwd": roofline_entry(mpst / (ms_f / 1e3), FLOP_PER_PX_STAGE_FWD, peak,
                                                    f"{pname} peak; 9408 flop per pixel-stage"),
                     "roofline_fwd_bwd": roofline_entry(
                         mpst / (ms_fb / 1e3), FLOP_PER_PX_STAGE_FWD_BWD, peak,
                         f"{pname} peak; 32928 flop per pixel-stage (z = K u of the parameter-"
                         "gradient pass runs FP32 in every mode)")}
        del wsf, wsb
    # the outputs on the oracle patches; the CPU-baseline leg compares them with the oracle
    res["_patch_inputs"] = mixed_patch_inputs(f, ugt, m, outs)
    res["workload"] = ("mixed precision: 8 x 2048 x 2048, L=1, 8 stages x 48 7x7; filter-bank "
                       "operands FP32/BF16/FP16 with FP32 accumulation; influence and prox FP32")
    return res


# 128 x 128 patches (image, row, column) on which the mixed-precision outputs are
# compared with the FP64 oracle: a corner, the interior, the bottom and the right border
MIXED_PATCHES = [(0, 0, 0), (3, 960, 960), (5, 1920, 512), (7, 600, 1920)]
MIXED_PATCH = 128


def mixed_patch_inputs(f, ugt, m, outs):
    """For each patch of MIXED_PATCHES: the crop of f holding the patch plus its
    receptive field (T stages x (k - 1) = 48 pixels per side, or up to the image
    border, which the crop then shares, so u_T on the patch is the whole image's),
    the patch's clean image, and each precision's u_T on the patch."""
    T = m["filters"].shape[0]
    radius = T * (m["filters"].shape[2] - 1)
    N, H, W = f.shape
    host = {k: v.cpu().numpy() for k, v in outs.items()}
    items = []
    for n, y0, x0 in MIXED_PATCHES:
        y1, x1 = y0 + MIXED_PATCH, x0 + MIXED_PATCH
        cy0, cy1 = max(0, y0 - radius), min(H, y1 + radius)
        cx0, cx1 = max(0, x0 - radius), min(W, x1 + radius)
        items.append({"crop": np.ascontiguousarray(f[n, cy0:cy1, cx0:cx1]),
                      "at": (y0 - cy0, x0 - cx0),
                      "clean": ugt[n, y0:y1, x0:x1].astype(np.float64),
                      "got": {k: host[k][n, y0:y1, x0:x1].astype(np.float64) for k in host}})
    return {"model": m, "items": items}


def mixed_vs_oracle(pin):
    """CPU-baseline leg: error of each precision's u_T against the FP64 oracle on
    MIXED_PATCHES (the oracle runs on each patch's crop).  Per precision: max |a - b| /
    max |b| and mean |a - b| over the patches, and the PSNR of u_T against the clean
    image on the patches (peak 255) minus the oracle's."""
    import oracle

    t0 = time.perf_counter()
    ref, clean, got = [], [], {}
    for it in pin["items"]:
        uT = oracle.forward(it["crop"], pin["model"])
        y, x = it["at"]
        ref.append(uT[y:y + MIXED_PATCH, x:x + MIXED_PATCH])
        clean.append(it["clean"])
        for k, v in it["got"].items():
            got.setdefault(k, []).append(v)
    ref, clean = np.stack(ref), np.stack(clean)

    def psnr(u):
        mse = float(np.mean((u - clean) ** 2))
        return 10 * math.log10(255.0 ** 2 / mse) if mse > 0 else float("inf")

    out = {"oracle_patches": {"patches": [list(p) for p in MIXED_PATCHES], "size": MIXED_PATCH,
                              "oracle_s": time.perf_counter() - t0,
                              "psnr_db_oracle": psnr(ref)}}
    for k, v in got.items():
        a = np.stack(v)
        d = np.abs(a - ref)
        out[k + "_vs_oracle"] = {"max_rel_err": float(d.max() / np.abs(ref).max()),
                                 "mean_abs_err": float(d.mean()),
                                 "dpsnr_db": psnr(a) - psnr(ref)}
    return out


def leg_fused_vs_split(args):
    """8 x 2048 x 2048, 8 stages x 48 7x7, FP32: the fused stage kernel against the
    split path (K and phi into Nk response maps in HBM, then K^T and prox).  Not a
    default leg; its HBM counters are in profiles/fused_vs_split_c2_c5.md."""
    import torch
    from paper_1702_07482_amd import synth, tnrd

    N, H, W, T = 8, 2048, 2048, 8
    m = synth.config_model(5)
    f = np.stack([synth.make_pair(H, W, 1, config_id=5, index=n)[1] for n in range(N)])
    dm = tnrd.DeviceModel.from_numpy(m)
    fd = torch.from_numpy(f).cuda().contiguous()
    out = {}
    for name, impl in (("split", tnrd.IMPL_SPLIT), ("fused", tnrd.IMPL_FUSED)):
        o = tnrd.default_opts(impl=impl)
        tnrd.forward(fd, dm, opts=o)  # warm-up (and workspace)
        torch.cuda.synchronize()
        a, b = _events()
        a.record()
        for _ in range(2):
            tnrd.forward(fd, dm, opts=o)
        b.record()
        torch.cuda.synchronize()
        ms = a.elapsed_time(b) / 2
        out[name] = {"ms_per_call": ms, "mpst_s": N * H * W * T / 1e6 / (ms / 1e3)}
    out["workload"] = "forward 8 x 2048 x 2048, L=1, 8 stages x 48 7x7, FP32, fused vs split"
    return out


def leg_projected(args):
    """The paper's comparison model (eq. diffusion_backP, projection onto u >= 1)
    at the shape of its comparison experiment (5 stages of 24 5x5 filters, L = 1),
    8 images of 512 x 512 whose clean version peaks at 6 (many pixels projected):
    forward, and forward + backward with dl/df."""
    import torch
    from paper_1702_07482_amd import synth, tnrd

    N, H, W = 8, 512, 512
    m = synth.config_model(6)
    T = m["filters"].shape[0]
    pairs = [synth.make_pair(H, W, 1, config_id=6, index=200 + n, peak=6.0) for n in range(N)]
    fd = torch.from_numpy(np.stack([p[1] for p in pairs])).cuda().contiguous()
    ud = torch.from_numpy(np.stack([p[0] for p in pairs])).cuda().contiguous()
    dm = tnrd.DeviceModel.from_numpy(m)
    mm = dm.abi()
    o = tnrd.default_opts()
    nbf = tnrd.tnrd_workspace_bytes(N, H, W, mm, o, 0)
    nbb = tnrd.tnrd_workspace_bytes(N, H, W, mm, o, 1)
    wsf = torch.empty(nbf, dtype=torch.uint8, device="cuda")
    wsb = torch.empty(nbb, dtype=torch.uint8, device="cuda")
    u = torch.empty_like(fd)
    states = torch.empty((T + 1, N, H, W), dtype=torch.float32, device="cuda")
    g = torch.empty_like(fd)
    gf = torch.empty_like(fd)
    dK, dW, dl = torch.empty_like(dm.filters), torch.empty_like(dm.rbf_w), torch.empty_like(dm.lam)

    def fwd(st=None):
        r = tnrd.tnrd_forward(fd, N, H, W, 1, mm, u, st, o, wsf, nbf)
        if r != 0:
            raise RuntimeError(tnrd.status_str(r))

    def fwd_bwd():
        fwd(states)
        torch.sub(u, ud, out=g)
        g.mul_(2.0 / g.numel())
        r = tnrd.tnrd_backward(fd, N, H, W, 1, mm, states, g, dK, dW, dl, None, gf, o, wsb, nbb)
        if r != 0:
            raise RuntimeError(tnrd.status_str(r))

    res = {}
    for name, fn in (("fwd", fwd), ("fwd_bwd", fwd_bwd)):
        for _ in range(2):
            fn()
        torch.cuda.synchronize()
        a, b = _events()
        reps = 5
        a.record()
        for _ in range(reps):
            fn()
        b.record()
        torch.cuda.synchronize()
        ms = a.elapsed_time(b) / reps
        res[f"{name}_mpst_s"] = N * H * W * T / 1e6 / (ms / 1e3)
        res[f"{name}_ms"] = ms
    fwd(states)
    torch.cuda.synchronize()
    res["projected_fraction_final"] = float((states[T] <= 1.0).float().mean().item())
    res["workload"] = ("projected variant (eq. diffusion_backP, c = 1): 8 x 512 x 512, clean peak 6, "
                       "L=1, 5 stages x 24 5x5, FP32; fwd_bwd includes dl/df")
    return res


def leg_denoise(args):
    """The framework's Gaussian-denoising reaction (quadratic data term, a gradient
    step) at TNRD's own shape, 5 stages of 48 7x7 filters: 8 images of 512 x 512
    with Gaussian noise of sigma 25, forward and forward + backward."""
    import torch
    from paper_1702_07482_amd import synth, tnrd

    N, H, W = 8, 512, 512
    m = synth.config_model(7)
    T = m["filters"].shape[0]
    pairs = [synth.make_gaussian_pair(H, W, 25.0, config_id=7, index=300 + n) for n in range(N)]
    fd = torch.from_numpy(np.stack([p[1] for p in pairs])).cuda().contiguous()
    ud = torch.from_numpy(np.stack([p[0] for p in pairs])).cuda().contiguous()
    dm = tnrd.DeviceModel.from_numpy(m)
    mm = dm.abi()
    o = tnrd.default_opts()
    nbf = tnrd.tnrd_workspace_bytes(N, H, W, mm, o, 0)
    nbb = tnrd.tnrd_workspace_bytes(N, H, W, mm, o, 1)
    wsf = torch.empty(nbf, dtype=torch.uint8, device="cuda")
    wsb = torch.empty(nbb, dtype=torch.uint8, device="cuda")
    u = torch.empty_like(fd)
    states = torch.empty((T + 1, N, H, W), dtype=torch.float32, device="cuda")
    g = torch.empty_like(fd)
    dK, dW, dl = torch.empty_like(dm.filters), torch.empty_like(dm.rbf_w), torch.empty_like(dm.lam)

    def fwd(st=None):
        r = tnrd.tnrd_forward(fd, N, H, W, 1, mm, u, st, o, wsf, nbf)
        if r != 0:
            raise RuntimeError(tnrd.status_str(r))

    def fwd_bwd():
        fwd(states)
        torch.sub(u, ud, out=g)
        g.mul_(2.0 / g.numel())
        r = tnrd.tnrd_backward(fd, N, H, W, 1, mm, states, g, dK, dW, dl, None, None, o, wsb, nbb)
        if r != 0:
            raise RuntimeError(tnrd.status_str(r))

    res = {}
    for name, fn in (("fwd", fwd), ("fwd_bwd", fwd_bwd)):
        for _ in range(2):
            fn()
        torch.cuda.synchronize()
        a, b = _events()
        reps = 5
        a.record()
        for _ in range(reps):
            fn()
        b.record()
        torch.cuda.synchronize()
        ms = a.elapsed_time(b) / reps
        res[f"{name}_mpst_s"] = N * H * W * T / 1e6 / (ms / 1e3)
        res[f"{name}_ms"] = ms
    res["workload"] = ("quadratic data term (Gaussian denoising reaction): 8 x 512 x 512, noise sigma 25, "
                       "5 stages x 48 7x7, lambda 0.1, FP32")
    return res


def leg_peaks(args):
    """Measured throughput of the units the kernels run on (copy, FP32 and BF16
    matrix instructions, FP32 vector FMA, hardware exp2), from the library's probes."""
    import torch
    from paper_1702_07482_amd import tnrd

    nbytes = 1 << 30
    src = torch.ones(nbytes // 4, device="cuda")
    dst = torch.empty_like(src)
    sink = torch.empty(tnrd.tnrd_peaks_sink_floats(), device="cuda")
    torch.cuda.synchronize()
    p = tnrd.tnrd_measure_peaks(src, dst, nbytes, sink)
    del src, dst, sink
    return p


def fractions(out):
    """Rates of the legs against the measured peaks.  The modelled ceiling of the
    FP32 forward counts the algorithmic work of a pixel-stage: 9408 flop of
    convolution on the FP32 matrix unit plus the influence function's 48 x 7
    FMAs (polynomial form) on the vector unit, which share one datapath, so
    their times add."""
    pk = out.get("peaks")
    if not pk:
        return None
    fr = {}
    conv = out["roofline"]["achieved"]
    fr["fwd_conv_vs_measured_mfma_f32"] = conv / pk["mfma_f32_tflops"]
    t_px = (FLOP_PER_PX_STAGE_FWD / (pk["mfma_f32_tflops"] * 1e12)
            + 2 * 48 * 7 / (pk["valu_f32_tflops"] * 1e12))
    ceiling = 1.0 / t_px / 1e6  # megapixel-stages/s
    fr["fwd_modelled_ceiling_mpst_s"] = ceiling
    fr["fwd_vs_modelled_ceiling"] = out["value"] / ceiling
    fr["fwd_hbm_algorithmic_gbs"] = out["roofline"]["algorithmic_bytes_per_launch"] / (
        out["roofline"]["per_launch_us"] * 1e-6) / 1e9
    fr["fwd_hbm_algorithmic_vs_measured_copy"] = fr["fwd_hbm_algorithmic_gbs"] / pk["copy_gbs"]
    if out["roofline"].get("traffic"):
        fr["fwd_hbm_counted_gbs"] = out["roofline"]["traffic"] / (out["roofline"]["per_launch_us"] * 1e-6) / 1e9
    mx = out.get("mixed")
    if mx:
        for name in ("fp32", "bf16", "fp16"):
            if name in mx:
                tf = mx[name]["fwd_mpst_s"] * 1e6 * FLOP_PER_PX_STAGE_FWD / 1e12
                peak = pk["mfma_f32_tflops"] if name == "fp32" else pk["mfma_bf16_k16_tflops"]
                fr[f"mixed_{name}_fwd_conv_tflops"] = tf
                fr[f"mixed_{name}_fwd_conv_vs_measured_peak"] = tf / peak
    fb = out.get("fwd_bwd")
    if fb:
        # forward (9408) + backward: recomputed K u, K e, K^T, two dK correlations (5 x 4704)
        tf = fb["value"] * 1e6 * (FLOP_PER_PX_STAGE_FWD + 5 * 4704) / 1e12
        fr["fwd_bwd_conv_tflops"] = tf
        fr["fwd_bwd_conv_vs_measured_mfma_f32"] = tf / pk["mfma_f32_tflops"]
    return fr


def resolve_auto_impl():
    """The implementation IMPL_AUTO runs for the headline workload."""
    import ctypes
    from paper_1702_07482_amd import synth, tnrd

    dm = tnrd.DeviceModel.from_numpy(synth.config_model(2))
    m, o = dm.abi(), tnrd.default_opts()
    impl = tnrd.load().tnrd_selected_impl(ctypes.byref(m), ctypes.byref(o))
    if impl not in (tnrd.IMPL_FUSED, tnrd.IMPL_SPLIT):
        raise RuntimeError(f"no implementation for the headline model: {tnrd.status_str(impl)}")
    return impl


def cpu_baseline(f, m, rows):
    import oracle

    strip = np.ascontiguousarray(f[:rows])
    # repeated until about 10 s of CPU work (at most 4 runs)
    runs, t0 = 0, time.perf_counter()
    while runs < 4 and (runs == 0 or time.perf_counter() - t0 < 10.0):
        oracle.forward(strip, m)
        runs += 1
    dt = (time.perf_counter() - t0) / runs
    T = m["filters"].shape[0]
    return {
        "value": strip.size * T / 1e6 / dt, "unit": "megapixel-stages/s",
        "cores": oracle.max_threads(), "kind": "oracle",
        "sample": f"FP64 oracle forward, all {T} stages, on rows 0..{rows - 1} of the "
                  f"512x512 image ({rows}x512 px), {runs} runs of {dt:.1f} s each",
        "single_thread": cpu_single_thread(f, m),
    }


def cpu_single_thread(f2, m2):
    """The oracle on one thread (the paper's CPU figures are single-threaded Matlab,
    Table runtime; context only): the whole 128 x 128 image of 5 stages x 24 5x5
    filters, and a 32-row strip of the 512 x 512 image with 8 stages x 48 7x7."""
    import oracle
    from paper_1702_07482_amd import synth

    out = {}
    m1 = synth.config_model(1)
    _, f1 = synth.make_pair(128, 128, 1, config_id=1)
    for name, img, m in (("plain forward 1x128x128, 5 stages x 24 5x5", f1, m1),
                         ("plain forward, rows 0..31 of 1x512x512, 8 stages x 48 7x7",
                          np.ascontiguousarray(f2[:32]), m2)):
        t0 = time.perf_counter()
        oracle.forward(img, m, nthreads=1)
        dt = time.perf_counter() - t0
        out[name] = {"value": img.size * m["filters"].shape[0] / 1e6 / dt,
                     "unit": "megapixel-stages/s", "seconds": dt, "cores": 1}
    return out


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only: --gpus {args.gpus} is not supported "
              "(images are independent: several GPUs would each run a share of them with no "
              "exchange in the forward and one small all-reduce of the parameter gradients)",
              file=sys.stderr)
        sys.exit(2)
    import torch
    from paper_1702_07482_amd import tnrd

    torch.cuda.set_device(0)
    tnrd.load()
    impl_code = {"auto": tnrd.IMPL_AUTO, "fused": tnrd.IMPL_FUSED, "split": tnrd.IMPL_SPLIT}[args.impl]
    if impl_code == tnrd.IMPL_AUTO:
        impl_code = resolve_auto_impl()
    legs = set(args.legs.split(","))
    if args.calib_copy_mib > 0:
        n = args.calib_copy_mib * (1 << 20) // 4
        src = torch.ones(n, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    fwd = leg_forward(args, impl_code)
    out = {
        "metric": "megapixel-stages/s fwd and fwd+bwd (48x7x7, 8 stages) vs plain FP32 at <=1e-4 rel",
        "value": fwd["value"],
        "unit": "megapixel-stages/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": fwd["ms_per_step"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32", "data": "synthetic",
        "config": {"workload": "plain forward, 1 image 512x512 FP32, L=1, 8 stages x 48 7x7 filters, "
                               "63 Gaussian RBFs/filter, lambda=1, reflective boundary",
                   "global_batch": 1, "H": 512, "W": 512, "stages": 8, "filters": 48, "ksize": 7,
                   "impl": fwd["impl"]},
        "roofline": fwd["roofline"],
        "min_ms_per_step": fwd["min_ms"],
    }
    if "fwd_bwd" in legs:
        out["fwd_bwd"] = leg_fwd_bwd(args)
    if "batched" in legs:
        out["batched"] = leg_batched(args)
    if "mixed" in legs:
        out["mixed"] = leg_mixed(args)
    if "fused_vs_split" in legs:
        out["fused_vs_split"] = leg_fused_vs_split(args)
    if "projected" in legs:
        out["projected"] = leg_projected(args)
    if "denoise" in legs:
        out["denoise"] = leg_denoise(args)
    if "train" in legs:
        out["train"] = leg_train(args)
    if "peaks" in legs:
        out["peaks"] = leg_peaks(args)
        out["fractions"] = fractions(out)
    pin = out["mixed"].pop("_patch_inputs", None) if "mixed" in out else None
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(fwd["f"], fwd["m"], args.cpu_rows)
        if pin is not None:
            out["mixed"].update(mixed_vs_oracle(pin))
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
