"""Batched uneven forward (tnrd_forward_batched: one launch per stage over the
tiles of every image, or one persistent launch over every (stage, tile),
replayed from a HIP graph) against per-image tnrd_forward and the FP64
oracle."""
import numpy as np
import pytest
import torch

import oracle
from paper_1702_07482_amd import autotune, synth, tnrd
from tests.helpers import oracle_uT_at, rel_inf

pytestmark = pytest.mark.gpu

TOL = 1e-4


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).cuda()


def _models(looks, cfg=4):
    return {L: synth.config_model(cfg, look=L) for L in sorted(set(looks))}


def _per_image(f, m, L, opts):
    dm = tnrd.DeviceModel.from_numpy(m, L=L)
    return tnrd.forward(_dev(f), dm, L=L, opts=opts).cpu().numpy()[0]


def test_small_uneven_batch_matches_per_image_and_oracle():
    sizes = [(40, 52), (96, 64), (33, 90), (64, 64), (120, 75), (7, 7)]
    looks = [1, 4, 1, 2, 4, 2]
    ms = _models(looks)
    fs = [synth.make_pair(h, w, L, config_id=4, index=i)[1] for i, ((h, w), L) in enumerate(zip(sizes, looks))]
    dms = [tnrd.DeviceModel.from_numpy(ms[L], L=L) for L in sorted(ms)]
    o = tnrd.default_opts(use_graph=0, validate=1)
    outs, _ = tnrd.forward_batched([_dev(f) for f in fs], looks, dms, opts=o)
    torch.cuda.synchronize()
    fo = tnrd.default_opts(tile_h=32, tile_w=32, wg_waves=8, impl=tnrd.IMPL_FUSED)
    for b, (f, L) in enumerate(zip(fs, looks)):
        ref = _per_image(f, ms[L], L, fo)
        np.testing.assert_array_equal(outs[b].cpu().numpy(), ref, err_msg=f"image {b}")
    for b in (2, 5):
        ref = oracle.forward(fs[b], ms[looks[b]])
        assert rel_inf(outs[b].cpu().numpy(), ref) <= TOL


def test_graph_replay_recomputes_with_new_inputs():
    sizes = [(64, 80), (50, 45), (96, 96)]
    looks = [1, 2, 1]
    ms = _models(looks)
    dms = [tnrd.DeviceModel.from_numpy(ms[L], L=L) for L in sorted(ms)]
    fs = [_dev(synth.make_pair(h, w, L, config_id=4, index=10 + i)[1])
          for i, ((h, w), L) in enumerate(zip(sizes, looks))]
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        og = tnrd.default_opts(use_graph=1)
        outs, ws = tnrd.forward_batched(fs, looks, dms, opts=og)  # records
        for rep in range(3):
            # new contents in the same buffers, then a replay
            for i, f in enumerate(fs):
                f.copy_(_dev(synth.make_pair(*sizes[i], looks[i], config_id=4, index=20 + 3 * rep + i)[1]))
            tnrd.forward_batched(fs, looks, dms, opts=og, outs=outs, ws=ws)
            got = [u.clone() for u in outs]
            ref, _ = tnrd.forward_batched(fs, looks, dms, opts=tnrd.default_opts(use_graph=0))
            s.synchronize()
            for a, b in zip(got, ref):
                torch.testing.assert_close(a, b, rtol=0, atol=0)


def test_model_selection_by_looks():
    ms = _models([1, 4])
    f = synth.make_pair(40, 40, 8, config_id=4, index=30)[1]
    d1 = tnrd.DeviceModel.from_numpy(ms[1], L=1)
    d0 = tnrd.DeviceModel.from_numpy(ms[4], L=0)  # matches any L
    o = tnrd.default_opts(use_graph=0)
    outs, _ = tnrd.forward_batched([_dev(f)], [8], [d1, d0], opts=o)
    ref = oracle.forward(f, ms[4])
    assert rel_inf(outs[0].cpu().numpy(), ref) <= TOL
    with pytest.raises(RuntimeError):
        tnrd.forward_batched([_dev(f)], [8], [d1], opts=o)


def _c4_inputs():
    sizes, looks = synth.c4_batch(64)
    ms = _models(looks)
    dms = [tnrd.DeviceModel.from_numpy(ms[L], L=L) for L in sorted(ms)]
    fs = [synth.make_pair(h, w, L, config_id=4, index=100 + i)[1]
          for i, ((h, w), L) in enumerate(zip(sizes, looks))]
    return sizes, looks, ms, dms, fs


def test_c4_full_batch_every_candidate_tile():
    """64 images from {256x256, 384x512, 512x512, 1024x768}, L in {1,2,4,8}, at
    every tile the autotuner may pick (so whichever it picks on a given GPU is
    covered): sampled images equal per-image tnrd_forward with the same tile bit
    for bit.  The tile the autotuner returns here, and the 96 x 32 x 8-wave tile
    (the tallest candidate), run as graph replays, and their outputs are
    compared with the oracle at sampled pixels (crops covering the receptive
    field)."""
    sizes, looks, ms, dms, fs = _c4_inputs()
    fd = [_dev(f) for f in fs]
    print(f"[c4 batch: {sum(h * w for h, w in sizes) / 1e6:.2f} MP]", flush=True)
    outs, ws = None, None
    tested = 0
    for th, tw, nw in autotune.CANDIDATES:
        o = tnrd.default_opts(tile_h=th, tile_w=tw, wg_waves=nw, use_graph=0)
        try:
            outs, ws = tnrd.forward_batched(fd, looks, dms, opts=o, outs=outs, ws=ws)
        except RuntimeError as e:
            assert "unsupported" in str(e), e
            continue
        torch.cuda.synchronize()
        fo = tnrd.default_opts(tile_h=th, tile_w=tw, wg_waves=nw, impl=tnrd.IMPL_FUSED)
        for b in (0, 17, 40, 63):
            ref = _per_image(fs[b], ms[looks[b]], looks[b], fo)
            np.testing.assert_array_equal(outs[b].cpu().numpy(), ref,
                                          err_msg=f"image {b} tile {th}x{tw}x{nw}")
        tested += 1
    print(f"[c4: {tested} candidate tiles bit-exact]", flush=True)
    assert tested >= 20
    tuned = tuple(autotune.tune_batched(fd, looks, dms))
    print(f"[c4: autotuned tile {tuned}]", flush=True)
    radius = 8 * 6
    for th, tw, nw in sorted({tuned, (96, 32, 8)}):
        o = tnrd.default_opts(tile_h=th, tile_w=tw, wg_waves=nw, use_graph=1, validate=1)
        s = torch.cuda.Stream()
        with torch.cuda.stream(s):
            outs, ws = tnrd.forward_batched(fd, looks, dms, opts=o, outs=outs, ws=ws)  # records
            outs, ws = tnrd.forward_batched(fd, looks, dms, opts=o, outs=outs, ws=ws)  # replays
        s.synchronize()
        for b in (5, 33):
            h, w = sizes[b]
            pts = [(0, 0), (h - 1, w // 2), (h // 2, w - 1), (h // 3, w // 3)]
            ref = oracle_uT_at(fs[b], ms[looks[b]], pts, radius)
            got = np.array([outs[b].cpu().numpy()[p] for p in pts])
            assert np.abs(got - ref).max() <= TOL * np.abs(ref).max(), (th, tw, nw, b, got, ref)


def test_graph_signature_covers_the_reaction():
    """Two calls on the same buffers and parameter tensors that differ only in
    the models' reaction (prox, then projected, then prox): each call's output
    equals the per-image forward of its own model (a cached graph must not
    replay the other reaction)."""
    sizes, looks = [(64, 70), (40, 90)], [1, 1]
    m = synth.config_model(4, look=1)
    fs = [_dev(synth.make_pair(h, w, 1, config_id=4, index=140 + i, peak=8.0)[1])
          for i, (h, w) in enumerate(sizes)]
    dm = tnrd.DeviceModel.from_numpy(m, L=1)
    s = torch.cuda.Stream()
    outs, ws = None, None
    fo = tnrd.default_opts(tile_h=32, tile_w=32, wg_waves=8, impl=tnrd.IMPL_FUSED)
    with torch.cuda.stream(s):
        for react in (tnrd.REACT_PROX, tnrd.REACT_PROJECTED, tnrd.REACT_PROX, tnrd.REACT_PROJECTED):
            dm.reaction = react
            outs, ws = tnrd.forward_batched(fs, looks, [dm], opts=tnrd.default_opts(use_graph=1),
                                            outs=outs, ws=ws)
            got = [u.clone() for u in outs]
            ref = [tnrd.forward(f[None].contiguous(), dm, L=1, opts=fo)[0] for f in fs]
            s.synchronize()
            for a, b in zip(got, ref):
                torch.testing.assert_close(a, b, rtol=0, atol=0)
    assert outs[0].min().item() >= 1.0  # the last call was the projected one


def _persistent_vs_per_stage(fd, looks, dms, th, tw, nw, graph):
    """Outputs of the single persistent launch and of one launch per stage
    (same tile), the persistent one checked for give-ups (validate)."""
    base = dict(tile_h=th, tile_w=tw, wg_waves=nw, use_graph=graph)
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        ref, _ = tnrd.forward_batched(fd, looks, dms, opts=tnrd.default_opts(persistent=0, **base))
        ref = [u.clone() for u in ref]
        po = tnrd.default_opts(persistent=1, validate=0 if graph else 1, **base)
        outs, ws = tnrd.forward_batched(fd, looks, dms, opts=po)
        if graph:  # records, then replays into the same buffers
            outs, ws = tnrd.forward_batched(fd, looks, dms, opts=po, outs=outs, ws=ws)
    s.synchronize()
    return [u.cpu().numpy() for u in outs], [u.cpu().numpy() for u in ref]


def test_persistent_launch_small_uneven_batch():
    """One persistent launch over every (stage, tile) of an uneven batch with
    per-look models (Sec. 4.5), tiles from 1 x 1 to 4 x 3 per image: bit for bit
    the per-stage launches, and the oracle at whole images."""
    sizes = [(40, 52), (96, 64), (33, 90), (64, 64), (120, 75), (7, 7)]
    looks = [1, 4, 1, 2, 4, 2]
    ms = _models(looks)
    fs = [synth.make_pair(h, w, L, config_id=4, index=i)[1] for i, ((h, w), L) in enumerate(zip(sizes, looks))]
    dms = [tnrd.DeviceModel.from_numpy(ms[L], L=L) for L in sorted(ms)]
    print("[persistent: small uneven batch, 32x32x8, direct launch]", flush=True)
    got, ref = _persistent_vs_per_stage([_dev(f) for f in fs], looks, dms, 32, 32, 8, 0)
    for b in range(len(fs)):
        np.testing.assert_array_equal(got[b], ref[b], err_msg=f"image {b}")
    for b in (2, 4, 5):
        assert rel_inf(got[b], oracle.forward(fs[b], ms[looks[b]])) <= TOL


def test_persistent_launch_c4_batch():
    """The 64-image batch of 256x256 .. 1024x768 images, L in {1, 2, 4, 8}: the
    persistent launch at the autotuned tile and at 96 x 32 x 8 waves, directly
    and as a graph replay, equals the per-stage launches on every image bit for
    bit, and the oracle at sampled pixels."""
    sizes, looks, ms, dms, fs = _c4_inputs()
    fd = [_dev(f) for f in fs]
    tuned = tuple(autotune.tune_batched(fd, looks, dms))
    radius = 8 * 6
    for th, tw, nw in sorted({tuned, (96, 32, 8)}):
        for graph in (0, 1):
            print(f"[persistent c4: tile {th}x{tw}x{nw} graph {graph}]", flush=True)
            got, ref = _persistent_vs_per_stage(fd, looks, dms, th, tw, nw, graph)
            for b in range(len(fs)):
                np.testing.assert_array_equal(got[b], ref[b], err_msg=f"image {b} tile {th}x{tw}x{nw}")
        for b in (9, 50):
            h, w = sizes[b]
            pts = [(0, w - 1), (h - 1, 0), (h // 2, w // 2)]
            want = oracle_uT_at(fs[b], ms[looks[b]], pts, radius)
            have = np.array([got[b][p] for p in pts])
            assert np.abs(have - want).max() <= TOL * np.abs(want).max(), (th, tw, nw, b, have, want)
