"""The allocation-free forward (tnrd_forward_noalloc, scratch in a fixed device
array) gives the same bits as tnrd_forward on a caller workspace, on two calls
in a row, the second with a smaller input, and matches the FP64 oracle there.

Collected last (tests/test_zz_*) so that a failure here cannot hide another test.
"""
import numpy as np
import pytest
import torch

import oracle
from paper_1702_07482_amd import synth, tnrd
from tests.helpers import rel_inf

pytestmark = pytest.mark.gpu


def _both(f, m, dm, L, opts, want_states):
    N, H, W = f.shape
    abi = dm.abi()
    ns = tnrd.tnrd_num_checkpoints(abi.T, opts.recompute_every)
    nb = tnrd.tnrd_workspace_bytes(N, H, W, abi, opts, 0)
    assert 0 < nb <= tnrd.NOALLOC_SCRATCH_BYTES
    ws = torch.empty(nb, dtype=torch.uint8, device="cuda")
    u_ref = torch.empty_like(f)
    u_na = torch.full_like(f, float("nan"))
    st_ref = st_na = None
    if want_states:
        st_ref = torch.empty((ns, N, H, W), dtype=torch.float32, device="cuda")
        st_na = torch.full_like(st_ref, float("nan"))
    assert tnrd.tnrd_forward(f, N, H, W, L, abi, u_ref, st_ref, opts, ws, nb) == tnrd.TNRD_OK
    # the workspace of the reference call is freed before the allocation-free one runs
    torch.cuda.synchronize()
    del ws
    assert tnrd.tnrd_forward_noalloc(f, N, H, W, L, abi, u_na, st_na, opts) == tnrd.TNRD_OK
    torch.cuda.synchronize()
    return u_ref, u_na, st_ref, st_na


def test_noalloc_forward_matches_tnrd_forward_twice_then_smaller():
    m = synth.config_model(2)
    dm = tnrd.DeviceModel.from_numpy(m)
    # call 1: the full 512 x 512 image with every state kept
    print("[noalloc call 1: 1 x 512 x 512, 8 x 48 7x7, states]", flush=True)
    _, f1 = synth.make_pair(512, 512, 1, config_id=2, index=0)
    f1d = torch.from_numpy(f1).cuda()[None].contiguous()
    u_ref, u_na, st_ref, st_na = _both(f1d, m, dm, 1, tnrd.default_opts(), True)
    assert torch.equal(u_ref, u_na)
    assert torch.equal(st_ref, st_na)
    # call 2: a smaller batch, checkpoints every 3 stages; the array still holds
    # call 1's planes and prepared constants, none of which may leak into call 2
    print("[noalloc call 2: 2 x 64 x 80, checkpoints every 3 stages]", flush=True)
    pairs = [synth.make_pair(64, 80, 1, config_id=2, index=40 + i) for i in range(2)]
    f2 = np.stack([p[1] for p in pairs])
    f2d = torch.from_numpy(f2).cuda()
    o2 = tnrd.default_opts(recompute_every=3)
    u_ref2, u_na2, st_ref2, st_na2 = _both(f2d, m, dm, 1, o2, True)
    assert torch.equal(u_ref2, u_na2)
    assert torch.equal(st_ref2, st_na2)
    ref = oracle.forward(f2, m)
    err = rel_inf(u_na2.cpu().numpy(), ref)
    print(f"noalloc 2 x 64 x 80 vs oracle: {err:.2e}", flush=True)
    assert err <= 1e-4


def test_noalloc_forward_mixed_precision_and_ragged():
    """BF16 operands (the same kernels tnrd_forward picks) and a ragged image."""
    m = synth.config_model(2)
    dm = tnrd.DeviceModel.from_numpy(m)
    print("[noalloc BF16: 1 x 97 x 131]", flush=True)
    _, f = synth.make_pair(97, 131, 1, config_id=2, index=7)
    fd = torch.from_numpy(f).cuda()[None].contiguous()
    u_ref, u_na, _, _ = _both(fd, m, dm, 1, tnrd.default_opts(prec=tnrd.PREC_BF16), False)
    assert torch.equal(u_ref, u_na)
