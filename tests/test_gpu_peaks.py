"""The throughput probes (a measurement aid of the library) run and report
plausible positive rates; argument errors are caught on the host."""
import math

import pytest
import torch

from paper_1702_07482_amd import tnrd

pytestmark = pytest.mark.gpu


def test_measure_peaks_positive_and_finite():
    nbytes = 64 << 20
    src = torch.ones(nbytes // 4, device="cuda")
    dst = torch.empty_like(src)
    sink = torch.empty(tnrd.tnrd_peaks_sink_floats(), device="cuda")
    p = tnrd.tnrd_measure_peaks(src, dst, nbytes, sink)
    torch.cuda.synchronize()
    print("peaks", p, flush=True)
    for k, v in p.items():
        assert math.isfinite(v) and v > 0, (k, v)
    assert torch.equal(dst, src)
    # the k32 BF16 instruction does at least the work per second of the FP32 one
    assert p["mfma_bf16_k32_tflops"] > p["mfma_f32_tflops"]


def test_measure_peaks_rejects_small_copy():
    sink = torch.empty(tnrd.tnrd_peaks_sink_floats(), device="cuda")
    src = torch.ones(1024, device="cuda")
    with pytest.raises(RuntimeError, match="argument"):
        tnrd.tnrd_measure_peaks(src, src.clone(), 4096, sink)
