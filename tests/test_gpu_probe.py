"""The FP32 FMA-rate probe (measurement support): the flop count it reports and a
rate between the non-packed and the packed FP32 vector peaks' plausible range."""

import pytest
import torch

from gpu_util import say

pytestmark = pytest.mark.gpu


def test_fma_probe_rate_is_plausible():
    import paper_1611_08779_amd as ocd
    out = torch.zeros(1024, device="cuda")
    blocks, iters = 2048, 256
    fl = ocd.ocd_probe_fma(blocks, iters, out)
    assert fl == 2.0 * blocks * 256 * iters * 16 * 8
    for _ in range(20):
        ocd.ocd_probe_fma(blocks, iters, out)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(10):
        ocd.ocd_probe_fma(blocks, iters, out)
    e1.record()
    torch.cuda.synchronize()
    tflops = fl * 10 / (e0.elapsed_time(e1) * 1e-3) / 1e12
    say("FP32 FMA rate %.1f TFLOP/s" % tflops)
    # 256 CUs x 64 lanes x 2 flop at 1.5-2.4 GHz without packed FMAs: 49-79 TFLOP/s
    assert 30.0 < tflops < 90.0
    assert float(out.abs().sum()) == 0.0   # the guarded store never fires
