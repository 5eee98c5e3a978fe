"""Box-constrained OCD at full size: B=256 antennas, U=32 users, 3300 subcarriers x
14 symbols, QPSK and 16-QAM, the box at the constellation edge, K=5, SNR from 0 to
20 dB in 2 dB steps, FP32 and FP16 storage of H and y.  Every slot is detected
whole on the GPU through the C ABI; its outputs at four subcarriers (56 vectors)
are compared with the FP64 oracle: FP32 z within 1e-4 and LLRs within 1e-3, FP16
storage z within 3e-3 of the oracle on the unrounded inputs; and the FP16 path's
bit errors are within 2% of the FP32 path's on the same noise wherever the FP32
path makes at least 500 errors."""

import numpy as np
import pytest
import torch

import synth
from gpu_util import (LLR_TOL_F32, Z_TOL_F16, Z_TOL_F32, host, llr_rel_err, oracle_ref, say,
                      z_rel_err)

pytestmark = pytest.mark.gpu

B, U, W, S, K = 256, 32, 3300, 14, 5


@pytest.fixture(scope="module")
def ocd():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_1611_08779_amd as m
    return m


@pytest.mark.parametrize("Q", [2, 4])
def test_snr_sweep(ocd, Q):
    dev = torch.device("cuda:0")
    ws = np.sort(np.random.default_rng(Q).choice(W, 4, replace=False))
    for snr in range(0, 21, 2):
        say("box B=256 U=32 W=3300 S=14 Q=%d K=5 snr=%d dB" % (Q, snr))
        wl = synth.make_workload_device(B, U, W, S, Q, float(snr), seed=7000 + 100 * Q + snr,
                                        device=dev)
        N0 = float(np.float32(wl["N0"]))
        z32, L32, _ = ocd.detect(wl["H"], wl["y"], K, Q, "box", N0)
        h16 = torch.view_as_real(wl["H"]).to(torch.float16).contiguous()
        y16 = torch.view_as_real(wl["y"]).to(torch.float16).contiguous()
        z16, L16, _ = ocd.detect(h16, y16, K, Q, "box", N0, storage="f16")
        torch.cuda.synchronize()
        # the slot's own outputs at the sampled subcarriers against the oracle
        zo, Lo, _ = oracle_ref(host(wl["H"][ws]), host(wl["y"][ws]), K, Q, "box", N0)
        ez = z_rel_err(host(z32[ws]), zo)
        el = llr_rel_err(host(L32[ws]), Lo)
        ez16 = z_rel_err(host(z16[ws]), zo)
        bits = wl["bits"]
        e32 = int(((L32 > 0).to(torch.uint8) != bits).sum().item())
        e16 = int(((L16 > 0).to(torch.uint8) != bits).sum().item())
        say("  z err %.2g llr err %.2g fp16 z err %.2g; bit errors fp32 %d fp16 %d of %d"
            % (ez, el, ez16, e32, e16, bits.numel()))
        assert ez <= Z_TOL_F32 and el <= LLR_TOL_F32
        assert ez16 <= Z_TOL_F16
        if e32 >= 500:
            assert abs(e16 - e32) <= 0.02 * e32
        del wl, z32, L32, z16, L16, h16, y16
