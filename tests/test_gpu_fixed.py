"""GPU parity of ocd_detect_fixed (the fixed-point datapath of Section IV-C)
against the fixed-point oracle, through the C ABI.  z is integer work: bit-exact.
The LLRs are formed in FP32 on the GPU and in FP64 by the oracle from the same
integer z and p: within 1e-3 of the vector's largest, the bar of the
floating-point path."""

import numpy as np
import pytest
import torch

import oracle
from gpu_util import LLR_TOL_F32, dev, host, llr_rel_err, say
from test_oracle_fixed_pins import deq, fixed_workload, q11

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ocd():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_1611_08779_amd as m
    return m


def f32(x):
    return float(np.float32(x))


def run_fixed(ocd, Hq, yq, K, Q, mode, N0, Es=1.0, beta=0.0):
    N0 = f32(N0)
    z, L = ocd.detect_fixed(dev(Hq), dev(yq), K, Q, mode, N0, Es, beta)
    torch.cuda.synchronize()
    zo, Lo = oracle.ocd_fixed(Hq, yq, K, Q, mode, N0=N0, Es=Es, beta=f32(beta), threads=0)
    zg = host(z)
    mism = int(np.sum(zg != zo))
    el = llr_rel_err(host(L), Lo)
    say("  z words differing: %d of %d, llr err %.3g" % (mism, zo.size, el))
    assert mism == 0
    assert el <= LLR_TOL_F32
    return zg, host(L)


@pytest.mark.parametrize("B,U,W,S,Q,K,mode,snr", [
    (128, 8, 40, 14, 6, 3, "mmse", 20.0),   # the headline shape, a slice
    (128, 8, 40, 14, 6, 3, "box", 20.0),
    (32, 8, 30, 4, 6, 4, "box", 15.0),      # the smallest array of the paper
    (64, 8, 30, 4, 4, 2, "mmse", 10.0),
    (100, 6, 20, 3, 6, 3, "mmse", 18.0),    # B not a power of two (b = 7)
    (33, 4, 20, 2, 2, 3, "box", 8.0),       # odd B
    (256, 16, 8, 3, 4, 3, "mmse", 20.0),    # NPL = 16
    (512, 8, 4, 2, 6, 3, "box", 20.0),      # L = 32, NPL = 16
    (1024, 4, 2, 2, 4, 2, "mmse", 20.0),    # the largest B (NPL = 32)
    (64, 32, 6, 2, 4, 3, "mmse", 25.0),     # the largest U
    (16, 1, 12, 5, 6, 1, "box", 10.0),      # one user, one sweep
])
def test_bit_exact(ocd, B, U, W, S, Q, K, mode, snr):
    say("fixed case B=%d U=%d W=%d S=%d Q=%d K=%d %s %s dB" % (B, U, W, S, Q, K, mode, snr))
    Hq, yq, N0, _ = fixed_workload(B, U, W, S, Q, snr, [70, B, U])
    run_fixed(ocd, Hq, yq, K, Q, mode, N0)


def test_symbol_energy_and_given_box(ocd):
    Hq, yq, N0, _ = fixed_workload(64, 8, 10, 4, 4, 12.0, [71])
    run_fixed(ocd, Hq, yq, 3, 4, "box", N0, Es=1.0, beta=0.8)
    run_fixed(ocd, Hq, yq, 3, 4, "box", N0, Es=1.0, beta=1e30)   # beyond the word range: no clip
    wl_scale = np.sqrt(2.0)
    run_fixed(ocd, Hq, np.clip(np.round(yq * wl_scale), -32768, 32767).astype(np.int16), 3, 4,
              "mmse", N0 * 2.0, Es=2.0)


def test_saturation_and_zero_columns(ocd):
    """Saturating words and all-zero columns take the same integer path on both sides."""
    H = q11(np.full((2, 2, 4), 0.5 + 0.25j))
    H[1, 1] = 0
    y = np.full((2, 3, 4, 2), 32767, np.int16)
    y[:, 1] = -32768
    for mode in ("mmse", "box"):
        zg, Lg = run_fixed(ocd, H, y, 2, 4, mode, 1e-3)
        assert np.all(zg[1, :, 1] == 0) and np.all(Lg[1, :, 1] == 0)


def test_headline_full_slot_sampled_and_ber(ocd):
    """B=128, U=8, 1200 x 14, 64-QAM, K=3, 20 dB at the fixed-point scale: the whole
    slot on the GPU; 24 subcarriers bit-exact against the oracle; and the bit
    errors of the fixed-point design within 10% of the FP32 path's on the same
    noise (the paper reports a loss below 0.2 dB)."""
    B, U, W, S, Q = 128, 8, 1200, 14, 6
    Hq, yq, N0, wl = fixed_workload(B, U, W, S, Q, 20.0, [72])
    N0 = f32(N0)
    z, L = ocd.detect_fixed(dev(Hq), dev(yq), 3, Q, "mmse", N0)
    torch.cuda.synchronize()
    ws = np.random.default_rng(72).choice(W, 24, replace=False)
    zo, _ = oracle.ocd_fixed(Hq[ws], yq[ws], 3, Q, "mmse", N0=N0, threads=0)
    assert np.array_equal(host(z)[ws], zo)
    zf, Lf, _ = ocd.detect(dev(deq(Hq).astype(np.complex64)), dev(deq(yq).astype(np.complex64)),
                           3, Q, "mmse", N0)
    torch.cuda.synchronize()
    e_fx = int(np.sum((host(L) > 0) != wl["bits"]))
    e_fp = int(np.sum((host(Lf) > 0) != wl["bits"]))
    say("bit errors: fixed point %d, FP32 %d of %d" % (e_fx, e_fp, wl["bits"].size))
    assert e_fp > 500 and abs(e_fx - e_fp) <= 0.1 * e_fp


def test_rejects_hybrid(ocd):
    Hq, yq, N0, _ = fixed_workload(32, 4, 2, 2, 4, 10.0, [73])
    with pytest.raises(ocd.OCDError) as ei:
        ocd.detect_fixed(dev(Hq), dev(yq), 2, 4, "hybrid", N0)
    assert ei.value.status == -2
