"""GPU parity of ocd_ofdm_demodulate (Section II-A's OFDM demodulation) against the
FP64 oracle, through the C ABI.  Tolerance: an FP32 radix-8 FFT's error grows like
c log2(N) u ||x|| (u = 2^-24); per (antenna, symbol) the used bins are within 1e-5
of the oracle's in relative L2 norm."""

import numpy as np
import pytest
import torch

import oracle
import synth
from gpu_util import dev, host, say

pytestmark = pytest.mark.gpu

TOL = 1e-5


@pytest.fixture(scope="module")
def ocd():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_1611_08779_amd as m
    return m


def rel_err(yg, yo):
    """max over (s, b) of ||y_gpu - y_oracle|| / ||y_oracle|| over the W bins."""
    d = np.linalg.norm(yg.astype(np.complex128) - yo, axis=0)
    n = np.linalg.norm(yo, axis=0)
    return float(np.max(d / np.maximum(n, 1e-300)))


@pytest.mark.parametrize("N,Ncp,W,B,S", [
    (256, 18, 180, 5, 3),       # radix 8, 8, 4; several FFTs per workgroup
    (512, 36, 300, 7, 2),       # radix 8 x 3
    (1024, 72, 600, 9, 2),      # radix 8 x 3 and 2
    (2048, 144, 1200, 16, 3),   # LTE 20 MHz: radix 8 x 3 and 4
    (4096, 288, 2400, 3, 2),    # radix 8 x 4, 512 threads per FFT
    (2048, 0, 2046, 2, 1),      # no cyclic prefix, every bin but DC and Nyquist
    (2048, 2048, 2, 3, 5),      # a prefix as long as the symbol, two subcarriers
    # batches large enough for the bigger workgroups on a 256-CU GPU
    (256, 18, 180, 64, 128),    # 1024 threads, 32 FFTs per workgroup
    (512, 36, 300, 64, 48),     # 512 threads (1024 would leave CUs idle)
    (4096, 288, 2400, 64, 8),   # 1024 threads, 2 FFTs per workgroup
])
def test_random_signals(ocd, N, Ncp, W, B, S):
    say("ofdm case N=%d Ncp=%d W=%d B=%d S=%d" % (N, Ncp, W, B, S))
    rng = np.random.default_rng([90, N, W])
    x = (rng.normal(size=(B, S, Ncp + N)) + 1j * rng.normal(size=(B, S, Ncp + N))).astype(np.complex64)
    y = ocd.ofdm_demodulate(dev(x), N, Ncp, W)
    torch.cuda.synchronize()
    e = rel_err(host(y), oracle.ofdm_demodulate(x, N, Ncp, W))
    say("  rel err %.3g" % e)
    assert e <= TOL


def test_single_tones_land_on_their_subcarriers(ocd):
    N, Ncp, W = 2048, 144, 1200
    n = np.arange(-Ncp, N)
    freqs = [-600, -1, 1, 600, 0, 601, -601]
    x = np.stack([np.exp(2j * np.pi * f * n / N) for f in freqs])[:, None, :].astype(np.complex64)
    y = host(ocd.ofdm_demodulate(dev(x), N, Ncp, W))[:, 0, :]   # [W, tones]
    for i, f in enumerate(freqs):
        col = np.abs(y[:, i])
        if f == 0 or abs(f) > W // 2:
            assert col.max() < 1e-3 * np.sqrt(N)
        else:
            w = f + W // 2 if f < 0 else f + W // 2 - 1
            assert abs(col[w] - np.sqrt(N)) < 1e-4 * np.sqrt(N)
            assert np.delete(col, w).max() < 1e-3 * np.sqrt(N)


def test_headline_slot_front_end_then_detection(ocd):
    """B=128 antennas, 1200 of 2048 subcarriers, 14 symbols, CP 144: the time-domain
    slot built from the frequency-domain model demodulates back to it, and OCD on
    the demodulated vectors gives the detector's results on the model's vectors."""
    B, U, W, S, Q, K, N, Ncp = 128, 8, 1200, 14, 6, 3, 2048, 144
    wl = synth.make_workload(B, U, W, S, Q, 20.0, seed=[91])
    x = synth.ofdm_time_domain(wl["y"], N, Ncp).astype(np.complex64)
    y = ocd.ofdm_demodulate(dev(x), N, Ncp, W)
    torch.cuda.synchronize()
    yo = oracle.ofdm_demodulate(x[:, :, :], N, Ncp, W)
    assert rel_err(host(y), yo) <= TOL
    assert rel_err(host(y), wl["y"].astype(np.complex128)) <= TOL
    N0 = float(np.float32(wl["N0"]))
    H = dev(wl["H"])
    _, L1, _ = ocd.detect(H, y, K, Q, "mmse", N0)
    _, L2, _ = ocd.detect(H, dev(wl["y"]), K, Q, "mmse", N0)
    torch.cuda.synchronize()
    L1, L2 = host(L1), host(L2)
    assert np.max(np.abs(L1 - L2)) <= 1e-3 * np.max(np.abs(L2))
    flips = int(np.sum((L1 > 0) != (L2 > 0)))
    say("decisions changed by the front end: %d of %d" % (flips, L1.size))
    assert flips <= 20
