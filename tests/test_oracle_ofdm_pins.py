"""Pins of the OFDM front-end oracle (Section II-A: cyclic-prefix removal and the
DFT at every receive antenna) against the DFT's definition, single tones, the
inverse transform of the transmitter model, and the cyclic prefix's role.  All
on the CPU."""

import cmath
import math

import numpy as np
import pytest

import oracle
import synth


def test_equals_the_dft_sum():
    """X[k] = N^-1/2 sum_n x[Ncp + n] e^{-2 pi i k n / N} at the used bins, written out."""
    rng = np.random.default_rng(80)
    N, Ncp, W, B, S = 64, 9, 40, 3, 2
    x = rng.normal(size=(B, S, Ncp + N)) + 1j * rng.normal(size=(B, S, Ncp + N))
    y = oracle.ofdm_demodulate(x, N, Ncp, W)
    for b in range(B):
        for s in range(S):
            for w in range(W):
                f = w - W // 2 if w < W // 2 else w - W // 2 + 1   # -W/2..-1, 1..W/2
                acc = sum(x[b, s, Ncp + n] * cmath.exp(-2j * math.pi * f * n / N) for n in range(N))
                assert abs(y[w, s, b] - acc / math.sqrt(N)) < 1e-12


@pytest.mark.parametrize("f", [-100, -1, 1, 37, 100])
def test_single_tone_lands_on_its_subcarrier(f):
    """A tone at frequency f (CP included) appears only on its subcarrier, with
    amplitude sqrt(N); a tone at DC or outside the used band appears nowhere."""
    N, Ncp, W = 256, 18, 200
    n = np.arange(-Ncp, N)
    x = np.exp(2j * math.pi * f * n / N)[None, None, :]
    y = oracle.ofdm_demodulate(x, N, Ncp, W)[:, 0, 0]
    w = f + W // 2 if f < 0 else f + W // 2 - 1
    expect = np.zeros(W, complex)
    expect[w] = math.sqrt(N)
    assert np.max(np.abs(y - expect)) < 1e-9
    for g in (0, W // 2 + 1, -W // 2 - 1):
        xg = np.exp(2j * math.pi * g * n / N)[None, None, :]
        assert np.max(np.abs(oracle.ofdm_demodulate(xg, N, Ncp, W))) < 1e-9


def test_inverts_the_transmitter_model():
    """synth's time-domain samples (unitary inverse DFT of the frequency-domain
    model, CP prepended) demodulate to the frequency-domain model itself."""
    wl = synth.make_workload(16, 4, 300, 3, 4, 10.0, seed=[81], dtype=np.complex128)
    x = synth.ofdm_time_domain(wl["y"], 512, 36)
    y = oracle.ofdm_demodulate(x, 512, 36, 300)
    assert np.max(np.abs(y - wl["y"])) < 1e-12


def test_cyclic_prefix_is_discarded_and_energy_is_preserved():
    rng = np.random.default_rng(82)
    N, Ncp, W = 128, 10, 126
    x = rng.normal(size=(2, 2, Ncp + N)) + 1j * rng.normal(size=(2, 2, Ncp + N))
    y = oracle.ofdm_demodulate(x, N, Ncp, W)
    x2 = x.copy()
    x2[..., :Ncp] = 0
    assert np.array_equal(oracle.ofdm_demodulate(x2, N, Ncp, W), y)
    # Parseval: the used bins carry all the energy but DC's and Nyquist's
    X = np.fft.fft(x[..., Ncp:], axis=-1, norm="ortho")
    rest = np.abs(X[..., 0]) ** 2 + np.abs(X[..., N // 2]) ** 2
    tot = np.sum(np.abs(x[..., Ncp:]) ** 2, axis=-1)
    assert np.allclose(np.sum(np.abs(y) ** 2, axis=0).T + rest, tot, rtol=1e-12)
