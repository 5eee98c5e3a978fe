"""Seeded synthetic uplink workloads for OCD detection.

This module is the one place that makes inputs; it serves both the FP64
oracle (``oracle/``) and the HIP detector (``paper_1611_08779_amd``) and
holds none of the detector's arithmetic.  It models the transmitter and the
channel only:

* Section II-A, the OFDM uplink model ``y_w = H_w s_w + n_w``
  (equation ``eq:OFDMsystem``): one channel matrix per subcarrier, i.i.d.
  circularly-symmetric Gaussian noise of variance ``N0`` per complex entry.
  The noise vector has B entries (the paper's text gives it dimension U,
  a typo: it is added to the B-dimensional receive vector).
* Section II-A, Gray-mapped square QAM with unit average energy
  ``E|s|^2 = 1`` (then scaled by ``sqrt(Es)``).

Conventions (stated once here, implemented independently by the oracle and
the kernels, never shared as code):

* Square QAM with ``Q`` in {2, 4, 6} bits.  Each axis carries ``Q/2`` bits,
  MSB first; the in-phase bits come first, then the quadrature bits.  The
  per-axis label of level index ``m`` (levels in increasing amplitude) is the
  binary-reflected Gray code ``m ^ (m >> 1)``.  Level ``m`` has amplitude
  ``(2m - M + 1) / sqrt(2 (M^2 - 1) / 3)`` with ``M = 2**(Q/2)``, which gives
  unit average symbol energy.
* Rayleigh fading: entries of ``H_w`` i.i.d. CN(0, 1/B), so that every
  column has unit expected squared norm; independent across subcarriers and
  fixed across the ``S`` OFDM symbols that share a subcarrier (block fading).
* SNR: ``N0 = Es * 10**(-snr_db/10)`` (per-user receive SNR, since
  ``E||h_u||^2 = 1``).  The paper's own SNR per bit (Section III-D) is
  ``Eb/N0 = E||s||^2 / (Q E||n||^2)``; :func:`ebn0_db` converts.

Memory layouts (interleaved complex, C order):

* ``H``    ``[W][U][B]``  column ``h_u`` of subcarrier ``w`` contiguous
* ``y``    ``[W][S][B]``
* ``s``    ``[W][S][U]``
* ``bits`` ``[W][S][U][Q]`` uint8, bit 0 = first (MSB of the I axis)
"""

from __future__ import annotations

import math

import numpy as np

__all__ = [
    "n0_from_snr",
    "ebn0_db",
    "qam_modulate",
    "rayleigh_channel",
    "make_workload",
    "batched_job_list",
    "ofdm_used_bins",
    "ofdm_time_domain",
    "ofdm_time_domain_device",
]


def n0_from_snr(snr_db: float, Es: float = 1.0) -> float:
    """Noise variance per complex entry for a per-user receive SNR in dB."""
    return float(Es) * 10.0 ** (-float(snr_db) / 10.0)


def ebn0_db(snr_db: float, B: int, U: int, Q: int) -> float:
    """The paper's SNR per bit (Section III-D) for the same noise level.

    E||s||^2 = U Es and E||n||^2 = B N0, so Eb/N0 = U Es / (Q B N0).
    """
    return float(snr_db) + 10.0 * math.log10(U / (Q * B))


def _axis_amplitudes(M: int) -> np.ndarray:
    # transmitter-side level table: M equally spaced levels, unit energy over 2 axes
    scale = math.sqrt(2.0 * (M * M - 1) / 3.0)
    return np.array([(2 * m - M + 1) / scale for m in range(M)], dtype=np.float64)


def _label_to_level(M: int) -> np.ndarray:
    # inverse of the binary-reflected Gray code: level index that carries a label
    inv = np.empty(M, dtype=np.int64)
    for m in range(M):
        inv[m ^ (m >> 1)] = m
    return inv


def qam_modulate(bits: np.ndarray, Q: int, Es: float = 1.0) -> np.ndarray:
    """Map ``[..., Q]`` bits (uint8) to Gray square-QAM symbols (complex128)."""
    if Q not in (2, 4, 6):
        raise ValueError("Q must be 2, 4 or 6")
    half = Q // 2
    M = 1 << half
    amp = _axis_amplitudes(M)
    lvl = _label_to_level(M)
    bits = np.asarray(bits, dtype=np.int64)
    weights = 1 << np.arange(half - 1, -1, -1)
    lab_i = (bits[..., :half] * weights).sum(-1)
    lab_q = (bits[..., half:] * weights).sum(-1)
    return math.sqrt(Es) * (amp[lvl[lab_i]] + 1j * amp[lvl[lab_q]])


def rayleigh_channel(rng: np.random.Generator, W: int, U: int, B: int) -> np.ndarray:
    """``[W][U][B]`` i.i.d. CN(0, 1/B) entries (complex128)."""
    sd = math.sqrt(0.5 / B)
    return rng.normal(0.0, sd, (W, U, B)) + 1j * rng.normal(0.0, sd, (W, U, B))


def make_workload(B: int, U: int, W: int, S: int, Q: int, snr_db: float,
                  seed, Es: float = 1.0, dtype=np.complex64,
                  channel: np.ndarray | None = None) -> dict:
    """One seeded slot: W subcarriers x S OFDM symbols sharing ``H_w``.

    Everything is drawn in FP64 and ``H`` and ``y`` are then cast to
    ``dtype``; consumers that need FP64 must promote the cast values, so that
    every side sees exactly the same inputs.
    """
    rng = np.random.default_rng(seed)
    N0 = n0_from_snr(snr_db, Es)
    H = rayleigh_channel(rng, W, U, B) if channel is None else np.asarray(channel, np.complex128)
    bits = rng.integers(0, 2, size=(W, S, U, Q), dtype=np.uint8)
    s = qam_modulate(bits, Q, Es)
    sd = math.sqrt(0.5 * N0)
    n = rng.normal(0.0, sd, (W, S, B)) + 1j * rng.normal(0.0, sd, (W, S, B))
    # y[w, s, b] = sum_u H[w, u, b] s[w, s, u] + n[w, s, b]
    y = np.einsum("wub,wsu->wsb", H, s) + n
    return {
        "H": np.ascontiguousarray(H.astype(dtype)),
        "y": np.ascontiguousarray(y.astype(dtype)),
        "s": s,
        "bits": bits,
        "N0": N0,
        "Es": float(Es),
        "snr_db": float(snr_db),
        "ebn0_db": ebn0_db(snr_db, B, U, Q),
        "shape": dict(B=B, U=U, W=W, S=S, Q=Q),
    }


def batched_job_list(n_jobs: int = 48, seed: int = 4) -> list[dict]:
    """Uneven detection jobs: B, U, W and K drawn uniformly and independently.

    B from {64, 128, 256}, U from {4, 8, 16, 32}, W from {300, 1200, 3300},
    K from {2, 3, 4}; 64-QAM, MMSE mode, S = 14 symbols sharing each H_w.
    """
    rng = np.random.default_rng(seed)
    jobs = []
    for j in range(n_jobs):
        jobs.append(dict(
            B=int(rng.choice([64, 128, 256])),
            U=int(rng.choice([4, 8, 16, 32])),
            W=int(rng.choice([300, 1200, 3300])),
            K=int(rng.choice([2, 3, 4])),
            S=14, Q=6, snr_db=20.0, seed=[4, j],
        ))
    return jobs


def make_workload_device(B: int, U: int, W: int, S: int, Q: int, snr_db: float, seed: int,
                         Es: float = 1.0, device="cuda"):
    """The same model as :func:`make_workload`, drawn with torch's seeded RNG on the
    device (for the large benchmark workloads).  Returns a dict with ``H``
    complex64 ``[W,U,B]``, ``y`` complex64 ``[W,S,B]``, ``bits`` uint8
    ``[W,S,U,Q]`` (device tensors) and ``N0``.  ``y = H s + n`` is formed in
    complex64 on the device."""
    import torch

    gen = torch.Generator(device=device)
    gen.manual_seed(int(seed))
    N0 = n0_from_snr(snr_db, Es)
    sd = math.sqrt(0.5 / B)

    def cn(shape, std):
        re = torch.randn(shape, generator=gen, device=device, dtype=torch.float32) * std
        im = torch.randn(shape, generator=gen, device=device, dtype=torch.float32) * std
        return torch.complex(re, im)

    H = cn((W, U, B), sd)
    bits = torch.randint(0, 2, (W, S, U, Q), generator=gen, device=device, dtype=torch.uint8)
    half = Q // 2
    M = 1 << half
    amp = torch.tensor(_axis_amplitudes(M), device=device, dtype=torch.float32)
    lvl = torch.tensor(_label_to_level(M), device=device, dtype=torch.long)
    weights = torch.tensor([1 << (half - 1 - i) for i in range(half)], device=device,
                           dtype=torch.long)
    lab_i = (bits[..., :half].long() * weights).sum(-1)
    lab_q = (bits[..., half:].long() * weights).sum(-1)
    s = math.sqrt(Es) * torch.complex(amp[lvl[lab_i]], amp[lvl[lab_q]])        # [W,S,U]
    y = torch.matmul(s, H.contiguous()) + cn((W, S, B), math.sqrt(0.5 * N0))     # [W,S,B]
    return {"H": H.contiguous(), "y": y.contiguous(), "bits": bits, "N0": N0, "Es": float(Es)}


# ---------------------------------------------------------------- OFDM transmitter side

def ofdm_used_bins(N: int, W: int) -> np.ndarray:
    """DFT bin that carries subcarrier w (the transmitter's mapping, LTE style):
    the W/2 lowest subcarriers on the negative frequencies -W/2 .. -1 (bins
    N - W/2 .. N - 1), the others on +1 .. +W/2; DC is left empty."""
    if W % 2 or W // 2 >= N // 2:
        raise ValueError("W must be even and below N - 1")
    w = np.arange(W)
    return np.where(w < W // 2, N - W // 2 + w, w - W // 2 + 1)


def ofdm_time_domain(y: np.ndarray, N: int, Ncp: int) -> np.ndarray:
    """Receive antennas' time-domain samples whose OFDM demodulation is ``y``.

    ``y`` [W][S][B] (frequency domain, the detector's layout) -> ``x``
    [B][S][Ncp + N] complex128: per antenna and symbol the W values are placed on
    their bins (zeros elsewhere), transformed by the unitary inverse DFT, and the
    last Ncp samples are prepended as the cyclic prefix (Section II-A: with a
    cyclic prefix at least as long as the channel, this is the same model)."""
    W, S, B = y.shape
    full = np.zeros((B, S, N), np.complex128)
    full[:, :, ofdm_used_bins(N, W)] = np.transpose(np.asarray(y, np.complex128), (2, 1, 0))
    sym = np.fft.ifft(full, axis=-1) * math.sqrt(N)
    return np.concatenate([sym[..., N - Ncp:], sym], axis=-1)


def ofdm_time_domain_device(y, N: int, Ncp: int):
    """:func:`ofdm_time_domain` with torch on the device: complex64 [W][S][B] ->
    complex64 [B][S][Ncp + N] (the inverse DFT in complex64)."""
    import torch

    W, S, B = y.shape
    full = torch.zeros((B, S, N), dtype=torch.complex64, device=y.device)
    bins = torch.as_tensor(ofdm_used_bins(N, W), device=y.device)
    full[:, :, bins] = y.permute(2, 1, 0)
    sym = torch.fft.ifft(full, dim=-1) * math.sqrt(N)
    return torch.cat([sym[..., N - Ncp:], sym], dim=-1).contiguous()
