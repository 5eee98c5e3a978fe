"""Pins of the fixed-point oracle (the datapath of Section IV-C, readings F1-F8 in
oracle/ocd_oracle.c) against what the mathematics fixes: the reciprocal unit's
error against the true reciprocal, exact recovery where every rounding is
absorbed, closeness to the pinned floating-point oracle on the same (dequantised)
inputs, the zero mean of round-half-up errors, saturation and clipping in closed
form, and the 36-bit range check.  All on the CPU."""

import math

import numpy as np
import pytest

import oracle
import synth

LSB = 2.0 ** -11


def q11(a, scale=1.0):
    """complex -> int16 (re, im) pairs in Q5.11, rounded half up, saturated."""
    a = np.asarray(a, np.complex128) * scale
    v = np.stack([a.real, a.imag], axis=-1) * 2048.0
    return np.clip(np.floor(v + 0.5), -32768, 32767).astype(np.int16)


def deq(a):
    a = np.asarray(a, np.float64)
    return (a[..., 0] + 1j * a[..., 1]) / 2048.0


def fixed_workload(B, U, W, S, Q, snr, seed):
    """A synth slot at the fixed-point scale of reading F2 (H and y times sqrt(B),
    N0 times B: unit-power channel entries, the same OCD estimate)."""
    wl = synth.make_workload(B, U, W, S, Q, snr, seed=seed, dtype=np.complex128)
    c = math.sqrt(B)
    return q11(wl["H"], c), q11(wl["y"], c), wl["N0"] * B, wl


@pytest.mark.parametrize("octave", range(17, 31))
def test_reciprocal_unit_error_bound(octave):
    """F5: an 11-bit index into a table of interval midpoints puts the normalised
    input within 2^-12 (relative) of the point whose reciprocal is stored; the
    18-bit entry and the final rounding to Q.11 add at most 2^-18 and half an LSB."""
    rng = np.random.default_rng(octave)
    xs = rng.integers(1 << octave, 1 << (octave + 1), 400)
    for x in xs:
        d = oracle.fx_recip(int(x))
        if d >= 32767:
            continue                               # saturated (F6)
        exact = 2.0 ** 33 / float(x)               # 1 / (x 2^-22) in Q.11 units
        assert abs(d - exact) <= exact * (2.0 ** -12 + 2.0 ** -18) + 0.5, (x, d, exact)


def test_reciprocal_of_zero_and_saturation():
    assert oracle.fx_recip(0) == 0
    assert oracle.fx_recip(1) == 32767          # 2^22 in Q.11 saturates


@pytest.mark.parametrize("mode,K", [("mmse", 1), ("mmse", 3), ("box", 1), ("box", 3)])
def test_exact_orthogonal_channels_recover_the_symbols(mode, K):
    """Columns 2^11 * (1, j, -1, -j) e_u on distinct antennas, y = H s exactly, no
    regulariser: OCD's fixed point is z = s.  The reciprocal's relative error is
    at most 2^-12 (F5), i.e. below half an LSB of a component of magnitude < 1, and
    the residual stays exactly zero, so the fixed-point z is s bit for bit
    (conjugates, the cancelling shifts, p z and the residual update all enter).
    The components stay inside the 16-QAM box (edge 3/sqrt(10))."""
    B, U = 12, 4
    phases = [1, 1j, -1, -1j]
    H = np.zeros((1, U, B), np.complex128)
    for u in range(U):
        H[0, u, 3 * u] = phases[u]
    s = np.array([0.5 + 0.25j, -0.75 + 0.125j, 0.375 - 0.875j, -0.5 - 0.5j])
    y = (s @ H[0])[None, None, :]
    z, _ = oracle.ocd_fixed(q11(H), q11(y), K, 4, mode, N0=1e-12)
    assert np.array_equal(deq(z)[0, 0], s)


@pytest.mark.parametrize("B,U,mode", [(128, 8, "mmse"), (128, 8, "box"), (100, 6, "mmse"),
                                      (32, 8, "box")])
def test_close_to_the_floating_point_oracle(B, U, mode):
    """On the dequantised inputs the floating-point oracle is the datapath without
    rounding: the fixed-point z stays within 4 LSB (K = 3; each narrowing adds at
    most half an LSB, amplified by at most the few updates that feed a component)."""
    Hq, yq, N0, _ = fixed_workload(B, U, 6, 4, 6, 20.0, [61, B, U])
    z, _ = oracle.ocd_fixed(Hq, yq, 3, 6, mode, N0=N0)
    zf = oracle.ocd(deq(Hq), deq(yq), 3, 6, mode, N0=N0)
    err = np.abs(deq(z) - zf) / LSB
    assert err.max() <= 4.0, err.max()


def test_rounding_is_unbiased():
    """F6 rounds half up: over many vectors the mean signed error of z against the
    floating-point oracle is a small fraction of an LSB (truncation would bias
    every narrowing by -1/2 LSB)."""
    Hq, yq, N0, _ = fixed_workload(64, 8, 40, 4, 4, 15.0, [62])
    z, _ = oracle.ocd_fixed(Hq, yq, 3, 4, "mmse", N0=N0)
    zf = oracle.ocd(deq(Hq), deq(yq), 3, 4, "mmse", N0=N0)
    d = (deq(z) - zf) / LSB
    assert abs(d.real.mean()) < 0.1 and abs(d.imag.mean()) < 0.1, (d.real.mean(), d.imag.mean())


def test_saturation_and_box_clip_closed_form():
    """One user, h = 1/2, y = 16 - 2^-11: the unconstrained c is ~32 and saturates to
    the largest Q5.11 word; in BOX mode it is clipped to beta; a negative y gives
    the most negative word / -beta."""
    H = q11(np.full((1, 1, 1), 0.5))
    for sign, sat in ((1, 32767), (-1, -32768)):
        y = np.array([[[[sign * 32767, 0]]]], np.int16)
        z, _ = oracle.ocd_fixed(H, y, 1, 2, "mmse", N0=1e-12)
        assert tuple(z[0, 0, 0]) == (sat, 0)
        zb, _ = oracle.ocd_fixed(H, y, 1, 2, "box", N0=0.1, beta=0.75)
        assert tuple(zb[0, 0, 0]) == (sign * 1536, 0)


def test_llr_signs_are_the_sliced_bits_of_the_fixed_point_estimate():
    """F8: the LLRs are the max-log LLRs of z_fx / mu; their signs are the bits of
    the nearest constellation point to it."""
    Hq, yq, N0, wl = fixed_workload(64, 8, 10, 3, 6, 25.0, [63])
    z, L = oracle.ocd_fixed(Hq, yq, 3, 6, "mmse", N0=N0)
    assert np.mean((L > 0).astype(np.uint8) != wl["bits"]) < 0.01
    pts, labels = oracle.constellation(6)
    bits = (labels[:, None] >> np.arange(5, -1, -1)) & 1
    G = np.sum(deq(Hq).real ** 2 + deq(Hq).imag ** 2, axis=2)      # [W, U]
    zd = deq(z)
    for w in range(10):
        for s in range(3):
            for u in range(8):
                mu = round(G[w, u] / (G[w, u] + N0) * 2048) / 2048   # p within one LSB
                x = zd[w, s, u] / mu
                nearest = np.argmin(np.abs(x - pts))
                agree = (L[w, s, u] > 0).astype(int) == bits[nearest]
                # a decision may differ only where the LLR is within rounding of 0
                assert np.all(agree | (np.abs(L[w, s, u]) < 1e-2 * np.abs(L[w, s, u]).max()))


def test_36_bit_range_is_enforced():
    """An inner product that does not fit the 36-bit adder tree is an error, not a
    silently different sum."""
    B = 1024
    H = np.full((1, 1, B, 2), 32767, np.int16)
    y = np.full((1, 1, B, 2), 32767, np.int16)
    with pytest.raises(ValueError):
        oracle.ocd_fixed(H, y, 1, 2, "mmse", N0=1.0)


def test_regulariser_must_fit_the_adder():
    """F4: alpha = round(lambda 2^22) is an operand of the 36-bit adder beside
    ||h_u||^2; a lambda whose alpha reaches 2^35 (lambda >= 8192) is rejected, one
    well inside it is not."""
    Hq, yq, N0, _ = fixed_workload(32, 4, 2, 2, 4, 10.0, [64])
    oracle.ocd_fixed(Hq, yq, 2, 4, "mmse", N0=4000.0)
    with pytest.raises(ValueError):
        oracle.ocd_fixed(Hq, yq, 2, 4, "mmse", N0=8192.0)
    with pytest.raises(ValueError):
        oracle.ocd_fixed(Hq, yq, 2, 4, "mmse", N0=1e7)


def test_box_bound_beyond_the_word_clips_nothing():
    """F4, F6: c is narrowed to a 16-bit word before the clip, so a box bound of 16
    or more leaves BOX mode with no regulariser and no clip: bit for bit the MMSE
    iteration with alpha = 0 (N0 so small that round(N0 2^22) = 0).  At low SNR
    some components of c exceed the constellation edge, so the edge bound would
    clip (checked: it changes z)."""
    Hq, yq, _, _ = fixed_workload(64, 8, 6, 3, 4, 0.0, [65])
    zb, _ = oracle.ocd_fixed(Hq, yq, 3, 4, "box", N0=0.1, beta=1e30)
    zb16, _ = oracle.ocd_fixed(Hq, yq, 3, 4, "box", N0=0.1, beta=16.0)
    zm, _ = oracle.ocd_fixed(Hq, yq, 3, 4, "mmse", N0=1e-9)
    ze, _ = oracle.ocd_fixed(Hq, yq, 3, 4, "box", N0=0.1)
    assert np.array_equal(zb, zm) and np.array_equal(zb16, zm)
    assert not np.array_equal(ze, zm)
