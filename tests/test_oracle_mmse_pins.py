"""Pins of the explicit-MMSE oracle (Sections II-B and II-E) against what the
mathematics fixes: the normal equations checked by matrix products, a library
linear solve, the limit of coordinate descent (the pinned OCD oracle at large
K), closed forms for one user and for orthogonal columns, the post-
equalisation SINR computed from the explicit error covariance, and the
transmitted bits at high SNR.  All on the CPU."""

import math

import numpy as np
import pytest
import scipy.linalg

import oracle
import synth

from test_oracle_pins import _exact_mmse_llr_peraxis, _orthogonal_channel


def _wl(B, U, W, S, Q, snr, seed, Es=1.0, **kw):
    return synth.make_workload(B, U, W, S, Q, snr, seed=seed, Es=Es, dtype=np.complex128, **kw)


@pytest.mark.parametrize("B,U,Es", [(16, 4, 1.0), (32, 8, 2.5), (12, 12, 0.7)])
def test_mmse_satisfies_the_normal_equations(B, U, Es):
    """Section II-B: z minimises ||y - Hz||^2 + (N0/Es)||z||^2, i.e.
    H^H (y - H z) = (N0/Es) z, checked with matrix products only."""
    wl = _wl(B, U, 4, 3, 4, 6.0, [40, B, U], Es=Es)
    z, _, _ = oracle.mmse(wl["H"], wl["y"], 4, N0=wl["N0"], Es=Es)
    lam = wl["N0"] / Es
    for w in range(4):
        Hm = wl["H"][w].T                       # [B, U]
        for s in range(3):
            lhs = Hm.conj().T @ (wl["y"][w, s] - Hm @ z[w, s])
            scale = np.linalg.norm(Hm.conj().T @ wl["y"][w, s])
            assert np.linalg.norm(lhs - lam * z[w, s]) <= 1e-11 * scale


def test_mmse_matches_a_library_solve():
    """The same estimate from LAPACK's Hermitian positive definite solver."""
    wl = _wl(64, 16, 3, 2, 6, 15.0, [41])
    z, _, _ = oracle.mmse(wl["H"], wl["y"], 6, N0=wl["N0"])
    for w in range(3):
        Hm = wl["H"][w].T
        A = Hm.conj().T @ Hm + wl["N0"] * np.eye(16)
        ref = scipy.linalg.solve(A, Hm.conj().T @ wl["y"][w].T, assume_a="pos").T
        assert np.max(np.abs(z[w] - ref)) <= 1e-12 * np.max(np.abs(ref))


def test_mmse_is_the_limit_of_coordinate_descent():
    """Section III: OCD in MMSE mode converges to the MMSE estimate; at large K the
    pinned Algorithm-1 oracle reaches the explicit solution."""
    wl = _wl(32, 8, 3, 2, 4, 10.0, [42])
    z, _, _ = oracle.mmse(wl["H"], wl["y"], 4, N0=wl["N0"])
    zk = oracle.ocd(wl["H"], wl["y"], 200, 4, "mmse", N0=wl["N0"])
    assert np.max(np.abs(z - zk)) <= 1e-10


@pytest.mark.parametrize("Es", [1.0, 3.0])
def test_gain_and_sinr_are_those_of_the_error_covariance(Es):
    """Section II-E: z_i = mu_i s_i + e_i with mu_i = [A^-1 G]_ii, and rho_i =
    mu_i/(1 - mu_i) is the SINR mu_i^2 Es / E|e_i|^2.  The test forms E|e_i|^2 from
    the explicit interference and noise terms, takes mu from the identity
    A^-1 G = I - lambda A^-1 (numpy's inverse), and rebuilds every LLR."""
    Q = 6
    wl = _wl(24, 6, 3, 4, Q, 5.0, [43], Es=Es)
    N0 = wl["N0"]
    lam = N0 / Es
    z, L, mu_o = oracle.mmse(wl["H"], wl["y"], Q, N0=N0, Es=Es)
    for w in range(3):
        Hm = wl["H"][w].T
        G = Hm.conj().T @ Hm
        Ainv = np.linalg.inv(G + lam * np.eye(6))
        mu = 1.0 - lam * np.real(np.diag(Ainv))
        np.testing.assert_allclose(mu_o[w], mu, rtol=1e-12)
        assert np.all((mu > 0) & (mu < 1))
        T = Ainv @ G                                   # z = T s + A^-1 H^H n
        for i in range(6):
            interf = Es * (np.sum(np.abs(T[i]) ** 2) - abs(T[i, i]) ** 2)
            noise = N0 * np.real((Ainv @ G @ Ainv)[i, i])
            sinr = mu[i] ** 2 * Es / (interf + noise)
            assert abs(sinr - mu[i] / (1 - mu[i])) <= 1e-10 * sinr
            for s in range(4):
                ref = _exact_mmse_llr_peraxis(z[w, s, i] / (mu[i] * math.sqrt(Es)), sinr, Q)
                np.testing.assert_allclose(L[w, s, i], ref, rtol=1e-9, atol=1e-9)


@pytest.mark.parametrize("Q", [2, 4, 6])
def test_single_user_closed_form(Q):
    """U = 1: z = h^H y / (||h||^2 + lambda), mu = g/(g + lambda), rho = g/lambda."""
    wl = _wl(8, 1, 5, 3, Q, 3.0, [44, Q], Es=1.7)
    N0, Es = wl["N0"], 1.7
    z, L, mu_o = oracle.mmse(wl["H"], wl["y"], Q, N0=N0, Es=Es)
    lam = N0 / Es
    for w in range(5):
        h = wl["H"][w, 0]
        g = float(np.vdot(h, h).real)
        assert abs(mu_o[w, 0] - g / (g + lam)) <= 1e-14
        for s in range(3):
            zs = np.vdot(h, wl["y"][w, s]) / (g + lam)
            assert abs(z[w, s, 0] - zs) <= 1e-14 * max(1.0, abs(zs))
            ref = _exact_mmse_llr_peraxis(zs / (g / (g + lam) * math.sqrt(Es)), g / lam, Q)
            np.testing.assert_allclose(L[w, s, 0], ref, rtol=1e-11, atol=1e-11)


@pytest.mark.parametrize("Q", [2, 6])
def test_orthogonal_columns_equal_one_ocd_sweep(Q):
    """With orthogonal columns G is diagonal: the explicit estimate, gain and SINR
    equal what one OCD sweep and Section III-C's approximations give."""
    rng = np.random.default_rng([45, Q])
    H = _orthogonal_channel(rng, 3, 4, 16)
    wl = _wl(16, 4, 3, 2, Q, 9.0, [45, Q], channel=H)
    z, L, _ = oracle.mmse(H, wl["y"], Q, N0=wl["N0"])
    zo = oracle.ocd(H, wl["y"], 1, Q, "mmse", N0=wl["N0"])
    Lo = oracle.llr(H, zo, 1, Q, "mmse", N0=wl["N0"])
    assert np.max(np.abs(z - zo)) <= 1e-13
    np.testing.assert_allclose(L, Lo, rtol=1e-11, atol=1e-11)


def test_high_snr_llr_signs_are_the_transmitted_bits():
    """At 40 dB every LLR sign is the transmitted bit (L > 0 favours 1)."""
    wl = _wl(32, 8, 6, 4, 6, 40.0, [46])
    _, L, _ = oracle.mmse(wl["H"], wl["y"], 6, N0=wl["N0"])
    assert np.array_equal((L > 0).astype(np.uint8), wl["bits"])


def test_zero_column_gives_zero_output():
    """An all-zero column: mu = 0, z = 0 and every LLR of that user is 0."""
    wl = _wl(16, 4, 2, 3, 4, 10.0, [47])
    H = wl["H"].copy()
    H[:, 2, :] = 0
    y = wl["y"]
    z, L, mu = oracle.mmse(H, y, 4, N0=wl["N0"])
    assert np.all(mu[:, 2] == 0) and np.all(z[:, :, 2] == 0) and np.all(L[:, :, 2] == 0)
    assert np.all(mu[:, [0, 1, 3]] > 0)


def test_symbol_energy_is_a_pure_scale():
    """Scaling the symbols by sqrt(Es) (and N0 with Es) scales z by sqrt(Es) and leaves
    the gains and LLRs unchanged."""
    a = _wl(16, 4, 3, 2, 4, 7.0, [48], Es=1.0)
    b = _wl(16, 4, 3, 2, 4, 7.0, [48], Es=4.0)
    za, La, ma = oracle.mmse(a["H"], a["y"], 4, N0=a["N0"], Es=1.0)
    zb, Lb, mb = oracle.mmse(b["H"], b["y"], 4, N0=b["N0"], Es=4.0)
    np.testing.assert_allclose(zb, 2.0 * za, rtol=1e-12, atol=1e-12)
    np.testing.assert_allclose(mb, ma, rtol=1e-12)
    np.testing.assert_allclose(Lb, La, rtol=1e-10, atol=1e-10)
