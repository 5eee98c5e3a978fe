"""Pins of the FP64 oracle against what the paper and the mathematics fix.

Every check here compares the oracle with something other than itself: a
textbook routine (Cholesky solve), brute force on tiny inputs (box QP by KKT
enumeration), closed forms (one user, orthogonal columns, the Rayleigh MRC
bit-error rate), invariants (monotone objective, LLR sign = sliced bit),
the transmitter of ``synth`` (an independent Gray mapper), values derived by
hand from Section II-D (``tests/golden``), and finite differences.
"""

import itertools
import math
import os

import numpy as np
import pytest
import scipy.linalg
import scipy.special

import fd_util
import oracle
import synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _rng(*seed):
    return np.random.default_rng(list(seed))


def _rayleigh(rng, W, U, B):
    return synth.rayleigh_channel(rng, W, U, B)


def _objective(h, y, z, lam):
    """f(z) = ||y - H z||^2 + lam ||z||^2 (eq:function); h is [U, B]."""
    res = y - h.T @ z
    return float(np.vdot(res, res).real + lam * np.vdot(z, z).real)


# ---------------------------------------------------------------- Alg. 1 == CD

@pytest.mark.parametrize("mode", ["mmse", "box", "hybrid"])
@pytest.mark.parametrize("B,U,K,Q", [(32, 8, 3, 4), (16, 5, 4, 6), (64, 16, 2, 2), (7, 7, 5, 4)])
def test_ocd_equals_plain_cd(mode, B, U, K, Q):
    """Section III-B: OCD and CD give exactly the same results (up to rounding)."""
    rng = _rng(11, B, U, K)
    wl = synth.make_workload(B, U, 3, 4, Q, 6.0, seed=[11, B, U, K, Q])
    lam = rng.uniform(0.05, 0.5, K) if mode == "hybrid" else None
    kw = dict(N0=wl["N0"], lam=lam)
    if mode != "mmse":
        kw["beta"] = 0.8 * (1 if Q == 2 else 1.1)
    z2 = oracle.ocd(wl["H"], wl["y"], K, Q, mode, **kw)
    z1 = oracle.cd(wl["H"], wl["y"], K, Q, mode, **kw)
    assert np.max(np.abs(z1 - z2)) <= 1e-12 * max(1.0, np.max(np.abs(z1)))


# ---------------------------------------------------------------- MMSE limit

@pytest.mark.parametrize("B,U", [(32, 8), (64, 16), (12, 12)])
def test_mmse_ocd_converges_to_cholesky_solution(B, U):
    """eq:CDrule is a Gauss-Seidel row update on (G + N0 I) z = H^H y (Section II-C),
    so many sweeps reach the explicit MMSE estimate A^-1 H^H y."""
    wl = synth.make_workload(B, U, 4, 2, 4, 10.0, seed=[1, B, U])
    K = 400 if B == U else 200
    z = oracle.ocd(wl["H"], wl["y"], K, 4, "mmse", N0=wl["N0"])
    H = wl["H"].astype(np.complex128)
    y = wl["y"].astype(np.complex128)
    for w in range(H.shape[0]):
        Hm = H[w].T                                   # B x U
        A = Hm.conj().T @ Hm + wl["N0"] * np.eye(U)   # regularised Gram matrix
        cf = scipy.linalg.cho_factor(A)
        for s in range(y.shape[1]):
            zs = scipy.linalg.cho_solve(cf, Hm.conj().T @ y[w, s])
            assert np.linalg.norm(z[w, s] - zs) <= 1e-10 * np.linalg.norm(zs)


# ---------------------------------------------------------------- BOX limit

def _box_qp_bruteforce(Hm, y, beta, lam=0.0):
    """min ||y - H z||^2 + lam||z||^2 over |Re z_i|, |Im z_i| <= beta, by KKT enumeration."""
    B, U = Hm.shape
    Hr = np.block([[Hm.real, -Hm.imag], [Hm.imag, Hm.real]])
    yr = np.concatenate([y.real, y.imag])
    if lam > 0:
        Hr = np.vstack([Hr, math.sqrt(lam) * np.eye(2 * U)])
        yr = np.concatenate([yr, np.zeros(2 * U)])
    best, best_f = None, np.inf
    n = 2 * U
    for pat in itertools.product((-1, 0, 1), repeat=n):
        pat = np.array(pat)
        x = np.zeros(n)
        fixed = pat != 0
        x[fixed] = beta * pat[fixed]
        free = ~fixed
        if free.any():
            rhs = yr - Hr[:, fixed] @ x[fixed]
            x[free] = np.linalg.lstsq(Hr[:, free], rhs, rcond=None)[0]
            if np.any(np.abs(x[free]) > beta + 1e-12):
                continue
        grad = Hr.T @ (Hr @ x - yr)
        if np.any(grad[pat == 1] > 1e-9) or np.any(grad[pat == -1] < -1e-9):
            continue
        f = float(np.sum((yr - Hr @ x) ** 2))
        if f < best_f:
            best, best_f = x, f
    return best[:U] + 1j * best[U:]


@pytest.mark.parametrize("U,lam", [(2, 0.0), (3, 0.0), (4, 0.0), (3, 0.2)])
def test_box_ocd_converges_to_bruteforce_box_qp(U, lam):
    """eq:BOXproblem is convex; CD with the projection eq:projection converges to its
    unique minimiser.  Brute force over all clip patterns gives that minimiser."""
    B, Q = 8, 4
    wl = synth.make_workload(B, U, 2, 2, Q, 0.0, seed=[2, U, int(lam * 10)])
    beta = 0.6  # tighter than the 16-QAM edge so that many components clip
    mode = "hybrid" if lam > 0 else "box"
    z = oracle.ocd(wl["H"], wl["y"], 500, Q, mode, N0=wl["N0"],
                   lam=[lam] * 500 if lam > 0 else None, beta=beta)
    H = wl["H"].astype(np.complex128)
    y = wl["y"].astype(np.complex128)
    nclip = 0
    for w in range(2):
        for s in range(2):
            zs = _box_qp_bruteforce(H[w].T, y[w, s], beta, lam)
            nclip += int(np.sum(np.isclose(np.abs(zs.real), beta)) + np.sum(np.isclose(np.abs(zs.imag), beta)))
            assert np.max(np.abs(z[w, s] - zs)) <= 1e-9
    assert nclip > 0, "the box must be active somewhere for this pin to mean anything"


# ---------------------------------------------------------------- invariants

@pytest.mark.parametrize("mode", ["mmse", "box", "hybrid"])
def test_objective_never_increases(mode):
    """Each update of eq:CDrule / eq:CDruleBOX is an exact coordinate minimisation of
    eq:function, so the objective cannot increase after any single update."""
    B, U, K, Q = 16, 6, 4, 4
    wl = synth.make_workload(B, U, 1, 3, Q, 3.0, seed=[3, 1])
    lam = {"mmse": wl["N0"], "box": 0.0, "hybrid": 0.3}[mode]
    beta = 0.7
    H = wl["H"].astype(np.complex128)[0]
    for s in range(3):
        y = wl["y"].astype(np.complex128)[0, s]
        tr = oracle.ocd_trace(H, y, K, Q, mode, N0=wl["N0"],
                              lam=[lam] * K if mode == "hybrid" else None, beta=beta)
        f_prev = _objective(H, y, np.zeros(U), lam)
        for k in range(K):
            for u in range(U):
                zc = tr[k, u]
                if mode != "mmse":
                    assert np.all(np.abs(zc.real) <= beta + 1e-15)
                    assert np.all(np.abs(zc.imag) <= beta + 1e-15)
                f = _objective(H, y, zc, lam)
                assert f <= f_prev + 1e-12 * max(1.0, f_prev)
                f_prev = f


def test_mmse_error_norm_never_increases():
    """For MMSE, f(z) - f(z*) = ||z - z*||_A^2 with A = G + N0 I: the A-norm error
    to the Cholesky solution is monotone along the updates."""
    B, U, K = 24, 8, 5
    wl = synth.make_workload(B, U, 1, 2, 4, 5.0, seed=[3, 2])
    H = wl["H"].astype(np.complex128)[0]
    A = H.conj() @ H.T + wl["N0"] * np.eye(U)
    for s in range(2):
        y = wl["y"].astype(np.complex128)[0, s]
        zs = np.linalg.solve(A, H.conj() @ y)
        tr = oracle.ocd_trace(H, y, K, 4, "mmse", N0=wl["N0"])
        e_prev = np.vdot(zs, A @ zs).real
        for k in range(K):
            for u in range(U):
                e = tr[k, u] - zs
                en = np.vdot(e, A @ e).real
                assert en <= e_prev * (1 + 1e-12)
                e_prev = en


# ---------------------------------------------------------------- closed forms

@pytest.mark.parametrize("mode", ["mmse", "box"])
def test_single_user_closed_form(mode):
    """U = 1: one sweep solves eq:MMSEproblem / eq:BOXproblem exactly,
    z = h^H y / (||h||^2 + N0) or clip(h^H y / ||h||^2); later sweeps change nothing."""
    B, Q = 32, 4
    wl = synth.make_workload(B, 1, 5, 3, Q, 2.0, seed=[4, 1])
    H = wl["H"].astype(np.complex128)
    y = wl["y"].astype(np.complex128)
    beta0 = 3 / math.sqrt(10)
    for K in (1, 4):
        z = oracle.ocd(wl["H"], wl["y"], K, Q, mode, N0=wl["N0"])
        for w in range(5):
            h = H[w, 0]
            g = np.vdot(h, h).real
            for s in range(3):
                mf = np.vdot(h, y[w, s])
                if mode == "mmse":
                    ref = mf / (g + wl["N0"])
                else:
                    c = mf / g
                    ref = np.clip(c.real, -beta0, beta0) + 1j * np.clip(c.imag, -beta0, beta0)
                assert abs(z[w, s, 0] - ref) <= 1e-13 * max(1, abs(ref))


def test_paper_qpsk_box_example():
    """Section II-D: the box around {+-1 +- j} has radius 1 and the projection
    clips each part independently (fixture tests/golden/qpsk_box_example.txt)."""
    rows = np.loadtxt(os.path.join(GOLDEN, "qpsk_box_example.txt"))
    for w_re, w_im, p_re, p_im in rows:
        H = np.ones((1, 1, 1), np.complex128)          # B = U = 1, h = 1
        y = np.array([[[w_re + 1j * w_im]]])
        z = oracle.ocd(H, y, 1, 2, "box", N0=1.0, beta=1.0)
        assert z[0, 0, 0] == pytest.approx(p_re + 1j * p_im, abs=1e-15)


def test_default_box_is_constellation_edge():
    """Section II-D: alpha = max Re{a} (hand-derived values in tests/golden/box_edges.txt)."""
    rows = np.loadtxt(os.path.join(GOLDEN, "box_edges.txt"))
    for Q, beta0 in rows:
        Q = int(Q)
        H = np.ones((1, 1, 1), np.complex128)
        y = np.array([[[50.0 - 50.0j]]])
        z = oracle.ocd(H, y, 1, Q, "box", N0=1.0)
        assert z[0, 0, 0].real == pytest.approx(beta0, abs=1e-15)
        assert z[0, 0, 0].imag == pytest.approx(-beta0, abs=1e-15)
        pts, _ = oracle.constellation(Q)
        assert np.max(pts.real) == pytest.approx(beta0, abs=1e-15)
        assert np.mean(np.abs(pts) ** 2) == pytest.approx(1.0, abs=1e-14)
        # Es scales the box with the constellation
        z = oracle.ocd(H, y * 3, 1, Q, "box", N0=1.0, Es=4.0)
        assert z[0, 0, 0].real == pytest.approx(2 * beta0, abs=1e-14)


def _orthogonal_channel(rng, W, U, B):
    H = np.empty((W, U, B), np.complex128)
    for w in range(W):
        M = rng.normal(size=(B, U)) + 1j * rng.normal(size=(B, U))
        Qm, _ = np.linalg.qr(M)
        H[w] = (Qm * rng.uniform(0.5, 1.5, U)).T     # orthogonal columns, unequal norms
    return H


def _exact_mmse_llr_peraxis(xhat, rho, Q):
    """Max-log LLR of eq:exactinversellr evaluated one axis at a time (square QAM is a
    product of two Gray PAMs; the other axis' minimum cancels in the difference)."""
    half = Q // 2
    M = 1 << half
    lev = np.array([(2 * m - M + 1) for m in range(M)]) / math.sqrt(2 * (M * M - 1) / 3)
    gray = np.array([m ^ (m >> 1) for m in range(M)])
    out = np.empty(Q)
    for b in range(Q):
        comp = xhat.real if b < half else xhat.imag
        bb = b % half
        bit = (gray >> (half - 1 - bb)) & 1
        d = (comp - lev) ** 2
        out[b] = rho * (d[bit == 0].min() - d[bit == 1].min())
    return out


@pytest.mark.parametrize("Q", [2, 4, 6])
def test_orthogonal_columns_match_exact_mmse_soft_output(Q):
    """With orthogonal columns G is diagonal: one OCD sweep equals the explicit MMSE
    estimate A^-1 H^H y (Section II-C), and Section III-C's approximate gain and SINR
    equal the exact ones of Section II-E (mu_i = [A^-1 G]_ii, rho = mu/(1-mu)), so the
    OCD LLRs equal the exact-MMSE max-log LLRs."""
    rng = _rng(5, Q)
    B, U, W, S = 16, 4, 3, 2
    H = _orthogonal_channel(rng, W, U, B)
    wl = synth.make_workload(B, U, W, S, Q, 8.0, seed=[5, Q], channel=H, dtype=np.complex128)
    N0 = wl["N0"]
    z = oracle.ocd(H, wl["y"], 1, Q, "mmse", N0=N0)
    L = oracle.llr(H, z, 1, Q, "mmse", N0=N0)
    for w in range(W):
        Hm = H[w].T
        G = Hm.conj().T @ Hm
        Ainv = np.linalg.inv(G + N0 * np.eye(U))
        mu = np.real(np.diag(Ainv @ G))
        rho = mu / (1 - mu)
        for s in range(S):
            zs = Ainv @ (Hm.conj().T @ wl["y"][w, s])
            assert np.max(np.abs(z[w, s] - zs)) <= 1e-13
            for u in range(U):
                ref = _exact_mmse_llr_peraxis(zs[u] / mu[u], rho[u], Q)
                np.testing.assert_allclose(L[w, s, u], ref, rtol=1e-11, atol=1e-11)


# ---------------------------------------------------------------- soft output

@pytest.mark.parametrize("Q,mode", [(2, "mmse"), (4, "mmse"), (6, "mmse"), (4, "box"), (6, "hybrid")])
def test_llr_2d_bruteforce_equals_per_axis(Q, mode):
    """For a Gray product constellation the 2-D minima of eq:exactinversellr split
    per axis; the oracle enumerates all 2^Q points, the test works per axis."""
    B, U, K = 32, 8, 3
    wl = synth.make_workload(B, U, 6, 3, Q, 4.0, seed=[6, Q])
    lam = [0.07] * K if mode == "hybrid" else None
    z = oracle.ocd(wl["H"], wl["y"], K, Q, mode, N0=wl["N0"], lam=lam)
    L = oracle.llr(wl["H"], z, K, Q, mode, N0=wl["N0"], lam=lam)
    H = wl["H"].astype(np.complex128)
    for w in range(6):
        g = np.sum(np.abs(H[w]) ** 2, axis=1)
        for s in range(3):
            for u in range(U):
                if mode == "mmse":
                    lamK = wl["N0"]
                elif mode == "hybrid":
                    lamK = 0.07
                else:
                    lamK = 0.0
                if lamK > 0:
                    mu, rho = g[u] / (g[u] + lamK), g[u] / lamK
                else:
                    mu, rho = 1.0, g[u] / wl["N0"]
                ref = _exact_mmse_llr_peraxis(z[w, s, u] / mu, rho, Q)
                np.testing.assert_allclose(L[w, s, u], ref, rtol=1e-12, atol=1e-12)


@pytest.mark.parametrize("Q,mode", [(2, "mmse"), (4, "box"), (6, "mmse"), (6, "box")])
def test_llr_sign_equals_sliced_bits(Q, mode):
    """eq:slicing on x = z/mu picks the nearest point; its bits are the signs of the
    max-log LLRs (L > 0 <=> bit 1)."""
    wl = synth.make_workload(32, 8, 10, 4, Q, 5.0, seed=[7, Q])
    z = oracle.ocd(wl["H"], wl["y"], 3, Q, mode, N0=wl["N0"])
    L = oracle.llr(wl["H"], z, 3, Q, mode, N0=wl["N0"])
    hb = oracle.hard(wl["H"], z, 3, Q, mode, N0=wl["N0"])
    assert np.array_equal((L > 0).astype(np.uint8), hb)


@pytest.mark.parametrize("Q,mode", [(2, "mmse"), (4, "mmse"), (6, "mmse"), (6, "box"), (4, "box")])
def test_high_snr_recovers_transmitted_bits(Q, mode):
    """At 40 dB with B/U = 16 and K = 3 sweeps every decision is right: this ties the
    oracle's demapper to the independent transmitter in synth (Gray labels, bit order)."""
    wl = synth.make_workload(128, 8, 20, 4, Q, 40.0, seed=[8, Q])
    z, L = oracle.detect(wl["H"], wl["y"], 3, Q, mode, N0=wl["N0"])
    assert np.array_equal((L > 0).astype(np.uint8), wl["bits"])


def test_mrc_ber_matches_rayleigh_closed_form():
    """U = 1, QPSK, MMSE: x = z/mu is the maximum-ratio-combining output, so the bit
    error rate is the textbook B-branch i.i.d. Rayleigh MRC BPSK formula with mean
    per-branch SNR per bit Es/(2 B N0)."""
    B, W, S, Q, snr = 4, 4000, 25, 2, 4.0
    wl = synth.make_workload(B, 1, W, S, Q, snr, seed=[9, 0])
    z, L = oracle.detect(wl["H"], wl["y"], 1, Q, "mmse", N0=wl["N0"])
    errs = np.sum((L > 0).astype(np.uint8) != wl["bits"])
    nbits = wl["bits"].size
    gbar = 1.0 / (2 * B * wl["N0"])
    mu = math.sqrt(gbar / (1 + gbar))
    pb = ((1 - mu) / 2) ** B * sum(scipy.special.comb(B - 1 + k, k) * ((1 + mu) / 2) ** k
                                   for k in range(B))
    sd = math.sqrt(pb * (1 - pb) / nbits)
    assert abs(errs / nbits - pb) < 4.5 * sd, (errs / nbits, pb)


def test_constellation_gray_neighbours_differ_in_one_bit():
    for Q in (2, 4, 6):
        pts, lab = oracle.constellation(Q)
        d = np.abs(pts[:, None] - pts[None, :])
        dmin = np.min(d[d > 1e-12])
        for i in range(len(pts)):
            for j in range(len(pts)):
                if abs(d[i, j] - dmin) < 1e-12:
                    assert bin(int(lab[i]) ^ int(lab[j])).count("1") == 1


# ---------------------------------------------------------------- gradients

def _bce_loss(L, bits):
    # mean over bits of softplus(L) - bit * L  (P(bit = 1) = sigmoid(L)); softplus(-L)
    # for bit 1, which does not cancel when the bit is confidently right
    return float(np.mean(np.logaddexp(0.0, np.where(bits != 0, -L, L))))


def _forward_loss(H, y, bits, K, Q, mode, N0, lam, beta):
    z = oracle.ocd(H, y, K, Q, mode, N0=N0, lam=lam, beta=beta)
    L = oracle.llr(H, z, K, Q, mode, N0=N0, lam=lam, beta=beta)
    return _bce_loss(L, bits)


def _evaluate(H, y, bits, K, Q, mode, N0, lam, beta):
    """(mean BCE loss, active set) of the oracle's forward pass."""
    z = oracle.ocd(H, y, K, Q, mode, N0=N0, lam=lam, beta=beta)
    L = oracle.llr(H, z, K, Q, mode, N0=N0, lam=lam, beta=beta)
    return _bce_loss(L, bits), oracle.active_set(H, y, K, Q, mode, N0=N0, lam=lam, beta=beta)


def _check(fd, analytic, tol=1e-7):
    """FP64 central difference against the reverse mode, relative 1e-7 (absolute below
    1e-3); None = the active set changed across every step: excluded."""
    if fd is None:
        return 0
    assert abs(fd - analytic) <= tol * max(1e-3, abs(fd)), (fd, analytic)
    return 1


@pytest.mark.parametrize("mode", ["hybrid", "mmse", "box"])
def test_reference_gradient_matches_finite_differences(mode):
    """Reverse mode (oracle_grad) against FP64 central differences of the forward pass,
    each taken across a step that leaves the active set unchanged (tests/fd_util.py)."""
    B, U, W, S, K, Q = 12, 3, 2, 2, 3, 4
    wl = synth.make_workload(B, U, W, S, Q, 6.0, seed=[10, K], dtype=np.complex128)
    H, y, bits = wl["H"], wl["y"], wl["bits"]
    N0 = wl["N0"]
    lam = np.array([0.3, 0.2, 0.25]) if mode in ("hybrid", "mmse") else None
    beta = 0.8 if mode != "mmse" else 0.0
    z = oracle.ocd(H, y, K, Q, mode, N0=N0, lam=lam, beta=beta)
    L = oracle.llr(H, z, K, Q, mode, N0=N0, lam=lam, beta=beta)
    dllr = (scipy.special.expit(L) - bits) / bits.size
    dlam, dbeta, dy = oracle.grad(H, y, dllr, K, Q, mode, N0=N0, lam=lam, beta=beta)
    compared = 0
    if lam is not None:
        for k in range(K):
            def f(v, k=k):
                l2 = lam.copy()
                l2[k] = v
                return _evaluate(H, y, bits, K, Q, mode, N0, l2, beta)
            compared += _check(fd_util.central(f, lam[k]), dlam[k])
    if mode != "mmse":
        compared += _check(fd_util.central(
            lambda v: _evaluate(H, y, bits, K, Q, mode, N0, lam, v), beta), dbeta)
        assert dbeta != 0.0
    for (w, s, b) in [(0, 0, 0), (0, 1, 5), (1, 0, 11), (1, 1, 3)]:
        for part in (1.0, 1j):
            def f(v, w=w, s=s, b=b, part=part):
                y2 = y.copy()
                y2[w, s, b] += part * v
                return _evaluate(H, y2, bits, K, Q, mode, N0, lam, beta)
            ana = dy[w, s, b].real if part == 1.0 else dy[w, s, b].imag
            compared += _check(fd_util.central(f, 0.0), ana)
    total = (K if lam is not None else 0) + (mode != "mmse") + 8
    assert compared >= total - 1, (compared, total)   # at most one coordinate on a kink


def test_active_set_describes_the_forward_pass():
    """oracle.active_set against the forward pass it describes: a component recorded as
    clipped ends the sweep at exactly +-beta on that side, one recorded inside does not
    sit beyond the box; every LLR equals rho (|x - a0|^2 - |x - a1|^2) with the two
    recorded minimisers, a0 carrying bit 0 and a1 bit 1."""
    B, U, W, S, K, Q = 16, 4, 3, 2, 3, 4
    wl = synth.make_workload(B, U, W, S, Q, 0.0, seed=[10, 7], dtype=np.complex128)
    H, y, N0 = wl["H"], wl["y"], wl["N0"]
    beta = 0.5
    lam = np.array([0.2, 0.1, 0.3])
    z, zh = oracle.ocd(H, y, K, Q, "hybrid", N0=N0, lam=lam, beta=beta, hist=True)
    clip, amin = oracle.active_set(H, y, K, Q, "hybrid", N0=N0, lam=lam, beta=beta)
    parts = np.stack([zh.real, zh.imag], axis=-1)
    assert np.all(parts[clip == 1] == beta) and np.all(parts[clip == -1] == -beta)
    assert np.all(np.abs(parts[clip == 0]) <= beta)
    assert np.any(clip != 0) and np.any(clip == 0)
    pts, lab = oracle.constellation(Q)
    L = oracle.llr(H, z, K, Q, "hybrid", N0=N0, lam=lam, beta=beta)
    g = np.sum(np.abs(H) ** 2, axis=2)                       # [W, U]
    mu = g / (g + lam[-1])
    rho = g / lam[-1]
    x = z / mu[:, None, :]
    for b in range(Q):
        a0, a1 = amin[..., b, 0], amin[..., b, 1]
        assert np.all((lab[a0] >> (Q - 1 - b)) & 1 == 0) and np.all((lab[a1] >> (Q - 1 - b)) & 1 == 1)
        want = rho[:, None, :] * (np.abs(x - pts[a0]) ** 2 - np.abs(x - pts[a1]) ** 2)
        np.testing.assert_allclose(L[..., b], want, rtol=1e-12, atol=1e-12)
    # box mode without a regulariser: every projection clips or not, LLR minimisers exist
    clip_b, amin_b = oracle.active_set(H, y, K, Q, "box", N0=N0, beta=beta)
    assert np.all(amin_b >= 0) and set(np.unique(clip_b)) <= {-1, 0, 1}


@pytest.mark.parametrize("mode", ["mmse", "box"])
def test_symbol_energy_is_a_pure_scale(mode):
    """Section II-A fixes unit symbol energy; with energy Es the symbols, the noise
    standard deviation and hence y all scale by sqrt(Es).  The equalised estimate must
    scale the same way (regulariser N0/Es, box edge times sqrt(Es)) and the LLRs must
    not change at all."""
    wl = synth.make_workload(32, 8, 4, 3, 6, 10.0, seed=[12, 0], dtype=np.complex128)
    z1, L1 = oracle.detect(wl["H"], wl["y"], 3, 6, mode, N0=wl["N0"], Es=1.0)
    z2, L2 = oracle.detect(wl["H"], 2.0 * wl["y"], 3, 6, mode, N0=4.0 * wl["N0"], Es=4.0)
    np.testing.assert_allclose(z2, 2.0 * z1, rtol=1e-12, atol=1e-12)
    np.testing.assert_allclose(L2, L1, rtol=1e-10, atol=1e-10)
