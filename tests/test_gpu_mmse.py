"""GPU parity of ocd_detect_mmse (explicit MMSE soft output, Sections II-B and
II-E) against the FP64 oracle, through the C ABI.

Tolerance.  The kernel inverts A = G + lambda I in FP32 by Gauss-Jordan
elimination; the forward error of an inverse computed this way is of order
cond(A) * u (u = 2^-24), and z, mu and rho inherit it, as do the LLRs through
rho and x = z / mu.  The bar is the OCD path's (z within 1e-4 per vector, LLRs
within 1e-3 of the vector's largest) raised where cond(A), computed from the
inputs, makes 64 * cond(A) * u larger: z within max(1e-4, 64 cond(A) u), LLRs
within max(1e-3, 10 times that).  Channels with B >= 4U have cond(A) < 10, so
the OCD bars hold; B = 2U reaches ~30 and a square system ~400."""

import numpy as np
import pytest
import torch

import oracle
import synth
from gpu_util import (LLR_TOL_F32, Z_TOL_F16, Z_TOL_F32, dev, from_f16_pairs, host, llr_rel_err,
                      say, to_f16_pairs, z_rel_err)

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ocd():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_1611_08779_amd as m
    return m


def f32(x):
    return float(np.float32(x))


def cond_max(H, lam):
    """Largest condition number of A = H^H H + lambda I over the subcarriers."""
    c = 0.0
    for w in range(H.shape[0]):
        Hm = H[w].astype(np.complex128).T
        ev = np.linalg.eigvalsh(Hm.conj().T @ Hm + lam * np.eye(Hm.shape[1]))
        c = max(c, ev[-1] / ev[0])
    return c


def run_mmse(ocd, B, U, W, S, Q, snr, seed, Es=1.0, plan=None, ztol=None, ltol=None, H=None):
    say("mmse case B=%d U=%d W=%d S=%d Q=%d snr=%s seed=%s plan=%s" % (B, U, W, S, Q, snr, seed,
                                                                       plan))
    wl = synth.make_workload(B, U, W, S, Q, snr, seed=seed, Es=Es, channel=H)
    N0 = f32(wl["N0"])
    if ztol is None:
        ztol = max(Z_TOL_F32, 64 * cond_max(wl["H"], N0 / Es) * 2.0 ** -24)
    if ltol is None:
        ltol = max(LLR_TOL_F32, 10 * ztol)
    z, L = ocd.detect_mmse(dev(wl["H"]), dev(wl["y"]), Q, N0, Es, plan=plan)
    torch.cuda.synchronize()
    zo, Lo, _ = oracle.mmse(wl["H"], wl["y"], Q, N0=N0, Es=Es, threads=0)
    ez, el = z_rel_err(host(z), zo), llr_rel_err(host(L), Lo)
    say("  z err %.3g  llr err %.3g" % (ez, el))
    assert ez <= ztol, ez
    assert el <= ltol, el
    return wl, z, L


# the headline shape on a slice of subcarriers, under several plans
@pytest.mark.parametrize("plan", [None, (0, 14, 0), (0, 0, 1), (16, 14, 0), (16, 28, 1), (16, 16, 0),
                                  (8, 14, 0), (32, 14, 0), (16, 5, 0),
                                  (8, 14, 0, 2), (16, 14, 1, 4), (0, 14, 0, 4)])   # staggered
def test_b128_u8_s14_64qam_plans(ocd, plan):
    run_mmse(ocd, 128, 8, 60, 14, 6, 20.0, [50, 1], plan=plan)


@pytest.mark.parametrize("B,U,W,S,Q,snr", [
    (64, 16, 30, 1, 4, 12.0),    # one H per vector
    (64, 32, 10, 2, 4, 20.0),    # the largest user count
    (256, 16, 6, 3, 6, 20.0),    # NPL = 8 at L = 32
    (512, 8, 3, 2, 4, 15.0),     # the largest antenna count (NPL = 16)
    (100, 8, 17, 3, 6, 18.0),    # padded lanes, ragged last workgroup
    (33, 4, 11, 2, 2, 8.0),      # odd B: scalar loads
    (16, 1, 9, 5, 4, 6.0),       # one user
    (24, 12, 7, 2, 4, 10.0),     # U not a power of two
])
def test_shapes(ocd, B, U, W, S, Q, snr):
    run_mmse(ocd, B, U, W, S, Q, snr, [51, B, U])


def test_square_system_tolerance_scales_with_conditioning(ocd):
    """B = U = 32: A is far worse conditioned; the bar is 64 cond(A) u."""
    run_mmse(ocd, 32, 32, 8, 2, 4, 20.0, [52])


def test_symbol_energy(ocd):
    run_mmse(ocd, 64, 8, 20, 4, 4, 10.0, [53], Es=2.5)


def test_zero_column(ocd):
    """An all-zero column: z_u = 0 and its LLRs are 0; the other users are unaffected."""
    wl = synth.make_workload(32, 4, 12, 3, 4, 10.0, seed=[54])
    H = wl["H"].copy()
    H[:, 1, :] = 0
    N0 = f32(wl["N0"])
    z, L = ocd.detect_mmse(dev(H), dev(wl["y"]), 4, N0)
    torch.cuda.synchronize()
    zo, Lo, _ = oracle.mmse(H, wl["y"], 4, N0=N0)
    assert np.all(host(z)[:, :, 1] == 0) and np.all(host(L)[:, :, 1] == 0)
    assert z_rel_err(host(z), zo) <= Z_TOL_F32
    assert llr_rel_err(host(L), Lo) <= LLR_TOL_F32


def test_fp16_storage(ocd):
    """FP16-stored H and y: the oracle on the FP16-rounded values, FP32 bars (all
    arithmetic after the load is FP32)."""
    B, U, W, S, Q = 128, 8, 40, 14, 6
    wl = synth.make_workload(B, U, W, S, Q, 20.0, seed=[55])
    H16, y16 = to_f16_pairs(wl["H"]), to_f16_pairs(wl["y"])
    N0 = f32(wl["N0"])
    z, L = ocd.detect_mmse(dev(H16), dev(y16), Q, N0, storage="f16")
    torch.cuda.synchronize()
    zo, Lo, _ = oracle.mmse(from_f16_pairs(H16), from_f16_pairs(y16), Q, N0=N0, threads=0)
    assert z_rel_err(host(z), zo) <= Z_TOL_F32
    assert llr_rel_err(host(L), Lo) <= LLR_TOL_F32
    # against the FP32-stored inputs, the FP16 storage tolerance
    z32, _ = ocd.detect_mmse(dev(wl["H"]), dev(wl["y"]), Q, N0)
    torch.cuda.synchronize()
    assert z_rel_err(host(z), host(z32).astype(np.complex128)) <= Z_TOL_F16


def test_outputs_are_optional_and_consistent(ocd):
    wl = synth.make_workload(64, 8, 20, 4, 6, 15.0, seed=[56])
    H, y = dev(wl["H"]), dev(wl["y"])
    N0 = f32(wl["N0"])
    z, L = ocd.detect_mmse(H, y, 6, N0)
    z1, none1 = ocd.detect_mmse(H, y, 6, N0, want_llr=False)
    none2, L1 = ocd.detect_mmse(H, y, 6, N0, want_z=False)
    torch.cuda.synchronize()
    assert none1 is None and none2 is None
    assert torch.equal(z, z1) and torch.equal(L, L1)


@pytest.mark.parametrize("plan", [None, (8, 14, 0, 2), (0, 14, 0, 4)])
def test_headline_full_size_sampled(ocd, plan):
    """B=128, U=8, 1200 subcarriers x 14 symbols, 64-QAM, 20 dB: the whole slot on
    the GPU (default plan, and staggered plans of both forms: every workgroup past
    the first 256 waits before its loads); a sample of subcarriers on the oracle."""
    B, U, W, S, Q = 128, 8, 1200, 14, 6
    wl = synth.make_workload(B, U, W, S, Q, 20.0, seed=[57])
    N0 = f32(wl["N0"])
    z, L = ocd.detect_mmse(dev(wl["H"]), dev(wl["y"]), Q, N0, plan=plan)
    torch.cuda.synchronize()
    ws = np.random.default_rng(57).choice(W, 24, replace=False)
    zo, Lo, _ = oracle.mmse(wl["H"][ws], wl["y"][ws], Q, N0=N0, threads=0)
    assert z_rel_err(host(z)[ws], zo) <= Z_TOL_F32
    assert llr_rel_err(host(L)[ws], Lo) <= LLR_TOL_F32
    # hard decisions of exact MMSE at 20 dB
    ber = float(np.mean((host(L) > 0) != wl["bits"]))
    say("exact MMSE BER at 20 dB: %.4g" % ber)
    assert ber < 0.05


def test_rejects_box_and_bad_plans(ocd):
    wl = synth.make_workload(32, 4, 4, 2, 4, 10.0, seed=[58])
    H, y = dev(wl["H"]), dev(wl["y"])
    pb = ocd.problem(32, 4, 4, 2, 4, 1, "box", "f32", 0.1)
    z = torch.empty(4, 2, 4, device="cuda", dtype=torch.complex64)
    with pytest.raises(ocd.OCDError) as ei:
        ocd.ocd_detect_mmse(pb, H, y, z)
    assert ei.value.status == -2
    with pytest.raises(ocd.OCDError) as ei:
        ocd.detect_mmse(H, y, 4, 0.1, plan=(4, 8))
    assert ei.value.status == -2


# the matrix-core form (plan lanes_per_vector = 0): U <= 8, S <= 16
@pytest.mark.parametrize("B,U,W,S,Q,snr", [
    (100, 8, 17, 3, 6, 18.0),    # B not a multiple of 8 (K padded to 100), S = 3
    (33, 4, 11, 2, 2, 8.0),      # odd B (K padded to 36)
    (16, 1, 9, 5, 4, 6.0),       # one user
    (64, 6, 10, 16, 4, 12.0),    # S = 16: all 32 columns of the matched-filter product
    (512, 8, 3, 1, 6, 15.0),     # the largest B, one symbol
    (128, 8, 40, 1, 6, 20.0),    # one H per vector at the headline's B and U
    (24, 7, 5, 9, 6, 20.0),      # U = 7, S = 9
])
def test_matrix_core_form(ocd, B, U, W, S, Q, snr):
    run_mmse(ocd, B, U, W, S, Q, snr, [59, B, U, S], plan=(0, S))


def test_matrix_core_form_zero_column_and_fp16(ocd):
    wl = synth.make_workload(32, 4, 12, 6, 4, 10.0, seed=[60])
    H = wl["H"].copy()
    H[:, 1, :] = 0
    N0 = f32(wl["N0"])
    z, L = ocd.detect_mmse(dev(H), dev(wl["y"]), 4, N0, plan=(0, 6))
    torch.cuda.synchronize()
    zo, Lo, _ = oracle.mmse(H, wl["y"], 4, N0=N0)
    assert np.all(host(z)[:, :, 1] == 0) and np.all(host(L)[:, :, 1] == 0)
    assert z_rel_err(host(z), zo) <= Z_TOL_F32
    H16, y16 = to_f16_pairs(wl["H"]), to_f16_pairs(wl["y"])
    z, L = ocd.detect_mmse(dev(H16), dev(y16), 4, N0, storage="f16", plan=(0, 6))
    torch.cuda.synchronize()
    zo, Lo, _ = oracle.mmse(from_f16_pairs(H16), from_f16_pairs(y16), 4, N0=N0)
    assert z_rel_err(host(z), zo) <= Z_TOL_F32
    assert llr_rel_err(host(L), Lo) <= LLR_TOL_F32


def test_matrix_core_form_rejects_shapes_it_does_not_cover(ocd):
    wl = synth.make_workload(64, 9, 4, 4, 4, 10.0, seed=[61])
    with pytest.raises(ocd.OCDError):
        ocd.detect_mmse(dev(wl["H"]), dev(wl["y"]), 4, 0.1, plan=(0, 4))     # U = 9
    wl = synth.make_workload(64, 8, 4, 4, 4, 10.0, seed=[61])
    with pytest.raises(ocd.OCDError):
        ocd.detect_mmse(dev(wl["H"]), dev(wl["y"]), 4, 0.1, plan=(0, 2))     # not S


@pytest.mark.parametrize("base", [(8, 14, 0), (16, 28, 1), (0, 14, 0)])
def test_stagger_changes_only_when_workgroups_start(ocd, base):
    """Staggered staging delays workgroups before their loads and nothing else: the
    outputs of both forms are bit-identical at every stagger value."""
    B, U, W, S, Q = 128, 8, 600, 14, 6
    wl = synth.make_workload(B, U, W, S, Q, 20.0, seed=[59])
    N0 = f32(wl["N0"])
    H, y = dev(wl["H"]), dev(wl["y"])
    z0, L0 = ocd.detect_mmse(H, y, Q, N0, plan=base + (0,))
    for sg in (1, 2, 4, 16):
        z, L = ocd.detect_mmse(H, y, Q, N0, plan=base + (sg,))
        torch.cuda.synchronize()
        assert torch.equal(z, z0) and torch.equal(L, L0), sg
