"""GPU parity of ocd_detect / ocd_preprocess against the FP64 oracle.

Every case generates seeded synthetic inputs (synth), runs the HIP path through
the C ABI and the oracle on exactly the same (FP32, promoted) values, and
compares element by element: z within 1e-4 and LLRs within 1e-3, per vector.
"""

import numpy as np
import pytest
import torch

import oracle
import synth
from gpu_util import (LLR_TOL_F32, Z_TOL_F16, Z_TOL_F32, dev, from_f16_pairs, host, llr_rel_err,
                      oracle_ref, say, to_f16_pairs, z_rel_err)

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ocd():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_1611_08779_amd as m
    return m


def f32(x):
    return float(np.float32(x))


def run_and_compare(ocd, B, U, W, S, Q, K, mode, snr, seed, lam=None, beta=0.0, Es=1.0,
                    hist=False, plan=None, ztol=Z_TOL_F32, ltol=LLR_TOL_F32):
    say("case B=%d U=%d W=%d S=%d Q=%d K=%d mode=%s snr=%s seed=%s plan=%s"
        % (B, U, W, S, Q, K, mode, snr, seed, plan))
    wl = synth.make_workload(B, U, W, S, Q, snr, seed=seed, Es=Es)
    N0 = f32(wl["N0"])
    lam_t = None if lam is None else dev(np.asarray(lam, np.float32))
    if plan is not None:
        pb = ocd.problem(B, U, W, S, Q, K, mode, "f32", N0, Es, beta)
        ocd.ocd_set_plan(pb, ocd.Plan(*(tuple(plan) + (0,) * (5 - len(plan)))))
    z, L, zh = ocd.detect(dev(wl["H"]), dev(wl["y"]), K, Q, mode, N0, Es, beta, lam=lam_t,
                          want_hist=hist)
    torch.cuda.synchronize()
    zo, Lo, zho = oracle_ref(wl["H"], wl["y"], K, Q, mode, N0, Es,
                             None if lam is None else np.asarray(lam, np.float32), f32(beta), hist)
    ez, el = z_rel_err(host(z), zo), llr_rel_err(host(L), Lo)
    say("  z err %.3g  llr err %.3g" % (ez, el))
    assert ez <= ztol, ez
    assert el <= ltol, el
    if hist:
        for k in range(K):
            assert z_rel_err(host(zh)[:, :, k], zho[:, :, k]) <= ztol
        assert np.array_equal(host(zh)[:, :, K - 1], host(z))
    return wl, z, L


# B=32, U=8, 64 subcarriers, 16-QAM, 10 dB, K=3 under every lane split
@pytest.mark.parametrize("plan", [(4, 16, 0), (4, 1, 0), (4, 3, 1), (8, 64, 0), (8, 7, 0),
                                  (16, 32, 1), (16, 5, 0), (32, 16, 0), (32, 2, 0)])
def test_b32_u8_every_plan(ocd, plan):
    run_and_compare(ocd, 32, 8, 64, 1, 4, 3, "mmse", 10.0, [1, 0, 0], hist=True, plan=plan)


# multiples of 8 users with at most 8 entries per lane beyond U = 16: the sweep runs
# as unrolled chunks of 8 users (3 and 4 chunks; at most 32 users), with the per-sweep
# history
@pytest.mark.parametrize("case", [
    (64, 24, 9, 3, 4, 3, "box", (8, 16, 0)),
    (128, 32, 5, 4, 6, 2, "mmse", (16, 8, 1)),
    (100, 24, 6, 2, 2, 3, "box", (16, 4, 0)),
    (256, 32, 3, 5, 4, 5, "box", (32, 5, 0, 0, 1)),
])
def test_chunked_user_loop(ocd, case):
    B, U, W, S, Q, K, mode, plan = case
    run_and_compare(ocd, B, U, W, S, Q, K, mode, 15.0, [1, 7, U], beta=0.9 * 3 / np.sqrt(10),
                    hist=True, plan=plan)


def test_b32_u8_default_plan(ocd):
    # W differs from the forced-plan cases above, so the heuristic plan is used
    run_and_compare(ocd, 32, 8, 63, 1, 4, 3, "mmse", 10.0, [1, 0, 1], hist=True)


def test_b128_u8_64qam_full_slot(ocd):
    """B=128, U=8, 1200 subcarriers x 14 symbols, 64-QAM, K=3, MMSE, 20 dB: the whole
    slot against the oracle (the workload the benchmark times)."""
    wl, z, L = run_and_compare(ocd, 128, 8, 1200, 14, 6, 3, "mmse", 20.0, [2, 0, 0])
    # hard decisions (LLR signs) agree with the oracle's wherever the oracle's LLR is not
    # within rounding of zero
    _, Lo, _ = oracle_ref(wl["H"], wl["y"], 3, 6, "mmse", f32(wl["N0"]))
    Lg = host(L)
    differ = (Lg > 0) != (Lo > 0)
    near_zero = np.abs(Lo) <= 1e-5 * np.max(np.abs(Lo), axis=(2, 3), keepdims=True)
    assert not np.any(differ & ~near_zero)
    ber = np.mean((Lg > 0).astype(np.uint8) != wl["bits"])
    say("  BER %.4g (64-QAM at 20 dB per-user SNR)" % ber)


def _full_slot_against_oracle(ocd, pb, wl, want_plan=None):
    """Detects the whole headline slot with the plan cached for `pb` and compares every
    vector with the oracle; returns the plan the launch used."""
    N0 = f32(wl["N0"])
    H, y = dev(wl["H"]), dev(wl["y"])
    used = ocd.ocd_get_plan(pb)
    say("  plan used %s" % used.as_dict())
    if want_plan is not None:
        assert (used.lanes_per_vector, used.vectors_per_block, used.xcd_remap,
                used.channel_in_registers, used.stagger) == want_plan
    z, L, _ = ocd.detect(H, y, 3, 6, "mmse", N0)
    torch.cuda.synchronize()
    zo, Lo, _ = oracle_ref(wl["H"], wl["y"], 3, 6, "mmse", N0)
    ez, el = z_rel_err(host(z), zo), llr_rel_err(host(L), Lo)
    say("  z err %.3g  llr err %.3g over %d vectors" % (ez, el, zo.shape[0] * zo.shape[1]))
    assert ez <= Z_TOL_F32, ez
    assert el <= LLR_TOL_F32, el
    return used


@pytest.mark.parametrize("plan", [(16, 14, 1, 0, 0), (16, 14, 1, 0, 2), (16, 16, 1, 0, 0),
                                  (16, 16, 1, 0, 2)])
def test_b128_u8_64qam_full_slot_bench_plan_forced(ocd, plan):
    """The headline slot whole (16,800 vectors) under the launch plans the benchmark's
    autotuner picks between on MI355X: 16 lanes per vector (8 complex entries per
    lane), XCD-aware tile order, with and without staggered staging, and either one
    subcarrier's 14 symbols per workgroup (the dense one-subcarrier staging path) or
    16 vectors per workgroup (tiles across two subcarriers, the general staging
    path); U = 8 takes the unrolled user loop.  That is the kernel instance
    k_forward<L=16, NPL=8, FP32, MMSE, U=8>, checked against the oracle."""
    B, U, W, S, Q, K = 128, 8, 1200, 14, 6, 3
    say("case headline slot, bench plan %s" % (plan,))
    wl = synth.make_workload(B, U, W, S, Q, 20.0, seed=[2, 0, 1])
    pb = ocd.problem(B, U, W, S, Q, K, "mmse", "f32", f32(wl["N0"]))
    ocd.ocd_set_plan(pb, ocd.Plan(*plan))
    _full_slot_against_oracle(ocd, pb, wl, want_plan=plan)


def test_b128_u8_64qam_full_slot_bench_autotuned(ocd):
    """The headline slot whole under whatever plan the autotuner chooses, tuned the way
    the benchmark tunes it (ocd_autotune_inputs over a stream of distinct slots, more
    than the caches hold, 2 passes); the plan used is the one the tuner returned."""
    B, U, W, S, Q, K = 128, 8, 1200, 14, 6, 3
    say("case headline slot, autotuned plan over 12 slots")
    wl = synth.make_workload(B, U, W, S, Q, 20.0, seed=[2, 0, 2])
    N0 = f32(wl["N0"])
    pb = ocd.problem(B, U, W, S, Q, K, "mmse", "f32", N0)
    others = [synth.make_workload_device(B, U, W, S, Q, 20.0, seed=3000 + i, device="cuda")
              for i in range(11)]
    Hs = [dev(wl["H"])] + [o["H"] for o in others]
    ys = [dev(wl["y"])] + [o["y"] for o in others]
    z = torch.empty(W, S, U, dtype=torch.complex64, device="cuda")
    L = torch.empty(W, S, U, Q, dtype=torch.float32, device="cuda")
    tuned = ocd.ocd_autotune_inputs(pb, Hs, ys, z, L, repeats=2)
    say("  autotuned %s" % tuned.as_dict())
    del others, Hs, ys
    _full_slot_against_oracle(ocd, pb, wl, want_plan=(
        tuned.lanes_per_vector, tuned.vectors_per_block, tuned.xcd_remap,
        tuned.channel_in_registers, tuned.stagger))


@pytest.mark.parametrize("plan", [(16, 4, 0, 1), (32, 4, 0, 1), (16, 4, 0, 1, 1)])
def test_b128_u8_64qam_one_h_per_vector_full_size(ocd, plan):
    """The S = 1 shape the benchmark times, whole: 16,800 vectors with one channel
    matrix each (B=128, U=8, 64-QAM, K=3, 20 dB), under the register plans its
    autotuner chooses between (with and without staggered starts), against the
    oracle."""
    run_and_compare(ocd, 128, 8, 16800, 1, 6, 3, "mmse", 20.0, [2, 5, 0], plan=plan)


@pytest.mark.parametrize("plan", [(4, 14, 0), (4, 16, 1), (8, 28, 0), (8, 64, 1), (16, 32, 0),
                                  (16, 14, 1), (16, 14, 0), (16, 28, 1), (16, 14, 1, 0, 4),
                                  (8, 28, 0, 0, 1), (16, 16, 1, 0, 2)])
def test_b128_u8_64qam_slice_plans(ocd, plan):
    run_and_compare(ocd, 128, 8, 60, 14, 6, 3, "mmse", 20.0, [2, 1, 0], plan=plan)


@pytest.mark.parametrize("Q", [2, 4])
@pytest.mark.parametrize("snr", [0.0, 10.0, 20.0])
def test_b256_u32_box(ocd, Q, snr):
    """B=256, U=32, 14 symbols per subcarrier, box at the constellation edge, K=5."""
    run_and_compare(ocd, 256, 32, 24, 14, Q, 5, "box", snr, [3, int(snr), Q])


EDGE = [
    # B, U, W, S, Q, K, mode
    (33, 5, 7, 3, 4, 2, "mmse"),      # odd B: scalar loads, padded lanes
    (100, 7, 5, 13, 6, 3, "box"),     # B not a power of two, S not dividing a tile
    (8, 8, 9, 2, 2, 4, "mmse"),       # U = B
    (1, 1, 4, 3, 2, 1, "box"),        # one antenna, one user
    (64, 1, 10, 5, 6, 3, "mmse"),     # one user
    (16, 4, 3, 1, 4, 256, "mmse"),    # maximum K
    (512, 32, 2, 3, 4, 2, "mmse"),    # large B
    (1024, 16, 1, 2, 2, 1, "box"),    # maximum B (H_w of 128 KB in LDS)
    (24, 3, 200, 1, 6, 3, "box"),     # many subcarriers, S = 1
]


@pytest.mark.parametrize("case", EDGE, ids=[str(c) for c in EDGE])
def test_edge_shapes(ocd, case):
    B, U, W, S, Q, K, mode = case
    run_and_compare(ocd, B, U, W, S, Q, K, mode, 8.0, [4] + list(case[:6]), hist=True)


def test_channel_too_large_for_lds_is_rejected(ocd):
    """B = 1024 with U = 32 needs 256 KB of LDS for one H_w: EUNSUPPORTED, nothing launched."""
    H = torch.zeros(1, 32, 1024, dtype=torch.complex64, device="cuda")
    y = torch.zeros(1, 2, 1024, dtype=torch.complex64, device="cuda")
    with pytest.raises(ocd.OCDError) as ei:
        ocd.detect(H, y, 1, 2, "box", 0.1)
    assert ei.value.status == -2


# channel columns held in registers (no LDS): the plans for channels few symbols share
REG_CASES = [
    # B, U, W, S, Q, K, mode, plan (L, vectors per workgroup, xcd, channel_in_registers)
    (128, 8, 300, 1, 6, 3, "mmse", (16, 16, 0, 1)),   # one H per vector, 64-QAM (a slice)
    (128, 8, 97, 1, 6, 3, "mmse", (32, 8, 0, 1)),     # ragged last workgroup
    (128, 6, 40, 2, 4, 4, "box", (16, 4, 0, 1)),      # U below the register bound, S = 2
    (100, 5, 30, 1, 2, 2, "box", (32, 3, 0, 1)),      # padded lanes (B < L * NPL)
    (64, 8, 50, 3, 4, 3, "mmse", (16, 16, 0, 1)),     # NPL = 4, three vectors per subcarrier
    (33, 4, 20, 1, 4, 2, "mmse", (16, 7, 0, 1)),      # odd B: scalar loads
    (32, 8, 64, 1, 4, 3, "mmse", (16, 16, 0, 1)),     # NPL = 2
    (256, 1, 12, 1, 6, 5, "box", (32, 2, 0, 1)),      # one user, NPL = 8 at L = 32
    (128, 8, 700, 1, 6, 3, "mmse", (16, 4, 0, 1, 2)),  # staggered starts, 175 workgroups
]


@pytest.mark.parametrize("case", REG_CASES, ids=[str(c[:7]) for c in REG_CASES])
def test_channel_in_registers_plans(ocd, case):
    B, U, W, S, Q, K, mode, plan = case
    run_and_compare(ocd, B, U, W, S, Q, K, mode, 12.0, [12] + list(case[:6]), hist=True, plan=plan)


def test_channel_in_registers_hybrid_and_preprocessed(ocd):
    """Per-sweep regularisers on the register path (S = 1 selects it by default); with
    caller-supplied preprocessing the same plan runs LDS-staged (the register kernel
    fuses the preprocessing)."""
    K = 4
    lam = np.array([0.3, 0.05, 0.12, 0.08], np.float32)
    run_and_compare(ocd, 128, 8, 40, 1, 4, K, "hybrid", 10.0, [12, 1], lam=lam, beta=0.9, hist=True)
    wl = synth.make_workload(128, 8, 50, 1, 6, 20.0, seed=[12, 2])
    N0 = f32(wl["N0"])
    H, y = dev(wl["H"]), dev(wl["y"])
    pb = ocd.problem(128, 8, 50, 1, 6, 3, "mmse", "f32", N0)
    assert ocd.ocd_get_plan(pb).channel_in_registers == 1
    g, dinv, p = ocd.preprocess(H, 3, 6, "mmse", N0)
    z2, L2, _ = ocd.detect(H, y, 3, 6, "mmse", N0, pre=(g, dinv, p))
    torch.cuda.synchronize()
    zo, Lo, _ = oracle_ref(wl["H"], wl["y"], 3, 6, "mmse", N0)
    assert z_rel_err(host(z2), zo) <= Z_TOL_F32
    assert llr_rel_err(host(L2), Lo) <= LLR_TOL_F32


@pytest.mark.parametrize("plan", [(32, 8, 0, 1), (16, 16, 0, 1), (16, 5, 0, 1), (32, 2, 0, 1),
                                  (16, 4, 0, 1, 1)])
def test_channel_in_registers_fp16(ocd, plan):
    """FP16 storage kept packed in registers (mixed-precision FMAs): the same values as
    the oracle on the FP16-rounded inputs, within the FP32 tolerance."""
    B, U, W, S, Q, K = 128, 8, 80, 1, 6, 3
    wl = synth.make_workload(B, U, W, S, Q, 15.0, seed=[12, 3])
    N0 = f32(wl["N0"])
    H16, y16 = to_f16_pairs(wl["H"]), to_f16_pairs(wl["y"])
    pb = ocd.problem(B, U, W, S, Q, K, "mmse", "f16", N0)
    ocd.ocd_set_plan(pb, ocd.Plan(*plan))
    z, L, _ = ocd.detect(dev(H16), dev(y16), K, Q, "mmse", N0, storage="f16")
    torch.cuda.synchronize()
    zo, Lo, _ = oracle_ref(from_f16_pairs(H16), from_f16_pairs(y16), K, Q, "mmse", N0)
    assert z_rel_err(host(z), zo) <= Z_TOL_F32
    assert llr_rel_err(host(L), Lo) <= LLR_TOL_F32


def test_hybrid_per_sweep_regulariser(ocd):
    K = 4
    lam = np.array([0.3, 0.05, 0.12, 0.08], np.float32)
    run_and_compare(ocd, 128, 16, 20, 4, 4, K, "hybrid", 10.0, [5, 0], lam=lam, beta=0.9, hist=True)


def test_mmse_with_explicit_regulariser(ocd):
    lam = np.array([0.5, 0.2, 0.1], np.float32)
    run_and_compare(ocd, 64, 8, 30, 3, 6, 3, "mmse", 15.0, [5, 1], lam=lam)


def test_symbol_energy_and_explicit_box(ocd):
    run_and_compare(ocd, 64, 8, 30, 3, 4, 3, "box", 12.0, [5, 2], Es=2.5, beta=1.2)
    run_and_compare(ocd, 64, 8, 30, 3, 6, 3, "mmse", 12.0, [5, 3], Es=0.4)


def test_empty_problem_is_a_no_op(ocd):
    H = torch.zeros(0, 8, 32, dtype=torch.complex64, device="cuda")
    y = torch.zeros(0, 3, 32, dtype=torch.complex64, device="cuda")
    z, L, _ = ocd.detect(H, y, 3, 4, "mmse", 0.1)
    torch.cuda.synchronize()
    assert z.numel() == 0 and L.numel() == 0


def test_zero_column_user_is_never_updated(ocd):
    """A user whose channel column is zero keeps z = 0 and gets LLR 0 (MMSE and BOX)."""
    wl = synth.make_workload(32, 4, 6, 2, 4, 10.0, seed=[6, 0])
    H = wl["H"].copy()
    H[:, 2, :] = 0
    for mode in ("mmse", "box"):
        z, L, _ = ocd.detect(dev(H), dev(wl["y"]), 3, 4, mode, f32(wl["N0"]))
        zo, Lo, _ = oracle_ref(H, wl["y"], 3, 4, mode, f32(wl["N0"]))
        assert np.all(host(z)[:, :, 2] == 0) and np.all(host(L)[:, :, 2] == 0)
        assert np.all(Lo[:, :, 2] == 0)
        assert z_rel_err(host(z), zo) <= Z_TOL_F32


def test_separate_preprocessing_matches_fused(ocd):
    B, U, W, S, Q, K = 128, 8, 40, 14, 6, 3
    wl = synth.make_workload(B, U, W, S, Q, 20.0, seed=[7, 0])
    N0 = f32(wl["N0"])
    H, y = dev(wl["H"]), dev(wl["y"])
    for lam in (None, dev(np.array([0.02, 0.01, 0.005], np.float32))):
        g, dinv, p = ocd.preprocess(H, K, Q, "mmse", N0, lam=lam)
        torch.cuda.synchronize()
        g_ref = np.sum(np.abs(wl["H"].astype(np.complex128)) ** 2, axis=2)
        np.testing.assert_allclose(host(g), g_ref, rtol=1e-5)
        lam_np = np.full(1, N0) if lam is None else host(lam).astype(np.float64)
        d_ref = 1.0 / (g_ref[:, None, :] + lam_np[None, :, None])
        np.testing.assert_allclose(host(dinv), d_ref, rtol=1e-5)
        np.testing.assert_allclose(host(p), d_ref * g_ref[:, None, :], rtol=1e-5)
        z1, L1, _ = ocd.detect(H, y, K, Q, "mmse", N0, lam=lam)
        z2, L2, _ = ocd.detect(H, y, K, Q, "mmse", N0, lam=lam, pre=(g, dinv, p))
        torch.cuda.synchronize()
        assert torch.equal(z1, z2) and torch.equal(L1, L2)


def test_runs_are_bitwise_reproducible(ocd):
    wl = synth.make_workload(128, 8, 100, 14, 6, 20.0, seed=[8, 0])
    H, y = dev(wl["H"]), dev(wl["y"])
    a = ocd.detect(H, y, 3, 6, "mmse", f32(wl["N0"]))
    b = ocd.detect(H, y, 3, 6, "mmse", f32(wl["N0"]))
    torch.cuda.synchronize()
    assert torch.equal(a[0], b[0]) and torch.equal(a[1], b[1])


def test_rejects_undersized_buffers_before_launch(ocd):
    wl = synth.make_workload(32, 4, 4, 2, 4, 10.0, seed=[9, 0])
    H, y = dev(wl["H"]), dev(wl["y"])
    pb = ocd.problem(32, 4, 5, 2, 4, 3, "mmse", "f32", 0.1)     # W=5 but H holds 4
    z = torch.empty(5, 2, 4, dtype=torch.complex64, device="cuda")
    with pytest.raises(ValueError):
        ocd.ocd_detect(pb, H, y, z=z)


# ---------------------------------------------------------------- FP16 storage

def test_fp16_storage_parity(ocd):
    """H and y stored as FP16 pairs, every computation in FP32: against the oracle on the
    FP16-rounded inputs (arithmetic error only, FP32 tolerance) and on the original FP32
    inputs (total error, 3e-3)."""
    B, U, W, S, Q, K = 256, 32, 20, 14, 4, 5
    wl = synth.make_workload(B, U, W, S, Q, 10.0, seed=[10, 0])
    N0 = f32(wl["N0"])
    H16, y16 = to_f16_pairs(wl["H"]), to_f16_pairs(wl["y"])
    z, L, _ = ocd.detect(dev(H16), dev(y16), K, Q, "box", N0, storage="f16")
    torch.cuda.synchronize()
    zo, Lo, _ = oracle_ref(from_f16_pairs(H16), from_f16_pairs(y16), K, Q, "box", N0)
    assert z_rel_err(host(z), zo) <= Z_TOL_F32
    assert llr_rel_err(host(L), Lo) <= LLR_TOL_F32
    zo32, _, _ = oracle_ref(wl["H"], wl["y"], K, Q, "box", N0)
    e = z_rel_err(host(z), zo32)
    say("  fp16 total z err %.3g" % e)
    assert e <= Z_TOL_F16


def test_fp16_storage_headline_full_slot(ocd):
    """The FP16-storage form the benchmark times, whole: B=128, U=8, 1200 x 14, 64-QAM,
    K=3, MMSE.  Against the oracle on the FP16-rounded inputs (FP32 tolerance) and on
    the FP32 inputs (3e-3); bit errors within 2% of the FP32 path's on the same noise
    (at 12 dB, where there are enough)."""
    B, U, W, S, Q, K = 128, 8, 1200, 14, 6, 3
    wl = synth.make_workload(B, U, W, S, Q, 12.0, seed=[10, 3])
    N0 = f32(wl["N0"])
    H16, y16 = to_f16_pairs(wl["H"]), to_f16_pairs(wl["y"])
    z, L, _ = ocd.detect(dev(H16), dev(y16), K, Q, "mmse", N0, storage="f16")
    _, L32, _ = ocd.detect(dev(wl["H"]), dev(wl["y"]), K, Q, "mmse", N0)
    torch.cuda.synchronize()
    zo, Lo, _ = oracle_ref(from_f16_pairs(H16), from_f16_pairs(y16), K, Q, "mmse", N0)
    assert z_rel_err(host(z), zo) <= Z_TOL_F32
    assert llr_rel_err(host(L), Lo) <= LLR_TOL_F32
    zo32, _, _ = oracle_ref(wl["H"], wl["y"], K, Q, "mmse", N0)
    assert z_rel_err(host(z), zo32) <= Z_TOL_F16
    e16 = int(np.sum((host(L) > 0) != wl["bits"]))
    e32 = int(np.sum((host(L32) > 0) != wl["bits"]))
    say("  errors fp32 %d fp16 %d of %d bits" % (e32, e16, wl["bits"].size))
    assert e32 >= 500 and abs(e16 - e32) <= 0.02 * e32


@pytest.mark.parametrize("case", [(128, 8, 60, 14, 6, 3, "mmse"), (33, 5, 7, 3, 4, 2, "box")])
def test_fp16_storage_shapes(ocd, case):
    B, U, W, S, Q, K, mode = case
    wl = synth.make_workload(B, U, W, S, Q, 15.0, seed=[10, 1] + list(case[:6]))
    N0 = f32(wl["N0"])
    H16, y16 = to_f16_pairs(wl["H"]), to_f16_pairs(wl["y"])
    z, L, zh = ocd.detect(dev(H16), dev(y16), K, Q, mode, N0, storage="f16", want_hist=True)
    torch.cuda.synchronize()
    zo, Lo, _ = oracle_ref(from_f16_pairs(H16), from_f16_pairs(y16), K, Q, mode, N0)
    assert z_rel_err(host(z), zo) <= Z_TOL_F32
    assert llr_rel_err(host(L), Lo) <= LLR_TOL_F32


def test_fp16_ber_matches_fp32_on_paired_noise(ocd):
    """Same channel and noise realisations through the FP32 and the FP16-storage paths:
    bit-error counts within 2% where there are at least 500 errors."""
    B, U, W, S, Q, K = 256, 32, 300, 14, 4, 5
    wl = synth.make_workload(B, U, W, S, Q, 2.0, seed=[10, 2])
    N0 = f32(wl["N0"])
    _, L32, _ = ocd.detect(dev(wl["H"]), dev(wl["y"]), K, Q, "box", N0)
    _, L16, _ = ocd.detect(dev(to_f16_pairs(wl["H"])), dev(to_f16_pairs(wl["y"])), K, Q, "box", N0,
                           storage="f16")
    torch.cuda.synchronize()
    e32 = int(np.sum((host(L32) > 0) != wl["bits"]))
    e16 = int(np.sum((host(L16) > 0) != wl["bits"]))
    say("  errors fp32 %d fp16 %d of %d bits" % (e32, e16, wl["bits"].size))
    assert e32 >= 500
    assert abs(e16 - e32) <= 0.02 * e32


# ---------------------------------------------------------------- autotuner

def test_autotune_over_several_inputs(ocd):
    """ocd_autotune_inputs: the plan it returns is valid and cached for the shape, and
    under it every input set it was timed on is detected as the oracle detects it."""
    B, U, W, S, Q, K = 64, 8, 40, 14, 4, 3
    wls = [synth.make_workload(B, U, W, S, Q, 12.0, seed=[11, 1, i]) for i in range(3)]
    N0 = f32(wls[0]["N0"])
    pb = ocd.problem(B, U, W, S, Q, K, "mmse", "f32", N0)
    Hs, ys = [dev(w["H"]) for w in wls], [dev(w["y"]) for w in wls]
    z = torch.empty(W, S, U, dtype=torch.complex64, device="cuda")
    L = torch.empty(W, S, U, Q, dtype=torch.float32, device="cuda")
    plan = ocd.ocd_autotune_inputs(pb, Hs, ys, z, L, repeats=2)
    say("  tuned plan", plan.as_dict())
    assert ocd.ocd_get_plan(pb).as_dict() == plan.as_dict()
    for w, H, y in zip(wls, Hs, ys):
        z2, L2, _ = ocd.detect(H, y, K, Q, "mmse", N0)
        torch.cuda.synchronize()
        zo, Lo, _ = oracle_ref(w["H"], w["y"], K, Q, "mmse", N0)
        assert z_rel_err(host(z2), zo) <= Z_TOL_F32
        assert llr_rel_err(host(L2), Lo) <= LLR_TOL_F32
    with pytest.raises(ValueError):
        ocd.ocd_autotune_inputs(pb, [], [], z, L)


def test_autotune_persists_its_plan(ocd, tmp_path, monkeypatch):
    """With OCD_TUNE_CACHE set, the tuner writes its choice to that file (one JSON
    object a line, keyed by GPU architecture and shape), stagger included."""
    import json
    cache = tmp_path / "plans.json"
    monkeypatch.setenv("OCD_TUNE_CACHE", str(cache))
    B, U, W, S, Q, K = 64, 8, 96, 6, 4, 2
    wl = synth.make_workload(B, U, W, S, Q, 12.0, seed=[11, 1])
    pb = ocd.problem(B, U, W, S, Q, K, "mmse", "f32", f32(wl["N0"]))
    H, y = dev(wl["H"]), dev(wl["y"])
    z = torch.empty(W, S, U, dtype=torch.complex64, device="cuda")
    L = torch.empty(W, S, U, Q, dtype=torch.float32, device="cuda")
    plan = ocd.ocd_autotune(pb, H, y, z, L, repeats=2)
    shape = "|fwd|B%d|U%d|W%d|S%d|K%d|Q%d|m0|s0|l" % (B, U, W, S, K, Q)
    recs = [json.loads(l) for l in cache.read_text().splitlines() if shape in l]
    say("  persisted %s" % recs)
    assert len(recs) == 2   # with and without per-sweep regularisers
    for r in recs:
        assert {k: r[k] for k in plan.as_dict()} == plan.as_dict()


def test_autotune_returns_a_valid_plan(ocd):
    B, U, W, S, Q, K = 32, 8, 64, 1, 4, 3
    wl = synth.make_workload(B, U, W, S, Q, 10.0, seed=[11, 0])
    N0 = f32(wl["N0"])
    pb = ocd.problem(B, U, W, S, Q, K, "mmse", "f32", N0)
    H, y = dev(wl["H"]), dev(wl["y"])
    z = torch.empty(W, S, U, dtype=torch.complex64, device="cuda")
    L = torch.empty(W, S, U, Q, dtype=torch.float32, device="cuda")
    plan = ocd.ocd_autotune(pb, H, y, z, L, repeats=2)
    say("  tuned plan", plan.as_dict())
    assert plan.lanes_per_vector in (4, 8, 16, 32)
    assert ocd.ocd_get_plan(pb).as_dict() == plan.as_dict()
    z2, L2, _ = ocd.detect(H, y, K, Q, "mmse", N0)
    torch.cuda.synchronize()
    zo, Lo, _ = oracle_ref(wl["H"], wl["y"], K, Q, "mmse", N0)
    assert z_rel_err(host(z2), zo) <= Z_TOL_F32
    assert llr_rel_err(host(L2), Lo) <= LLR_TOL_F32
