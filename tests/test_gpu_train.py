"""GPU parity of the one-launch training step (ocd_detect_train_bce): detection, the
mean bit cross-entropy of the LLRs and its gradients.  Against the two-launch path
(ocd_detect with the per-sweep history, then ocd_detect_backward_bce) under the same
plan, where z, the LLRs and dy must agree bit for bit, and against the FP64 oracle:
its loss, and its reverse mode within 1e-3 relative L2 per gradient."""

import numpy as np
import pytest
import scipy.special
import torch

import oracle
import synth
from gpu_util import LLR_TOL_F32, Z_TOL_F32, dev, host, say

pytestmark = pytest.mark.gpu

GRAD_TOL = 1e-3
LOSS_TOL = 1e-5      # FP32 sums of about 10^4..10^6 terms against an FP64 mean
REDUCE_TOL = 1e-5    # the same partial sums reduced over a different workgroup split


@pytest.fixture(scope="module")
def ocd():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_1611_08779_amd as m
    return m


def f32(x):
    return float(np.float32(x))


def rel(a, b):
    a, b = np.asarray(a, np.complex128).ravel(), np.asarray(b, np.complex128).ravel()
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def _setup(mode, B, U, W, S, Q, K, seed, snr=10.0):
    wl = synth.make_workload(B, U, W, S, Q, snr, seed=[21, seed])
    N0 = f32(wl["N0"])
    lam = (np.full(K, N0, np.float32) * np.array([1.0, 0.8, 1.3, 0.9, 1.1, 1.0][:K], np.float32)
           if mode == "hybrid" else None)
    beta = f32(0.9 * 3 / np.sqrt(10)) if mode != "mmse" else 0.0
    return wl, N0, lam, beta


def _two_launch(ocd, H, y, bits, K, Q, mode, N0, beta, lam_t, storage="f32"):
    z, L, zh = ocd.detect(H, y, K, Q, mode, N0, 1.0, beta, lam=lam_t, storage=storage,
                          want_z=True, want_hist=True)
    dlam, dbeta, dy = ocd.backward(H, y, zh, None, K, Q, mode, N0, 1.0, beta, lam=lam_t,
                                   storage=storage, bits=bits)
    return z, L, dlam, dbeta, dy


@pytest.mark.parametrize("mode", ["hybrid", "box", "mmse"])
def test_train_step_reproduces_the_two_launch_path(ocd, mode):
    """B=128, U=16, 36 subcarriers x 4 symbols, 16-QAM, K=4 (a ragged last workgroup):
    the forward plan is set to the training step's, so z, the LLRs and dy must match the
    two launches bit for bit; dlambda and dbeta are the same partial sums reduced over
    possibly different workgroups."""
    B, U, W, S, Q, K = 128, 16, 36, 4, 4, 4
    say("train vs two-launch mode=%s" % mode)
    wl, N0, lam, beta = _setup(mode, B, U, W, S, Q, K, seed=0)
    H, y = dev(wl["H"]), dev(wl["y"])
    lam_t = dev(lam) if lam is not None else None
    bits = torch.from_numpy(wl["bits"]).cuda()
    pb = ocd.problem(B, U, W, S, Q, K, mode, "f32", N0, 1.0, beta)
    tp = ocd.ocd_train_plan(pb)
    say("  train plan", tp.as_dict())
    ocd.ocd_set_plan(pb, tp)
    z2, L2, dlam2, dbeta2, dy2 = _two_launch(ocd, H, y, bits, K, Q, mode, N0, beta, lam_t)
    loss, dlam, dbeta, dy, z, L = ocd.train_step(H, y, bits, K, Q, mode, N0, 1.0, beta,
                                                 lam=lam_t, want_z=True, want_llr=True)
    torch.cuda.synchronize()
    assert torch.equal(z, z2)
    assert torch.equal(L, L2)
    assert torch.equal(dy, dy2)
    assert rel(host(dlam), host(dlam2)) <= REDUCE_TOL
    if mode == "mmse":
        assert float(host(dbeta)[0]) == 0.0
    else:
        assert abs(float(host(dbeta)[0]) - float(host(dbeta2)[0])) <= \
            REDUCE_TOL * abs(float(host(dbeta2)[0]))
    want = torch.nn.functional.binary_cross_entropy_with_logits(L2.double(), bits.double())
    say("  loss %.9g torch %.9g" % (float(host(loss)[0]), float(want)))
    assert abs(float(host(loss)[0]) - float(want)) <= LOSS_TOL * float(want)


@pytest.mark.parametrize("mode", ["hybrid", "box", "mmse"])
def test_train_step_matches_the_oracle(ocd, mode):
    """A 32-subcarrier slice of the differentiable workload against the FP64 oracle:
    z and the LLRs per vector, the loss, and the reverse mode seeded from the oracle's
    own LLRs and the bits."""
    B, U, W, S, Q, K = 128, 16, 32, 4, 4, 4
    say("train vs oracle mode=%s" % mode)
    wl, N0, lam, beta = _setup(mode, B, U, W, S, Q, K, seed=1)
    H, y = dev(wl["H"]), dev(wl["y"])
    lam_t = dev(lam) if lam is not None else None
    bits = torch.from_numpy(wl["bits"]).cuda()
    loss, dlam, dbeta, dy, z, L = ocd.train_step(H, y, bits, K, Q, mode, N0, 1.0, beta,
                                                 lam=lam_t, want_z=True, want_llr=True)
    torch.cuda.synchronize()
    zo, Lo = oracle.detect(wl["H"], wl["y"], K, Q, mode, N0=N0, lam=lam, beta=beta, threads=0)
    zg, Lg = host(z).astype(np.complex128), host(L).astype(np.float64)
    ez = np.linalg.norm((zg - zo).reshape(W * S, -1), axis=1) / \
        np.maximum(np.linalg.norm(zo.reshape(W * S, -1), axis=1), 1e-30)
    eL = np.linalg.norm((Lg - Lo).reshape(W * S, -1), axis=1) / \
        np.maximum(np.linalg.norm(Lo.reshape(W * S, -1), axis=1), 1e-30)
    assert ez.max() <= Z_TOL_F32 and eL.max() <= LLR_TOL_F32
    loss_o = float(np.mean(np.logaddexp(0.0, np.where(wl["bits"] != 0, -Lo, Lo))))
    say("  loss gpu %.9g oracle %.9g" % (float(host(loss)[0]), loss_o))
    assert abs(float(host(loss)[0]) - loss_o) <= 1e-4 * loss_o
    dllr_o = (scipy.special.expit(Lo) - wl["bits"]) / wl["bits"].size
    dlam_o, dbeta_o, dy_o = oracle.grad(wl["H"], wl["y"], dllr_o, K, Q, mode, N0=N0, lam=lam,
                                        beta=beta)
    say("  dlam gpu", host(dlam), "oracle", dlam_o)
    assert rel(host(dlam), dlam_o) <= GRAD_TOL
    assert rel(host(dy), dy_o) <= GRAD_TOL
    if mode == "mmse":
        assert float(host(dbeta)[0]) == 0.0
    else:
        assert abs(float(host(dbeta)[0]) - dbeta_o) <= GRAD_TOL * abs(dbeta_o)


@pytest.mark.parametrize("case", [
    # (B, U, W, S, Q, K, mode, storage): run-time user loop, ragged antennas, one
    # symbol per channel, one sweep, QPSK and 64-QAM, FP16 storage
    (36, 5, 21, 3, 2, 3, "hybrid", "f32"),
    (64, 8, 50, 1, 6, 2, "box", "f32"),
    (128, 16, 17, 4, 4, 1, "hybrid", "f32"),
    (128, 8, 24, 4, 4, 3, "hybrid", "f16"),
    (200, 12, 9, 7, 6, 3, "mmse", "f32"),
    (256, 32, 4, 2, 4, 2, "hybrid", "f32"),   # the most users, the largest H_w
])
def test_train_step_edge_shapes(ocd, case):
    B, U, W, S, Q, K, mode, storage = case
    say("train edge", case)
    wl, N0, lam, beta = _setup(mode, B, U, W, S, Q, K, seed=2)
    if storage == "f16":
        pairs = lambda a: torch.view_as_real(dev(a)).to(torch.float16).contiguous()
        H, y = pairs(wl["H"]), pairs(wl["y"])
    else:
        H, y = dev(wl["H"]), dev(wl["y"])
    lam_t = dev(lam) if lam is not None else None
    bits = torch.from_numpy(wl["bits"]).cuda()
    z2, L2, dlam2, dbeta2, dy2 = _two_launch(ocd, H, y, bits, K, Q, mode, N0, beta, lam_t,
                                             storage)
    loss, dlam, dbeta, dy, z, L = ocd.train_step(H, y, bits, K, Q, mode, N0, 1.0, beta,
                                                 lam=lam_t, storage=storage, want_z=True,
                                                 want_llr=True)
    torch.cuda.synchronize()
    # the two paths may run different lane mappings: FP32 rounding apart (the
    # tolerances of the GPU path against the oracle)
    assert rel(host(z), host(z2)) <= Z_TOL_F32
    assert rel(host(L), host(L2)) <= LLR_TOL_F32
    assert rel(host(dy), host(dy2)) <= GRAD_TOL
    assert rel(host(dlam), host(dlam2)) <= GRAD_TOL
    if mode != "mmse":
        assert abs(float(host(dbeta)[0]) - float(host(dbeta2)[0])) <= \
            GRAD_TOL * max(abs(float(host(dbeta2)[0])), 1e-12)
    want = torch.nn.functional.binary_cross_entropy_with_logits(L.double(), bits.double())
    assert abs(float(host(loss)[0]) - float(want)) <= LOSS_TOL * float(want)


def test_train_step_empty_problem_and_null_outputs(ocd):
    """W = 0 writes zero gradients and a zero loss; a training step without z, LLR or
    dy outputs gives the same loss and parameter gradients, bitwise, and repeated calls
    on one workspace give identical bits (the completion counter returns to zero)."""
    K, Q = 3, 4
    pb = ocd.problem(64, 4, 0, 2, Q, K, "hybrid", "f32", 0.1, 1.0, 0.7)
    H = torch.empty(0, 4, 64, dtype=torch.complex64, device="cuda")
    y = torch.empty(0, 2, 64, dtype=torch.complex64, device="cuda")
    bits = torch.empty(0, 2, 4, Q, dtype=torch.uint8, device="cuda")
    lam = torch.full((K,), 0.1, device="cuda")
    loss = torch.full((1,), 7.0, device="cuda")
    dlam = torch.full((K,), 7.0, device="cuda")
    dbeta = torch.full((1,), 7.0, device="cuda")
    ws = torch.zeros(ocd.ocd_backward_workspace_bytes(pb), dtype=torch.uint8, device="cuda")
    ocd.ocd_detect_train_bce(pb, H, y, lam, bits, None, None, loss, dlam, dbeta, None, ws)
    torch.cuda.synchronize()
    assert np.all(host(dlam) == 0.0) and host(dbeta)[0] == 0.0 and host(loss)[0] == 0.0

    B, U, W, S, Q, K = 128, 16, 40, 4, 4, 4
    wl, N0, lam, beta = _setup("hybrid", B, U, W, S, Q, K, seed=3)
    H, y, lam_t = dev(wl["H"]), dev(wl["y"]), dev(lam)
    bits = torch.from_numpy(wl["bits"]).cuda()
    pb = ocd.problem(B, U, W, S, Q, K, "hybrid", "f32", N0, 1.0, beta)
    ws = torch.zeros(ocd.ocd_backward_workspace_bytes(pb), dtype=torch.uint8, device="cuda")
    outs = []
    for full in (True, False, True):
        loss = torch.empty(1, device="cuda")
        dlam = torch.empty(K, device="cuda")
        dbeta = torch.empty(1, device="cuda")
        z = torch.empty(W, S, U, dtype=torch.complex64, device="cuda") if full else None
        L = torch.empty(W, S, U, Q, device="cuda") if full else None
        dy = torch.empty(W, S, B, dtype=torch.complex64, device="cuda") if full else None
        ocd.ocd_detect_train_bce(pb, H, y, lam_t, bits, z, L, loss, dlam, dbeta, dy, ws)
        outs.append((loss, dlam, dbeta, z, L, dy))
    torch.cuda.synchronize()
    for o in outs[1:]:
        for a, b in zip(o[:3], outs[0][:3]):
            assert torch.equal(a, b)
    for a, b in zip(outs[2][3:], outs[0][3:]):
        assert torch.equal(a, b)
    assert int(host(ws[:4].view(torch.int32))[0]) == 0


def test_train_autotuner_keeps_the_results(ocd):
    """ocd_autotune_train picks and caches a plan; the training step under it gives the
    untuned step's loss and gradients (FP32 rounding apart) and reports it."""
    B, U, W, S, Q, K = 128, 16, 44, 4, 4, 4
    wl, N0, lam, beta = _setup("hybrid", B, U, W, S, Q, K, seed=4)
    H, y, lam_t = dev(wl["H"]), dev(wl["y"]), dev(lam)
    bits = torch.from_numpy(wl["bits"]).cuda()
    pb = ocd.problem(B, U, W, S, Q, K, "hybrid", "f32", N0, 1.0, beta)
    before = ocd.train_step(H, y, bits, K, Q, "hybrid", N0, 1.0, beta, lam=lam_t)
    ws = torch.zeros(ocd.ocd_backward_workspace_bytes(pb), dtype=torch.uint8, device="cuda")
    loss, dlam, dbeta = (torch.empty(1, device="cuda"), torch.empty(K, device="cuda"),
                         torch.empty(1, device="cuda"))
    dy = torch.empty(W, S, B, dtype=torch.complex64, device="cuda")
    tuned = ocd.ocd_autotune_train(pb, H, y, lam_t, bits, loss, dlam, dbeta, dy, ws, repeats=1)
    say("  tuned train plan", tuned.as_dict())
    assert ocd.ocd_train_plan(pb).as_dict() == tuned.as_dict()
    after = ocd.train_step(H, y, bits, K, Q, "hybrid", N0, 1.0, beta, lam=lam_t)
    torch.cuda.synchronize()
    assert abs(float(host(after[0])[0]) - float(host(before[0])[0])) <= \
        LOSS_TOL * float(host(before[0])[0])
    assert rel(host(after[1]), host(before[1])) <= GRAD_TOL
    assert abs(float(host(after[2])[0]) - float(host(before[2])[0])) <= \
        GRAD_TOL * abs(float(host(before[2])[0]))
    assert rel(host(after[3]), host(before[3])) <= GRAD_TOL


def test_train_step_rejects_bad_arguments(ocd):
    B, U, W, S, Q, K = 64, 4, 4, 2, 4, 2
    pb = ocd.problem(B, U, W, S, Q, K, "hybrid", "f32", 0.1, 1.0, 0.7)
    H = torch.zeros(W, U, B, dtype=torch.complex64, device="cuda")
    y = torch.zeros(W, S, B, dtype=torch.complex64, device="cuda")
    bits = torch.zeros(W, S, U, Q, dtype=torch.uint8, device="cuda")
    loss, dlam, dbeta = (torch.empty(1, device="cuda"), torch.empty(K, device="cuda"),
                         torch.empty(1, device="cuda"))
    small = torch.zeros(ocd.ocd_backward_workspace_bytes(pb) - 16, dtype=torch.uint8,
                        device="cuda")
    with pytest.raises(ValueError):   # the binding checks the size before the library
        ocd.ocd_detect_train_bce(pb, H, y, None, bits, None, None, loss, dlam, dbeta, None, small)
    st = ocd._lib.ocd_detect_train_bce(
        ocd.ctypes.byref(pb),
        H.data_ptr(), y.data_ptr(), None, bits.data_ptr(), None, None, None, dlam.data_ptr(),
        dbeta.data_ptr(), None, small.data_ptr(), small.numel(), None)
    assert st == -1   # OCD_EINVAL: no loss output


def test_train_step_at_the_full_differentiable_workload(ocd):
    """The differentiable workload the benchmark times, whole: B=128, U=16, 2048
    subcarriers x 4 symbols, 16-QAM, K=4, HYBRID, 10 dB, one training-step launch;
    against the oracle's loss and reverse mode seeded from its own LLRs and the bits."""
    B, U, W, S, Q, K = 128, 16, 2048, 4, 4, 4
    wl = synth.make_workload(B, U, W, S, Q, 10.0, seed=[20, 11])
    N0 = f32(wl["N0"])
    lam = np.full(K, N0, np.float32)
    beta = f32(3 / np.sqrt(10))
    H, y = dev(wl["H"]), dev(wl["y"])
    bits = torch.from_numpy(wl["bits"]).cuda()
    say("train full workload, plan",
        ocd.ocd_train_plan(ocd.problem(B, U, W, S, Q, K, "hybrid", "f32", N0, 1.0, beta)).as_dict())
    loss, dlam, dbeta, dy, _, _ = ocd.train_step(H, y, bits, K, Q, "hybrid", N0, 1.0, beta,
                                                 lam=dev(lam))
    torch.cuda.synchronize()
    _, Lo = oracle.detect(wl["H"], wl["y"], K, Q, "hybrid", N0=N0, lam=lam, beta=beta, threads=0)
    loss_o = float(np.mean(np.logaddexp(0.0, np.where(wl["bits"] != 0, -Lo, Lo))))
    dllr_o = (scipy.special.expit(Lo) - wl["bits"]) / wl["bits"].size
    dlam_o, dbeta_o, dy_o = oracle.grad(wl["H"], wl["y"], dllr_o, K, Q, "hybrid", N0=N0, lam=lam,
                                        beta=beta)
    say("  loss gpu %.9g oracle %.9g" % (float(host(loss)[0]), loss_o))
    say("  dlam gpu", host(dlam), "oracle", dlam_o)
    assert abs(float(host(loss)[0]) - loss_o) <= 1e-4 * loss_o
    assert rel(host(dlam), dlam_o) <= GRAD_TOL
    assert rel(host(dy), dy_o) <= GRAD_TOL
    assert abs(float(host(dbeta)[0]) - dbeta_o) <= GRAD_TOL * abs(dbeta_o)
