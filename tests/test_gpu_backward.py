"""GPU parity of the adjoint kernel (ocd_detect_backward) and of the autograd
wrapper: gradients of the bit cross-entropy of the LLRs with respect to the
per-sweep regularisers, the box half-width and y, against the FP64 oracle's
reverse mode and against FP64 central differences of the oracle's forward pass;
relative L2 error within 1e-3 for each gradient."""

import numpy as np
import pytest
import scipy.special
import torch

import fd_util
import oracle
import synth
from gpu_util import dev, host, say

pytestmark = pytest.mark.gpu

GRAD_TOL = 1e-3


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


def _bce(L, bits):
    return float(np.mean(np.logaddexp(0.0, np.where(bits != 0, -L, L))))


def _case(ocd, mode, B=128, U=16, W=32, S=4, Q=4, K=4, snr=10.0, seed=0):
    """Slice of the differentiable workload: B=128, U=16, 32 subcarriers x 4 symbols,
    16-QAM, K=4, 10 dB."""
    say("backward case mode=%s B=%d U=%d W=%d S=%d Q=%d K=%d" % (mode, B, U, W, S, Q, K))
    wl = synth.make_workload(B, U, W, S, Q, snr, seed=[20, seed])
    N0 = f32(wl["N0"])
    lam = np.full(K, N0, np.float32) * np.array([1.0, 0.8, 1.3, 0.9, 1.1, 1.0][:K], np.float32) \
        if mode == "hybrid" else None
    beta = f32(0.9 * 3 / np.sqrt(10)) if mode != "mmse" else 0.0
    H, y = dev(wl["H"]), dev(wl["y"])
    lam_t = dev(lam) if lam is not None else None
    _, L, zh = ocd.detect(H, y, K, Q, mode, N0, 1.0, beta, lam=lam_t, want_z=False, want_hist=True)
    bits = torch.from_numpy(wl["bits"]).cuda().float()
    dllr = (torch.sigmoid(L) - bits) / bits.numel()
    dlam, dbeta, dy = ocd.backward(H, y, zh, dllr, K, Q, mode, N0, 1.0, beta, lam=lam_t)
    torch.cuda.synchronize()
    return dict(wl=wl, N0=N0, lam=lam, beta=beta, K=K, Q=Q, L=host(L), dllr=host(dllr),
                dlam=host(dlam), dbeta=float(host(dbeta)[0]), dy=host(dy), H=H, y=y, zh=zh,
                lam_t=lam_t, dllr_t=dllr)


@pytest.mark.parametrize("mode", ["hybrid", "box", "mmse"])
def test_adjoint_matches_oracle_reverse_mode(ocd, mode):
    c = _case(ocd, mode)
    wl = c["wl"]
    dlam_o, dbeta_o, dy_o = oracle.grad(wl["H"], wl["y"], c["dllr"].astype(np.float64), c["K"],
                                        c["Q"], mode, N0=c["N0"], lam=c["lam"], beta=c["beta"])
    say("  dlam gpu", c["dlam"], "oracle", dlam_o)
    say("  dbeta gpu %.6g oracle %.6g" % (c["dbeta"], dbeta_o))
    assert rel(c["dlam"], dlam_o) <= GRAD_TOL
    assert rel(c["dy"], dy_o) <= GRAD_TOL
    if mode == "mmse":
        assert c["dbeta"] == 0.0
    else:
        assert dbeta_o != 0.0
        assert abs(c["dbeta"] - dbeta_o) <= GRAD_TOL * abs(dbeta_o)


@pytest.mark.parametrize("mode", ["hybrid", "box"])
def test_adjoint_matches_fp64_finite_differences(ocd, mode):
    """The GPU adjoint against FP64 finite differences of the oracle's loss (Algorithm 1,
    the soft output, the mean bit cross-entropy) on a 32-subcarrier slice of the
    differentiable workload.  Every difference is taken across a step that leaves the
    oracle's active set unchanged (clip sides and max-log minimisers; the step is halved
    up to four times, then the coordinate is excluded and counted; tests/fd_util.py).
    Held to 1e-3 relative L2, separately for d lambda, d beta and a sample of dy.

    Regularisers: HYBRID takes central differences at the learnable lambda_k.  BOX runs
    with lambda_k = 0, the edge of their domain, so its differences are one-sided
    (second order) and lambda_K is left out: the soft output switches from the
    matched-filter SINR at lambda_K = 0 to g / lambda_K above it (reading C3), so the
    loss is not continuous there; the sweep lambdas enter only through d_u^-1 and p_u."""
    c = _case(ocd, mode, seed=1)
    wl = c["wl"]
    H = wl["H"].astype(np.complex128)
    y = wl["y"].astype(np.complex128)
    bits = wl["bits"]
    K, Q, N0, beta = c["K"], c["Q"], c["N0"], c["beta"]
    nbits = bits.size
    lam0 = c["lam"].astype(np.float64) if mode == "hybrid" else np.zeros(K)

    def evaluate(lam, beta_, Hs=H, ys=y, bs=bits):
        z = oracle.ocd(Hs, ys, K, Q, mode, N0=N0, lam=lam, beta=beta_, threads=0)
        L = oracle.llr(Hs, z, K, Q, mode, N0=N0, lam=lam, beta=beta_, threads=0)
        act = oracle.active_set(Hs, ys, K, Q, mode, N0=N0, lam=lam, beta=beta_)
        return fd_util.bce_sum(L, bs) / nbits, act

    excluded = 0
    # d lambda_k
    ks = list(range(K)) if mode == "hybrid" else list(range(K - 1))
    fd_lam, gpu_lam = [], []
    for k in ks:
        def f(v, k=k):
            l2 = lam0.copy()
            l2[k] = v
            return evaluate(l2, beta)
        d = fd_util.central(f, lam0[k]) if mode == "hybrid" else fd_util.one_sided(f, 0.0)
        if d is None:
            excluded += 1
            continue
        fd_lam.append(d)
        gpu_lam.append(c["dlam"][k])
    # d beta
    fdb = fd_util.central(lambda v: evaluate(lam0, v), beta)
    # dy: 24 (vector, antenna) entries, real and imaginary part; only that vector's bits
    # change, so its loss alone is differenced
    W, S, B = y.shape
    rng = np.random.default_rng(11)
    fd_y, gpu_y = [], []
    for _ in range(24):
        w, s_, b = int(rng.integers(W)), int(rng.integers(S)), int(rng.integers(B))
        for part in (1.0, 1j):
            def f(v, w=w, s_=s_, b=b, part=part):
                yv = y[w:w + 1, s_:s_ + 1].copy()
                yv[0, 0, b] += part * v
                return evaluate(lam0, beta, H[w:w + 1], yv, bits[w:w + 1, s_:s_ + 1])
            d = fd_util.central(f, 0.0)
            if d is None:
                excluded += 1
                continue
            fd_y.append(d)
            gpu_y.append(c["dy"][w, s_, b].real if part == 1.0 else c["dy"][w, s_, b].imag)
    say("  %s: fd dlam %s gpu %s" % (mode, np.array(fd_lam), np.array(gpu_lam)))
    say("  %s: fd dbeta %s gpu %.8g; dy entries %d; excluded coordinates %d"
        % (mode, fdb, c["dbeta"], len(fd_y), excluded))
    assert excluded <= 2, excluded
    assert len(fd_lam) >= len(ks) - 1
    e_lam = rel(gpu_lam, fd_lam)
    e_y = rel(gpu_y, fd_y)
    say("  %s: rel err dlam %.3g dy %.3g" % (mode, e_lam, e_y))
    assert e_lam <= GRAD_TOL, e_lam
    assert e_y <= GRAD_TOL, e_y
    assert fdb is not None
    e_b = abs(c["dbeta"] - fdb) / abs(fdb)
    say("  %s: rel err dbeta %.3g" % (mode, e_b))
    assert e_b <= GRAD_TOL, e_b


def test_adjoint_is_bitwise_reproducible(ocd):
    c = _case(ocd, "hybrid", W=16, seed=2)
    d2 = ocd.backward(c["H"], c["y"], c["zh"], c["dllr_t"], c["K"], c["Q"], "hybrid", c["N0"], 1.0,
                      c["beta"], lam=c["lam_t"])
    torch.cuda.synchronize()
    assert np.array_equal(host(d2[0]), c["dlam"])
    assert np.array_equal(host(d2[2]), c["dy"])


@pytest.mark.parametrize("case", [(33, 5, 7, 3, 6, 2, "box"), (256, 32, 4, 14, 2, 3, "hybrid"),
                                  (16, 4, 3, 1, 4, 9, "mmse"),
                                  # S = 1: z_hist from the channel-in-registers forward plan
                                  (128, 8, 20, 1, 6, 3, "hybrid")])
def test_adjoint_edge_shapes(ocd, case):
    B, U, W, S, Q, K, mode = case
    c = _case(ocd, mode, B, U, W, S, Q, K, 8.0, seed=3)
    wl = c["wl"]
    dlam_o, dbeta_o, dy_o = oracle.grad(wl["H"], wl["y"], c["dllr"].astype(np.float64), K, Q, mode,
                                        N0=c["N0"], lam=c["lam"], beta=c["beta"])
    assert rel(c["dlam"], dlam_o) <= GRAD_TOL
    assert rel(c["dy"], dy_o) <= GRAD_TOL
    if mode != "mmse" and dbeta_o != 0.0:
        assert abs(c["dbeta"] - dbeta_o) <= GRAD_TOL * abs(dbeta_o)


def test_backward_autotuner_keeps_the_gradients(ocd):
    """The adjoint autotuner returns an LDS plan; gradients with the tuned plan equal
    those of the default plan up to the order of the partial sums."""
    B, U, W, S, Q, K = 128, 16, 24, 4, 4, 4
    c = _case(ocd, "hybrid", B, U, W, S, Q, K, seed=4)
    pb = ocd.problem(B, U, W, S, Q, K, "hybrid", "f32", c["N0"], 1.0, c["beta"])
    dlam = torch.empty(K, device="cuda")
    dbeta = torch.empty(1, device="cuda")
    dy = torch.empty(W, S, B, dtype=torch.complex64, device="cuda")
    ws = torch.zeros(ocd.ocd_backward_workspace_bytes(pb), dtype=torch.uint8, device="cuda")
    plan = ocd.ocd_autotune_backward(pb, c["H"], c["y"], c["lam_t"], c["zh"], c["dllr_t"], dlam,
                                     dbeta, dy, ws, repeats=1)
    say("  tuned adjoint plan", plan.as_dict())
    assert plan.lanes_per_vector in (4, 8, 16, 32) and plan.channel_in_registers == 0
    d2 = ocd.backward(c["H"], c["y"], c["zh"], c["dllr_t"], K, Q, "hybrid", c["N0"], 1.0, c["beta"],
                      lam=c["lam_t"])
    torch.cuda.synchronize()
    assert rel(host(d2[0]), c["dlam"]) <= 1e-5
    assert rel(host(d2[2]), c["dy"]) <= 1e-6
    assert abs(float(host(d2[1])[0]) - c["dbeta"]) <= 1e-5 * abs(c["dbeta"])


def test_autograd_function_drives_the_kernels(ocd):
    from paper_1611_08779_amd.autograd import ocd_llr
    B, U, W, S, Q, K = 128, 16, 16, 4, 4, 4
    wl = synth.make_workload(B, U, W, S, Q, 10.0, seed=[21, 0])
    N0 = f32(wl["N0"])
    H = dev(wl["H"])
    y = dev(wl["y"]).requires_grad_(True)
    lam = torch.full((K,), N0, device="cuda", requires_grad=True)
    beta = torch.tensor([3 / np.sqrt(10)], device="cuda", dtype=torch.float32, requires_grad=True)
    L = ocd_llr(y, H, K, Q, "hybrid", N0, 1.0, lam, beta)
    bits = torch.from_numpy(wl["bits"]).cuda().float()
    loss = torch.nn.functional.binary_cross_entropy_with_logits(L, bits)
    loss.backward()
    torch.cuda.synchronize()
    dlam_o, dbeta_o, dy_o = oracle.grad(wl["H"], wl["y"],
                                        host((torch.sigmoid(L) - bits) / bits.numel()).astype(np.float64),
                                        K, Q, "hybrid", N0=N0, lam=host(lam.detach()),
                                        beta=float(host(beta.detach())[0]))
    assert rel(host(lam.grad), dlam_o) <= GRAD_TOL
    assert rel(host(y.grad), dy_o) <= GRAD_TOL
    assert abs(float(host(beta.grad)[0]) - dbeta_o) <= GRAD_TOL * max(abs(dbeta_o), 1e-12)


@pytest.mark.parametrize("mode", ["hybrid", "box", "mmse"])
def test_fused_cross_entropy_adjoint(ocd, mode):
    """ocd_detect_backward_bce forms dLoss/dLLR = (sigmoid(L) - bit) / N itself from
    the bits: the same gradients as the two-step path (torch's sigmoid of the
    forward LLRs, then ocd_detect_backward), and as the FP64 oracle's reverse mode
    seeded from the oracle's own LLRs and the same bits."""
    c = _case(ocd, mode)
    wl = c["wl"]
    bits_u8 = torch.from_numpy(wl["bits"].astype(np.uint8)).cuda()
    dlam, dbeta, dy = ocd.backward(c["H"], c["y"], c["zh"], None, c["K"], c["Q"], mode, c["N0"],
                                   1.0, c["beta"], lam=c["lam_t"], bits=bits_u8)
    torch.cuda.synchronize()
    say("  fused dlam", host(dlam), "two-step", c["dlam"])
    assert rel(host(dlam), c["dlam"]) <= 1e-4
    assert rel(host(dy), c["dy"]) <= 1e-4
    assert abs(float(host(dbeta)[0]) - c["dbeta"]) <= 1e-4 * max(abs(c["dbeta"]), 1e-12)
    _, Lo = oracle.detect(wl["H"], wl["y"], c["K"], c["Q"], mode, N0=c["N0"], lam=c["lam"],
                          beta=c["beta"])
    dllr_o = (scipy.special.expit(Lo) - wl["bits"]) / wl["bits"].size
    dlam_o, dbeta_o, dy_o = oracle.grad(wl["H"], wl["y"], dllr_o, c["K"], c["Q"], mode,
                                        N0=c["N0"], lam=c["lam"], beta=c["beta"])
    assert rel(host(dlam), dlam_o) <= GRAD_TOL
    assert rel(host(dy), dy_o) <= GRAD_TOL
    if mode != "mmse":
        assert abs(float(host(dbeta)[0]) - dbeta_o) <= GRAD_TOL * abs(dbeta_o)


def test_fused_loss_function_matches_llr_function_plus_torch_loss(ocd):
    """ocd_bce_loss (one training-step launch: the loss summed in FP32 in the kernel and
    its gradients) gives the loss and the gradients of ocd_llr followed by torch's BCE
    with logits, including a non-unit upstream gradient."""
    from paper_1611_08779_amd.autograd import ocd_bce_loss, ocd_llr
    B, U, W, S, Q, K = 128, 16, 16, 4, 4, 4
    wl = synth.make_workload(B, U, W, S, Q, 10.0, seed=[21, 1])
    N0 = f32(wl["N0"])
    H = dev(wl["H"])
    bits = torch.from_numpy(wl["bits"]).cuda()
    grads = []
    for fused in (False, True):
        y = dev(wl["y"]).requires_grad_(True)
        lam = torch.full((K,), N0, device="cuda", requires_grad=True)
        beta = torch.tensor([3 / np.sqrt(10)], device="cuda", dtype=torch.float32,
                            requires_grad=True)
        if fused:
            loss = ocd_bce_loss(y, H, bits, K, Q, "hybrid", N0, 1.0, lam, beta)
        else:
            L = ocd_llr(y, H, K, Q, "hybrid", N0, 1.0, lam, beta)
            loss = torch.nn.functional.binary_cross_entropy_with_logits(L, bits.float())
        (2.5 * loss).backward()
        torch.cuda.synchronize()
        grads.append((float(loss.detach()), host(lam.grad), float(host(beta.grad)[0]), host(y.grad)))
    (l0, gl0, gb0, gy0), (l1, gl1, gb1, gy1) = grads
    assert abs(l1 - l0) <= 1e-5 * abs(l0)
    assert rel(gl1, gl0) <= 1e-4
    assert rel(gy1, gy0) <= 1e-4
    assert abs(gb1 - gb0) <= 1e-4 * max(abs(gb0), 1e-12)


def test_fused_cross_entropy_adjoint_empty_and_fp16(ocd):
    """The fused adjoint on an empty problem writes zero gradients; with FP16 storage
    of H and y it gives the two-step path's gradients."""
    K, Q = 3, 4
    pb = ocd.problem(64, 4, 0, 2, Q, K, "hybrid", "f32", 0.1, 1.0, 0.7)
    H = torch.empty(0, 4, 64, dtype=torch.complex64, device="cuda")
    y = torch.empty(0, 2, 64, dtype=torch.complex64, device="cuda")
    zh = torch.empty(0, 2, K, 4, dtype=torch.complex64, device="cuda")
    bits = torch.empty(0, 2, 4, Q, dtype=torch.uint8, device="cuda")
    lam = torch.full((K,), 0.1, device="cuda")
    dlam = torch.full((K,), 7.0, device="cuda")
    dbeta = torch.full((1,), 7.0, device="cuda")
    ws = torch.zeros(ocd.ocd_backward_workspace_bytes(pb), dtype=torch.uint8, device="cuda")
    ocd.ocd_detect_backward_bce(pb, H, y, lam, zh, bits, dlam, dbeta, None, ws)
    torch.cuda.synchronize()
    assert np.all(host(dlam) == 0.0) and host(dbeta)[0] == 0.0

    B, U, W, S = 128, 8, 24, 4
    wl = synth.make_workload(B, U, W, S, Q, 10.0, seed=[20, 9])
    N0 = f32(wl["N0"])
    pairs = lambda a: torch.view_as_real(dev(a)).to(torch.float16).contiguous()
    H16, y16 = pairs(wl["H"]), pairs(wl["y"])
    lam = torch.full((K,), N0, device="cuda")
    beta = f32(0.9 * 3 / np.sqrt(10))
    _, L, zh = ocd.detect(H16, y16, K, Q, "hybrid", N0, 1.0, beta, lam=lam, storage="f16",
                          want_z=False, want_hist=True)
    bits = torch.from_numpy(wl["bits"]).cuda()
    dllr = (torch.sigmoid(L) - bits.float()) / bits.numel()
    two = ocd.backward(H16, y16, zh, dllr, K, Q, "hybrid", N0, 1.0, beta, lam=lam, storage="f16")
    fused = ocd.backward(H16, y16, zh, None, K, Q, "hybrid", N0, 1.0, beta, lam=lam, storage="f16",
                         bits=bits)
    torch.cuda.synchronize()
    assert rel(host(fused[0]), host(two[0])) <= 1e-4
    assert rel(host(fused[2]), host(two[2])) <= 1e-4
    assert abs(float(host(fused[1])[0]) - float(host(two[1])[0])) <= \
        1e-4 * max(abs(float(host(two[1])[0])), 1e-12)


def test_fused_adjoint_at_the_full_differentiable_workload(ocd):
    """The differentiable workload the benchmark times, whole: B=128, U=16, 2048
    subcarriers x 4 symbols, 16-QAM, K=4, HYBRID, 10 dB, with the fused cross-entropy
    adjoint; against the oracle's reverse mode seeded from its own LLRs and the bits."""
    B, U, W, S, Q, K = 128, 16, 2048, 4, 4, 4
    wl = synth.make_workload(B, U, W, S, Q, 10.0, seed=[20, 11])
    N0 = f32(wl["N0"])
    lam = np.full(K, N0, np.float32)
    beta = f32(3 / np.sqrt(10))
    H, y = dev(wl["H"]), dev(wl["y"])
    _, _, zh = ocd.detect(H, y, K, Q, "hybrid", N0, 1.0, beta, lam=dev(lam), want_z=False,
                          want_hist=True)
    bits = torch.from_numpy(wl["bits"]).cuda()
    dlam, dbeta, dy = ocd.backward(H, y, zh, None, K, Q, "hybrid", N0, 1.0, beta, lam=dev(lam),
                                   bits=bits)
    torch.cuda.synchronize()
    _, Lo = oracle.detect(wl["H"], wl["y"], K, Q, "hybrid", N0=N0, lam=lam, beta=beta, threads=0)
    dllr_o = (scipy.special.expit(Lo) - wl["bits"]) / wl["bits"].size
    dlam_o, dbeta_o, dy_o = oracle.grad(wl["H"], wl["y"], dllr_o, K, Q, "hybrid", N0=N0, lam=lam,
                                        beta=beta)
    say("  dlam gpu", host(dlam), "oracle", dlam_o)
    assert rel(host(dlam), dlam_o) <= GRAD_TOL
    assert rel(host(dy), dy_o) <= GRAD_TOL
    assert abs(float(host(dbeta)[0]) - dbeta_o) <= GRAD_TOL * abs(dbeta_o)
