"""Randomised GPU parity of the one-launch training step (ocd_detect_train_bce):
seeded draws of shape, mode and storage.

What is continuous in the inputs is held to the oracle: z and the LLRs per vector
(the FP32 bars) and the mean cross-entropy (1e-4 relative, down to FP32's range).  The gradients are held
to the two-launch path (ocd_detect with the z history, then ocd_detect_backward_bce,
the same device code for the reverse updates) on the same inputs, within 1e-4
relative L2: FP32 against FP32, the two launches may split the work differently.
Against the FP64 reverse mode a random draw could land a component on a clip
point or an LLR on a max-log level boundary, where the gradient jumps and the two
precisions may take different sides; the fixed cases of test_gpu_train and the
finite-difference procedure treat those points explicitly.
"""

import numpy as np
import pytest
import torch

import oracle
import synth
from gpu_util import (LLR_TOL_F32, Z_TOL_F32, dev, from_f16_pairs, host, llr_rel_err, say,
                      to_f16_pairs, z_rel_err)

pytestmark = pytest.mark.gpu

PATH_TOL = 1e-4


@pytest.fixture(scope="module")
def ocd():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_1611_08779_amd as m
    return m


def rel(a, b):
    a, b = np.asarray(a, np.complex128).ravel(), np.asarray(b, np.complex128).ravel()
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def _draw(seed, n):
    rng = np.random.default_rng(seed)
    out = []
    for i in range(n):
        B = int(rng.choice([int(rng.integers(2, 33)), int(rng.integers(33, 257))]))
        U = int(rng.integers(1, max(1, min(32, B // 2)) + 1))
        S = int(rng.choice([1, 2, 4, int(rng.integers(3, 15))]))
        W = int(rng.integers(1, max(1, 200 // S) + 1))
        out.append((i, B, U, W, S, int(rng.choice([2, 4, 6])), int(rng.integers(1, 6)),
                    str(rng.choice(["mmse", "box", "hybrid"])),
                    "f16" if rng.random() < 0.25 else "f32", round(float(rng.uniform(5.0, 20.0)), 1)))
    return out


CASES = _draw(20261208, 30)


@pytest.mark.parametrize("case", CASES, ids=["t%02d-%s" % (c[0], "-".join(map(str, c[1:9])))
                                             for c in CASES])
def test_random_train_step(ocd, case):
    i, B, U, W, S, Q, K, mode, storage, snr = case
    say("train case %s" % (case,))
    wl = synth.make_workload(B, U, W, S, Q, snr, seed=[99, i])
    N0 = float(np.float32(wl["N0"]))
    rng = np.random.default_rng([100, i])
    lam = (N0 * rng.uniform(0.5, 2.0, K)).astype(np.float32) if mode == "hybrid" else None
    beta = float(np.float32(0.9 * rng.uniform(0.8, 1.2))) if mode != "mmse" else 0.0
    if storage == "f16":
        H16, y16 = to_f16_pairs(wl["H"]), to_f16_pairs(wl["y"])
        H, y, Hr, yr = dev(H16), dev(y16), from_f16_pairs(H16), from_f16_pairs(y16)
    else:
        H, y, Hr, yr = dev(wl["H"]), dev(wl["y"]), wl["H"], wl["y"]
    lam_t = dev(lam) if lam is not None else None
    bits = torch.from_numpy(wl["bits"]).cuda()
    loss, dlam, dbeta, dy, z, L = ocd.train_step(H, y, bits, K, Q, mode, N0, 1.0, beta, lam=lam_t,
                                                 storage=storage, want_z=True, want_llr=True)
    z2, L2, zh = ocd.detect(H, y, K, Q, mode, N0, 1.0, beta, lam=lam_t, storage=storage,
                            want_hist=True)
    dlam2, dbeta2, dy2 = ocd.backward(H, y, zh, None, K, Q, mode, N0, 1.0, beta, lam=lam_t,
                                      storage=storage, bits=bits)
    torch.cuda.synchronize()
    zo, Lo = oracle.detect(Hr, yr, K, Q, mode, N0=N0, lam=lam, beta=beta, threads=0)
    ez, el = z_rel_err(host(z), zo), llr_rel_err(host(L), Lo)
    loss_o = float(np.mean(np.logaddexp(0.0, np.where(wl["bits"] != 0, -Lo, Lo))))
    say("  z err %.3g  llr err %.3g  loss %.9g oracle %.9g" % (ez, el, float(host(loss)[0]), loss_o))
    assert ez <= Z_TOL_F32, ez
    assert el <= LLR_TOL_F32, el
    # a loss near the bottom of FP32's range (every bit confidently right) keeps the
    # relative bar down to that range; below it the terms underflow to zero
    assert abs(float(host(loss)[0]) - loss_o) <= 1e-4 * loss_o + 1e-37
    assert rel(host(dy), host(dy2)) <= PATH_TOL
    assert rel(host(dlam), host(dlam2)) <= PATH_TOL
    if mode == "mmse":
        assert float(host(dbeta)[0]) == 0.0 and float(host(dbeta2)[0]) == 0.0
    else:
        b1, b2 = float(host(dbeta)[0]), float(host(dbeta2)[0])
        assert abs(b1 - b2) <= PATH_TOL * max(abs(b2), 1e-30) or b1 == b2
