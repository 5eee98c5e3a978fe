"""Arrays past 4 GiB: the kernels address caller buffers from a 64-bit workgroup
base plus 32-bit lane offsets, so a byte offset formed in 32 bits anywhere would
show up here.  The headline shape widened to 300,000 subcarriers (4.2 M vectors:
y 4.3 GB, H 2.5 GB) in FP32 and FP16 storage, checked against the oracle on
subcarriers spread over the whole range up to the last one; one H per vector on
the register path with 2.2 M vectors (H 18 GB); and the training step on the wide
shape, whose dy (4.3 GB) must equal the two-launch path's bit for bit at the far
end of the array."""

import numpy as np
import pytest
import torch

import oracle
import synth
from gpu_util import (LLR_TOL_F32, Z_TOL_F32, from_f16_pairs, host, llr_rel_err, say, z_rel_err)

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ocd():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_1611_08779_amd as m
    return m


def _as_f16(t):
    return torch.view_as_real(t).to(torch.float16).contiguous()


def _check_sampled(wl, z, L, ws, K, Q, mode, N0, f16=False, beta=0.0):
    H = wl["H"][ws].cpu().numpy()
    y = wl["y"][ws].cpu().numpy()
    if f16:   # the oracle on exactly the values the GPU received
        H = from_f16_pairs(_as_f16(wl["H"][ws]).cpu().numpy())
        y = from_f16_pairs(_as_f16(wl["y"][ws]).cpu().numpy())
    zo, Lo = oracle.detect(H, y, K, Q, mode, N0=N0, beta=beta, threads=0)
    ez, el = z_rel_err(host(z[ws]), zo), llr_rel_err(host(L[ws]), Lo)
    say("  sampled subcarriers %s: z err %.3g, llr err %.3g" % (list(ws[-3:]), ez, el))
    assert ez <= Z_TOL_F32, ez
    assert el <= LLR_TOL_F32, el


def _sample(W):
    return np.array(sorted(set([0, 1, W // 3, W // 2, (2 ** 31) // (14 * 128 * 8) % W,
                                W - 3, W - 2, W - 1])))


@pytest.mark.parametrize("storage", ["f32", "f16"])
def test_headline_shape_over_four_gib(ocd, storage):
    B, U, W, S, Q, K = 128, 8, 300_000, 14, 6, 3
    say("large case: B=%d U=%d W=%d S=%d (y %.2f GB) %s" % (B, U, W, S, W * S * B * 8 / 1e9, storage))
    wl = synth.make_workload_device(B, U, W, S, Q, 20.0, seed=777, device="cuda")
    N0 = float(np.float32(wl["N0"]))
    H, y = (wl["H"], wl["y"]) if storage == "f32" else (_as_f16(wl["H"]), _as_f16(wl["y"]))
    z, L, _ = ocd.detect(H, y, K, Q, "mmse", N0, storage=storage)
    torch.cuda.synchronize()
    _check_sampled(wl, z, L, _sample(W), K, Q, "mmse", N0, f16=storage == "f16")
    del wl, H, y, z, L
    torch.cuda.empty_cache()


def test_one_h_per_vector_over_four_gib(ocd):
    B, U, W, Q, K = 128, 8, 2_200_000, 6, 3
    say("large case S=1: %d vectors (H %.1f GB)" % (W, W * U * B * 8 / 1e9))
    wl = synth.make_workload_device(B, U, W, 1, Q, 20.0, seed=778, device="cuda")
    N0 = float(np.float32(wl["N0"]))
    pb = ocd.problem(B, U, W, 1, Q, K, "mmse", "f32", N0)
    ocd.ocd_set_plan(pb, ocd.Plan(32, 2, 0, 1))   # the register plan the S = 1 form takes
    z, L, _ = ocd.detect(wl["H"], wl["y"], K, Q, "mmse", N0)
    torch.cuda.synchronize()
    _check_sampled(wl, z, L, np.array([0, W // 2, W - 2, W - 1]), K, Q, "mmse", N0)
    del wl, z, L
    torch.cuda.empty_cache()


def test_training_step_over_four_gib(ocd):
    B, U, W, S, Q, K = 128, 8, 300_000, 14, 6, 3
    say("large training step: %d vectors (dy %.2f GB)" % (W * S, W * S * B * 8 / 1e9))
    wl = synth.make_workload_device(B, U, W, S, Q, 10.0, seed=779, device="cuda")
    N0 = float(np.float32(wl["N0"]))
    beta = float(np.float32(0.9 * 7 / np.sqrt(42)))
    pb = ocd.problem(B, U, W, S, Q, K, "box", "f32", N0, 1.0, beta)
    ocd.ocd_set_plan(pb, ocd.ocd_train_plan(pb))   # the two launches under the step's plan
    bits = wl["bits"]
    loss, dlam, dbeta, dy, z, L = ocd.train_step(wl["H"], wl["y"], bits, K, Q, "box", N0, 1.0,
                                                 beta, want_z=True, want_llr=True)
    z2, L2, zh = ocd.detect(wl["H"], wl["y"], K, Q, "box", N0, 1.0, beta, want_hist=True)
    del z2, L2
    _, _, dy2 = ocd.backward(wl["H"], wl["y"], zh, None, K, Q, "box", N0, 1.0, beta, bits=bits)
    torch.cuda.synchronize()
    tail = slice(W * S - 4 * S, W * S)   # the last four subcarriers, at offsets past 4 GiB
    a = dy.reshape(W * S, B)[tail]
    b = dy2.reshape(W * S, B)[tail]
    say("  dy at the far end: identical %s, |dy| %.3g" % (bool(torch.equal(a, b)),
                                                         float(a.abs().max())))
    assert torch.equal(a, b)
    assert torch.equal(dy, dy2)
    assert torch.isfinite(loss).all() and float(a.abs().max()) > 0
    _check_sampled(wl, z, L, np.array([0, W // 2, W - 1]), K, Q, "box", N0, beta=beta)
