"""The entry points inside captured graphs (torch.cuda.CUDAGraph over the caller's
stream), the way the benchmark times them and a serving loop would run them:
every replay, with eager work and synchronisation between replays, equals the
eager call on the same buffers bit for bit.  None of these entry points records a
memset or allocates device memory, so their captured launches replay unchanged;
the training step's and the adjoint's completion counters return to zero at the
end of every launch, so their workspaces need no clearing between replays."""

import numpy as np
import pytest
import torch

import synth
from gpu_util import dev, say

pytestmark = pytest.mark.gpu

REPLAYS = 5


@pytest.fixture(scope="module")
def ocd():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_1611_08779_amd as m
    return m


def _capture_and_replay(call, outputs, name):
    """Runs `call` eagerly (the reference), captures it into a graph, clears the
    outputs, then replays the graph REPLAYS times with eager work between the
    replays; returns how many replays matched."""
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        call()                      # warm the plan cache outside capture
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    ref = [o.clone() for o in outputs]
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        call()
    torch.cuda.synchronize()
    ok = 0
    for rep in range(REPLAYS):
        for o in outputs:
            o.fill_(float("nan")) if o.is_floating_point() or o.is_complex() else o.zero_()
        g.replay()
        torch.cuda.synchronize()
        _ = (torch.randn(4096, device="cuda") ** 2).sum().item()   # eager work between
        for o, r in zip(outputs, ref):
            assert torch.equal(o, r), (name, rep)
        ok += 1
    say("  %s: %d replays equal the eager call" % (name, ok))
    return ok


def test_detection_in_a_graph(ocd):
    B, U, W, S, Q, K = 128, 8, 60, 14, 6, 3
    wl = synth.make_workload(B, U, W, S, Q, 20.0, seed=[120, 0])
    N0 = float(np.float32(wl["N0"]))
    pb = ocd.problem(B, U, W, S, Q, K, "mmse", "f32", N0)
    ocd.ocd_set_plan(pb, ocd.Plan(16, 14, 1, 0, 2))   # staggered, XCD-ordered
    H, y = dev(wl["H"]), dev(wl["y"])
    z = torch.empty(W, S, U, dtype=torch.complex64, device="cuda")
    L = torch.empty(W, S, U, Q, device="cuda")
    zh = torch.empty(W, S, K, U, dtype=torch.complex64, device="cuda")
    assert _capture_and_replay(lambda: ocd.ocd_detect(pb, H, y, z=z, llr=L, z_hist=zh),
                               [z, L, zh], "ocd_detect") == REPLAYS


@pytest.mark.parametrize("mode", ["hybrid", "box"])
def test_training_step_and_adjoints_in_a_graph(ocd, mode):
    B, U, W, S, Q, K = 128, 16, 32, 4, 4, 4
    wl = synth.make_workload(B, U, W, S, Q, 10.0, seed=[120, 1])
    N0 = float(np.float32(wl["N0"]))
    beta = float(np.float32(0.9 * 3 / np.sqrt(10)))
    lam = dev(np.full(K, N0, np.float32)) if mode == "hybrid" else None
    pb = ocd.problem(B, U, W, S, Q, K, mode, "f32", N0, 1.0, beta)
    H, y = dev(wl["H"]), dev(wl["y"])
    bits = torch.from_numpy(wl["bits"]).cuda()
    ws = torch.zeros(ocd.ocd_backward_workspace_bytes(pb), dtype=torch.uint8, device="cuda")
    loss = torch.empty(1, device="cuda")
    dlam = torch.empty(K, device="cuda")
    dbeta = torch.empty(1, device="cuda")
    dy = torch.empty(W, S, B, dtype=torch.complex64, device="cuda")
    assert _capture_and_replay(
        lambda: ocd.ocd_detect_train_bce(pb, H, y, lam, bits, None, None, loss, dlam, dbeta, dy, ws),
        [loss, dlam, dbeta, dy], "ocd_detect_train_bce") == REPLAYS
    assert int(ws[:4].view(torch.int32)[0]) == 0          # the completion counter is back at zero
    # the two-launch adjoint on a workspace, and the no-allocation one on the static scratch
    zh = torch.empty(W, S, K, U, dtype=torch.complex64, device="cuda")
    ocd.ocd_detect(pb, H, y, lam, z=None, llr=None, z_hist=zh)
    torch.cuda.synchronize()
    dl2, db2 = torch.empty(K, device="cuda"), torch.empty(1, device="cuda")
    dy2 = torch.empty(W, S, B, dtype=torch.complex64, device="cuda")
    assert _capture_and_replay(
        lambda: ocd.ocd_detect_backward_bce(pb, H, y, lam, zh, bits, dl2, db2, dy2, ws),
        [dl2, db2, dy2], "ocd_detect_backward_bce") == REPLAYS
    dl3, db3 = torch.empty(K, device="cuda"), torch.empty(1, device="cuda")
    dy3 = torch.empty(W, S, B, dtype=torch.complex64, device="cuda")
    assert _capture_and_replay(
        lambda: ocd.ocd_detect_backward_bce_noalloc(pb, H, y, lam, zh, bits, dl3, db3, dy3),
        [dl3, db3, dy3], "ocd_detect_backward_bce_noalloc") == REPLAYS
    assert torch.equal(dy2, dy3) and torch.equal(dl2, dl3) and torch.equal(db2, db3)


def test_mmse_and_ofdm_in_a_graph(ocd):
    B, U, W, S, Q = 128, 8, 40, 14, 6
    wl = synth.make_workload(B, U, W, S, Q, 20.0, seed=[120, 2])
    N0 = float(np.float32(wl["N0"]))
    pb = ocd.problem(B, U, W, S, Q, 1, "mmse", "f32", N0)
    H, y = dev(wl["H"]), dev(wl["y"])
    z = torch.empty(W, S, U, dtype=torch.complex64, device="cuda")
    L = torch.empty(W, S, U, Q, device="cuda")
    for plan in (ocd.Plan(8, 14, 0, 0), ocd.Plan(0, 14, 0, 0)):   # VALU and matrix-core forms
        assert _capture_and_replay(lambda: ocd.ocd_detect_mmse(pb, H, y, z, L, plan), [z, L],
                                   "ocd_detect_mmse %d" % plan.lanes_per_vector) == REPLAYS
    N, Ncp, Wo, Bo, So = 2048, 144, 1200, 16, 3
    rng = np.random.default_rng([120, 3])
    x = dev((rng.normal(size=(Bo, So, Ncp + N)) + 1j * rng.normal(size=(Bo, So, Ncp + N)))
            .astype(np.complex64))
    yo = torch.empty(Wo, So, Bo, dtype=torch.complex64, device="cuda")
    sh = ocd.OfdmShape(Bo, So, N, Ncp, Wo)
    assert _capture_and_replay(lambda: ocd.ocd_ofdm_demodulate(sh, x, yo), [yo],
                               "ocd_ofdm_demodulate") == REPLAYS
