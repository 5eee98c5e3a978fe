"""The adjoint entry point that allocates nothing, ocd_detect_backward_bce_noalloc,
against the workspace form it varies, ocd_detect_backward_bce, through the C ABI.

Two calls in a row on the library's static scratch, the second with a smaller problem
(fewer workgroups than the first left partial sums for): each equals the workspace
form bit for bit (same plan, same kernels, same reduction order) and so lies within the
gradient tolerance, 1e-3 relative, of it.  A problem whose partial sums do not fit the
scratch is rejected on the host with OCD_ESCRATCH, and the empty problem writes zero
gradients."""

import ctypes

import numpy as np
import pytest
import torch

import synth
from gpu_util import dev, host, say

pytestmark = pytest.mark.gpu

GRAD_TOL = 1e-3


@pytest.fixture(scope="module")
def ocd():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_1611_08779_amd as m
    return m


def _problem(ocd, B, U, W, S, Q, K, mode, seed):
    wl = synth.make_workload(B, U, W, S, Q, 10.0, seed=[30, seed])
    N0 = float(np.float32(wl["N0"]))
    beta = float(np.float32(0.9 * 3 / np.sqrt(10))) if mode != "mmse" else 0.0
    lam = None
    if mode == "hybrid":
        lam = torch.tensor(np.float32(N0) * np.array([1.0, 0.8, 1.3, 0.9, 1.1][:K], np.float32),
                           device="cuda")
    pb = ocd.problem(B, U, W, S, Q, K, mode, "f32", N0, 1.0, beta)
    H, y = dev(wl["H"]), dev(wl["y"])
    zh = torch.empty(W, S, K, U, dtype=torch.complex64, device="cuda")
    ocd.ocd_detect(pb, H, y, lam, z=None, llr=None, z_hist=zh)
    bits = torch.from_numpy(wl["bits"]).cuda()
    return pb, H, y, lam, zh, bits


def _outputs(pb):
    nan = float("nan")
    return (torch.full((pb.K,), nan, device="cuda"), torch.full((1,), nan, device="cuda"),
            torch.full((pb.W, pb.S, pb.B), complex(nan, nan), dtype=torch.complex64,
                       device="cuda"))


def _rel(a, b):
    a, b = np.asarray(a, np.complex128).ravel(), np.asarray(b, np.complex128).ravel()
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


@pytest.mark.parametrize("order", ["noalloc_first", "workspace_first"])
def test_noalloc_adjoint_matches_the_workspace_form_twice(ocd, order):
    cases = [(128, 16, 64, 4, 4, 4, "hybrid", 1),   # 256 vectors
             (64, 8, 9, 3, 6, 3, "box", 2)]         # then a smaller one: 27 vectors
    for B, U, W, S, Q, K, mode, seed in cases:
        say("noalloc case B=%d U=%d W=%d S=%d Q=%d K=%d %s (%s)" % (B, U, W, S, Q, K, mode, order))
        pb, H, y, lam, zh, bits = _problem(ocd, B, U, W, S, Q, K, mode, seed)
        ws = torch.zeros(ocd.ocd_backward_workspace_bytes(pb), dtype=torch.uint8, device="cuda")
        ref, got = _outputs(pb), _outputs(pb)

        def run_ws():
            ocd.ocd_detect_backward_bce(pb, H, y, lam, zh, bits, *ref, ws)

        def run_noalloc():
            ocd.ocd_detect_backward_bce_noalloc(pb, H, y, lam, zh, bits, *got)

        for f in ((run_noalloc, run_ws) if order == "noalloc_first" else (run_ws, run_noalloc)):
            f()
        torch.cuda.synchronize()
        r, g = [host(t) for t in ref], [host(t) for t in got]
        for name, a, b in zip(("dlambda", "dbeta", "dy"), g, r):
            assert np.all(np.isfinite(a)), name
            e = _rel(a, b)
            say("  %s rel diff %.3g, identical %s" % (name, e, np.array_equal(a, b)))
            assert e <= GRAD_TOL, (name, e)
            assert np.array_equal(a, b), name
        if mode == "box":
            assert r[0][0] != 0.0 or r[1][0] != 0.0


def test_noalloc_adjoint_over_a_random_sequence_of_shapes(ocd):
    """Twelve calls in a row on the shared scratch, seeded random shapes growing and
    shrinking (B, U, W, S, Q, K and the mode drawn; each within the scratch): every
    call equals the workspace form bit for bit, whatever the previous call left."""
    rng = np.random.default_rng(20261209)
    for n in range(12):
        B = int(rng.integers(2, 257))
        U = int(rng.integers(1, max(1, min(32, B // 2)) + 1))
        S = int(rng.integers(1, 9))
        W = int(rng.integers(1, max(1, 400 // S) + 1))
        Q, K = int(rng.choice([2, 4, 6])), int(rng.integers(1, 6))
        mode = str(rng.choice(["mmse", "box", "hybrid"]))
        say("noalloc sequence %d: B=%d U=%d W=%d S=%d Q=%d K=%d %s" % (n, B, U, W, S, Q, K, mode))
        pb, H, y, lam, zh, bits = _problem(ocd, B, U, W, S, Q, K, mode, 100 + n)
        ws = torch.zeros(ocd.ocd_backward_workspace_bytes(pb), dtype=torch.uint8, device="cuda")
        ref, got = _outputs(pb), _outputs(pb)
        ocd.ocd_detect_backward_bce(pb, H, y, lam, zh, bits, *ref, ws)
        ocd.ocd_detect_backward_bce_noalloc(pb, H, y, lam, zh, bits, *got)
        torch.cuda.synchronize()
        for name, a, b in zip(("dlambda", "dbeta", "dy"), [host(t) for t in got],
                              [host(t) for t in ref]):
            assert np.all(np.isfinite(a)), (n, name)
            assert np.array_equal(a, b), (n, name)


def test_noalloc_adjoint_rejects_what_does_not_fit_and_handles_empty(ocd):
    # 2^22 subcarriers x 4 symbols: several hundred thousand workgroups of partial sums,
    # far beyond the scratch; rejected on the host before anything is read or launched
    big = ocd.problem(128, 16, 1 << 22, 4, 4, 4, "hybrid", "f32", 0.1, 1.0, 0.9)
    dummy = torch.zeros(64, device="cuda")
    p = ctypes.c_void_p(dummy.data_ptr())
    st = ocd._lib.ocd_detect_backward_bce_noalloc(ctypes.byref(big), p, p, None, p, p, p, p, None,
                                                  None)
    say("oversized problem: status %d" % st)
    assert st == -4
    assert b"ESCRATCH" in ocd._lib.ocd_status_str(st)
    # the empty problem: zero gradients
    empty = ocd.problem(32, 4, 0, 2, 4, 3, "box", "f32", 0.1, 1.0, 0.0)
    dl, db, _ = _outputs(empty)
    st = ocd._lib.ocd_detect_backward_bce_noalloc(
        ctypes.byref(empty), None, None, None, None, None, ctypes.c_void_p(dl.data_ptr()),
        ctypes.c_void_p(db.data_ptr()), None, None)
    torch.cuda.synchronize()
    assert st == 0
    assert np.all(host(dl) == 0.0) and host(db)[0] == 0.0
