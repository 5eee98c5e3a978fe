"""Randomised GPU parity: seeded draws of problem shapes and launch plans.

The fixed cases elsewhere cover the shapes the benchmark times and the edges one
thinks of; these cover combinations one does not: antenna counts that are not
powers of two, tiles that straddle subcarriers at odd vectors per workgroup,
ragged last workgroups, the XCD tile order and staggered starts on small grids,
register plans, per-sweep regularisers, FP16 storage.  Every draw is fixed by
its seed (the list below is the same on every run), goes through the public C
ABI (ocd_set_plan, then ocd_detect) and is compared with the FP64 oracle on the
values the GPU received, element by element, with the z history.  A drawn plan
the library rejects for the shape (OCD_EUNSUPPORTED on the host) is redrawn.
"""

import numpy as np
import pytest
import torch

import synth
from gpu_util import (LLR_TOL_F32, Z_TOL_F32, dev, from_f16_pairs, host, llr_rel_err, oracle_ref,
                      say, to_f16_pairs, z_rel_err)

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ocd():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_1611_08779_amd as m
    return m


def _draw_cases(seed, n):
    rng = np.random.default_rng(seed)
    cases = []
    for i in range(n):
        B = int(rng.choice([int(rng.integers(1, 33)), int(rng.integers(33, 129)),
                            int(rng.integers(129, 257))]))
        U = int(rng.integers(1, max(1, min(32, B // 2)) + 1))
        S = int(rng.choice([1, 1, 2, 3, int(rng.integers(4, 17))]))
        W = int(rng.integers(1, max(1, 300 // S) + 1))
        Q = int(rng.choice([2, 4, 6]))
        K = int(rng.integers(1, 7))
        mode = str(rng.choice(["mmse", "box", "hybrid"]))
        storage = "f16" if rng.random() < 0.25 else "f32"
        snr = float(rng.uniform(8.0, 25.0))
        cases.append((i, B, U, W, S, Q, K, mode, storage, round(snr, 1), int(rng.integers(1 << 30))))
    return cases


CASES = _draw_cases(20261203, 60)


def _set_random_plan(ocd, pb, S, plan_seed):
    rng = np.random.default_rng(plan_seed)
    for _ in range(40):
        L = int(rng.choice([4, 8, 16, 32]))
        cir = int(rng.integers(0, 2)) if S <= 2 else 0
        cap = (256 if cir else 512) // L
        vpb = int(rng.integers(1, cap + 1))
        plan = (L, vpb, int(rng.integers(0, 2)), cir, int(rng.integers(0, 4)))
        try:
            ocd.ocd_set_plan(pb, ocd.Plan(*plan))
        except ocd.OCDError:
            continue
        return plan
    return None   # no drawn plan fits: the library's own choice runs


@pytest.mark.parametrize("case", CASES, ids=["r%02d-%s" % (c[0], "-".join(map(str, c[1:9])))
                                             for c in CASES])
def test_random_shape_and_plan(ocd, case):
    i, B, U, W, S, Q, K, mode, storage, snr, plan_seed = case
    wl = synth.make_workload(B, U, W, S, Q, snr, seed=[91, i])
    N0 = float(np.float32(wl["N0"]))
    lam = None
    beta = 0.0
    if mode == "hybrid":
        lam = (N0 * np.random.default_rng([92, i]).uniform(0.3, 3.0, K)).astype(np.float32)
        beta = 0.9
    pb = ocd.problem(B, U, W, S, Q, K, mode, storage, N0, 1.0, beta)
    plan = _set_random_plan(ocd, pb, S, plan_seed)
    say("case %s plan %s" % (case, plan))
    if plan is not None:
        used = ocd.ocd_get_plan(pb)
        assert (used.lanes_per_vector, used.vectors_per_block, used.xcd_remap,
                used.channel_in_registers, used.stagger) == plan
    if storage == "f16":
        H16, y16 = to_f16_pairs(wl["H"]), to_f16_pairs(wl["y"])
        H, y = dev(H16), dev(y16)
        Hr, yr = from_f16_pairs(H16), from_f16_pairs(y16)
    else:
        H, y = dev(wl["H"]), dev(wl["y"])
        Hr, yr = wl["H"], wl["y"]
    lam_t = None if lam is None else dev(lam)
    z, L, zh = ocd.detect(H, y, K, Q, mode, N0, 1.0, beta, lam=lam_t, storage=storage,
                          want_hist=True)
    torch.cuda.synchronize()
    zo, Lo, zho = oracle_ref(Hr, yr, K, Q, mode, N0, 1.0, lam, float(np.float32(beta)), True)
    ez, el = z_rel_err(host(z), zo), llr_rel_err(host(L), Lo)
    say("  z err %.3g  llr err %.3g" % (ez, el))
    assert ez <= Z_TOL_F32, ez
    assert el <= LLR_TOL_F32, el
    for k in range(K):
        assert z_rel_err(host(zh)[:, :, k], zho[:, :, k]) <= Z_TOL_F32
    assert np.array_equal(host(zh)[:, :, K - 1], host(z))
