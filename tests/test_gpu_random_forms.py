"""Randomised GPU parity of the other entry points: seeded draws of shapes (and
launch plans) for explicit MMSE detection, the fixed-point datapath and the OFDM
front end, each against the oracle with the bar its fixed tests use (MMSE: the
FP32 bars, widened with the condition number of A as in test_gpu_mmse; fixed
point: bit for bit; OFDM: 1e-5 relative per (symbol, antenna)).  A drawn MMSE plan
the library rejects for the shape is redrawn.
"""

import numpy as np
import pytest
import torch

import oracle
import synth
from gpu_util import (LLR_TOL_F32, Z_TOL_F32, dev, from_f16_pairs, host, llr_rel_err, say,
                      to_f16_pairs, z_rel_err)
from test_gpu_fixed import run_fixed
from test_gpu_mmse import cond_max
from test_gpu_ofdm import TOL as OFDM_TOL
from test_gpu_ofdm import rel_err as ofdm_rel_err
from test_oracle_fixed_pins import fixed_workload

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ocd():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_1611_08779_amd as m
    return m


def _antennas(rng, hi):
    return int(rng.choice([int(rng.integers(1, 33)), int(rng.integers(33, hi + 1))]))


def _mmse_cases(seed, n):
    rng = np.random.default_rng(seed)
    out = []
    for i in range(n):
        B = _antennas(rng, 256)
        U = int(rng.integers(1, max(1, min(32, B // 2)) + 1))
        S = int(rng.choice([1, 2, int(rng.integers(3, 17))]))
        W = int(rng.integers(1, max(1, 240 // S) + 1))
        out.append((i, B, U, W, S, int(rng.choice([2, 4, 6])), "f16" if rng.random() < 0.25 else "f32",
                    round(float(rng.uniform(8.0, 25.0)), 1), int(rng.integers(1 << 30))))
    return out


MMSE_CASES = _mmse_cases(20261205, 30)


def _mmse_plans(U, S, plan_seed):
    rng = np.random.default_rng(plan_seed)
    for _ in range(40):
        if U <= 8 and S <= 16 and rng.random() < 0.25:
            yield (0, S, int(rng.integers(0, 2)))       # the matrix-core form
        else:
            L = int(rng.choice([8, 16, 32]))
            yield (L, int(rng.integers(1, 512 // L + 1)), int(rng.integers(0, 2)))
    yield None                                          # the library's own choice


@pytest.mark.parametrize("case", MMSE_CASES, ids=["m%02d-%s" % (c[0], "-".join(map(str, c[1:7])))
                                                  for c in MMSE_CASES])
def test_random_mmse(ocd, case):
    i, B, U, W, S, Q, storage, snr, plan_seed = case
    wl = synth.make_workload(B, U, W, S, Q, snr, seed=[96, i])
    N0 = float(np.float32(wl["N0"]))
    if storage == "f16":
        H16, y16 = to_f16_pairs(wl["H"]), to_f16_pairs(wl["y"])
        H, y, Hr, yr = dev(H16), dev(y16), from_f16_pairs(H16), from_f16_pairs(y16)
    else:
        H, y, Hr, yr = dev(wl["H"]), dev(wl["y"]), wl["H"], wl["y"]
    for plan in _mmse_plans(U, S, plan_seed):
        try:   # a plan that does not fit the shape is rejected on the host, before a launch
            z, L = ocd.detect_mmse(H, y, Q, N0, storage=storage, plan=plan)
            break
        except ocd.OCDError:
            continue
    say("mmse case %s plan %s" % (case, plan))
    torch.cuda.synchronize()
    zo, Lo, _ = oracle.mmse(Hr, yr, Q, N0=N0, threads=0)
    ztol = max(Z_TOL_F32, 64 * cond_max(Hr, N0) * 2.0 ** -24)
    ltol = max(LLR_TOL_F32, 10 * ztol)
    ez, el = z_rel_err(host(z), zo), llr_rel_err(host(L), Lo)
    say("  z err %.3g (bar %.3g)  llr err %.3g" % (ez, ztol, el))
    assert ez <= ztol, ez
    assert el <= ltol, el


def _fixed_cases(seed, n):
    rng = np.random.default_rng(seed)
    out = []
    for i in range(n):
        B = _antennas(rng, 1024)
        U = int(rng.integers(1, max(1, min(32, B // 2)) + 1))
        S = int(rng.integers(1, 15))
        W = int(rng.integers(1, max(1, 160 // S) + 1))
        out.append((i, B, U, W, S, int(rng.choice([2, 4, 6])), int(rng.integers(1, 7)),
                    str(rng.choice(["mmse", "box"])), round(float(rng.uniform(8.0, 25.0)), 1)))
    return out


FIXED_CASES = _fixed_cases(20261206, 24)


@pytest.mark.parametrize("case", FIXED_CASES, ids=["f%02d-%s" % (c[0], "-".join(map(str, c[1:8])))
                                                   for c in FIXED_CASES])
def test_random_fixed_point(ocd, case):
    i, B, U, W, S, Q, K, mode, snr = case
    say("fixed case %s" % (case,))
    Hq, yq, N0, _ = fixed_workload(B, U, W, S, Q, snr, [97, i])
    run_fixed(ocd, Hq, yq, K, Q, mode, N0)


def _ofdm_cases(seed, n):
    rng = np.random.default_rng(seed)
    out = []
    for i in range(n):
        N = int(rng.choice([256, 512, 1024, 2048, 4096]))
        Ncp = int(rng.choice([0, int(rng.integers(1, N // 8 + 1)), int(rng.integers(1, N + 1))]))
        W = 2 * int(rng.integers(1, N // 2))
        B = int(rng.integers(1, 65))
        S = int(rng.integers(1, 17))
        while B * S * (N + Ncp) > (1 << 21) and S > 1:
            S -= 1
        while B * S * (N + Ncp) > (1 << 21) and B > 1:
            B -= 1
        out.append((i, N, Ncp, W, B, S))
    return out


OFDM_CASES = _ofdm_cases(20261207, 24)


@pytest.mark.parametrize("case", OFDM_CASES, ids=["o%02d-%s" % (c[0], "-".join(map(str, c[1:])))
                                                  for c in OFDM_CASES])
def test_random_ofdm(ocd, case):
    i, N, Ncp, W, B, S = case
    say("ofdm case %s" % (case,))
    rng = np.random.default_rng([98, i])
    x = (rng.normal(size=(B, S, Ncp + N)) + 1j * rng.normal(size=(B, S, Ncp + N))).astype(np.complex64)
    y = ocd.ofdm_demodulate(dev(x), N, Ncp, W)
    torch.cuda.synchronize()
    e = ofdm_rel_err(host(y), oracle.ofdm_demodulate(x, N, Ncp, W))
    say("  rel err %.3g" % e)
    assert e <= OFDM_TOL
