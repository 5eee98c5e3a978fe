"""Randomised GPU parity of the batched launch (ocd_detect_jobs): seeded draws of
job lists and flags.

Each draw is a batch of 2-10 uneven jobs under the entry point's rules (one
storage and one projection family per batch, the default regulariser, B <= 256)
with shapes drawn independently per job: B 1-256, U up to 32, 1-30 subcarriers
of 1-14 symbols, every modulation, K 1-5.  The flags force a lane mode and a
schedule, or ask the batch tuner, with and without graph capture.  Every job is
compared with the FP64 oracle; captured batches are replayed and must repeat the
eager outputs bit for bit; the schedule query must name a valid choice.
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


def _draw_batches(seed, n):
    rng = np.random.default_rng(seed)
    batches = []
    for i in range(n):
        family = str(rng.choice(["mmse", "box"]))
        storage = "f16" if rng.random() < 0.3 else "f32"
        jobs = []
        for _ in range(int(rng.integers(2, 11))):
            B = int(rng.choice([int(rng.integers(1, 65)), int(rng.integers(65, 257))]))
            U = int(rng.integers(1, max(1, min(32, B // 2)) + 1))
            mode = "mmse" if family == "mmse" else str(rng.choice(["box", "hybrid"]))
            jobs.append((B, U, int(rng.integers(1, 31)), int(rng.integers(1, 15)),
                         int(rng.choice([2, 4, 6])), int(rng.integers(1, 6)), mode,
                         round(float(rng.uniform(8.0, 25.0)), 1)))
        kind = int(rng.integers(0, 4))   # 0-2: forced lane mode, 3: tuned
        persistent = bool(rng.integers(0, 2))
        graph = bool(rng.integers(0, 2))
        batches.append((i, storage, jobs, kind, persistent, graph))
    return batches


BATCHES = _draw_batches(20261204, 16)


@pytest.mark.parametrize("batch", BATCHES, ids=["b%02d-%s-%djobs-k%d-p%d-g%d" % (
    b[0], b[1], len(b[2]), b[3], b[4], b[5]) for b in BATCHES])
def test_random_job_batch(ocd, batch):
    i, storage, jobs, kind, persistent, graph = batch
    say("batch %d: %s, kind %d, persistent %s, graph %s, jobs %s" % (i, storage, kind, persistent,
                                                                      graph, jobs))
    probs, Hs, ys, refs = [], [], [], []
    for j, (B, U, W, S, Q, K, mode, snr) in enumerate(jobs):
        wl = synth.make_workload(B, U, W, S, Q, snr, seed=[95, i, j])
        N0 = float(np.float32(wl["N0"]))
        probs.append(ocd.problem(B, U, W, S, Q, K, mode, storage, N0))
        if storage == "f16":
            H16, y16 = to_f16_pairs(wl["H"]), to_f16_pairs(wl["y"])
            Hs.append(dev(H16))
            ys.append(dev(y16))
            refs.append((from_f16_pairs(H16), from_f16_pairs(y16), N0))
        else:
            Hs.append(dev(wl["H"]))
            ys.append(dev(wl["y"]))
            refs.append((wl["H"], wl["y"], N0))
    flags = ocd.OCD_JOBS_TUNE if kind == 3 else ocd.OCD_JOBS_LANE_MODE(kind)
    if persistent:
        flags |= ocd.OCD_JOBS_PERSISTENT
    z, L, ws = ocd.detect_jobs(probs, Hs, ys, flags=flags)
    torch.cuda.synchronize()
    for j, (pb, (H, y, N0)) in enumerate(zip(probs, refs)):
        mode = jobs[j][6]
        zo, Lo, _ = oracle_ref(H, y, pb.K, pb.Q, mode, N0)
        ez, el = z_rel_err(host(z[j]), zo), llr_rel_err(host(L[j]), Lo)
        assert ez <= Z_TOL_F32, (j, ez)
        assert el <= LLR_TOL_F32, (j, el)
    sched = ocd.ocd_jobs_schedule(probs)
    assert sched["persistent"] in (0, 1) and sched["tile_policy"] in (0, 1, 2)
    assert sched["lane_mode"] in (0, 1, 2)
    if graph:
        # captured on the first call, replayed on the next ones: every replay repeats the
        # eager outputs bit for bit, with eager work and synchronisation between replays
        gflags = (flags & ~ocd.OCD_JOBS_TUNE) | ocd.OCD_JOBS_GRAPH
        for rep in range(3):
            zg, Lg, ws = ocd.detect_jobs(probs, Hs, ys, flags=gflags, workspace=ws)
            torch.cuda.synchronize()
            _ = torch.ones(1024, device="cuda").sum().item()
            for j in range(len(probs)):
                assert torch.equal(zg[j], z[j]) and torch.equal(Lg[j], L[j]), (rep, j)
        ocd.ocd_release_graphs()
