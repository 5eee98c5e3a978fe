"""GPU parity of the batched persistent launch (ocd_detect_jobs): every job against
the FP64 oracle and bit-for-bit against a one-problem launch with the same lane
split; graph replays checked against the eager result on every replay."""

import numpy as np
import pytest
import torch

import synth
from gpu_util import (LLR_TOL_F32, Z_TOL_F32, dev, host, llr_rel_err, oracle_ref, say, to_f16_pairs,
                      z_rel_err)

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ocd():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_1611_08779_amd as m
    return m


def f32(x):
    return float(np.float32(x))


# uneven shapes drawn like the 48-job batch, cut down so the oracle stays fast; with
# U = 24 (three chunks of the chunked user loop) at a B that is not a power of two
JOBS = [
    (64, 4, 21, 2), (128, 8, 30, 3), (256, 32, 5, 4), (128, 16, 11, 2), (64, 32, 9, 3),
    (256, 4, 17, 2), (128, 32, 3, 4), (64, 8, 40, 3), (256, 16, 7, 2), (33, 5, 6, 3),
    (96, 24, 4, 3), (200, 24, 3, 2),
]


def _make(ocd, storage="f32", jobs=JOBS, S=14, Q=6):
    probs, Hs, ys, wls = [], [], [], []
    for j, (B, U, W, K) in enumerate(jobs):
        wl = synth.make_workload(B, U, W, S, Q, 20.0, seed=[30, j])
        N0 = f32(wl["N0"])
        probs.append(ocd.problem(B, U, W, S, Q, K, "mmse", storage, N0))
        if storage == "f16":
            Hs.append(dev(to_f16_pairs(wl["H"])))
            ys.append(dev(to_f16_pairs(wl["y"])))
        else:
            Hs.append(dev(wl["H"]))
            ys.append(dev(wl["y"]))
        wls.append(wl)
    return probs, Hs, ys, wls


def _lanes(B):
    # the batched kernel gives each vector B/8 lanes (8 complex entries per lane)
    L = 4
    while 8 * L < B:
        L *= 2
    return L


def test_jobs_match_oracle_and_single_launches(ocd):
    probs, Hs, ys, wls = _make(ocd)
    say("jobs: %d uneven problems" % len(probs))
    z, L, ws = ocd.detect_jobs(probs, Hs, ys)
    torch.cuda.synchronize()
    for j, (pb, wl) in enumerate(zip(probs, wls)):
        zo, Lo, _ = oracle_ref(wl["H"], wl["y"], pb.K, pb.Q, "mmse", pb.N0)
        assert z_rel_err(host(z[j]), zo) <= Z_TOL_F32, j
        assert llr_rel_err(host(L[j]), Lo) <= LLR_TOL_F32, j
        # same lane split and entries per lane as the batched kernel: same bits
        ocd.ocd_set_plan(pb, ocd.Plan(_lanes(pb.B), 14, 0, 0))
        z1, L1, _ = ocd.detect(Hs[j], ys[j], pb.K, pb.Q, "mmse", pb.N0)
        torch.cuda.synchronize()
        assert torch.equal(z1, z[j]) and torch.equal(L1, L[j]), j


def _lanes_npl(B, mode):
    # lane modes of the batched kernel: entries per lane by B, lanes per vector B / NPL
    npl = 16 if (mode >= 1 and B > 128) else 4 if (mode == 2 and B > 32) else 8
    L = 4
    while npl * L < B:
        L *= 2
    if not ((npl == 8 and L in (4, 8, 16, 32)) or (npl in (4, 16) and L in (16, 32))):
        npl, L = 8, _lanes(B)
    return L, npl


@pytest.mark.parametrize("mode", [0, 1, 2])
@pytest.mark.parametrize("persistent", [False, True])
def test_jobs_every_lane_mode(ocd, mode, persistent):
    """Each lane mode of the batched kernel (8 entries per lane; 16 for B > 128; and 4
    for 32 < B <= 128), forced through the flags, in both schedules: every job against
    the oracle, and bit for bit against a one-problem launch with the same lanes per
    vector (the one-problem kernel unrolls U = 8 and 16 where the batched one may run the
    loop over a run-time U: the same arithmetic in the same order)."""
    probs, Hs, ys, wls = _make(ocd)
    flags = ocd.OCD_JOBS_LANE_MODE(mode) | (ocd.OCD_JOBS_PERSISTENT if persistent else 0)
    say("jobs: lane mode %d persistent %s" % (mode, persistent))
    z, L, ws = ocd.detect_jobs(probs, Hs, ys, flags=flags)
    torch.cuda.synchronize()
    for j, (pb, wl) in enumerate(zip(probs, wls)):
        zo, Lo, _ = oracle_ref(wl["H"], wl["y"], pb.K, pb.Q, "mmse", pb.N0)
        assert z_rel_err(host(z[j]), zo) <= Z_TOL_F32, j
        assert llr_rel_err(host(L[j]), Lo) <= LLR_TOL_F32, j
        lanes, npl = _lanes_npl(pb.B, mode)
        ocd.ocd_set_plan(pb, ocd.Plan(lanes, 14, 0, 0))
        z1, L1, _ = ocd.detect(Hs[j], ys[j], pb.K, pb.Q, "mmse", pb.N0)
        torch.cuda.synchronize()
        assert torch.equal(z1, z[j]) and torch.equal(L1, L[j]), (j, lanes, npl)


def test_jobs_schedule_reports_the_tuned_choice(ocd):
    probs, Hs, ys, wls = _make(ocd, jobs=JOBS[:4])
    before = ocd.ocd_jobs_schedule(probs)
    z, L, ws = ocd.detect_jobs(probs, Hs, ys, flags=ocd.OCD_JOBS_TUNE)
    torch.cuda.synchronize()
    after = ocd.ocd_jobs_schedule(probs)
    say("jobs schedule default %s tuned %s" % (before, after))
    assert before == {"persistent": 0, "tile_policy": 1, "lane_mode": 0} or before == after
    assert after["persistent"] in (0, 1) and after["tile_policy"] in (0, 1, 2)
    assert after["lane_mode"] in (0, 1, 2)


@pytest.mark.parametrize("mode", [0, 1, 2])
def test_jobs_small_antenna_counts(ocd, mode):
    """Jobs with B <= 16 have fewer antennas than 4 lanes of 8 entries: they run at
    that width with the antennas past B zero-padded, beside larger jobs, in every lane
    mode; each against the oracle."""
    jobs = [(1, 1, 9, 2), (4, 2, 10, 2), (6, 3, 7, 3), (13, 6, 5, 4), (16, 8, 6, 2),
            (128, 8, 6, 3)]
    probs, Hs, ys, wls = _make(ocd, jobs=jobs)
    say("jobs: small antenna counts, lane mode %d" % mode)
    z, L, ws = ocd.detect_jobs(probs, Hs, ys, flags=ocd.OCD_JOBS_LANE_MODE(mode))
    torch.cuda.synchronize()
    for j, (pb, wl) in enumerate(zip(probs, wls)):
        zo, Lo, _ = oracle_ref(wl["H"], wl["y"], pb.K, pb.Q, "mmse", pb.N0)
        assert z_rel_err(host(z[j]), zo) <= Z_TOL_F32, j
        assert llr_rel_err(host(L[j]), Lo) <= LLR_TOL_F32, j


def test_jobs_persistent_schedule_matches(ocd):
    """The persistent schedule (workgroups popping tiles from the device queue)
    computes the same bits as one workgroup per tile."""
    probs, Hs, ys, wls = _make(ocd)
    z0, L0, ws = ocd.detect_jobs(probs, Hs, ys)
    z1, L1, _ = ocd.detect_jobs(probs, Hs, ys, flags=ocd.OCD_JOBS_PERSISTENT, workspace=ws)
    torch.cuda.synchronize()
    for j in range(len(probs)):
        assert torch.equal(z1[j], z0[j]) and torch.equal(L1[j], L0[j]), j


@pytest.mark.parametrize("extra", [0, 4])
def test_jobs_graph_replays_match_eager(ocd, extra):
    probs, Hs, ys, wls = _make(ocd)
    z0, L0, ws = ocd.detect_jobs(probs, Hs, ys)
    torch.cuda.synchronize()
    for rep in range(3):
        z = [torch.full_like(t, float("nan")) for t in z0]
        L = [torch.full_like(t, float("nan")) for t in L0]
        ocd.ocd_detect_jobs(probs, Hs, ys, z, L, ws, flags=ocd.OCD_JOBS_GRAPH | extra)
        torch.cuda.synchronize()
        # eager work and a synchronisation between replays
        _ = ocd.detect(Hs[1], ys[1], probs[1].K, probs[1].Q, "mmse", probs[1].N0)
        torch.cuda.synchronize()
        for j in range(len(probs)):
            assert torch.equal(z[j], z0[j]) and torch.equal(L[j], L0[j]), (rep, j)


def test_jobs_graph_follows_new_buffers(ocd):
    """The graph reads job pointers from the workspace tables: new output buffers on a
    replay must be the ones written."""
    probs, Hs, ys, _ = _make(ocd)
    z0, L0, ws = ocd.detect_jobs(probs, Hs, ys, flags=ocd.OCD_JOBS_GRAPH)
    torch.cuda.synchronize()
    z1, L1, _ = ocd.detect_jobs(probs, Hs, ys, flags=ocd.OCD_JOBS_GRAPH, workspace=ws)
    torch.cuda.synchronize()
    for j in range(len(probs)):
        assert torch.equal(z1[j], z0[j]) and torch.equal(L1[j], L0[j])


def test_jobs_tuner_and_fp16_storage(ocd):
    probs, Hs, ys, wls = _make(ocd, storage="f16", jobs=JOBS[:5])
    z, L, ws = ocd.detect_jobs(probs, Hs, ys, flags=ocd.OCD_JOBS_TUNE)
    torch.cuda.synchronize()
    from gpu_util import from_f16_pairs
    for j, (pb, wl) in enumerate(zip(probs, wls)):
        zo, Lo, _ = oracle_ref(from_f16_pairs(host(Hs[j])), from_f16_pairs(host(ys[j])), pb.K, pb.Q,
                               "mmse", pb.N0)
        assert z_rel_err(host(z[j]), zo) <= Z_TOL_F32, j
        assert llr_rel_err(host(L[j]), Lo) <= LLR_TOL_F32, j
    ocd.ocd_release_graphs()


def test_the_48_job_batch_at_full_size_sampled(ocd):
    """The batched workload the benchmark times, whole (48 jobs drawn by
    synth.batched_job_list, 865,200 vectors, one launch with the tuner): three
    subcarriers (all their symbols) of every job against the oracle."""
    jl = synth.batched_job_list()
    probs, Hs, ys = [], [], []
    for j, jd in enumerate(jl):
        wl = synth.make_workload_device(jd["B"], jd["U"], jd["W"], jd["S"], jd["Q"], jd["snr_db"],
                                        seed=3000 + j, device="cuda")
        probs.append(ocd.problem(jd["B"], jd["U"], jd["W"], jd["S"], jd["Q"], jd["K"], "mmse", "f32",
                                 f32(wl["N0"])))
        Hs.append(wl["H"])
        ys.append(wl["y"])
    say("jobs: the 48-job batch, %d vectors" % sum(p.W * p.S for p in probs))
    z, L, _ = ocd.detect_jobs(probs, Hs, ys, flags=ocd.OCD_JOBS_TUNE)
    torch.cuda.synchronize()
    rng = np.random.default_rng(48)
    for j, pb in enumerate(probs):
        ws = torch.as_tensor(np.sort(rng.choice(pb.W, 3, replace=False)), device="cuda")
        zo, Lo, _ = oracle_ref(host(Hs[j][ws]), host(ys[j][ws]), pb.K, pb.Q, "mmse", pb.N0)
        assert z_rel_err(host(z[j][ws]), zo) <= Z_TOL_F32, j
        assert llr_rel_err(host(L[j][ws]), Lo) <= LLR_TOL_F32, j
