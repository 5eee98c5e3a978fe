"""The library under concurrent host threads: several threads call the C ABI at
once (ctypes releases the interpreter lock for the call), each on its own stream
and its own problem shapes, mixing detections, plan queries and plans set by the
caller, and batched launches with their own workspaces.  Every output equals the
one the same call gave sequentially, bit for bit (same plans, same kernels)."""

import threading

import numpy as np
import pytest
import torch

import synth
from gpu_util import dev, say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ocd():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_1611_08779_amd as m
    return m


# one shape set per thread (distinct shapes: a thread's plans are its own)
SHAPES = [
    [(64, 8, 30, 14, 6, 3, "mmse"), (32, 4, 50, 3, 4, 2, "box")],
    [(128, 16, 12, 4, 4, 4, "hybrid"), (96, 6, 20, 2, 2, 3, "mmse")],
    [(48, 12, 25, 5, 6, 2, "box"), (200, 8, 6, 14, 4, 3, "mmse")],
    [(33, 5, 40, 1, 4, 3, "mmse"), (64, 32, 8, 7, 2, 2, "box")],
]


def _inputs(shapes, t):
    out = []
    for n, (B, U, W, S, Q, K, mode) in enumerate(shapes):
        wl = synth.make_workload(B, U, W, S, Q, 15.0, seed=[110, t, n])
        N0 = float(np.float32(wl["N0"]))
        lam = dev(np.full(K, N0, np.float32)) if mode == "hybrid" else None
        out.append((B, U, W, S, Q, K, mode, N0, lam, dev(wl["H"]), dev(wl["y"])))
    return out


def _detect(ocd, x):
    B, U, W, S, Q, K, mode, N0, lam, H, y = x
    beta = 0.9 if mode == "hybrid" else 0.0
    z, L, _ = ocd.detect(H, y, K, Q, mode, N0, 1.0, beta, lam=lam)
    return z, L


def _jobs(ocd, xs):
    probs = [ocd.problem(x[0], x[1], x[2], x[3], x[4], x[5], "mmse", "f32", x[7]) for x in xs]
    z, L, _ = ocd.detect_jobs(probs, [x[9] for x in xs], [x[10] for x in xs])
    return z, L


def test_concurrent_threads_match_sequential_calls(ocd):
    per_thread = [_inputs(s, t) for t, s in enumerate(SHAPES)]
    jobs_in = [x for x in per_thread[0] + per_thread[2] if x[6] == "mmse"]
    # plans fixed before the threads start, so that each call's plan is known
    for xs in per_thread:
        for x in xs:
            B, U, W, S, Q, K, mode, N0 = x[:8]
            pb = ocd.problem(B, U, W, S, Q, K, mode, "f32", N0, 1.0, 0.9 if mode == "hybrid" else 0.0)
            ocd.ocd_set_plan(pb, ocd.ocd_get_plan(pb))
    ref = [[_detect(ocd, x) for x in xs] for xs in per_thread]
    ref_jobs = _jobs(ocd, jobs_in)
    torch.cuda.synchronize()

    errors, results = [], {}

    def worker(t):
        try:
            s = torch.cuda.Stream()
            with torch.cuda.stream(s):
                got = []
                for it in range(12):
                    for n, x in enumerate(per_thread[t]):
                        B, U, W, S, Q, K, mode, N0 = x[:8]
                        pb = ocd.problem(B, U, W, S, Q, K, mode, "f32", N0, 1.0,
                                         0.9 if mode == "hybrid" else 0.0)
                        ocd.ocd_get_plan(pb)            # queries beside the launches
                        got.append((n, _detect(ocd, x)))
                    if t == 1 and it % 4 == 0:          # one thread also runs batches
                        got.append(("jobs", _jobs(ocd, jobs_in)))
                s.synchronize()
                results[t] = got
        except Exception as e:   # reported after the join
            errors.append((t, repr(e)))

    threads = [threading.Thread(target=worker, args=(t,)) for t in range(len(SHAPES))]
    for th in threads:
        th.start()
    for th in threads:
        th.join(timeout=300)
    assert not errors, errors
    torch.cuda.synchronize()
    checked = 0
    for t, got in results.items():
        for n, out in got:
            if n == "jobs":
                for j in range(len(jobs_in)):
                    assert torch.equal(out[0][j], ref_jobs[0][j]) and torch.equal(out[1][j], ref_jobs[1][j])
            else:
                assert torch.equal(out[0], ref[t][n][0]) and torch.equal(out[1], ref[t][n][1]), (t, n)
            checked += 1
    say("  %d concurrent results checked" % checked)
    assert checked == sum(12 * len(s) for s in SHAPES) + 3
