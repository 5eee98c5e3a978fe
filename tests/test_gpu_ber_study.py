"""The error-rate study's counts (paper_1611_08779_amd/ber_study.py) against the
FP64 oracle's decisions on the same seeded inputs.  A decision is the sign of a
max-log LLR; the GPU's LLRs are within ~1e-6 of the oracle's, so the two can
disagree only on bits whose LLR is that close to zero: at most 2 per detector
on these 26,880 bits."""

import numpy as np
import pytest
import torch

import oracle
import synth
from gpu_util import say

pytestmark = pytest.mark.gpu


def test_study_counts_match_the_oracle():
    from paper_1611_08779_amd import ber_study as bs
    B, U, Q, W, S, eb, seed = 32, 8, 6, 40, 14, 6.0, 77
    res = bs.study([B], [eb], 1, U=U, Q=Q, W=W, S=S, seed=seed)[(B, eb)]
    wl = synth.make_workload_device(B, U, W, S, Q, bs.snr_for_ebn0(eb, B, U, Q), seed=seed,
                                    device=torch.device("cuda:0"))
    H, y = wl["H"].cpu().numpy(), wl["y"].cpu().numpy()
    bits = wl["bits"].cpu().numpy()
    N0 = float(np.float32(wl["N0"]))
    assert res["bits"] == bits.size
    c = np.sqrt(B)
    Hq = bs.quantize_q11(wl["H"], c).cpu().numpy()
    yq = bs.quantize_q11(wl["y"], c).cpu().numpy()
    for det, K in bs.DETECTORS:
        if det.endswith("-fx"):
            N0f = float(np.float32(float(np.float32(wl["N0"])) * B))   # as the study forms it
            _, L = oracle.ocd_fixed(Hq, yq, K, Q, "box", N0=N0f, threads=0)
            key = "%s/%d" % (det, K)
        elif det == "mmse":
            _, L, _ = oracle.mmse(H, y, Q, N0=N0, threads=0)
            key = "mmse"
        else:
            mode = "mmse" if det == "ocd-mmse" else "box"
            _, L = oracle.detect(H, y, K, Q, mode, N0=N0, threads=0)
            key = "%s/%d" % (det, K)
        e = int(np.sum((L > 0).astype(np.uint8) != bits))
        say("%s: GPU %d, oracle %d errors" % (key, res[key], e))
        assert abs(res[key] - e) <= 2, key
