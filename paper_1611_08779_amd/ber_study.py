#!/usr/bin/env python
"""Uncoded bit-error rates of OCD (MMSE and BOX modes, K = 1..4) and of explicit
MMSE detection on synthetic slots: a stand-in for the paper's error-rate study
(Section III-D), whose packet-error rates use a rate-3/4 turbo code and
WINNER-II channels; neither is reproduced here.  Channels are i.i.d. Rayleigh
(block fading over the S symbols of a subcarrier), 64-QAM with Gray labels,
U = 8 users, B in {32, 64, 128} antennas, and the SNR per bit of Section III-D,
Eb/N0 = E||s||^2 / (Q E||n||^2).  A bit decision is the sign of its max-log LLR
(L > 0 favours 1), the slicer's decision.

Every detection runs on the GPU through the C ABI (ocd_detect, ocd_detect_mmse);
the inputs come from synth.make_workload_device, seeded per (B, Eb/N0, slot), so
every detector sees the same channel and noise realisations (paired counts).

    python paper_1611_08779_amd/ber_study.py [--antennas 32,64,128]
        [--ebn0 0,2,4,6,8,10,12] [--slots 8] [--out results.json]

prints one markdown table per antenna count and, with --out, writes the counts.
"""

from __future__ import annotations

import argparse
import json
import math
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

DETECTORS = ([("ocd-mmse", k) for k in (1, 2, 3, 4)] + [("ocd-box", k) for k in (1, 2, 3, 4)]
             + [("mmse", 0)] + [("ocd-box-fx", k) for k in (3, 4)])


def quantize_q11(t, scale):
    """complex64 device tensor -> int16 (re, im) pairs in Q5.11 of t * scale, rounded
    half up and saturated (the fixed-point detector's input format)."""
    import torch
    v = torch.view_as_real(t).to(torch.float64) * (scale * 2048.0)
    return torch.clamp(torch.floor(v + 0.5), -32768, 32767).to(torch.int16).contiguous()


def snr_for_ebn0(ebn0_db: float, B: int, U: int, Q: int) -> float:
    """Per-user receive SNR (N0 = Es 10^(-snr/10), E||h_u||^2 = 1) whose SNR per bit
    is ebn0_db: Eb/N0 = U Es / (Q B N0)."""
    return ebn0_db - 10.0 * math.log10(U / (Q * B))


def count_errors(ocd, torch, wl, Q, K, det):
    """Bit errors of one detector on one slot (device tensors from synth)."""
    N0 = float(wl["N0"])
    if det == "mmse":
        _, L = ocd.detect_mmse(wl["H"], wl["y"], Q, N0, want_z=False)
    elif det.endswith("-fx"):
        # the datapath's shifts assume unit-power channel entries: H, y times sqrt(B)
        # and N0 times B, which leaves OCD's estimate unchanged
        B = wl["H"].shape[-1]
        c = math.sqrt(B)
        mode = "box" if det.startswith("ocd-box") else "mmse"
        _, L = ocd.detect_fixed(quantize_q11(wl["H"], c), quantize_q11(wl["y"], c), K, Q, mode,
                                float(torch.tensor(N0 * B, dtype=torch.float32)), want_z=False)
    else:
        mode = "mmse" if det == "ocd-mmse" else "box"
        _, L, _ = ocd.detect(wl["H"], wl["y"], K, Q, mode, N0, want_z=False)
    return int(((L > 0).to(torch.uint8) != wl["bits"]).sum().item())


def study(antennas, ebn0s, slots, U=8, Q=6, W=1200, S=14, seed=9000, log=None):
    """Error counts {(B, ebn0): {"bits": n, "ocd-mmse/K": e, ..., "mmse": e}}."""
    import torch

    import paper_1611_08779_amd as ocd
    import synth

    dev = torch.device("cuda:0")
    out = {}
    for bi, B in enumerate(antennas):
        for ei, eb in enumerate(ebn0s):
            snr = snr_for_ebn0(eb, B, U, Q)
            rec = {"bits": 0}
            for sl in range(slots):
                wl = synth.make_workload_device(B, U, W, S, Q, snr,
                                                seed=seed + 100000 * bi + 1000 * ei + sl,
                                                device=dev)
                wl["N0"] = float(torch.tensor(wl["N0"], dtype=torch.float32))
                rec["bits"] += wl["bits"].numel()
                for det, K in DETECTORS:
                    key = det if det == "mmse" else "%s/%d" % (det, K)
                    rec[key] = rec.get(key, 0) + count_errors(ocd, torch, wl, Q, K, det)
            out[(B, eb)] = rec
            if log:
                log("B=%d Eb/N0=%g dB: %s" % (B, eb, " ".join(
                    "%s=%.3g" % (k, v / rec["bits"]) for k, v in rec.items() if k != "bits")))
    return out


def ebn0_at(res, B, ebn0s, key, target):
    """Eb/N0 (dB) where the BER of detector `key` crosses `target`, by linear
    interpolation of log10(BER) between the two sweep points around it; None if
    the sweep does not cross it."""
    pts = [(eb, res[(B, eb)][key] / res[(B, eb)]["bits"]) for eb in ebn0s]
    for (e0, b0), (e1, b1) in zip(pts, pts[1:]):
        if b0 >= target > b1 and b1 > 0:
            l0, l1, lt = math.log10(b0), math.log10(b1), math.log10(target)
            return e0 + (e1 - e0) * (l0 - lt) / (l0 - l1)
    return None


def fixed_point_loss(res, B, ebn0s, K, target):
    """SNR loss (dB) of the fixed-point OCD-BOX against the floating-point one at a BER."""
    a = ebn0_at(res, B, ebn0s, "ocd-box/%d" % K, target)
    b = ebn0_at(res, B, ebn0s, "ocd-box-fx/%d" % K, target)
    return None if a is None or b is None else b - a


def table(res, B, ebn0s):
    keys = ["%s/%d" % d for d in DETECTORS if d[0] != "mmse"]
    keys = keys[:8] + ["mmse"] + keys[8:]
    lines = ["| Eb/N0 (dB) | " + " | ".join(keys) + " |",
             "|---" * (len(keys) + 1) + "|"]
    for eb in ebn0s:
        r = res[(B, eb)]
        lines.append("| %g | " % eb + " | ".join("%.2e" % (r[k] / r["bits"]) for k in keys) + " |")
    return "\n".join(lines)


def main():
    ap = argparse.ArgumentParser(description=__doc__,
                                 formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--antennas", default="32,64,128")
    ap.add_argument("--ebn0", default="0,2,4,6,8,10,12")
    ap.add_argument("--slots", type=int, default=8)
    ap.add_argument("--out", default=None)
    a = ap.parse_args()
    antennas = [int(x) for x in a.antennas.split(",")]
    ebn0s = [float(x) for x in a.ebn0.split(",")]

    def log(m):
        print("[ber] " + m, file=sys.stderr, flush=True)

    res = study(antennas, ebn0s, a.slots, log=log)
    for B in antennas:
        print("\nB = %d, U = 8, 64-QAM, %d slots of 1200 x 14 vectors (%d bits per point)\n"
              % (B, a.slots, res[(B, ebn0s[0])]["bits"]))
        print(table(res, B, ebn0s))
        for K in (3, 4):
            for target in (1e-2, 1e-3):
                loss = fixed_point_loss(res, B, ebn0s, K, target)
                print("\nfixed-point OCD-BOX K=%d, loss at BER %.0e: %s" % (
                    K, target, "%.3f dB" % loss if loss is not None else "not crossed"))
    if a.out:
        with open(a.out, "w") as fh:
            json.dump([{"B": B, "ebn0_db": eb, **r} for (B, eb), r in sorted(res.items())], fh,
                      indent=1)


if __name__ == "__main__":
    main()
