#!/usr/bin/env python
"""Benchmark of OCD soft-output detection on one MI355X.

Headline workload: B=128 antennas, U=8 users, 1200 subcarriers x 14 OFDM symbols
sharing H_w, 64-QAM, K=3 sweeps, MMSE, 20 dB, FP32 storage (synthetic
Rayleigh-fading slots).  A step is one fused launch of the whole path (stage
H_w, preprocessing, Algorithm 1, soft output, stores) over one slot of 16,800
vectors; consecutive steps cycle through distinct slots (> 1 GB in total) so the
256 MB Infinity Cache cannot hold the inputs.  The launch plan is tuned over
those slots (ocd_autotune_inputs), the regime the steps run in.  The timed steps
are captured in a hipGraph (through torch.cuda.CUDAGraph) and replayed, so host
launch overhead is not timed; HIP events on the replay stream bracket exactly
the timed steps, and the kernel's average launch time is that region divided by
its launches (one per step).

One JSON line goes to stdout; progress goes to stderr.  Besides the contract's
fields it carries the roofline of the dominant kernel, the FP64 oracle timed on
this host's cores, and the other forms: FP16 storage (speedup at equal BER),
the S=1 variant (one H per vector, HBM-bound), the OFDM front end (alone and
followed by detection), the paper's 16-bit fixed-point datapath, explicit MMSE
detection (the detector OCD approximates, at paired bit errors), 48 uneven jobs
in one graph launch against one launch per job, the forward+backward step of the
differentiable form in vectors/s, and the measured FP32 FMA and device-copy rates.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--main-only]
"""

from __future__ import annotations

import argparse
import glob
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBPS = 8000.0          # MI355X HBM3E
FP32_VECTOR_PEAK_TFLOPS = 157.3  # MI355X FP32 vector (packed FMA)
FP32_NONPACKED_TFLOPS = 78.6     # 256 CU x 4 SIMD x 16 lanes x 2 flop x 2.4 GHz
FPGA_MBPS_K3 = 376.0             # Virtex-7, 128x8, 64-QAM, K=3 (Table III)


def log(msg):
    print("[bench] " + msg, file=sys.stderr, flush=True)


def algorithmic(B, U, S, K, Q, cbytes=8):
    """Per-vector work the method itself must do: 16 B U K flops for the K sweeps
    (two B-long complex MAC passes per coordinate update, 8BU+4U real
    multiplications per sweep in the paper's count) plus 4 B U / S for the
    preprocessing shared by S symbols; bytes = H share + y + LLRs + z."""
    flops = 16.0 * B * U * K + 4.0 * B * U / S
    nbytes = cbytes * B * U / S + cbytes * B + 4.0 * U * Q + 8.0 * U
    return flops, nbytes


def algorithmic_mmse(B, U, S, Q, cbytes=8):
    """Per-vector work of explicit MMSE detection (Sections II-B, II-E), in real
    flops (8 per complex MAC): the Gram matrix's upper triangle U(U+1)/2 B and the
    Gauss-Jordan inverse U^3 per subcarrier, shared by S symbols, then the matched
    filter U B and z = A^-1 s, U^2, per vector.  Bytes as for OCD."""
    flops = 8.0 * (U * (U + 1) / 2 * B + U ** 3) / S + 8.0 * (U * B + U * U)
    nbytes = cbytes * B * U / S + cbytes * B + 4.0 * U * Q + 8.0 * U
    return flops, nbytes


# the sources the one-problem detection kernel and its launch are built from
FORWARD_SOURCES = ("ocd_api.hip", "ocd_forward.hip", "ocd_tile.h", "ocd_stage.h", "ocd_device.h",
                   "ocd_internal.h")


def source_hash():
    """Hash of the detection kernel's sources: counter summaries taken on other
    sources no longer describe the kernel."""
    h = hashlib.sha256()
    for name in FORWARD_SOURCES:
        h.update(open(os.path.join(ROOT, "paper_1611_08779_amd", "csrc", name), "rb").read())
    return h.hexdigest()[:16]


TRAFFIC_TAG = "ocd_forward_b128_u8_w1200_s14_64qam_k3"


def plan_fields(plan):
    """The fields of a launch plan that decide which bytes a launch moves (the
    stagger only delays workgroup starts)."""
    return [int(plan["lanes_per_vector"]), int(plan["vectors_per_block"]), int(plan["xcd_remap"]),
            int(plan["channel_in_registers"])]


def read_traffic(kernel_tag, plan):
    """Measured HBM bytes per launch from a committed rocprofv3 counter summary
    (one record per profiled plan), if one was taken under this plan on the
    current kernel sources; else None."""
    path = os.path.join(ROOT, "profiles", "traffic_%s.json" % kernel_tag)
    if not os.path.exists(path):
        return None
    try:
        d = json.load(open(path))
    except ValueError:
        return None
    for rec in d.get("records", []):
        if rec.get("source_hash") == source_hash() and rec.get("plan") == plan_fields(plan):
            return rec.get("bytes_per_launch")
    return None


class GraphedSteps:
    """Captures `fns` (one launch each) into one graph replayed as a block of steps."""

    def __init__(self, torch, fns):
        self.torch = torch
        s = torch.cuda.Stream()
        s.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(s):
            for f in fns:      # warm the plan cache and allocator outside capture
                f()
        torch.cuda.current_stream().wait_stream(s)
        torch.cuda.synchronize()
        self.g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(self.g):
            for f in fns:
                f()
        torch.cuda.synchronize()
        self.n = len(fns)

    def replay(self):
        self.g.replay()


WARM_SECONDS = 0.25   # sustained load before timing: the GPU's clocks ramp up under load


def time_graph(torch, gs, steps, warmup, tail=None):
    """Replays the graph until `steps` steps ran; returns (seconds per step, steps
    timed).  Without `tail` the count is rounded up to whole replays; with `tail`, a
    graph of the first steps % n launches replayed once after the whole ones, it is
    exactly `steps`.

    Warm-up: whole-graph replays until at least `warmup` steps ran and at least
    WARM_SECONDS passed (a few milliseconds of load leave the clocks below their
    sustained level: the same kernel runs ~10% longer in the first milliseconds),
    and the tail once (a graph's first replay uploads it).  One more untimed replay
    runs right before the start event with nothing synchronised after it, so the host
    queues every timed launch while the GPU is busy: the events bracket exactly the
    timed steps' GPU time."""
    reps = steps // gs.n if tail is not None else max(1, math.ceil(steps / gs.n))
    t0, done = time.perf_counter(), 0
    while done < warmup or time.perf_counter() - t0 < WARM_SECONDS:
        for _ in range(max(1, math.ceil(warmup / gs.n))):
            gs.replay()
            done += gs.n
        torch.cuda.synchronize()
    if tail is not None:
        tail.replay()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    gs.replay()
    e0.record()
    for _ in range(reps):
        gs.replay()
    if tail is not None:
        tail.replay()
    e1.record()
    torch.cuda.synchronize()
    n = reps * gs.n + (tail.n if tail is not None else 0)
    return e0.elapsed_time(e1) / 1e3 / n, n


def warm_up(torch, fn):
    """Runs fn until WARM_SECONDS of sustained load have passed (then synchronises)."""
    t0 = time.perf_counter()
    while time.perf_counter() - t0 < WARM_SECONDS:
        for _ in range(4):
            fn()
        torch.cuda.synchronize()


def kernel_durations(torch, fns, rounds=2):
    """Average time of single eager launches: HIP events around each launch on the
    stream it runs on (torch's current stream).  The queue is empty before each
    launch, so this includes the host's launch path (the binding's marshalling and
    the runtime's submission); the kernel's own duration is the graph-replayed
    per-launch time (time_graph), which rocprofv3 confirms."""
    evs = []
    for _ in range(rounds):
        for f in fns:
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record()
            f()
            b.record()
            evs.append((a, b))
    torch.cuda.synchronize()
    ts = [a.elapsed_time(b) / 1e3 for a, b in evs]
    return sum(ts) / len(ts)


def _cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def _time_oracle(fn, target_s, unit_vectors, unit_bits):
    """Runs fn (one pass over a sample) once, then repeatedly for about target_s seconds;
    returns (repetitions, seconds, vectors/s, Gb/s)."""
    t0 = time.perf_counter()
    fn()
    one = time.perf_counter() - t0
    reps = max(1, int(target_s / max(one, 1e-3)))
    t0 = time.perf_counter()
    for _ in range(reps):
        fn()
    dt = time.perf_counter() - t0
    return reps, dt, unit_vectors * reps / dt, unit_bits * reps / dt / 1e9


def cpu_baseline(wl_host, K, Q, N0, target_s, synth):
    """The FP64 oracle (Algorithm 1 plus the brute-force max-log soft output) timed on
    this host's cores, single-threaded and with OpenMP over vectors on every core the
    process may run on: on the headline slot, and on a slice of the box-constrained
    configuration (B=256, U=32, 14 symbols, 16-QAM, box at the constellation edge, K=5,
    10 dB).  Each timing runs about target_s / 4 seconds; a single-threaded pass over
    the whole box slice would take far longer, so that one runs on its first 33
    subcarriers.  `value` is the all-core rate on the headline slot."""
    import oracle
    threads = len(os.sched_getaffinity(0))
    quarter = target_s / 4.0
    H, y = wl_host["H"], wl_host["y"]
    W, S, U = y.shape[0], y.shape[1], H.shape[1]
    Wb, Sb, Bb, Ub, Qb, Kb = 330, 14, 256, 32, 4, 5
    box = synth.make_workload(Bb, Ub, Wb, Sb, Qb, 10.0, seed=[3, 5, 0])
    Nb = float(box["N0"])
    Hb, yb = box["H"], box["y"]
    Ws = 33
    timings = {}
    for name, fn, nv, nb, sample in [
        ("headline_all_cores",
         lambda: oracle.detect(H, y, K, Q, "mmse", N0=N0, threads=threads),
         W * S, W * S * U * Q, "the whole headline slot (%d x %d vectors)" % (W, S)),
        ("headline_one_thread",
         lambda: oracle.detect(H, y, K, Q, "mmse", N0=N0, threads=1),
         W * S, W * S * U * Q, "the whole headline slot (%d x %d vectors)" % (W, S)),
        ("box_b256_u32_all_cores",
         lambda: oracle.detect(Hb, yb, Kb, Qb, "box", N0=Nb, threads=threads),
         Wb * Sb, Wb * Sb * Ub * Qb, "%d subcarriers x %d symbols" % (Wb, Sb)),
        ("box_b256_u32_one_thread",
         lambda: oracle.detect(Hb[:Ws], yb[:Ws], Kb, Qb, "box", N0=Nb, threads=1),
         Ws * Sb, Ws * Sb * Ub * Qb, "the first %d subcarriers x %d symbols" % (Ws, Sb)),
    ]:
        log("cpu baseline: %s" % name)
        reps, dt, vps, gbps = _time_oracle(fn, quarter, nv, nb)
        timings[name] = {"threads": 1 if "one_thread" in name else threads,
                         "vectors_per_s": vps, "gbps": gbps, "repetitions": reps,
                         "seconds": dt, "sample": sample}
    head = timings["headline_all_cores"]
    return {"value": head["gbps"], "unit": "Gb/s", "cores": threads, "kind": "oracle",
            "cpu_model": _cpu_model(),
            "sample": "%d repetitions of one full headline slot (%d subcarriers x %d symbols, "
                      "%d vectors), FP64 oracle (Alg. 1 + brute-force max-log LLR), OpenMP over "
                      "vectors on %d threads, %.1f s wall; timings holds the single-threaded "
                      "rate and the box-constrained slice" % (head["repetitions"], W, S, W * S,
                                                              threads, head["seconds"]),
            "vectors_per_s": head["vectors_per_s"],
            "timings": timings}


# ------------------------------------------------------------------ rocprofv3 summaries

COPY_BYTES = 256 << 20   # the --calibrate-copy transfer


def _csv_rows(d, suffix):
    import csv
    rows = []
    for path in sorted(glob.glob(os.path.join(d, "**", "*" + suffix), recursive=True)):
        with open(path, newline="") as f:
            rows.extend(csv.DictReader(f))
    return rows


def _col(row, *names):
    for n in names:
        if n in row:
            return row[n]
    raise KeyError("none of %s in rocprofv3 CSV columns %s" % (names, sorted(row)))


def _kernel_key(row):
    name = _col(row, "Kernel_Name", "Name").split("(")[0]
    grid = int(_col(row, "Grid_Size_X", "Grid_Size"))
    wg = int(_col(row, "Workgroup_Size_X", "Workgroup_Size"))
    return name, grid, wg


def summarize_profile(dirs, traffic_out, command, plan=None):
    """Prints the rocprofv3 --stats table and a per-(kernel, grid, workgroup) breakdown
    of the kernel trace; on --pmc FETCH_SIZE / WRITE_SIZE directories prints the
    per-dispatch counters, scales them by what the same counters read for the
    256 MiB calibration copy and (with traffic_out) writes the per-launch bytes of
    the detection kernel."""
    import statistics
    out = []
    counters = {}
    for d in dirs:
        stats = _csv_rows(d, "kernel_stats.csv")
        if stats:
            out.append("rocprofv3 --stats (%s):" % os.path.basename(d.rstrip("/")))
            out.append("%-60s %8s %12s %12s %12s" % ("kernel", "calls", "avg_us", "min_us", "max_us"))
            for r in sorted(stats, key=lambda r: -float(_col(r, "TotalDurationNs"))):
                out.append("%-60s %8s %12.3f %12.3f %12.3f" % (
                    _col(r, "Name")[:60], _col(r, "Calls"), float(_col(r, "AverageNs")) / 1e3,
                    float(_col(r, "MinNs")) / 1e3, float(_col(r, "MaxNs")) / 1e3))
        trace = _csv_rows(d, "kernel_trace.csv")
        if trace:
            per = {}
            for r in trace:
                dur = int(_col(r, "End_Timestamp")) - int(_col(r, "Start_Timestamp"))
                per.setdefault(_kernel_key(r), []).append(dur)
            out.append("kernel trace by launch shape (%s):" % os.path.basename(d.rstrip("/")))
            out.append("%-60s %9s %5s %7s %10s %10s" % ("kernel", "grid", "wg", "calls", "mean_us",
                                                        "median_us"))
            for (name, grid, wg), v in sorted(per.items(), key=lambda kv: -sum(kv[1])):
                out.append("%-60s %9d %5d %7d %10.3f %10.3f" % (
                    name[:60], grid, wg, len(v), statistics.mean(v) / 1e3,
                    statistics.median(v) / 1e3))
        for r in _csv_rows(d, "counter_collection.csv"):
            cname = _col(r, "Counter_Name")
            counters.setdefault(cname, {}).setdefault(_kernel_key(r), []).append(
                float(_col(r, "Counter_Value")))
    traffic = {}
    per_kernel = {}   # (kernel shape) -> {counter: median}
    for cname, per in sorted(counters.items()):
        if cname not in ("FETCH_SIZE", "WRITE_SIZE"):
            out.append("%s (per dispatch, summed over the device's instances):" % cname)
            for key, v in sorted(per.items(), key=lambda kv: -sum(kv[1])):
                med = statistics.median(v)
                per_kernel.setdefault(key, {})[cname] = med
                out.append("  %-58s grid=%-8d wg=%-4d n=%-4d median=%.6g" % (
                    key[0][:58], key[1], key[2], len(v), med))
            continue
        # calibration: the largest copy kernel dispatch is the 256 MiB copy
        copies = [(max(v), k) for k, v in per.items() if "copyBuffer" in k[0] or "copy" in k[0].lower()]
        cal = max(copies)[0] if copies else None
        scale = COPY_BYTES / (cal * 1024.0) if cal else None
        out.append("%s (KiB per dispatch; calibration copy of %d MiB reads %s KiB -> scale %s):" % (
            cname, COPY_BYTES >> 20, cal, "%.4f" % scale if scale else None))
        for (name, grid, wg), v in sorted(per.items(), key=lambda kv: -sum(kv[1])):
            med = statistics.median(v)
            out.append("  %-58s grid=%-8d wg=%-4d n=%-4d median=%.1f KiB  scaled=%.3f MB" % (
                name[:58], grid, wg, len(v), med, med * 1024 * (scale or 0) / 1e6))
            if "k_forward" in name:
                traffic.setdefault(cname, []).append((len(v), name, grid, wg, med, scale))
    for (name, grid, wg), c in sorted(per_kernel.items()):
        if "SQ_INSTS_VALU" not in c or "SQ_WAVES" not in c or not c["SQ_WAVES"]:
            continue
        out.append("derived, %s grid=%d wg=%d:" % (name[:58], grid, wg))
        out.append("  VALU instructions per wave %.1f" % (c["SQ_INSTS_VALU"] / c["SQ_WAVES"]))
        if "SQ_INSTS_VALU_FMA_F32" in c:
            out.append("  FP32 FMA share of VALU instructions %.3f" % (
                c["SQ_INSTS_VALU_FMA_F32"] / c["SQ_INSTS_VALU"]))
        if "SQ_ACTIVE_INST_VALU" in c and "SQ_BUSY_CYCLES" in c and c["SQ_BUSY_CYCLES"]:
            # SQ_ACTIVE_INST_VALU: quad-cycles, summed over waves; SQ_BUSY_CYCLES: cycles
            # with waves present, summed over the 32 shader engines (8 XCDs x 4); 1024
            # SIMDs.  (GRBM_GUI_ACTIVE spans more than the kernel under counter collection.)
            se_cycles = c["SQ_BUSY_CYCLES"] / 32.0
            out.append("  shader-engine busy cycles per dispatch %.0f" % se_cycles)
            out.append("  VALU busy (active VALU cycles over SIMD cycles) %.3f" % (
                4.0 * c["SQ_ACTIVE_INST_VALU"] / (se_cycles * 1024)))
        if "SQ_WAVE_CYCLES" in c:
            out.append("  wave cycles per wave %.0f" % (c["SQ_WAVE_CYCLES"] / c["SQ_WAVES"]))
    print("\n".join(out))
    if traffic_out:
        if "FETCH_SIZE" not in traffic or "WRITE_SIZE" not in traffic:
            print("no FETCH_SIZE/WRITE_SIZE dispatches of the detection kernel", file=sys.stderr)
            return 1
        f = max(traffic["FETCH_SIZE"])
        w = max(traffic["WRITE_SIZE"])
        if plan is None:
            print("--traffic-out needs the profiled plan (--plan L,VPB,XCD[,STAGGER])",
                  file=sys.stderr)
            return 1
        rec = {
            "kernel": f[1], "grid": f[2], "workgroup": f[3],
            "plan": plan_fields(plan),
            "workload": "B=128 U=8, 1200 subcarriers x 14 symbols, 64-QAM, K=3, MMSE, FP32",
            "fetch_kib_per_launch": f[4], "fetch_scale": f[5],
            "write_kib_per_launch": w[4], "write_scale": w[5],
            "bytes_per_launch": f[4] * 1024 * f[5] + w[4] * 1024 * w[5],
            "source_hash": source_hash(),
            "command": command,
        }
        # one record per profiled plan: a record of the same plan is replaced
        recs = []
        if os.path.exists(traffic_out):
            try:
                recs = json.load(open(traffic_out)).get("records", [])
            except (ValueError, AttributeError):
                recs = []
        recs = [r for r in recs if r.get("plan") != rec["plan"]] + [rec]
        doc = {"about": "HBM bytes per launch of the detection kernel from rocprofv3 FETCH_SIZE and "
                        "WRITE_SIZE, one record per profiled plan (lanes per vector, vectors per "
                        "workgroup, XCD remap, channel in registers); bench.py reports a record as "
                        "roofline.traffic when the timed plan and the kernel sources' hash match it",
               "records": sorted(recs, key=lambda r: r["plan"])}
        with open(traffic_out, "w") as fh:
            json.dump(doc, fh, indent=1)
        print("wrote %s: %.3f MB per launch" % (traffic_out, rec["bytes_per_launch"] / 1e6))
    return 0


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2000)
    ap.add_argument("--warmup", type=int, default=100)
    ap.add_argument("--slots", type=int, default=34, help="distinct config slots cycled (31 MB each)")
    ap.add_argument("--cpu-seconds", type=float, default=20.0)
    ap.add_argument("--main-only", action="store_true",
                    help="only the headline workload (for profiler runs)")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="run a 256 MiB device copy first (counter calibration under rocprofv3)")
    ap.add_argument("--plan", default=None,
                    help="L,VPB[,XCD[,STAGGER]]: fix the launch plan instead of autotuning "
                         "(profiled runs, so that every traced launch of the kernel is the timed one)")
    ap.add_argument("--mmse-only", default=None, metavar="L,VPB[,XCD[,STAGGER]]",
                    help="only the explicit-MMSE detector on the headline slots with this plan "
                         "(profiled runs); prints its own JSON line")
    ap.add_argument("--ofdm-only", action="store_true",
                    help="only the OFDM front end on the headline slots (profiled runs)")
    ap.add_argument("--fixed-only", action="store_true",
                    help="only the fixed-point datapath on the headline slots (profiled runs)")
    ap.add_argument("--s1-only", action="store_true",
                    help="only the S=1 form (one H per vector); with --plan L,VPB the register "
                         "plan is fixed instead of autotuned (profiled runs)")
    ap.add_argument("--jobs-only", action="store_true",
                    help="only the 48-job batched form")
    ap.add_argument("--fwdbwd-only", action="store_true",
                    help="only the forward+backward step of the differentiable workload "
                         "(profiled runs)")
    ap.add_argument("--summarize-profile", nargs="+", metavar="DIR", default=None,
                    help="no GPU work: summarise rocprofv3 CSV output (a --kernel-trace --stats "
                         "directory, or FETCH_SIZE and WRITE_SIZE --pmc directories) and exit")
    ap.add_argument("--traffic-out", default=None,
                    help="with --summarize-profile on counter directories: write the HBM traffic "
                         "summary that fills roofline.traffic")
    ap.add_argument("--command", default="", help="with --summarize-profile: the profiled command")
    args = ap.parse_args()
    if args.summarize_profile:
        pl = None
        if args.plan:
            f = [int(x) for x in args.plan.split(",")] + [0, 0]
            pl = {"lanes_per_vector": f[0], "vectors_per_block": f[1], "xcd_remap": f[2],
                  "channel_in_registers": 0}
        sys.exit(summarize_profile(args.summarize_profile, args.traffic_out, args.command, pl))
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU: this build has no multi-GPU path (subcarriers would be "
              "sharded with no exchange; see the design notes). Run with --gpus 1.", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_1611_08779_amd as ocd
    import synth

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)

    if args.calibrate_copy:
        n = 256 << 20
        src = torch.empty(n, dtype=torch.uint8, device=dev).fill_(1)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        log("calibration copy of %d bytes done" % n)
        del src, dst

    # ---------------------------------------------------------------- headline
    B, U, W, S, Q, K, snr = 128, 8, 1200, 14, 6, 3, 20.0
    if args.s1_only or args.fwdbwd_only or args.jobs_only:
        args.slots = 1          # the headline slot only fixes N0
    log("generating %d slots of B=%d U=%d W=%d S=%d (64-QAM, %g dB)" % (args.slots, B, U, W, S, snr))
    slots = [synth.make_workload_device(B, U, W, S, Q, snr, seed=1000 + i, device=dev)
             for i in range(args.slots)]
    N0 = float(np.float32(slots[0]["N0"]))
    pb = ocd.problem(B, U, W, S, Q, K, "mmse", "f32", N0)
    outs = [(torch.empty(W, S, U, dtype=torch.complex64, device=dev),
             torch.empty(W, S, U, Q, dtype=torch.float32, device=dev)) for _ in slots]
    if args.s1_only or args.fwdbwd_only or args.jobs_only:
        if args.s1_only:
            fixed = [int(x) for x in args.plan.split(",")][:2] if args.plan else None
            res = s1_form(torch, ocd, synth, dev, args, pb, plan=fixed)
        elif args.jobs_only:
            res = jobs_form(torch, np, ocd, synth, dev)
        else:
            res = fwd_bwd_form(torch, np, ocd, synth, dev)
        print(json.dumps(res), flush=True)
        return
    if args.ofdm_only or args.fixed_only:
        pb32 = ocd.problem(B, U, W, S, Q, K, "mmse", "f32", N0)
        if args.ofdm_only:
            del slots[8:]
            res = ofdm_form(torch, ocd, synth, dev, args, slots, pb32, float("nan"))
        else:
            res = fixed_form(torch, ocd, dev, args, slots, pb32, float("nan"), 0, 0)
        print(json.dumps(res), flush=True)
        return
    if args.mmse_only:
        f = [int(x) for x in args.mmse_only.split(",")] + [0, 0]
        mp = ocd.Plan(f[0], f[1], f[2], 0, f[3])
        pbm = ocd.problem(B, U, W, S, Q, 1, "mmse", "f32", N0)
        fns = [(lambda i=i: ocd.ocd_detect_mmse(pbm, slots[i]["H"], slots[i]["y"], outs[i][0],
                                                outs[i][1], mp)) for i in range(len(slots))]
        tk = kernel_durations(torch, fns)
        t, n = time_graph(torch, GraphedSteps(torch, fns), args.steps, args.warmup)
        flops, nbytes = algorithmic_mmse(B, U, S, Q)
        print(json.dumps({"form": "exact_mmse", "plan": mp.as_dict(), "steps": n,
                          "avg_kernel_us": t * 1e6, "single_eager_launch_us": tk * 1e6,
                          "gbps": W * S * U * Q / t / 1e9, "tflops": flops * W * S / t / 1e12,
                          "hbm_frac": nbytes * W * S / t / 1e9 / HBM_PEAK_GBPS}), flush=True)
        return
    if args.plan:
        f = [int(x) for x in args.plan.split(",")] + [0, 0]
        plan = ocd.Plan(f[0], f[1], f[2], 0, f[3])
        ocd.ocd_set_plan(pb, plan)
        log("fixed plan %s" % plan.as_dict())
    else:
        # timed over every slot in turn: the steady state the bench measures, inputs
        # read from HBM (one slot alone would stay cache-resident between launches)
        plan = ocd.ocd_autotune_inputs(pb, [s["H"] for s in slots], [s["y"] for s in slots],
                                       outs[0][0], outs[0][1], repeats=4)
        log("autotuned plan %s" % plan.as_dict())

    def step_fn(i, prob=pb, ins=slots, o=outs):
        return lambda: ocd.ocd_detect(prob, ins[i]["H"], ins[i]["y"], z=o[i][0], llr=o[i][1])

    fns = [step_fn(i) for i in range(len(slots))]
    t_single = kernel_durations(torch, fns)
    gs = GraphedSteps(torch, fns)
    rem = args.steps % len(fns)
    gs_tail = GraphedSteps(torch, fns[:rem]) if rem else None   # exactly --steps steps
    log("timing %d steps" % args.steps)
    t_step, nsteps = time_graph(torch, gs, args.steps, args.warmup, tail=gs_tail)
    # one launch per step: the kernel's average launch duration over the timed
    # region (HIP events on the stream the graph replays on)
    t_kernel = t_step
    nvec = W * S
    bits_per_step = nvec * U * Q
    flops_v, bytes_v = algorithmic(B, U, S, K, Q)
    value = bits_per_step / t_step / 1e9
    hbm_gbps = bytes_v * nvec / t_step / 1e9
    ach_tflops = flops_v * nvec / t_kernel / 1e12
    # the two ceilings re-measured on this GPU, after the timed region
    fma_tflops = fma_rate(torch, ocd, dev)
    copy_gbps = device_copy_rate(torch, dev, 256 << 20)
    log("%.3f us/step, %.2f Gb/s, single eager launch %.3f us" % (t_step * 1e6, value,
                                                                  t_single * 1e6))

    # spot parity of the timed outputs against the FP64 oracle (sampled subcarriers)
    import oracle
    rng = np.random.default_rng(7)
    ws_s = np.sort(rng.choice(W, 24, replace=False))
    Hs = slots[0]["H"][ws_s].cpu().numpy()
    ys = slots[0]["y"][ws_s].cpu().numpy()
    zo, Lo = oracle.detect(Hs, ys, K, Q, "mmse", N0=N0, threads=0)
    zg = outs[0][0][ws_s].cpu().numpy()
    Lg = outs[0][1][ws_s].cpu().numpy()
    z_err = float(np.max(np.linalg.norm((zg - zo).reshape(-1, U), axis=1) /
                         np.linalg.norm(zo.reshape(-1, U), axis=1)))
    l_err = float(np.max(np.max(np.abs(Lg - Lo).reshape(-1, U * Q), axis=1) /
                         np.max(np.abs(Lo).reshape(-1, U * Q), axis=1)))
    ber = float(torch.mean(((outs[0][1] > 0).to(torch.uint8) != slots[0]["bits"]).float()).item())

    npl = max(2, 1 << math.ceil(math.log2(max(2, math.ceil(B / plan.lanes_per_vector)))))
    if plan.channel_in_registers:
        fwd_kernel = "ocd::k_forward_reg<%d, %d, 8, false, false>" % (plan.lanes_per_vector, npl)
    else:
        # the instantiation the launcher picks: unrolled users for U = 8 or 16, their
        # chunked form for other multiples of 8 (entries per lane <= 8); one-ahead
        # column reads only with at most two waves per SIMD (not at this size)
        uc = U if (U in (8, 16) and npl <= 8) else (8 if (U % 8 == 0 and npl <= 8) else 0)
        chunked = uc == 8 and U != 8
        fwd_kernel = "ocd::k_forward<%d, %d, false, false, %d, false, %s>" % (
            plan.lanes_per_vector, npl, uc, "true" if chunked else "false")
    traffic = read_traffic(TRAFFIC_TAG, plan.as_dict())
    result = {
        "metric": "detected Gb/s & % HBM peak (B=128,U=8,64QAM,K=3); fwd+bwd vectors/s",
        "value": value,
        "unit": "Gb/s",
        "n_gpus": 1,
        "steps": nsteps,
        "warmup": args.warmup,
        "ms_per_step": t_step * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": value / (FPGA_MBPS_K3 / 1e3),
        "vs_baseline_ref": "paper's FPGA design, Virtex-7 XC7VX690T, 376 Mb/s (Table III), another "
                           "machine: context only",
        "dtype": "f32",
        "data": "synthetic i.i.d. Rayleigh CN(0,1/B) channels, Gray 64-QAM, AWGN at 20 dB; %d "
                "distinct slots cycled" % len(slots),
        "config": {"workload": "OCD MMSE detection + max-log LLR, B=128 U=8, 1200 subcarriers x 14 "
                               "OFDM symbols (H shared over 14), 64-QAM, K=3, 20 dB, FP32 storage",
                   "vectors_per_step": nvec, "bits_per_step": bits_per_step,
                   "plan": plan.as_dict()},
        "hbm_frac": hbm_gbps / HBM_PEAK_GBPS,
        "hbm_GBps_algorithmic": hbm_gbps,
        "roofline": {
            "bound": "alu",
            "kernel": fwd_kernel,
            "achieved": ach_tflops,
            "peak": FP32_VECTOR_PEAK_TFLOPS,
            "unit": "TFLOP/s",
            "frac": ach_tflops / FP32_VECTOR_PEAK_TFLOPS,
            "frac_of_nonpacked_fp32": ach_tflops / FP32_NONPACKED_TFLOPS,
            "traffic": traffic,
            "avg_kernel_us": t_kernel * 1e6,
            "avg_kernel_us_source": "HIP events around the timed graph replays / launches",
            "single_eager_launch_us": t_single * 1e6,
            "flops_per_vector": flops_v,
            "bytes_per_vector": bytes_v,
            "vectors_per_launch": nvec,
            "hbm_achieved_GBps": bytes_v * nvec / t_kernel / 1e9,
            "hbm_frac_kernel": bytes_v * nvec / t_kernel / 1e9 / HBM_PEAK_GBPS,
            "measured_peaks": {
                "fp32_fma_TFLOPs": fma_tflops,
                "fp32_fma_source": "ocd_probe_fma (non-packed FP32 FMA chains, same build flags)",
                "frac_of_measured_fma": ach_tflops / fma_tflops,
                "device_copy_GBps": copy_gbps,
                "device_copy_source": "torch device-to-device copy of 256 MiB, 4 sources cycled",
            },
        },
        "parity": {"z_rel_err_max": z_err, "llr_rel_err_max": l_err, "tol_z": 1e-4, "tol_llr": 1e-3,
                   "sample": "24 subcarriers x 14 symbols of the first slot vs FP64 oracle",
                   "ber": ber},
    }
    if not args.main_only:
        result["forms"] = other_forms(torch, np, ocd, synth, dev, args, slots, pb, t_step, value)
        log("cpu baseline (FP64 oracle)")
        wl_host = {"H": slots[0]["H"].cpu().numpy(), "y": slots[0]["y"].cpu().numpy()}
        result["cpu_baseline"] = cpu_baseline(wl_host, K, Q, N0, args.cpu_seconds, synth)
    print(json.dumps(result), flush=True)


def ofdm_form(torch, ocd, synth, dev, args, slots, pb32, t_ocd, N=2048, Ncp=144):
    """The OFDM front end on the headline slots: time-domain slots (per antenna and
    symbol, a 144-sample cyclic prefix and 2048 samples) built from the slots'
    frequency-domain vectors, demodulated into the detector's layout; timed alone
    (HBM roofline: every sample read once, every used bin written once) and
    followed by detection."""
    log("form: OFDM front end")
    B, U, W, S, Q, K = pb32.B, pb32.U, pb32.W, pb32.S, pb32.Q, pb32.K
    xs = [synth.ofdm_time_domain_device(sl["y"], N, Ncp) for sl in slots[:8]]
    ys = [torch.empty(W, S, B, dtype=torch.complex64, device=dev) for _ in xs]
    sh = ocd.OfdmShape(B, S, N, Ncp, W)
    fns = [(lambda i=i: ocd.ocd_ofdm_demodulate(sh, xs[i], ys[i])) for i in range(len(xs))]
    tk = kernel_durations(torch, fns)
    t, _ = time_graph(torch, GraphedSteps(torch, fns), max(200, args.steps // 4), 20)
    err = float(torch.max(torch.abs(ys[0] - slots[0]["y"])).item() /
                torch.max(torch.abs(slots[0]["y"])).item())
    outs = [(torch.empty(W, S, U, dtype=torch.complex64, device=dev),
             torch.empty(W, S, U, Q, dtype=torch.float32, device=dev)) for _ in xs]

    def both(i):
        ocd.ocd_ofdm_demodulate(sh, xs[i], ys[i])
        ocd.ocd_detect(pb32, slots[i]["H"], ys[i], z=outs[i][0], llr=outs[i][1])
    t2, _ = time_graph(torch, GraphedSteps(torch, [(lambda i=i: both(i)) for i in range(len(xs))]),
                       max(200, args.steps // 4), 20)
    nbytes = B * S * N * 8 + W * S * B * 8   # samples after each prefix + used bins
    return {"us_per_slot": t * 1e6, "eager_launch_us": tk * 1e6,
            "hbm_GBps": nbytes / t / 1e9, "hbm_frac": nbytes / t / 1e9 / HBM_PEAK_GBPS,
            "bytes_per_slot": nbytes, "max_rel_dev_from_model": err,
            "front_end_plus_ocd_us_per_slot": t2 * 1e6,
            "front_end_plus_ocd_gbps": W * S * U * Q / t2 / 1e9,
            "ocd_alone_us_per_slot": t_ocd * 1e6,
            "kernel": "ocd::k_ofdm_fft<2048, 1024>", "shape": "N=2048, CP=144, W=1200, B=128, S=14"}


def fixed_form(torch, ocd, dev, args, slots, pb32, t_ocd, errs_ocd, nbits):
    """OCD in the paper's 16-bit fixed-point datapath on the headline slots, its
    inputs quantised to Q5.11 at the unit-power channel scale (H, y times sqrt(B),
    N0 times B: the same OCD estimate); bit errors paired with the FP32 path's."""
    log("form: fixed-point datapath")
    B, U, W, S, Q, K = pb32.B, pb32.U, pb32.W, pb32.S, pb32.Q, pb32.K
    c = math.sqrt(B) * 2048.0

    def q(t):
        v = torch.view_as_real(t).to(torch.float64) * c
        return torch.clamp(torch.floor(v + 0.5), -32768, 32767).to(torch.int16).contiguous()

    N0 = float(torch.tensor(pb32.N0 * B, dtype=torch.float32))
    pbf = ocd.problem(B, U, W, S, Q, K, "mmse", "f32", N0)
    ins = [{"H": q(sl["H"]), "y": q(sl["y"])} for sl in slots]
    outs = [(torch.empty(W, S, U, 2, dtype=torch.int16, device=dev),
             torch.empty(W, S, U, Q, dtype=torch.float32, device=dev)) for _ in slots]
    fns = [(lambda i=i: ocd.ocd_detect_fixed(pbf, ins[i]["H"], ins[i]["y"], outs[i][0],
                                             outs[i][1])) for i in range(len(slots))]
    tk = kernel_durations(torch, fns)
    t, _ = time_graph(torch, GraphedSteps(torch, fns), max(200, args.steps // 4), 20)
    errs = sum(int(((outs[i][1] > 0).to(torch.uint8) != slots[i]["bits"]).sum().item())
               for i in range(len(slots)))
    return {"gbps": W * S * U * Q / t / 1e9, "ms_per_step": t * 1e3, "eager_launch_us": tk * 1e6,
            "slowdown_vs_fp32": t / t_ocd, "bit_errors_fixed": errs, "bit_errors_fp32": errs_ocd,
            "bits": nbits, "kernel": "ocd::k_forward_fx<16, 8, true>",
            "inputs": "Q5.11 int16 pairs of sqrt(B) H and sqrt(B) y, N0 B"}


def mmse_form(torch, ocd, synth, dev, args, slots, pb32, t_ocd, errs_ocd, nbits):
    """Explicit MMSE detection on the headline slots: a small plan search timed like
    the form (graph replays over the slots), then the same graph-replayed timing as
    the headline; bit errors
    paired with OCD's (same channels and noise); and the S = 1 shape, where the
    Gram matrix is no longer shared."""
    log("form: explicit MMSE")
    B, U, W, S, Q = pb32.B, pb32.U, pb32.W, pb32.S, pb32.Q
    N0 = pb32.N0
    pbm = ocd.problem(B, U, W, S, Q, 1, "mmse", "f32", N0)
    outs = [(torch.empty(W, S, U, dtype=torch.complex64, device=dev),
             torch.empty(W, S, U, Q, dtype=torch.float32, device=dev)) for _ in slots]

    def best_plan(prob, ins, o, cands):
        """The fastest candidate timed as the form is then timed: graph replays over
        the input sets in turn (inputs read from HBM), not one cache-resident set."""
        best = None
        for c in cands:
            pl = ocd.Plan(c[0], c[1], c[2], 0, c[3] if len(c) > 3 else 0)
            fs = [(lambda i=i: ocd.ocd_detect_mmse(prob, ins[i]["H"], ins[i]["y"], o[i][0],
                                                   o[i][1], pl)) for i in range(len(ins))]
            try:
                fs[0]()
            except ocd.OCDError:   # the plan does not fit the shape (host check, no launch)
                continue
            t, _ = time_graph(torch, GraphedSteps(torch, fs), 2 * len(fs), len(fs))
            if best is None or t < best[0]:
                best = (t, pl)
        return best[1]

    cands = [(16, 14, 0), (16, 28, 0), (16, 14, 1), (32, 14, 0), (8, 14, 0), (8, 28, 0),
             (16, 7, 0), (32, 7, 0), (16, 16, 0), (0, 14, 0), (0, 14, 1)]
    plan = best_plan(pbm, slots, outs, cands)
    fns = [(lambda i=i: ocd.ocd_detect_mmse(pbm, slots[i]["H"], slots[i]["y"], outs[i][0],
                                            outs[i][1], plan)) for i in range(len(slots))]
    tk = kernel_durations(torch, fns)
    t, _ = time_graph(torch, GraphedSteps(torch, fns), args.steps, args.warmup)
    errs = sum(int(((outs[i][1] > 0).to(torch.uint8) != slots[i]["bits"]).sum().item())
               for i in range(len(slots)))
    flops, nbytes = algorithmic_mmse(B, U, S, Q)
    res = {
        "gbps": W * S * U * Q / t / 1e9, "ms_per_step": t * 1e3, "eager_launch_us": tk * 1e6,
        "speedup_vs_ocd_k3": t_ocd / t, "bit_errors_mmse": errs, "bit_errors_ocd_k3": errs_ocd,
        "bits": nbits, "tflops": flops * W * S / t / 1e12,
        "hbm_frac": nbytes * W * S / t / 1e9 / HBM_PEAK_GBPS, "plan": plan.as_dict(),
        "kernel": ("ocd::k_mmse_mfma<false>" if plan.lanes_per_vector == 0 else
                   "ocd::k_mmse<%d, %d, false>" % (plan.lanes_per_vector,
                                                   max(2, 1 << math.ceil(math.log2(
                                                       max(2, math.ceil(B / plan.lanes_per_vector))))))),
    }
    del outs
    # S = 1: every vector has its own H
    W1 = W * S
    pb1 = ocd.problem(B, U, W1, 1, Q, 1, "mmse", "f32", N0)
    ins = [synth.make_workload_device(B, U, W1, 1, Q, 20.0, seed=2000 + i, device=dev)
           for i in range(4)]
    o1 = [(torch.empty(W1, 1, U, dtype=torch.complex64, device=dev),
           torch.empty(W1, 1, U, Q, dtype=torch.float32, device=dev)) for _ in ins]
    plan1 = best_plan(pb1, ins, o1, [(16, 16, 0), (16, 8, 0), (16, 4, 0), (32, 8, 0),
                                           (32, 4, 0), (8, 32, 0), (8, 16, 0), (0, 1, 0),
                                           (0, 1, 1)])
    fns = [(lambda i=i: ocd.ocd_detect_mmse(pb1, ins[i]["H"], ins[i]["y"], o1[i][0], o1[i][1],
                                            plan1)) for i in range(len(ins))]
    t1, _ = time_graph(torch, GraphedSteps(torch, fns), max(200, args.steps // 4), 20)
    flops1, bytes1 = algorithmic_mmse(B, U, 1, Q)
    res["s1"] = {"gbps": W1 * U * Q / t1 / 1e9, "ms_per_step": t1 * 1e3,
                 "tflops": flops1 * W1 / t1 / 1e12,
                 "hbm_frac": bytes1 * W1 / t1 / 1e9 / HBM_PEAK_GBPS, "plan": plan1.as_dict()}
    return res


def fma_rate(torch, ocd, dev, blocks=4096, iters=512, reps=10):
    """Non-packed FP32 FMA rate (TFLOP/s) this GPU reaches: ocd_probe_fma (8 independent
    FMA chains per thread, built like the detection kernels), timed with HIP events
    after a sustained warm-up; the reachable ceiling for the VALU fraction."""
    out = torch.zeros(1024, device=dev)
    fl = 0.0
    warm_up(torch, lambda: ocd.ocd_probe_fma(blocks, iters, out))
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        fl = ocd.ocd_probe_fma(blocks, iters, out)
    e1.record()
    torch.cuda.synchronize()
    return fl * reps / (e0.elapsed_time(e1) * 1e-3) / 1e12


def device_copy_rate(torch, dev, nbytes, reps=50):
    """HBM rate (GB/s, bytes read + written) of torch's device-to-device copy of
    `nbytes`, cycling over 4 sources so that no source stays in the caches: what a
    plain streaming kernel attains on this GPU, next to the published peak."""
    n = nbytes // 4
    src = [torch.randn(n, device=dev) for _ in range(4)]
    dst = torch.empty(n, device=dev)
    for i in range(8):
        dst.copy_(src[i % 4])
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for i in range(reps):
        dst.copy_(src[i % 4])
    e1.record()
    torch.cuda.synchronize()
    t = e0.elapsed_time(e1) * 1e-3 / reps
    del src, dst
    return 2.0 * n * 4 / t / 1e9


def as_f16(torch, t):
    """complex64 tensor -> FP16 (re, im) pairs, the FP16-storage input format."""
    return torch.view_as_real(t).to(torch.float16).contiguous()


def s1_form(torch, ocd, synth, dev, args, pb32, storages=("f32", "f16"), plan=None):
    """The headline vectors with one channel matrix each (S = 1, W = 1200 * 14): no H_w
    to share, so the kernel streams H and y from HBM.  Autotuned plans unless `plan`
    (then channel columns in registers with that lane split), graph replays over 4
    distinct slots; the device-copy rate of a buffer of the slot's size is measured
    beside it."""
    log("form: S=1 variant")
    B, U, W, S, Q, K = pb32.B, pb32.U, pb32.W, pb32.S, pb32.Q, pb32.K
    N0 = pb32.N0
    W1 = W * S
    _, bytes_f32 = algorithmic(B, U, 1, K, Q, cbytes=8)
    res = {"device_copy_GBps": device_copy_rate(torch, dev, int(bytes_f32 * W1))}
    for storage in storages:
        pbs = ocd.problem(B, U, W1, 1, Q, K, "mmse", storage, N0)
        ins = []
        for i in range(4):
            wl = synth.make_workload_device(B, U, W1, 1, Q, 20.0, seed=2000 + i, device=dev)
            if storage == "f16":
                wl = {"H": as_f16(torch, wl["H"]), "y": as_f16(torch, wl["y"])}
            ins.append(wl)
        outs = [(torch.empty(W1, 1, U, dtype=torch.complex64, device=dev),
                 torch.empty(W1, 1, U, Q, dtype=torch.float32, device=dev)) for _ in ins]
        if plan is None:
            ocd.ocd_autotune_inputs(pbs, [x["H"] for x in ins], [x["y"] for x in ins], outs[0][0],
                                    outs[0][1], repeats=3)
        else:
            ocd.ocd_set_plan(pbs, ocd.Plan(plan[0], plan[1], 0, 1))
        fns = [(lambda i=i: ocd.ocd_detect(pbs, ins[i]["H"], ins[i]["y"], z=outs[i][0], llr=outs[i][1]))
               for i in range(len(ins))]
        tk = kernel_durations(torch, fns)
        t1, _ = time_graph(torch, GraphedSteps(torch, fns), max(200, args.steps // 4), 20)
        _, bytes1 = algorithmic(B, U, 1, K, Q, cbytes=4 if storage == "f16" else 8)
        res[storage] = {"gbps": W1 * U * Q / t1 / 1e9, "ms_per_step": t1 * 1e3,
                        "eager_launch_us": tk * 1e6,
                        "hbm_frac": bytes1 * W1 / t1 / 1e9 / HBM_PEAK_GBPS,
                        "frac_of_device_copy": bytes1 * W1 / t1 / 1e9 / res["device_copy_GBps"],
                        "bytes_per_launch": bytes1 * W1,
                        "plan": ocd.ocd_get_plan(pbs).as_dict()}
        del ins, outs
    if "f32" in res and "f16" in res:
        res["fp16_speedup"] = res["f32"]["ms_per_step"] / res["f16"]["ms_per_step"]
    return res


def fwd_bwd_form(torch, np, ocd, synth, dev):
    """Forward + backward step of the differentiable workload (B=128, U=16, 2048 x 4,
    16-QAM, K=4, HYBRID with learnable lambda_k and beta, BCE of the LLRs), tuned
    forward and backward plans, graph replays."""
    log("form: forward+backward")
    B5, U5, W5, S5, Q5, K5 = 128, 16, 2048, 4, 4, 4
    wl = synth.make_workload_device(B5, U5, W5, S5, Q5, 10.0, seed=4000, device=dev)
    N05 = float(np.float32(wl["N0"]))
    lam = torch.full((K5,), N05, device=dev)
    beta5 = float(3 / math.sqrt(10))
    pb5 = ocd.problem(B5, U5, W5, S5, Q5, K5, "hybrid", "f32", N05, 1.0, beta5)
    L5 = torch.empty(W5, S5, U5, Q5, device=dev)
    zh = torch.empty(W5, S5, K5, U5, dtype=torch.complex64, device=dev)
    dlam = torch.empty(K5, device=dev)
    dbeta = torch.empty(1, device=dev)
    dy = torch.empty(W5, S5, B5, dtype=torch.complex64, device=dev)
    wsb = torch.zeros(ocd.ocd_backward_workspace_bytes(pb5), dtype=torch.uint8, device=dev)
    bits = wl["bits"].float()
    inv_n = 1.0 / bits.numel()
    nbits_s = bits * -inv_n          # -bit / N, fixed labels
    z5 = torch.empty(W5, S5, U5, dtype=torch.complex64, device=dev)
    plan_f = ocd.ocd_autotune(pb5, wl["H"], wl["y"], z5, L5, repeats=3)
    del z5

    def fwd_bwd():
        ocd.ocd_detect(pb5, wl["H"], wl["y"], lam, z=None, llr=L5, z_hist=zh)
        # gradient of the mean BCE with logits: (sigmoid(L) - bit) / N, two elementwise ops
        dllr = torch.add(nbits_s, torch.sigmoid(L5), alpha=inv_n)
        ocd.ocd_detect_backward(pb5, wl["H"], wl["y"], lam, zh, dllr, dlam, dbeta, dy, wsb)

    bits_u8 = wl["bits"].to(torch.uint8).contiguous()

    def fwd_bwd_fused():
        # the loss gradient formed inside the adjoint kernel from the bits
        ocd.ocd_detect(pb5, wl["H"], wl["y"], lam, z=None, llr=L5, z_hist=zh)
        ocd.ocd_detect_backward_bce(pb5, wl["H"], wl["y"], lam, zh, bits_u8, dlam, dbeta, dy, wsb)

    def fwd_only():
        ocd.ocd_detect(pb5, wl["H"], wl["y"], lam, z=None, llr=L5, z_hist=zh)

    fwd_only_once = lambda: ocd.ocd_detect(pb5, wl["H"], wl["y"], lam, z=None, llr=L5, z_hist=zh)
    fwd_only_once()
    dllr0 = (torch.sigmoid(L5) - bits) * inv_n
    plan_b = ocd.ocd_autotune_backward(pb5, wl["H"], wl["y"], lam, zh, dllr0, dlam, dbeta, dy, wsb,
                                       repeats=3)
    del dllr0
    # the two ways of forming dLoss/dLLR agree (same forward, same bits)
    fwd_bwd()
    ref = [t.clone() for t in (dlam, dbeta, dy)]
    fwd_bwd_fused()
    torch.cuda.synchronize()
    agree = all(float((a - b).abs().max()) <= 1e-4 * max(float(b.abs().max()), 1e-30)
                for a, b in zip((dlam, dbeta, dy), ref))
    loss1 = torch.empty(1, device=dev)

    def train_step():
        # one launch: forward, loss, loss gradient and the reverse sweeps
        ocd.ocd_detect_train_bce(pb5, wl["H"], wl["y"], lam, bits_u8, None, None, loss1, dlam,
                                 dbeta, dy, wsb)

    ref = [t.clone() for t in (dlam, dbeta, dy)]
    loss_ref = float(torch.nn.functional.binary_cross_entropy_with_logits(L5.double(),
                                                                          bits.double()))
    train_step()
    torch.cuda.synchronize()
    train_agree = all(float((a - b).abs().max()) <= 1e-4 * max(float(b.abs().max()), 1e-30)
                      for a, b in zip((dlam, dbeta, dy), ref))
    train_agree = train_agree and abs(float(loss1) - loss_ref) <= 1e-5 * loss_ref
    plan_t = ocd.ocd_autotune_train(pb5, wl["H"], wl["y"], lam, bits_u8, loss1, dlam, dbeta, dy,
                                    wsb, repeats=3)
    tts, _ = time_graph(torch, GraphedSteps(torch, [train_step] * 8), 400, 16)
    tfb, _ = time_graph(torch, GraphedSteps(torch, [fwd_bwd_fused] * 8), 400, 16)
    tfb2, _ = time_graph(torch, GraphedSteps(torch, [fwd_bwd] * 8), 400, 16)
    tf, _ = time_graph(torch, GraphedSteps(torch, [fwd_only] * 8), 400, 16)
    fl, _ = algorithmic(B5, U5, S5, K5, Q5)
    return {
        "vectors_per_s": W5 * S5 / tts, "ms_per_step": tts * 1e3,
        "step": "one launch of ocd_detect_train_bce: detection, mean BCE of the LLRs, "
                "dLoss/dlambda_k, dLoss/dbeta, dLoss/dy",
        "train_step_matches_two_launch": bool(train_agree),
        "two_launch_vectors_per_s": W5 * S5 / tfb,
        "two_launch_loss_gradient": "formed in the adjoint kernel from the bits "
                                    "(ocd_detect + ocd_detect_backward_bce)",
        "three_step_vectors_per_s": W5 * S5 / tfb2,
        "fused_matches_two_step": bool(agree),
        "fwd_vectors_per_s": W5 * S5 / tf, "step_over_fwd_time": tts / tf,
        "workload": "B=128 U=16, 2048 subcarriers x 4 symbols, 16-QAM, K=4, HYBRID (learnable "
                    "lambda_k, beta), BCE of LLRs, 10 dB",
        "fwd_tflops": fl * W5 * S5 / tf / 1e12,
        "plan_forward": plan_f.as_dict(), "plan_backward": plan_b.as_dict(),
        "plan_train": plan_t.as_dict(),
    }


def jobs_form(torch, np, ocd, synth, dev):
    """48 uneven jobs (B, U, W, K drawn independently; S = 14, 64-QAM, MMSE): one
    persistent launch of ocd_detect_jobs (batch-tuned, graph-captured) against one
    graph-captured launch per job with each job's autotuned plan."""
    log("form: 48 batched jobs")
    jl = synth.batched_job_list()
    probs, Hs, ys = [], [], []
    for j, jd in enumerate(jl):
        wl = synth.make_workload_device(jd["B"], jd["U"], jd["W"], jd["S"], jd["Q"], jd["snr_db"],
                                        seed=3000 + j, device=dev)
        probs.append(ocd.problem(jd["B"], jd["U"], jd["W"], jd["S"], jd["Q"], jd["K"], "mmse", "f32",
                                 float(np.float32(wl["N0"]))))
        Hs.append(wl["H"])
        ys.append(wl["y"])
    z, L, ws = ocd.detect_jobs(probs, Hs, ys, flags=ocd.OCD_JOBS_TUNE)
    torch.cuda.synchronize()
    schedule = ocd.ocd_jobs_schedule(probs)
    log("batched jobs: tuned schedule %s" % schedule)
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(4)]
    reps = 20
    call = ocd.JobsCall(probs, Hs, ys, z, L, ws, flags=ocd.OCD_JOBS_GRAPH)
    warm_up(torch, call)
    ev[0].record()
    for _ in range(reps):
        call()
    ev[1].record()
    torch.cuda.synchronize()
    t_batched = ev[0].elapsed_time(ev[1]) / reps
    # the same launch without the graph (host path included)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        call(flags=0)
    e1.record()
    torch.cuda.synchronize()
    t_batched_eager = e0.elapsed_time(e1) / reps
    # one launch per job, each with its own autotuned plan, captured in a graph
    zs = [torch.empty_like(t) for t in z]
    Ls = [torch.empty_like(t) for t in L]
    for j, pbj in enumerate(probs):
        ocd.ocd_autotune(pbj, Hs[j], ys[j], zs[j], Ls[j], repeats=2)
    fns = [(lambda j=j: ocd.ocd_detect(probs[j], Hs[j], ys[j], z=zs[j], llr=Ls[j]))
           for j in range(len(probs))]
    gs = GraphedSteps(torch, fns)
    warm_up(torch, gs.replay)
    ev[2].record()
    for _ in range(reps):
        gs.replay()
    ev[3].record()
    torch.cuda.synchronize()
    t_sep = ev[2].elapsed_time(ev[3]) / reps
    # eager per-job launches (what a caller without graphs gets)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        for f in fns:
            f()
    e1.record()
    torch.cuda.synchronize()
    t_eager = e0.elapsed_time(e1) / reps
    agree = all(torch.allclose(z[j], zs[j], rtol=1e-5, atol=1e-6) for j in range(len(probs)))
    total_bits = sum(p.W * p.S * p.U * p.Q for p in probs)
    total_flops = sum(algorithmic(p.B, p.U, p.S, p.K, p.Q)[0] * p.W * p.S for p in probs)
    res = {
        "ms_one_launch_graph": t_batched, "ms_one_launch_eager": t_batched_eager,
        "ms_per_job_launches_graph": t_sep,
        "ms_per_job_launches_eager": t_eager,
        "speedup_vs_per_job_graph": t_sep / t_batched, "speedup_vs_per_job_eager": t_eager / t_batched,
        "gbps_one_launch": total_bits / (t_batched / 1e3) / 1e9, "results_agree": bool(agree),
        "tflops_one_launch": total_flops / (t_batched / 1e3) / 1e12,
        "jobs": len(probs), "vectors": sum(p.W * p.S for p in probs),
        "schedule": {"persistent": bool(schedule["persistent"]),
                     "tile_policy": ["512/L vectors", "whole subcarriers", "half-size"][
                         schedule["tile_policy"]],
                     "lane_mode": ["8 entries per lane", "16 per lane for B > 128",
                                   "16 for B > 128, 4 for 32 < B <= 128"][schedule["lane_mode"]],
                     "chosen_by": "ocd_detect_jobs' batch tuner (OCD_JOBS_TUNE)"},
    }
    del Hs, ys, z, L, zs, Ls, ws, gs, call
    return res



def slots_per_launch_form(torch, ocd, synth, dev, pb32, plan):
    """The headline detection with n slots' subcarriers in one launch (W = 1200 n,
    n = 1, 2, 4, 8), same plan, graph replays over 4 distinct inputs: how much of a
    launch is start-up that more work per launch amortises.  The headline value
    stays one slot per step."""
    log("form: slots per launch")
    B, U, W, S, Q, K = pb32.B, pb32.U, pb32.W, pb32.S, pb32.Q, pb32.K
    res = {}
    for n in (1, 2, 4, 8):
        Wn = W * n
        pbn = ocd.problem(B, U, Wn, S, Q, K, "mmse", "f32", pb32.N0)
        ocd.ocd_set_plan(pbn, plan)
        ins = [synth.make_workload_device(B, U, Wn, S, Q, 20.0, seed=3000 + 10 * n + i, device=dev)
               for i in range(4)]
        z = torch.empty(Wn, S, U, dtype=torch.complex64, device=dev)
        L = torch.empty(Wn, S, U, Q, dtype=torch.float32, device=dev)
        fns = [(lambda i=i: ocd.ocd_detect(pbn, ins[i]["H"], ins[i]["y"], z=z, llr=L))
               for i in range(len(ins))]
        t, _ = time_graph(torch, GraphedSteps(torch, fns), max(100, 800 // n), 20)
        res[str(n)] = {"us_per_launch": t * 1e6, "us_per_slot": t * 1e6 / n,
                       "gbps": Wn * S * U * Q / t / 1e9}
        del ins, z, L
    return res


def other_forms(torch, np, ocd, synth, dev, args, slots, pb32, t32, gbps32):
    forms = {}
    B, U, W, S, Q, K = pb32.B, pb32.U, pb32.W, pb32.S, pb32.Q, pb32.K
    N0 = pb32.N0

    # ---- FP16 storage of H and y, same slots
    log("form: FP16 storage")
    pb16 = ocd.problem(B, U, W, S, Q, K, "mmse", "f16", N0)
    s16 = [{"H": as_f16(torch, s["H"]), "y": as_f16(torch, s["y"])} for s in slots]
    o16 = [(torch.empty(W, S, U, dtype=torch.complex64, device=dev),
            torch.empty(W, S, U, Q, dtype=torch.float32, device=dev)) for _ in slots]
    ocd.ocd_autotune_inputs(pb16, [s["H"] for s in s16], [s["y"] for s in s16], o16[0][0],
                            o16[0][1], repeats=2)
    fns = [(lambda i=i: ocd.ocd_detect(pb16, s16[i]["H"], s16[i]["y"], z=o16[i][0], llr=o16[i][1]))
           for i in range(len(slots))]
    tk16 = kernel_durations(torch, fns)
    t16, _ = time_graph(torch, GraphedSteps(torch, fns), args.steps, args.warmup)
    # paired BER on the same channel and noise realisations (all slots)
    e32 = e16 = nb = 0
    o32 = [(torch.empty(W, S, U, dtype=torch.complex64, device=dev),
            torch.empty(W, S, U, Q, dtype=torch.float32, device=dev))]
    for i in range(len(slots)):
        ocd.ocd_detect(pb32, slots[i]["H"], slots[i]["y"], z=o32[0][0], llr=o32[0][1])
        e32 += int(((o32[0][1] > 0).to(torch.uint8) != slots[i]["bits"]).sum().item())
        e16 += int(((o16[i][1] > 0).to(torch.uint8) != slots[i]["bits"]).sum().item())
        nb += slots[i]["bits"].numel()
    _, bytes16 = algorithmic(B, U, S, K, Q, cbytes=4)
    forms["fp16_storage"] = {
        "gbps": W * S * U * Q / t16 / 1e9, "ms_per_step": t16 * 1e3,
        "speedup_vs_fp32": t32 / t16, "eager_launch_us": tk16 * 1e6,
        "bit_errors_fp32": e32, "bit_errors_fp16": e16, "bits": nb,
        "ber_rel_diff": abs(e16 - e32) / max(e32, 1),
        "hbm_frac": bytes16 * W * S / t16 / 1e9 / HBM_PEAK_GBPS,
    }
    del s16, o16

    # ---- the fixed-point datapath of Section IV-C on the same slots
    forms["fixed_point_q11"] = fixed_form(torch, ocd, dev, args, slots, pb32, t32, e32, nb)

    # ---- OFDM front end (Section II-A) feeding the detector
    forms["ofdm_front_end"] = ofdm_form(torch, ocd, synth, dev, args, slots, pb32, t32)

    # ---- explicit MMSE (Sections II-B, II-E): the detector OCD approximates
    forms["exact_mmse"] = mmse_form(torch, ocd, synth, dev, args, slots, pb32, t32, e32, nb)

    # ---- several slots per launch (start-up amortised)
    forms["slots_per_launch"] = slots_per_launch_form(torch, ocd, synth, dev, pb32,
                                                      ocd.ocd_get_plan(pb32))

    # ---- S = 1: one channel matrix per vector (HBM-bound shape)
    forms["s1_one_H_per_vector"] = s1_form(torch, ocd, synth, dev, args, pb32)

    # ---- 48 uneven jobs: one persistent graph launch vs one launch per job
    forms["batched_48_jobs"] = jobs_form(torch, np, ocd, synth, dev)

    # ---- differentiable form: forward + backward step (B=128, U=16, 2048 x 4, 16-QAM, K=4)
    forms["fwd_bwd_differentiable"] = fwd_bwd_form(torch, np, ocd, synth, dev)
    return forms


if __name__ == "__main__":
    main()
