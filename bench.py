#!/usr/bin/env python3
"""Throughput of the boxcar search on one MI355X.

One step = one whole search of one spectrum (normalisation, power, boxcars
of every width 1..zmax, per-chunk maxima, threshold, candidate extraction
and ordering) through the C ABI, asynchronously on torch's current stream,
with the spectrum already in HBM.  Prints one JSON line on stdout; progress
goes to stderr.

  python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload plain_2e23]
"""

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "G bin-widths/s + % HBM roofline, batched/served vs plain; p99 latency"
HBM_PEAK_GBS = 8000.0
# non-packed 32-bit VALU: 256 CUs x 4 SIMDs x 16 lanes per clock x 2.4 GHz
VALU_PEAK_TOPS = 256 * 4 * 16 * 2.4e9 / 1e12
# minimum VALU work of the dense bank per (bin, width): one add of the
# running sum and half of a three-input max (two comparisons per v_max3_f32)
BANK_OPS_PER_BIN_WIDTH = 1.5


TRAFFIC_FILE = os.path.join(ROOT, "profiles", "bank_kernel_plain_2e23_traffic.json")
BANK_SOURCE = os.path.join(ROOT, "paper_2406_15186_amd", "csrc", "bank.hip")


def measured_traffic():
    """HBM bytes per bank-kernel launch from the committed counter summary, or
    None when there is none or the kernel source has changed since it was taken."""
    import hashlib
    try:
        rec = json.load(open(TRAFFIC_FILE))
    except (OSError, ValueError):
        return None
    src = hashlib.sha256(open(BANK_SOURCE, "rb").read()).hexdigest()
    if rec.get("bank_source_sha256") != src:
        return None
    return int(rec["bytes_per_launch"])


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--workload", default="plain_2e23")
    ap.add_argument("--latency-calls", type=int, default=100)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--dense", action="store_true",
                    help="evaluate every width block (no pruning bound): same candidates")
    ap.add_argument("--copy-reference-mib", type=int, default=0,
                    help="after timing, copy a buffer of this many MiB once on the device, so "
                         "that hardware byte counters can be scaled by a copy of known size")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (asked for {args.gpus}): the search shards by "
              "spectrum with no exchange, so there is no multi-GPU path to time.", file=sys.stderr)
        sys.exit(2)

    import torch

    import paper_2406_15186_amd as pk
    import synth

    wl = synth.workload(args.workload)
    n, Z, C, sigma = wl.nbins, wl.zmax, wl.chunk, wl.sigma
    log(f"bench: workload {wl.name} nbins={n} zmax={Z} chunk={C} sigma={sigma}")
    ctx = pk.Context(0)

    def tone_power(A, w, nt):
        return float(ctx.pulscan_threshold_table(w, A, nt)[w - 1])

    x, tones = synth.make_spectrum(wl, tone_power)
    d = torch.from_numpy(x).to("cuda:0")
    stream = torch.cuda.current_stream()
    cap = ((n + C - 1) // C) * Z
    out_buf = torch.empty(cap * pk.CANDIDATE_DTYPE.itemsize, dtype=torch.uint8, device="cuda:0")
    cnt = torch.zeros(1, dtype=torch.int64, device="cuda:0")

    ref, ref_count = ctx.pulscan_search_ex(d, Z, C, sigma)
    log(f"bench: {ref_count} candidates per step")
    opts = pk.make_opts(async_=True, stream=stream, dense=args.dense)

    def step():
        ctx.pulscan_search_ex(d, Z, C, sigma, capacity=cap, opts=opts, out_device=out_buf,
                              count_device=cnt)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    log(f"bench: warmup {args.warmup} done; timing {args.steps} steps")

    ctx.pulscan_ctx_kernel_time()
    ctx.pulscan_ctx_set_timing(True)
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ev0.record(stream)
    for _ in range(args.steps):
        step()
    ev1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    gpu_ms = ev0.elapsed_time(ev1)
    kms, launches = ctx.pulscan_ctx_kernel_time()
    ctx.pulscan_ctx_set_timing(False)
    assert int(cnt.item()) == ref_count, "timed steps disagree with the reference call"
    ms_per_step = wall * 1e3 / args.steps
    value = n * Z * args.steps / wall / 1e9
    bank_ms = kms / max(launches, 1)
    log(f"bench: {ms_per_step:.4f} ms/step wall, {gpu_ms / args.steps:.4f} ms/step GPU, "
        f"bank kernel {bank_ms * 1e3:.1f} us")

    # synchronous single calls: per-call latency including the host round trip
    lat = []
    for _ in range(args.latency_calls):
        torch.cuda.synchronize()
        a = time.perf_counter()
        ctx.pulscan_search_ex(d, Z, C, sigma, capacity=cap, opts=pk.make_opts(dense=args.dense))
        lat.append((time.perf_counter() - a) * 1e3)
    lat = np.array(lat) if lat else np.zeros(1)

    if args.copy_reference_mib > 0:
        nb = args.copy_reference_mib << 20
        src = torch.ones(nb // 4, dtype=torch.float32, device="cuda:0")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        log(f"bench: copied {args.copy_reference_mib} MiB device to device")
        del src, dst

    if args.dense:
        # every width evaluated: bounded by the VALU work of the recursion
        achieved = n * Z * BANK_OPS_PER_BIN_WIDTH / (bank_ms * 1e-3) / 1e12
        roofline = {"bound": "alu", "achieved": round(achieved, 3),
                    "peak": round(VALU_PEAK_TOPS, 3), "unit": "TOP/s",
                    "frac": round(achieved / VALU_PEAK_TOPS, 4), "traffic": None,
                    "kernel": "bank_kernel", "kernel_us": round(bank_ms * 1e3, 2),
                    "ops_per_bin_width": BANK_OPS_PER_BIN_WIDTH}
    else:
        # pruned bank: one read of the complex spectrum, 8 bytes per bin
        achieved = 8.0 * n / (bank_ms * 1e-3) / 1e9
        roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                    "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": measured_traffic(),
                    "kernel": "bank_kernel", "kernel_us": round(bank_ms * 1e3, 2),
                    "bytes_per_bin": 8}

    cpu = None
    if not args.no_cpu_baseline:
        import oracle
        ns = min(n, 1 << 22)
        log(f"bench: oracle on the first {ns} bins ({oracle.num_threads()} threads)")
        a = time.perf_counter()
        r = oracle.search(x[:ns], Z, C, sigma)
        dt = time.perf_counter() - a
        cpu = {"value": round(ns * Z / dt / 1e9, 4), "unit": "G bin-widths/s",
               "cores": oracle.num_threads(), "kind": "oracle",
               "sample": f"the first {ns} bins of the same spectrum searched as one spectrum, "
                         f"zmax {Z}, chunk {C}: FP64 normalisation, dense bank, maxima, sigma "
                         f"({dt:.2f} s wall)",
               "candidates": int(len(r.cands))}

    line = {
        "metric": METRIC, "value": round(value, 3), "unit": "G bin-widths/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms_per_step, 5),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": wl.name, "nbins": n, "zmax": Z, "chunk": C, "sigma": sigma,
                   "tones": len(tones), "red_frac": wl.red_frac,
                   "path": "plain, async, " + ("dense" if args.dense else "pruned")},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "hbm_frac_step": round(8.0 * n / (ms_per_step * 1e-3) / (HBM_PEAK_GBS * 1e9), 5),
        "gpu_ms_per_step": round(gpu_ms / args.steps, 5),
        "plain_sync_latency_ms": {"p50": round(float(np.percentile(lat, 50)), 4),
                                  "p99": round(float(np.percentile(lat, 99)), 4)},
        "candidates_per_step": ref_count,
    }
    ctx.close()
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
