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


TIMING_EVERY = 16  # bank launches per timed one (each timed launch costs ~5 us of step)
SATURATED_REQUESTS = 60000  # the serving capacity run


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


def batched_leg(ctx, pk, synth, args, stream, tone_power):
    """DM-trial batch: spectra of 2^20..2^23 bins (uniform), zmax in {64, 128,
    200}, 0-5 tones each, generated on the device.  One fused launch per
    batch, the chunk and tile picked by the autotuner on the first call, then
    replayed from a captured graph; compared with one launch per spectrum at
    the same chunk on the same stream."""
    import torch
    wls = synth.batched_workload(nspec=args.batch_spectra)
    log(f"bench: batched leg, {len(wls)} spectra")
    xs = []
    for w in wls:
        x, _ = synth.make_spectrum_device(w, tone_power)
        xs.append(x)
    torch.cuda.synchronize()
    zs = [w.zmax for w in wls]
    nb = sum(w.nbins for w in wls)
    bw = sum(w.nbins * w.zmax for w in wls)
    cap = 1 << 22
    buf = torch.empty(cap * pk.CANDIDATE_DTYPE.itemsize, dtype=torch.uint8, device="cuda:0")
    cnt = torch.zeros(1, dtype=torch.int64, device="cuda:0")
    t0 = time.perf_counter()
    _, n0, chunk = ctx.pulscan_search_batched(xs, zs, 0, 6.0, capacity=cap, out_device=buf,
                                              count_device=cnt)
    tune_s = time.perf_counter() - t0
    log(f"bench: autotuned chunk {chunk} in {tune_s:.2f} s; {n0} candidates per batch")
    opts = pk.make_opts(async_=True, stream=stream, graph=True)

    def batch():
        ctx.pulscan_search_batched(xs, zs, chunk, 6.0, capacity=cap, opts=opts, out_device=buf,
                                   count_device=cnt)

    batch()   # direct run, then capture
    batch()   # first replay
    torch.cuda.synchronize()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    ev0.record(stream)
    for _ in range(args.batch_steps):
        batch()
    ev1.record(stream)
    torch.cuda.synchronize()
    ms = ev0.elapsed_time(ev1) / args.batch_steps
    assert int(cnt.item()) == n0, "graph replays disagree with the direct batched call"

    # the same spectra one launch each
    popts = pk.make_opts(async_=True, stream=stream)
    pbuf = torch.empty((1 << 16) * pk.CANDIDATE_DTYPE.itemsize, dtype=torch.uint8,
                       device="cuda:0")
    pcnt = torch.zeros(1, dtype=torch.int64, device="cuda:0")

    def plain_all():
        for x, z in zip(xs, zs):
            ctx.pulscan_search_ex(x, z, chunk, 6.0, capacity=1 << 16, opts=popts, out_device=pbuf,
                                  count_device=pcnt)

    plain_all()
    torch.cuda.synchronize()
    ev0.record(stream)
    plain_all()
    ev1.record(stream)
    torch.cuda.synchronize()
    pms = ev0.elapsed_time(ev1)
    log(f"bench: batched {ms:.3f} ms per batch (graph), plain {pms:.3f} ms for the same spectra")

    # FP16 power storage on the same batch (candidates within the re-check
    # band of the threshold re-decided on their FP32 power), against the FP32
    # result above
    isz = pk.CANDIDATE_DTYPE.itemsize
    ref = buf[: n0 * isz].cpu().numpy().view(pk.CANDIDATE_DTYPE).copy()
    hopts = pk.make_opts(async_=True, stream=stream, graph=True, power_fp16=True)
    hbuf = torch.empty_like(buf)
    hcnt = torch.zeros_like(cnt)

    def batch16():
        ctx.pulscan_search_batched(xs, zs, chunk, 6.0, capacity=cap, opts=hopts, out_device=hbuf,
                                   count_device=hcnt)

    batch16()
    batch16()
    torch.cuda.synchronize()
    ev0.record(stream)
    for _ in range(args.batch_steps):
        batch16()
    ev1.record(stream)
    torch.cuda.synchronize()
    ms16 = ev0.elapsed_time(ev1) / args.batch_steps
    n16 = int(hcnt.item())
    got = hbuf[: n16 * isz].cpu().numpy().view(pk.CANDIDATE_DTYPE)

    def keyed(c):
        return {(int(e["spectrum"]), int(e["harmonics"]), int(e["chunk"]), int(e["width"])): e
                for e in c}

    r, g = keyed(ref), keyed(got)
    both = set(r) & set(g)
    rel = max((abs(float(g[k]["power"]) - float(r[k]["power"])) / float(r[k]["power"])
               for k in both), default=0.0)
    dsig = max((abs(float(g[k]["sigma"]) - float(r[k]["sigma"])) for k in both), default=0.0)
    fp16 = {"ms_per_batch": round(ms16, 4), "value": round(bw / (ms16 * 1e-3) / 1e9, 3),
            "candidates": n16, "only_fp32": len(set(r) - set(g)), "only_fp16": len(set(g) - set(r)),
            "max_rel_power_diff": float(f"{rel:.3g}"), "max_abs_sigma_diff": float(f"{dsig:.3g}"),
            "against": "the FP32 batched result (FP32 parity with the oracle is tested)"}
    log(f"bench: FP16 batch {ms16:.3f} ms, {n16} candidates, {fp16['only_fp32']} only in FP32, "
        f"{fp16['only_fp16']} only in FP16, max rel power diff {rel:.2e}")
    del xs
    torch.cuda.empty_cache()
    return {"workload": f"dm_trials_{len(wls)}", "spectra": len(wls), "bins": nb,
            "bin_widths": bw, "value": round(bw / (ms * 1e-3) / 1e9, 3),
            "unit": "G bin-widths/s", "ms_per_batch": round(ms, 4),
            "hbm_frac": round(8.0 * nb / (ms * 1e-3) / (HBM_PEAK_GBS * 1e9), 4),
            "chunk": chunk, "graph": True, "candidates": n0,
            "plain_value": round(bw / (pms * 1e-3) / 1e9, 3), "plain_ms": round(pms, 4),
            "speedup_vs_plain": round(pms / ms, 3), "autotune_s": round(tune_s, 2),
            "fp16": fp16}


def serve_stream(pk, pool, rate, seconds, host, max_batch, seed, count=None):
    """Poisson arrivals at `rate` per second for `seconds`, each a spectrum
    drawn from `pool` (device tensors, or pinned host pointers if `host`); or,
    with `count`, that many requests submitted back to back.  Returns
    (completed, bin-widths, wall seconds, latencies in ms, launches)."""
    import threading
    srv = pk.Server(0, hbm_budget=4 << 30, max_batch=max_batch, chunk=1024, sigma_thresh=6.0)
    rng = np.random.default_rng(seed)
    if count is not None:
        gaps = np.zeros(count)
        seconds = float("inf")
    else:
        gaps = rng.exponential(1.0 / rate, size=int(rate * seconds * 1.5) + 16)
    picks = rng.integers(0, len(pool), size=gaps.size)
    sent = []

    def feeder():
        t = time.perf_counter()
        t_end = t + seconds
        nxt = t
        for g, k in zip(gaps, picks):
            nxt += g
            if nxt > t_end:
                break
            d = nxt - time.perf_counter()
            if d > 0:
                time.sleep(d)
            ptr, n, z = pool[k]
            srv.pulscan_server_submit(ptr, n, z, not host)
            sent.append(n * z)

    th = threading.Thread(target=feeder)
    t0 = time.perf_counter()
    th.start()
    lat = []
    work = 0
    while th.is_alive() or len(lat) < len(sent):
        for (tk, status, total, ts, tb, td, c) in srv.pulscan_server_poll(wait_ms=20):
            assert status == pk.PULSCAN_OK, status
            lat.append((td - ts) * 1e3)
    wall = time.perf_counter() - t0
    th.join()
    launches = srv.pulscan_server_stats()[2]
    srv.close()
    work = sum(sent)
    return len(lat), work, wall, np.array(lat), launches


def serving_leg(pk, synth, args, tone_power):
    """Serving stream: Poisson arrivals at 200 spectra/s of 2^21..2^23 bins,
    zmax 200, chunk 1024, a 4 GiB device admission budget; device-resident
    spectra (the paper's timing excludes transfers) for the main figure, then
    pinned host spectra copied by the server, and the same arrivals served
    one launch per spectrum (max_batch 1) for comparison."""
    import torch
    rng = np.random.default_rng(4)
    pool, host_pool, hosts = [], [], []
    for k in range(32):
        n = int(rng.integers(1 << 21, (1 << 23) + 1))
        w = synth.Workload(f"serve_{k}", n, 200, 1024, 6.0, 4 * 1000003 + k, int(rng.integers(0, 6)),
                           None, (1, 200), (5.0, 20.0), (1000, n - 202))
        x, _ = synth.make_spectrum_device(w, tone_power)
        pool.append((x, n, 200))
        hp = pk.pulscan_host_alloc(n * 8)
        hosts.append(hp)
        torch.cuda.synchronize()
        import ctypes
        xh = x.cpu().numpy()  # held while copied: .ctypes.data alone keeps no reference
        ctypes.memmove(hp, xh.ctypes.data, n * 8)
        del xh
        host_pool.append((hp, n, 200))
    dev_pool = [(x.data_ptr(), n, z) for x, n, z in pool]
    out = {}
    for name, p, host, secs, mb, rate in (
            ("device", dev_pool, False, args.serve_seconds, 256, args.serve_rate),
            ("host", host_pool, True, min(10.0, args.serve_seconds), 256, args.serve_rate),
            ("device_plain", dev_pool, False, min(10.0, args.serve_seconds), 1, args.serve_rate),
            # requests submitted back to back: the server's capacity
            ("device_saturated", dev_pool, False, None, 256, None)):
        if rate is None:
            log(f"bench: serving leg {name}, {SATURATED_REQUESTS} requests back to back")
            done, work, wall, lat, launches = serve_stream(pk, p, 1.0, 0.0, host, mb, seed=4,
                                                           count=SATURATED_REQUESTS)
        else:
            log(f"bench: serving leg {name}, {secs:.0f} s at {rate:.0f}/s")
            done, work, wall, lat, launches = serve_stream(pk, p, rate, secs, host, mb, seed=4)
        out[name] = {"completed": done, "seconds": round(wall, 2), "arrivals_per_s": rate,
                     "value": round(work / wall / 1e9, 3), "unit": "G bin-widths/s",
                     "p50_ms": round(float(np.percentile(lat, 50)), 3),
                     "p99_ms": round(float(np.percentile(lat, 99)), 3),
                     "launches": launches, "max_batch": mb}
        log(f"bench: {name}: {done} spectra, p50 {out[name]['p50_ms']} ms, "
            f"p99 {out[name]['p99_ms']} ms, {launches} launches")
    for hp in hosts:
        pk.pulscan_host_free(hp)
    del pool
    torch.cuda.empty_cache()
    out["arrivals_per_s"] = args.serve_rate
    out["workload"] = "poisson_2e21_2e23_z200"
    return out


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
    ap.add_argument("--no-batched", action="store_true",
                    help="skip the batched DM-trial leg (512 spectra of 2^20..2^23 bins)")
    ap.add_argument("--batch-spectra", type=int, default=512)
    ap.add_argument("--batch-steps", type=int, default=10)
    ap.add_argument("--serve-seconds", type=float, default=30.0,
                    help="duration of the Poisson arrival stream (device-resident spectra); "
                         "0 skips the serving leg")
    ap.add_argument("--serve-rate", type=float, default=200.0)
    ap.add_argument("--no-copy-peak", dest="copy_peak", action="store_false",
                    help="skip the 1 GiB device-copy bandwidth measurement")
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
    # HIP events around every TIMING_EVERY-th bank launch of the timed
    # steps: their average is the kernel's duration, and the other steps
    # carry no event overhead
    ctx.pulscan_ctx_set_timing(TIMING_EVERY)
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

    # a measured stream-copy peak (a device-to-device copy of 1 GiB, read
    # plus write), to set the HBM figures against what a plain stream reaches
    copy_gbs = None
    if args.copy_peak:
        src = torch.empty(1 << 28, dtype=torch.float32, device="cuda:0")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        c0 = torch.cuda.Event(enable_timing=True)
        c1 = torch.cuda.Event(enable_timing=True)
        c0.record()
        for _ in range(10):
            dst.copy_(src)
        c1.record()
        torch.cuda.synchronize()
        copy_gbs = 2.0 * (1 << 30) * 10 / (c0.elapsed_time(c1) * 1e-3) / 1e9
        log(f"bench: device copy {copy_gbs:.0f} GB/s (read + write)")
        del src, dst
        torch.cuda.empty_cache()

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
        if copy_gbs:
            roofline["copy_peak"] = round(copy_gbs, 1)
            roofline["frac_of_copy"] = round(achieved / copy_gbs, 4)

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

    batched = None
    if not args.no_batched:
        batched = batched_leg(ctx, pk, synth, args, stream, tone_power)

    served = None
    if args.serve_seconds > 0:
        served = serving_leg(pk, synth, args, tone_power)

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
        "batched": batched,
        "served": served,
    }
    ctx.close()
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
