#!/usr/bin/env python3
"""Throughput of the boxcar search on one MI355X.

One step = one whole search of one spectrum (normalisation, power, boxcars
of every width 1..zmax, per-chunk maxima, threshold, candidate extraction
and ordering) through the C ABI, asynchronously on torch's current stream,
with the spectrum already in HBM.  Prints one JSON line on stdout; progress
goes to stderr.

Beside the headline 2^23-bin search the line carries: the same search with
logarithmic width sampling and with four harmonics summed; the 2^16-bin
search's per-call latency; a batch of 512 DM-trial spectra (graph-replayed
fused launch against one launch per spectrum, per-batch p50/p99, FP16 power
storage checked against the FP64 oracle on sampled spectra); a serving
stream of Poisson arrivals; and the FP64 oracle timed on the host cores.

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

# HBM bytes per launch of each bank kernel at the headline workload, from
# committed rocprofv3 counter summaries (valid while the kernel's source is
# the one the counters were taken on)
KERNEL_NAMES = {0: "stream_kernel", 1: "bank_kernel"}   # PULSCAN_KERNEL_STREAM / _TILED
TRAFFIC = {
    "stream_kernel": ("stream_kernel_plain_2e23_traffic.json", ("stream.hip", "mom.hpp")),
    "bank_kernel": ("bank_kernel_plain_2e23_traffic.json", ("bank.hip", "mom.hpp")),
}

TIMING_EVERY = 16           # bank launches per timed one (each timed launch costs ~5 us of step)
SATURATED_REQUESTS = 20000  # the serving capacity run
SERVE_POOL = 256            # distinct device spectra the serving legs draw from
HOST_POOL = 32              # of which pinned host copies serve the host leg
C5_SAMPLES = 3              # spectra of the FP16 batch checked against the oracle
# FP16 storage: entries this close to the threshold may fall on either side
C5_SIGMA_BAND = 0.05


def measured_traffic(kname):
    """HBM bytes per launch of bank kernel `kname` from its committed counter
    summary, or None when there is none or the kernel's source has changed
    since the counters were taken."""
    fname, sources = TRAFFIC[kname]
    try:
        rec = json.load(open(os.path.join(ROOT, "profiles", fname)))
    except (OSError, ValueError):
        return None
    if rec.get("source_sha256") != source_digest(sources):
        return None
    return int(rec["bytes_per_launch"])


def source_digest(sources):
    """SHA-256 over the kernel's source files, in order (the key of a counter
    summary)."""
    import hashlib
    h = hashlib.sha256()
    for name in sources:
        with open(os.path.join(ROOT, "paper_2406_15186_amd", "csrc", name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def pct(a, q):
    return round(float(np.percentile(np.asarray(a), q)), 4)


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def timed_steps(ctx, pk, d, Z, C, sigma, stream, steps, warmup, **kw):
    """Time `steps` asynchronous searches of device spectrum d (after `warmup`
    untimed ones); HIP events around every TIMING_EVERY-th bank launch give
    the bank kernel's duration.  Returns (wall ms per step, GPU ms per step,
    bank-kernel ms, candidate count)."""
    import torch
    n = d.shape[0]
    nh = max(int(kw.get("numharm", 1)), 1)
    cap = sum(((n // H) + C - 1) // C for H in range(1, nh + 1)) * Z
    out_buf = torch.empty(cap * pk.CANDIDATE_DTYPE.itemsize, dtype=torch.uint8, device="cuda:0")
    cnt = torch.zeros(1, dtype=torch.int64, device="cuda:0")
    _, ref_count = ctx.pulscan_search_ex(d, Z, C, sigma, opts=pk.make_opts(**kw))
    opts = pk.make_opts(async_=True, stream=stream, **kw)

    def step():
        ctx.pulscan_search_ex(d, Z, C, sigma, capacity=cap, opts=opts, out_device=out_buf,
                              count_device=cnt)

    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    ctx.pulscan_ctx_kernel_time()
    ctx.pulscan_ctx_set_timing(TIMING_EVERY)
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ev0.record(stream)
    for _ in range(steps):
        step()
    ev1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    kms, launches = ctx.pulscan_ctx_kernel_time()
    ctx.pulscan_ctx_set_timing(False)
    assert int(cnt.item()) == ref_count, "timed steps disagree with the reference call"
    return wall * 1e3 / steps, ev0.elapsed_time(ev1) / steps, kms / max(launches, 1), ref_count


def variant_leg(ctx, pk, d, wl, stream, args, base_ms, name, **kw):
    """The headline search with one option changed, timed like it."""
    n, Z, C = wl.nbins, wl.zmax, wl.chunk
    ms, gms, kms, count = timed_steps(ctx, pk, d, Z, C, wl.sigma, stream, args.steps,
                                      args.warmup, **kw)
    nh = max(int(kw.get("numharm", 1)), 1)
    stage_bins = sum(n // H for H in range(1, nh + 1))
    rec = {"ms_per_step": round(ms, 5), "gpu_ms_per_step": round(gms, 5),
           "bank_kernel_us": round(kms * 1e3, 2), "candidates": count,
           "bin_widths_per_step": stage_bins * Z,
           "value": round(stage_bins * Z / (ms * 1e-3) / 1e9, 3), "unit": "G bin-widths/s",
           "hbm_frac_step": round(8.0 * n / (ms * 1e-3) / (HBM_PEAK_GBS * 1e9), 4),
           "time_vs_all_widths": round(ms / base_ms, 3)}
    log(f"bench: {name}: {ms:.4f} ms/step, bank kernel {kms * 1e3:.1f} us, {count} candidates")
    return rec


def latency_leg(ctx, pk, synth, oracle_free_tone_power, calls):
    """The small plain spectrum: per-call latency of synchronous searches
    (host round trip included, candidates copied to the host)."""
    import torch
    wl = synth.workload("plain_2e16")
    x, _ = synth.make_spectrum(wl, oracle_free_tone_power)
    d = torch.from_numpy(x).to("cuda:0")
    for _ in range(10):
        ctx.pulscan_search_ex(d, wl.zmax, wl.chunk, wl.sigma)
    lat = []
    for _ in range(calls):
        torch.cuda.synchronize()
        a = time.perf_counter()
        _, count = ctx.pulscan_search_ex(d, wl.zmax, wl.chunk, wl.sigma)
        lat.append((time.perf_counter() - a) * 1e3)
    log(f"bench: {wl.name} synchronous calls p50 {pct(lat, 50)} ms, p99 {pct(lat, 99)} ms")
    return {"workload": wl.name, "nbins": wl.nbins, "zmax": wl.zmax, "chunk": wl.chunk,
            "calls": calls, "candidates": count, "p50_ms": pct(lat, 50), "p99_ms": pct(lat, 99)}


def compare_with_oracle(oracle, gpu, x, z, chunk, sigma, band):
    """GPU candidates of one spectrum against the FP64 oracle's: counts of the
    set difference (outside and inside `band` sigma of the threshold) and the
    largest relative power and absolute sigma differences of matched ones."""
    ref = oracle.search(x, z, chunk, sigma)
    g = {(int(c["chunk"]), int(c["width"])): c for c in gpu}
    o = {(int(c["chunk"]), int(c["width"])): c for c in ref.cands}
    only_o = [k for k in set(o) - set(g)]
    only_g = [k for k in set(g) - set(o)]
    nt = float(x.shape[0]) * z
    out_band = sum(1 for k in only_o if abs(float(o[k]["sigma"]) - sigma) >= band)
    out_band += sum(1 for k in only_g
                    if abs(oracle.candidate_sigma(float(g[k]["power"]), k[1], nt) - sigma) >= band)
    both = set(g) & set(o)
    rel = max((abs(float(g[k]["power"]) - o[k]["power"]) / o[k]["power"] for k in both),
              default=0.0)
    ds = max((abs(float(g[k]["sigma"]) - o[k]["sigma"]) for k in both), default=0.0)
    return {"oracle": len(o), "gpu": len(g), "only_oracle": len(only_o), "only_gpu": len(only_g),
            "differing_outside_band": out_band, "max_rel_power_err": rel, "max_abs_sigma_err": ds}


def batched_leg(ctx, pk, synth, args, stream, tone_power):
    """DM-trial batch: spectra of 2^20..2^23 bins (uniform), zmax in {64, 128,
    200}, 0-5 tones each, generated on the device.  One fused launch per
    batch, the chunk picked by the autotuner on the first call, then replayed
    from a captured graph; compared with one launch per spectrum at the same
    chunk on the same stream, both with their threshold tables cached."""
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
    isz = pk.CANDIDATE_DTYPE.itemsize
    buf = torch.empty(cap * isz, dtype=torch.uint8, device="cuda:0")
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
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
           for _ in range(args.batch_steps)]
    for a, b in evs:
        a.record(stream)
        batch()
        b.record(stream)
    torch.cuda.synchronize()
    per = [a.elapsed_time(b) for a, b in evs]
    ms = float(np.mean(per))
    assert int(cnt.item()) == n0, "graph replays disagree with the direct batched call"
    bkernel = KERNEL_NAMES[ctx.pulscan_ctx_last_kernel()]
    ref = buf[: n0 * isz].cpu().numpy().view(pk.CANDIDATE_DTYPE).copy()

    # the same spectra one launch each; the first pass fills the threshold
    # cache, so that the timed pass, like the batch, computes none
    popts = pk.make_opts(async_=True, stream=stream)
    pbuf = torch.empty((1 << 16) * isz, dtype=torch.uint8, device="cuda:0")
    pcnt = torch.zeros(1, dtype=torch.int64, device="cuda:0")

    def plain_all():
        for x, z in zip(xs, zs):
            ctx.pulscan_search_ex(x, z, chunk, 6.0, capacity=1 << 16, opts=popts, out_device=pbuf,
                                  count_device=pcnt)

    plain_all()
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    plain_all()
    e1.record(stream)
    torch.cuda.synchronize()
    pms = e0.elapsed_time(e1)
    log(f"bench: batched {ms:.3f} ms per batch (graph; p50 {pct(per, 50)}, p99 {pct(per, 99)}), "
        f"plain {pms:.3f} ms for the same spectra")

    # FP16 power storage on the same batch (candidates within the re-check
    # band of the threshold re-decided on their FP32 power)
    hopts = pk.make_opts(async_=True, stream=stream, graph=True, power_fp16=True)
    hbuf = torch.empty_like(buf)
    hcnt = torch.zeros_like(cnt)

    def batch16():
        ctx.pulscan_search_batched(xs, zs, chunk, 6.0, capacity=cap, opts=hopts, out_device=hbuf,
                                   count_device=hcnt)

    batch16()
    batch16()
    torch.cuda.synchronize()
    e0.record(stream)
    for _ in range(args.batch_steps):
        batch16()
    e1.record(stream)
    torch.cuda.synchronize()
    ms16 = e0.elapsed_time(e1) / args.batch_steps
    n16 = int(hcnt.item())
    got = hbuf[: n16 * isz].cpu().numpy().view(pk.CANDIDATE_DTYPE).copy()
    log(f"bench: FP16 batch {ms16:.3f} ms, {n16} candidates")

    # sampled spectra of the batch against the FP64 oracle, FP16 and FP32
    fp16_vs_oracle, fp32_vs_oracle = [], []
    if args.c5_samples > 0:
        import oracle
        oracle.set_num_threads(len(os.sched_getaffinity(0)))
        rng = np.random.default_rng(5)
        picks = sorted(int(i) for i in rng.choice(len(wls), size=min(args.c5_samples, len(wls)),
                                                  replace=False))
        for s in picks:
            xh = xs[s].cpu().numpy()
            for res, dst in ((got, fp16_vs_oracle), (ref, fp32_vs_oracle)):
                mine = res[res["spectrum"] == s]
                r = compare_with_oracle(oracle, mine, xh, zs[s], chunk, 6.0, C5_SIGMA_BAND)
                r["spectrum"] = s
                r["nbins"] = int(xh.shape[0])
                r["zmax"] = zs[s]
                dst.append(r)
            log(f"bench: spectrum {s} ({xh.shape[0]} bins, zmax {zs[s]}) against the oracle: "
                f"FP16 {fp16_vs_oracle[-1]}, FP32 {fp32_vs_oracle[-1]}")

    def summary(rs):
        if not rs:
            return None
        return {"spectra": [r["spectrum"] for r in rs],
                "bins": [r["nbins"] for r in rs],
                "candidates_oracle": sum(r["oracle"] for r in rs),
                "only_oracle": sum(r["only_oracle"] for r in rs),
                "only_gpu": sum(r["only_gpu"] for r in rs),
                "differing_outside_band": sum(r["differing_outside_band"] for r in rs),
                "band_sigma": C5_SIGMA_BAND,
                "max_rel_power_err": float(f"{max(r['max_rel_power_err'] for r in rs):.3g}"),
                "max_abs_sigma_err": float(f"{max(r['max_abs_sigma_err'] for r in rs):.3g}")}

    fp16 = {"ms_per_batch": round(ms16, 4), "value": round(bw / (ms16 * 1e-3) / 1e9, 3),
            "candidates": n16, "vs_oracle": summary(fp16_vs_oracle)}
    del xs
    torch.cuda.empty_cache()
    return {"workload": f"dm_trials_{len(wls)}", "spectra": len(wls), "bins": nb,
            "bin_widths": bw, "value": round(bw / (ms * 1e-3) / 1e9, 3),
            "unit": "G bin-widths/s", "ms_per_batch": round(ms, 4),
            "p50_ms": pct(per, 50), "p99_ms": pct(per, 99),
            "hbm_frac": round(8.0 * nb / (ms * 1e-3) / (HBM_PEAK_GBS * 1e9), 4),
            "chunk": chunk, "graph": True, "candidates": n0, "kernel": bkernel,
            "plain_value": round(bw / (pms * 1e-3) / 1e9, 3), "plain_ms": round(pms, 4),
            "speedup_vs_plain": round(pms / ms, 3),
            "thresholds": "cached on both sides", "autotune_s": round(tune_s, 2),
            "fp32_vs_oracle": summary(fp32_vs_oracle), "fp16": fp16}


def serve_stream(pk, pool, rate, seconds, host, max_batch, seed, count=None):
    """Poisson arrivals at `rate` per second for `seconds`, each a spectrum
    drawn from `pool` (device pointers, or pinned host pointers if `host`);
    or, with `count`, that many requests submitted back to back, cycling
    through the pool in order.  Returns (completed, bin-widths, wall seconds,
    latencies in ms, launches)."""
    import threading
    srv = pk.Server(0, hbm_budget=4 << 30, max_batch=max_batch, chunk=1024, sigma_thresh=6.0)
    rng = np.random.default_rng(seed)
    if count is not None:
        gaps = np.zeros(count)
        seconds = float("inf")
        picks = np.arange(count) % len(pool)
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
    while th.is_alive() or len(lat) < len(sent):
        for (tk, status, total, ts, tb, td, c) in srv.pulscan_server_poll(wait_ms=20):
            assert status == pk.PULSCAN_OK, status
            lat.append((td - ts) * 1e3)
    wall = time.perf_counter() - t0
    th.join()
    launches = srv.pulscan_server_stats()[2]
    srv.close()
    return len(lat), sum(sent), wall, np.array(lat), launches


def serving_leg(pk, synth, args, tone_power):
    """Serving stream: Poisson arrivals at 200 spectra/s of 2^21..2^23 bins,
    zmax 200, chunk 1024, a 4 GiB device admission budget, drawn from
    SERVE_POOL distinct device-resident spectra (the paper's timing excludes
    transfers); then pinned host spectra copied by the server, the same
    arrivals served one launch per spectrum (max_batch 1), and requests
    submitted back to back (the server's capacity), which cycle through the
    whole pool so that no launch finds its spectra in the on-chip cache."""
    import ctypes
    import torch
    rng = np.random.default_rng(4)
    pool, host_pool, hosts = [], [], []
    for k in range(args.serve_pool):
        n = int(rng.integers(1 << 21, (1 << 23) + 1))
        w = synth.Workload(f"serve_{k}", n, 200, 1024, 6.0, 4 * 1000003 + k, int(rng.integers(0, 6)),
                           None, (1, 200), (5.0, 20.0), (1000, n - 202))
        x, _ = synth.make_spectrum_device(w, tone_power)
        pool.append((x, n, 200))
        if k < HOST_POOL:
            hp = pk.pulscan_host_alloc(n * 8)
            hosts.append(hp)
            torch.cuda.synchronize()
            xh = x.cpu().numpy()  # held while copied: .ctypes.data alone keeps no reference
            ctypes.memmove(hp, xh.ctypes.data, n * 8)
            del xh
            host_pool.append((hp, n, 200))
    torch.cuda.synchronize()
    dev_pool = [(x.data_ptr(), n, z) for x, n, z in pool]
    pool_bytes = sum(8 * n for _, n, _ in dev_pool)
    out = {}
    for name, p, host, secs, mb, rate in (
            ("device", dev_pool, False, args.serve_seconds, 256, args.serve_rate),
            ("host", host_pool, True, min(10.0, args.serve_seconds), 256, args.serve_rate),
            ("device_plain", dev_pool, False, min(10.0, args.serve_seconds), 1, args.serve_rate),
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
                     "p50_ms": pct(lat, 50), "p99_ms": pct(lat, 99),
                     "launches": launches, "max_batch": mb, "distinct_spectra": len(p)}
        log(f"bench: {name}: {done} spectra, p50 {out[name]['p50_ms']} ms, "
            f"p99 {out[name]['p99_ms']} ms, {launches} launches")
    for hp in hosts:
        pk.pulscan_host_free(hp)
    del pool
    torch.cuda.empty_cache()
    out["arrivals_per_s"] = args.serve_rate
    out["pool_gib"] = round(pool_bytes / 2**30, 2)
    out["workload"] = "poisson_2e21_2e23_z200"
    return out


def cpu_leg(x, Z, C, sigma, repeats, single_bins):
    """The FP64 oracle on the host cores: the whole spectrum with every core
    (median of `repeats` runs), and its first `single_bins` bins on one core."""
    import oracle
    n = x.shape[0]
    cores = len(os.sched_getaffinity(0))
    oracle.set_num_threads(cores)
    ts = []
    count = 0
    for r in range(repeats):
        a = time.perf_counter()
        res = oracle.search(x, Z, C, sigma)
        ts.append(time.perf_counter() - a)
        count = int(len(res.cands))
        log(f"bench: oracle, {n} bins on {cores} threads: {ts[-1]:.2f} s")
    dt = float(np.median(ts))
    oracle.set_num_threads(1)
    ns = min(n, single_bins)
    a = time.perf_counter()
    oracle.search(x[:ns], Z, C, sigma)
    dt1 = time.perf_counter() - a
    oracle.set_num_threads(cores)
    log(f"bench: oracle, first {ns} bins on 1 thread: {dt1:.2f} s")
    return {"value": round(n * Z / dt / 1e9, 4), "unit": "G bin-widths/s", "cores": cores,
            "kind": "oracle",
            "sample": f"the whole {n}-bin spectrum, zmax {Z}, chunk {C}: FP64 normalisation, dense "
                      f"bank, maxima, sigma; median of {repeats} runs on {cores} threads "
                      f"({dt:.2f} s each)",
            "runs_s": [round(t, 3) for t in ts], "candidates": count,
            "single_core": {"value": round(ns * Z / dt1 / 1e9, 4), "unit": "G bin-widths/s",
                            "sample": f"the first {ns} bins of the same spectrum, 1 thread",
                            "seconds": round(dt1, 3)},
            "nproc": os.cpu_count(), "affinity_cpus": cores, "cpu_model": cpu_model()}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--workload", default="plain_2e23")
    ap.add_argument("--latency-calls", type=int, default=100)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-repeats", type=int, default=3)
    ap.add_argument("--cpu-single-bins", type=int, default=1 << 20)
    ap.add_argument("--numharm", type=int, default=1,
                    help="harmonic stages searched by the timed leg (1: the power only); the "
                         "throughput then counts every stage's bin-widths")
    ap.add_argument("--dense", action="store_true",
                    help="evaluate every width block (no pruning bound): same candidates")
    ap.add_argument("--kernel", choices=("auto", "stream", "tiled"), default="auto",
                    help="bank kernel: the library's choice per launch (default), or one forced")
    ap.add_argument("--no-variants", action="store_true",
                    help="skip the log-z and four-harmonic searches of the headline spectrum")
    ap.add_argument("--no-batched", action="store_true",
                    help="skip the batched DM-trial leg (512 spectra of 2^20..2^23 bins)")
    ap.add_argument("--batch-spectra", type=int, default=512)
    ap.add_argument("--batch-steps", type=int, default=20)
    ap.add_argument("--c5-samples", type=int, default=C5_SAMPLES)
    ap.add_argument("--serve-seconds", type=float, default=60.0,
                    help="duration of the Poisson arrival stream (device-resident spectra); "
                         "0 skips the serving leg")
    ap.add_argument("--serve-rate", type=float, default=200.0)
    ap.add_argument("--serve-pool", type=int, default=SERVE_POOL)
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
    ctx.pulscan_ctx_set_kernel({"auto": pk.PULSCAN_KERNEL_AUTO, "stream": pk.PULSCAN_KERNEL_STREAM,
                                "tiled": pk.PULSCAN_KERNEL_TILED}[args.kernel])

    def tone_power(A, w, nt):
        return float(ctx.pulscan_threshold_table(w, A, nt)[w - 1])

    x, tones = synth.make_spectrum(wl, tone_power)
    d = torch.from_numpy(x).to("cuda:0")
    stream = torch.cuda.current_stream()

    nh = max(args.numharm, 1)
    ms_per_step, gpu_ms, bank_ms, ref_count = timed_steps(
        ctx, pk, d, Z, C, sigma, stream, args.steps, args.warmup, dense=args.dense, numharm=nh)
    stage_bins = sum(n // H for H in range(1, nh + 1))
    value = stage_bins * Z / (ms_per_step * 1e-3) / 1e9
    kname = KERNEL_NAMES[ctx.pulscan_ctx_last_kernel()]
    log(f"bench: {ref_count} candidates per step; {ms_per_step:.4f} ms/step wall, "
        f"{gpu_ms:.4f} ms/step GPU, bank kernel ({kname}) {bank_ms * 1e3:.1f} us")

    # synchronous single calls: per-call latency including the host round trip
    cap = sum(((n // H) + C - 1) // C for H in range(1, nh + 1)) * Z
    lat = []
    for _ in range(args.latency_calls):
        torch.cuda.synchronize()
        a = time.perf_counter()
        ctx.pulscan_search_ex(d, Z, C, sigma, capacity=cap,
                              opts=pk.make_opts(dense=args.dense, numharm=nh))
        lat.append((time.perf_counter() - a) * 1e3)
    lat = lat or [0.0]

    variants = None
    if not args.no_variants and not args.dense and nh == 1:
        variants = {
            "log_z": variant_leg(ctx, pk, d, wl, stream, args, ms_per_step, "log-z widths",
                                 width_search=pk.PULSCAN_W_LOG2),
            "numharm_4": variant_leg(ctx, pk, d, wl, stream, args, ms_per_step,
                                     "four harmonics", numharm=4),
        }

    small = None
    if args.latency_calls > 0:
        small = latency_leg(ctx, pk, synth, tone_power, args.latency_calls)

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
                    "kernel": kname, "kernel_us": round(bank_ms * 1e3, 2),
                    "ops_per_bin_width": BANK_OPS_PER_BIN_WIDTH}
    else:
        # pruned bank: one read of the complex spectrum, 8 bytes per bin
        achieved = 8.0 * n / (bank_ms * 1e-3) / 1e9
        roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                    "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                    "traffic": measured_traffic(kname),
                    "kernel": kname,
                    "kernel_us": round(bank_ms * 1e3, 2), "bytes_per_bin": 8}
        if copy_gbs:
            roofline["copy_peak"] = round(copy_gbs, 1)
            roofline["frac_of_copy"] = round(achieved / copy_gbs, 4)

    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_leg(x, Z, C, sigma, args.cpu_repeats, args.cpu_single_bins)

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
                   "path": "plain, async, " + ("dense" if args.dense else "pruned")
                           + (f", {nh} harmonic stages (the bank kernel figure averages the "
                              "power pass and the stage search)" if nh > 1 else ""),
                   "kernel": args.kernel},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "hbm_frac_step": round(8.0 * n / (ms_per_step * 1e-3) / (HBM_PEAK_GBS * 1e9), 5),
        "gpu_ms_per_step": round(gpu_ms, 5),
        "post_bank_us_per_step": round(gpu_ms * 1e3 - bank_ms * 1e3, 2),
        "plain_sync_latency_ms": {"p50": pct(lat, 50), "p99": pct(lat, 99)},
        "candidates_per_step": ref_count,
        "variants": variants,
        "small_latency": small,
        "batched": batched,
        "served": served,
    }
    ctx.close()
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
