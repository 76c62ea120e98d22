"""Throughput and slice-close latency of the ATVC hot path on one MI355X.

One step = one pass of the whole path over the realistic-link workload:
10 slices of 5M (aip, bip) pairs (50M pairs), k = 10, a 2^26-AT pool
(c=9, s=7, u=3, g=4096).  Per slice: open + scan (at_ingest_slice), close
(at_close_slice), restore (at_restore) and the estimates of the window's true
super points (at_estimate).  Inputs are resident in HBM before timing starts.

Prints one JSON line.  `value` is pairs per second over whole steps (Mpps);
the ingest-only rate, slice-close latency p50/p99, the mean relative error of
the plain estimator over the true super points, the roofline of the dominant
kernel (the fused pair scan) and the single-core oracle baseline ride along.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
LINK = dict(k=10, r=4, c=9, s=7, u=3, log2g=12, theta=1024.0, seed=0)
WORKLOAD = ("link: 50M pairs in 10 slices of 5M, aip Zipf 1.2 over 2^22 hosts, bips from 2^26 values, "
            "30% repeats, 371 planted log-uniform [1024, 2^18]; k=10, 2^26-AT pool (c=9,s=7,u=3,g=4096,r=4), "
            "theta=1024")


def log(msg: str):
    print(msg, file=sys.stderr, flush=True)


SERVE_SHAPE = dict(r=4, c=9, s=8, u=1, log2g=12, theta=1024.0)   # 2^24 ATs per link


def serve_phase(dev, n_links: int = 16, slices: int = 10, period_scale: float = 0.1, seed: int = 0, mlp=None):
    """Streaming workload: n_links links, k drawn from {5, 10, 30}, per-slice
    pair counts lognormal (median 2M, sigma 1, clipped to [100k, 20M]), slice
    periods U[50, 200] ms times period_scale with a random phase, chunks of
    65536 pairs arriving uniformly within each slice.  A producer thread
    submits events on that schedule while the main thread runs server steps.
    Latency is taken per slice from its end call to its result on the host."""
    import torch

    from paper_1807_01527_amd import traffic_gpu as tg
    from paper_1807_01527_amd.binding import Server

    rng = np.random.default_rng(seed)
    ks = rng.choice([5, 10, 30], n_links)
    sizes = np.clip(np.exp(np.log(2e6) + rng.standard_normal((n_links, slices))), 1e5, 2e7).astype(np.int64) // 4 * 4
    stream_len = 20_000_000
    streams = []
    for li in range(n_links):
        a, b, planted = tg.link_stream(seed * 1000 + li, stream_len, dev)
        streams.append((a, b, planted))
    torch.cuda.synchronize()
    pool_bytes = (1 << (SERVE_SHAPE["c"] + SERVE_SHAPE["u"])) * SERVE_SHAPE["r"] * (1 << SERVE_SHAPE["log2g"])
    srv = Server(hbm_budget=n_links * (pool_bytes + (8 << 20)), max_links=n_links, cand_cap=2048, watch_cap=64,
                 **SERVE_SHAPE)
    if mlp is not None:
        srv.set_mlp(mlp)
    ids = []
    for li in range(n_links):
        # a tuple budget of 2^24: at these loads windows with more column tuples
        # answer AT_E_BUDGET at once instead of running a long join
        lid, adm = srv.open_link(int(ks[li]), seed * 1000 + li, tuple_budget=1 << 24)
        srv.set_watch(lid, streams[li][2])
        ids.append(lid)
    # event timeline
    chunk = 65536
    events = []
    for li in range(n_links):
        period = rng.uniform(50.0, 200.0) * period_scale * 1e-3
        t = rng.uniform(0, period)
        pos = 0
        for sl in range(slices):
            n = int(sizes[li, sl])
            nch = (n + chunk - 1) // chunk
            times = np.sort(rng.uniform(t, t + period, nch))
            for c in range(nch):
                lo = c * chunk
                hi = min(n, lo + chunk)
                start = (pos + lo) % (stream_len - chunk)
                events.append((times[c], li, "chunk", start, hi - lo))
            events.append((t + period, li, "end", int(ks[li]), 0))
            pos += n
            t += period
    events.sort(key=lambda e: (e[0], e[1], e[2] == "end"))
    total_pairs = int(sizes.sum())
    # device pointers of every event, computed before the clock starts
    lib = srv.lib
    plan = []
    for (ts, li, kind, x, n) in events:
        a, b, _ = streams[li]
        if kind == "chunk":
            plan.append((ts, 0, ids[li], a[x:].data_ptr(), b[x:].data_ptr(), n))
        else:
            plan.append((ts, 1, ids[li], x, 0, 0))
    import ctypes as C
    results = []
    srv.start()                     # the server steps on its own native thread
    t_start = time.perf_counter()
    for (ts, kind, lid, x, y, n) in plan:
        wait = ts - (time.perf_counter() - t_start)
        if wait > 0:
            time.sleep(wait)
        if kind == 0:
            lib.at_serve_submit(srv.h, lid, C.c_void_p(x), C.c_void_p(y), n)
        else:
            lib.at_serve_end_slice(srv.h, lid, x)
    while not all(srv.link_state(lid)[2] == 0 for lid in ids):
        time.sleep(0.0005)
    srv.stop()
    results += srv.results()
    wall = time.perf_counter() - t_start
    st = srv.stats()
    lat = np.array([r["latency_ms"] for r in results])
    srv.destroy()
    return {
        "workload": f"{n_links} links, k from {{5,10,30}}, 2^24-AT pools (c=9,s=8,u=1,g=4096,r=4), {slices} slices "
                    f"per link, lognormal slice sizes (median 2M, sigma 1, [100k, 20M]), 64k-pair chunks, slice "
                    f"periods U[50,200] ms x {period_scale}",
        "closes": len(results), "pairs": total_pairs, "wall_s": wall, "mpps_offered": total_pairs / wall / 1e6,
        "steps": st["steps"],
        "slice_close_ms": {"p50": float(np.percentile(lat, 50)), "p99": float(np.percentile(lat, 99)),
                           "max": float(lat.max())},
        "restore_rc_counts": {str(k): int(v) for k, v in zip(*np.unique([r["restore_rc"] for r in results],
                                                                          return_counts=True))},
    }


def scatter_sweep(n: int = 5_000_000):
    """Random byte-store throughput against buffer size: n items with r = 1 and
    r = 4 uniformly random stores each, the input read as the scan reads it."""
    import torch

    from paper_1807_01527_amd import traffic_gpu as tg
    from paper_1807_01527_amd.binding import probe_scatter
    dev = torch.device("cuda", 0)
    a = tg.as_u32_device(tg.rand_u32(1, 1, n, dev))
    b = tg.as_u32_device(tg.rand_u32(1, 2, n, dev))
    rows = []
    for mb in (1, 2, 4, 8, 16, 32, 64, 128, 256, 512, 1024):
        buf = torch.empty(mb << 20, dtype=torch.uint8, device=dev)
        for r in (1, 4):
            for _ in range(2):
                probe_scatter(buf, a, b, n, r)
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record()
            for _ in range(5):
                probe_scatter(buf, a, b, n, r)
            e1.record()
            torch.cuda.synchronize()
            ms = e0.elapsed_time(e1) / 5
            rows.append({"buffer_mib": mb, "r": r, "us": 1e3 * ms, "gstores_per_s": n * r / ms / 1e6})
            log(f"{mb:5d} MiB r={r}: {1e3 * ms:8.1f} us {n * r / ms / 1e6:7.1f} Gstores/s")
        del buf
    print(json.dumps({"scatter_sweep": rows}), flush=True)


# 2^32 16-bit ATs (8 GiB).  At this load U (column tuples) exceeds 2^32 while
# the pruned join stays cheap, so the guard is raised.
PAPER = dict(k=300, r=4, c=14, s=6, u=4, log2g=12, theta=1024.0, seed=0, tuple_budget=1 << 40)


def paper_scale(slices: int, seed: int = 0) -> dict:
    """The paper's sliding-window shape on synthetic traffic: k = 300 1-s
    slices in the (14, 6, 4, 4096) geometry (2^32 ATs, 16-bit since 2k+1 >
    256), `slices` slices (3600 gives the windows W(0,300)..W(3299,300)).
    Per slice, device time of the opening preserve, the scan and the close
    (HIP events on the handle's stream), and host time of restore plus the
    estimates of the planted hosts; the paper's per-slice figures on its GPU
    are 2 ms (preserve), 20 ms (scan) and 15 ms (estimation)."""
    import torch

    from paper_1807_01527_amd import traffic_gpu as tg
    from paper_1807_01527_amd.binding import AtPool

    dev = torch.device("cuda", 0)
    stream = torch.cuda.current_stream()
    shape = tg.SlidingShape(k=PAPER["k"])
    planted, m = tg.sliding_planted(shape, seed, dev)
    truth = shape.k * m
    watch = planted[truth >= PAPER["theta"]]
    watch_n = truth[truth >= PAPER["theta"]]
    pool = AtPool(**PAPER, stream=stream)
    rec = {"open": [], "scan": [], "close": [], "restore_estimate_ms": [], "pairs": 0}
    errs, fnr, n_out, rcs = [], [], [], {}
    t_all = time.perf_counter()
    for t in range(slices):
        a, b = tg.sliding_slice(shape, seed, t, dev)
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(6)]
        ev[0].record(stream)
        pool.ingest(a[:0], b[:0], n=0)
        ev[1].record(stream)
        ev[2].record(stream)
        pool.ingest(a, b)
        ev[3].record(stream)
        ev[4].record(stream)
        pool.close(PAPER["k"])
        ev[5].record(stream)
        h0 = time.perf_counter()
        full = t >= shape.k - 1
        if full and (t % 10 == 0 or t == slices - 1):
            rc, cand, _, fl, mo = pool.restore(cap=1 << 20)
            e, f, _ = pool.estimate(watch)
            rec["restore_estimate_ms"].append(1e3 * (time.perf_counter() - h0))
            rcs[rc] = rcs.get(rc, 0) + 1
            n_out.append(mo)
            rel = np.abs(e - watch_n) / watch_n
            errs.append((float(rel.mean()), float(rel[watch_n <= 4 * pool.g].mean())))
            if rc == 0:
                fnr.append(1.0 - float(np.isin(watch, cand[(fl & 8) != 0]).mean()))
        torch.cuda.synchronize()
        rec["open"].append(ev[0].elapsed_time(ev[1]))
        rec["scan"].append(ev[2].elapsed_time(ev[3]))
        rec["close"].append(ev[4].elapsed_time(ev[5]))
        rec["pairs"] += a.numel()
        if t % 300 == 0:
            log(f"paper-scale slice {t}/{slices}")
    wall = time.perf_counter() - t_all
    pool_gib = pool.pool_bytes / 2**30
    pool.destroy()
    scan = np.array(rec["scan"])
    close = np.array(rec["close"])
    return {
        "workload": f"paper-scale sliding window: k=300 1-s slices, (c,s,u,g)=(14,6,4,4096), r=4, 2^32 16-bit ATs "
                    f"({pool_gib:.0f} GiB); per slice {shape.distinct} fresh background pairs x{shape.repeat} "
                    f"(Zipf {shape.zipf_s} over 2^22 hosts) + {shape.planted} planted hosts with window "
                    f"cardinality log-uniform [{shape.lo}, {shape.hi}]",
        "slices": slices, "pairs": rec["pairs"], "wall_s": wall,
        "per_slice_ms": {"preserve": float(np.mean(rec["open"])), "scan": float(scan.mean()),
                         "close": float(close.mean()),
                         "restore_plus_estimate_host": float(np.mean(rec["restore_estimate_ms"]))
                         if rec["restore_estimate_ms"] else None},
        "scan_mpps": rec["pairs"] / (scan.sum() / 1e3) / 1e6,
        "close_read_gbs": pool_gib * 2**30 / (close.mean() / 1e3) / 1e9,
        "planted_mean_rel_err": {"all": float(np.mean([e[0] for e in errs])),
                                 "up_to_4g": float(np.mean([e[1] for e in errs])),
                                 "note": "linear counting in g = 4096 ATs saturates for n >> g"} if errs else None,
        "planted_fnr": float(np.mean(fnr)) if fnr else None,
        "restore": {"rc_counts": {str(k): v for k, v in rcs.items()},
                    "n_out_mean": float(np.mean(n_out)) if n_out else None},
        "paper_per_slice_ms": {"preserve": 2, "scan": 20, "estimation": 15, "hardware": "NVIDIA Titan Xp"},
    }


def measured_traffic():
    """HBM bytes per scan launch from the committed counter runs, or None when
    the kernel source has changed since they were taken."""
    import hashlib
    try:
        with open(os.path.join(ROOT, "profiles", "ingest_link_pmc.json")) as fh:
            rec = json.load(fh)
        with open(os.path.join(ROOT, "paper_1807_01527_amd", "csrc", "kernels.hip"), "rb") as fh:
            sha = hashlib.sha256(fh.read()).hexdigest()
    except OSError:
        return None
    if not sha.startswith(rec["kernels_hip_sha256_prefix"]):
        return None
    return rec["traffic_bytes_per_launch"]


def cpu_baseline(tr, truth_hosts, budget_s: float = 15.0) -> dict:
    """The oracle as it stands, single-threaded on a host core, over the
    slices of the same trace (passing over them again while the window keeps
    sliding) until about budget_s of work is done."""
    from oracle import oracle
    o = oracle.Oracle(**LINK)
    t0 = time.perf_counter()
    pairs = 0
    closes = []
    n = 0
    while time.perf_counter() - t0 <= budget_s and n < 4 * tr.n_slices:
        t = n % tr.n_slices
        o.ingest(tr.aip[t], tr.bip[t])
        pairs += tr.aip[t].size
        c0 = time.perf_counter()
        o.close(LINK["k"])
        o.estimate(truth_hosts)
        closes.append(time.perf_counter() - c0)
        n += 1
    el = time.perf_counter() - t0
    return {"value": pairs / el / 1e6, "unit": "Mpps", "cores": 1, "kind": "oracle",
            "sample": f"{n} slices of the {tr.n_slices}-slice trace, in order and again ({pairs} pairs): eager "
                      f"preserve + scan + close + estimate of the {truth_hosts.size} true super points, single thread",
            "slice_close_ms_mean": 1e3 * float(np.mean(closes)), "seconds": el}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--slices", type=int, default=10)
    ap.add_argument("--pairs", type=int, default=5_000_000)
    ap.add_argument("--no-serve", action="store_true", help="skip the streaming-server phase")
    ap.add_argument("--scatter-sweep", action="store_true",
                    help="only sweep the random byte-store probe over buffer sizes (1 MiB .. 1 GiB) and exit")
    ap.add_argument("--paper-scale", type=int, default=0, metavar="SLICES",
                    help="only run the k=300, 2^32-AT sliding shape over SLICES slices (3600 for 3300 windows) "
                         "and exit")
    ap.add_argument("--copy-probe", action="store_true",
                    help="also run a plain 256 MiB device copy (calibrates the HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU only; --gpus above 1 is not supported"}))
        sys.exit(2)
    if args.warmup < 1:
        args.warmup = 1  # the first pass fills the window; measured windows hold all slices

    import torch

    if args.scatter_sweep:
        scatter_sweep()
        return
    if args.paper_scale:
        print(json.dumps({"paper_scale": paper_scale(args.paper_scale)}), flush=True)
        return

    from paper_1807_01527_amd import traffic
    from paper_1807_01527_amd import learned
    from paper_1807_01527_amd.binding import AtPool, Mlp, probe_ace_age, probe_scatter

    t0 = time.perf_counter()
    tr = traffic.generate(traffic.config_link(seed=0, n_slices=args.slices, pairs_per_slice=args.pairs))
    truth_h, truth_n = traffic.window_counts(tr.aip, tr.bip, min_count=int(LINK["theta"]))
    log(f"trace ready in {time.perf_counter() - t0:.1f}s: {tr.cfg.total_pairs} pairs, "
        f"{truth_h.size} true super points")

    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    aip_d = [torch.from_numpy(a.view(np.int32)).to(dev) for a in tr.aip]
    bip_d = [torch.from_numpy(b.view(np.int32)).to(dev) for b in tr.bip]
    stream = torch.cuda.current_stream()
    pool = AtPool(**LINK, stream=stream)
    weights = learned.load_weights("link")
    mlp = Mlp(weights) if weights is not None else None
    S = tr.n_slices
    K = LINK["k"]
    cap = 1 << 20

    def step(record):
        ev = []
        lat = []
        last = None

        def ingest(t):
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            pool.ingest(aip_d[t], bip_d[t])    # opens the slice (lazy preserve) and scans its pairs
            e1.record(stream)
            ev.append((e0, e1))

        # Slice t's queries are queued, then slice t+1's pairs behind them, and
        # only then does the host wait for t's results: the device never idles
        # while the host copies results out.
        ingest(0)
        for t in range(S):
            c0 = time.perf_counter()
            pool.close(K)
            if mlp is not None:
                pool.estimate_learned_begin(mlp, truth_h)
            rc, sip, est, fl, m = pool.restore(cap=cap)
            if mlp is None:
                e_plain, f_plain = pool.estimate_plain(truth_h)
                e_learn = None
            if t + 1 < S:
                ingest(t + 1)
            if mlp is not None:
                e_learn, f_learn, e_plain = pool.estimate_learned_end()
            lat.append(time.perf_counter() - c0)
            last = (rc, m, e_plain, e_learn)
        if record is not None:
            torch.cuda.synchronize()
            record["ingest_ms"].extend(a.elapsed_time(b) for a, b in ev)
            record["close_ms"].extend(1e3 * x for x in lat)
            record["last"] = last

    for _ in range(args.warmup):
        step(None)
    torch.cuda.synchronize()
    rec = {"ingest_ms": [], "close_ms": [], "last": None}
    torch.cuda.synchronize()
    step_ms = []
    t_start = time.perf_counter()
    for s in range(args.steps):
        s0 = time.perf_counter()
        step(rec)
        step_ms.append(1e3 * (time.perf_counter() - s0))
        log(f"step {s + 1}/{args.steps} done")
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t_start

    total_pairs = tr.cfg.total_pairs * args.steps
    ms_step = 1e3 * elapsed / args.steps
    ingest_ms = np.array(rec["ingest_ms"])
    close_ms = np.array(rec["close_ms"])
    rc, m, e_plain, e_learn = rec["last"]
    rel = np.abs(e_plain - truth_n) / truth_n
    rel_l = np.abs(e_learn - truth_n) / truth_n if e_learn is not None else None
    per_launch = args.pairs
    avg_ingest_s = float(ingest_ms.mean()) / 1e3
    # at_ingest_slice's automatic choice (the rule stated with at_set_scan_mode)
    tiles = pool.pool_bytes % 65536 == 0 and pool.pool_bytes // 65536 <= 4096
    tiled = tiles and per_launch * LINK["r"] * 12 >= pool.pool_bytes
    # algorithmic bytes of one call: 8 B read + r B of AT state written per
    # pair; a tiled call that opens the slice (the step's only call) also does
    # the window count of the close: one read of the pool, 4 B per ATV written
    alg_pairs = (8 + LINK["r"]) * per_launch
    alg_count = pool.pool_bytes + 4 * pool.n_atv if tiled and per_launch <= (8 << 20) else 0
    achieved = (alg_pairs + alg_count) / avg_ingest_s / 1e9
    if tiled:
        scan_kernels = ("k_tile_count + k_tile_chunksum + k_tile_scan + k_tile_rowpre + k_tile_scatter + k_tile_apply "
                        "(tiled scan: AT stores grouped per 64 KiB tile, applied in LDS; the opening preserve and the "
                        "close's window count run in k_tile_apply)")
    elif LINK["u"] >= 3 and pool.pool_bytes >= (32 << 20) and per_launch >= 65536:
        scan_kernels = "k_bin_pairs + k_scan_bins (binned scan: XCD-local frame bins, then the r byte stores)"
    else:
        scan_kernels = "k_ingest (fused pair hash + r byte scatter)"
    out = {
        "metric": "Mpps ingested + slice-close p99 ms; mean rel. error plain vs learned at θ=1024",
        "value": total_pairs / elapsed / 1e6,
        "unit": "Mpps",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u8",
        "data": "synthetic",
        "config": {"workload": WORKLOAD, "slices": S, "pairs_per_slice": args.pairs, "k": K,
                   "pool_ats": pool.pool_bytes, "parallelism": "single GPU"},
        "step_ms": {"min": min(step_ms), "median": float(np.median(step_ms)), "max": max(step_ms),
                    "all": [round(x, 3) for x in step_ms]},
        "ingest_mpps": per_launch / avg_ingest_s / 1e6,
        "slice_close_ms": {"p50": float(np.percentile(close_ms, 50)), "p99": float(np.percentile(close_ms, 99)),
                           "includes": "close + restore + plain and learned estimates of the true super points, "
                                       "host wall clock from the close call to the estimates on the host (the next "
                                       "slice's ingest is queued meanwhile)"},
        "restore": {"rc": int(rc), "n_out": int(m), "note": "AT_E_BUDGET (-6) at this load: every ATV is super"},
        "mean_rel_err": {"plain": float(rel.mean()), "learned": float(rel_l.mean()) if rel_l is not None else None,
                         "hosts": int(truth_h.size),
                         "over": "true super points of the window (exact distinct count >= 1024)"},
        "roofline": {"kernel": scan_kernels, "bound": "hbm",
                     "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
                     "traffic": measured_traffic(), "traffic_of": "the scan kernels of one call, rocprofv3 "
                                                                  "FETCH_SIZE x2 + WRITE_SIZE x1 (copy-calibrated)",
                     "bytes_per_pair": 8 + LINK["r"],
                     "algorithmic_bytes_per_launch": {"pairs": alg_pairs, "window_count": alg_count},
                     "avg_launch_ms": float(ingest_ms.mean()), "pairs_per_launch": per_launch},
    }
    # the two scans of at_ingest_slice on the same slices (one pass each)
    modes = {}
    for mode, name in ((1, "direct"), (2, "binned"), (3, "tiled")):
        pool.set_scan_mode(mode)
        evs = []
        for t in range(S):
            pool.ingest(aip_d[t][:0], bip_d[t][:0], n=0)
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            pool.ingest(aip_d[t], bip_d[t])
            e1.record(stream)
            evs.append((e0, e1))
            pool.close(K)
        torch.cuda.synchronize()
        ms = float(np.mean([a.elapsed_time(b) for a, b in evs]))
        modes[name] = {"avg_ms": ms, "mpps": per_launch / (ms / 1e3) / 1e6}
    pool.set_scan_mode(0)
    out["scan_modes"] = modes
    # scatter roofline: the same input stream and r byte stores per pair at
    # uniformly random positions of a pool-sized buffer
    probe_buf = torch.empty(pool.pool_bytes, dtype=torch.uint8, device=dev)
    pr = []
    for rep in range(2):
        for t in range(S):
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            probe_scatter(probe_buf, aip_d[t], bip_d[t], args.pairs, LINK["r"], stream=stream)
            e1.record(stream)
            if rep:
                pr.append((e0, e1))
    torch.cuda.synchronize()
    probe_ms = float(np.mean([a.elapsed_time(b) for a, b in pr]))
    del probe_buf
    out["scatter_probe"] = {
        "what": "uniform random byte stores, r per pair, into a buffer of the pool's size, same input stream",
        "mpps": per_launch / (probe_ms / 1e3) / 1e6, "avg_launch_ms": probe_ms,
        "stores_per_s": LINK["r"] * per_launch / (probe_ms / 1e3),
        "ingest_frac_of_probe": (per_launch / avg_ingest_s) / (per_launch / (probe_ms / 1e3)),
    }
    # the paper's comparison of slice maintenance: aging counters (ACE) rewrite
    # the whole pool at every slice end, asynchronous timestamps preserve two
    # blocks of every ATV (measured on the opening call of each slice)
    ace_buf = torch.full((pool.pool_bytes,), 7, dtype=torch.uint8, device=dev)
    pres, ages = [], []
    for t in range(S):
        e0, e1, e2, e3 = (torch.cuda.Event(enable_timing=True) for _ in range(4))
        e0.record(stream)
        pool.ingest(aip_d[t][:0], bip_d[t][:0], n=0)
        e1.record(stream)
        e2.record(stream)
        probe_ace_age(ace_buf, stream=stream)
        e3.record(stream)
        pool.ingest(aip_d[t], bip_d[t])
        pool.close(K)
        pres.append((e0, e1))
        ages.append((e2, e3))
    torch.cuda.synchronize()
    pm = float(np.mean([a.elapsed_time(b) for a, b in pres]))
    am = float(np.mean([a.elapsed_time(b) for a, b in ages]))
    del ace_buf
    out["slice_maintenance"] = {"at_lazy_preserve_ms": pm, "ace_aging_ms": am, "ratio": am / pm,
                                "note": f"per slice, {pool.pool_bytes >> 20} MiB pool, k={K}: the timestamps touch "
                                        f"2 of 2k blocks per ATV, the aging counters all of them"}
    if args.copy_probe:
        x = torch.empty(256 << 20, dtype=torch.uint8, device=dev)
        y = torch.empty_like(x)
        for _ in range(3):
            y.copy_(x)
        torch.cuda.synchronize()
        out["copy_probe_bytes"] = {"read": x.numel(), "write": y.numel(), "launches": 3}
        del x, y
    if not args.no_serve:
        log("streaming-server phase ...")
        pool.destroy()
        del aip_d, bip_d
        torch.cuda.empty_cache()
        smlp = None
        w_small = learned.load_weights("serve")
        if w_small is not None:
            smlp = Mlp(w_small)
        out["serving"] = serve_phase(dev, mlp=smlp)
    if not args.no_cpu_baseline:
        log("timing the oracle on the host ...")
        out["cpu_baseline"] = cpu_baseline(tr, truth_h)
    pool.destroy()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
