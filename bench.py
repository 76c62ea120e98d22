"""Throughput, slice-close latency and accuracy of the ATVC hot path on one MI355X.

Headline (the large configuration): four links served together, each 200M
(aip, bip) pairs in 60 slices of 3,333,333, k = 60 (7-bit ATs in bytes), a
2^28-AT pool per link ((c, s, u, g) = (10, 6, 4, 4096), r = 4; 1 GiB of
pools), aip Zipf 1.1 over 2^24 hosts, uniform 32-bit bips, 661 planted hosts
log-uniform over [1024, 2^20], seeds 0-3, with the learned correction and the
streaming server on.  One step = one pass of every link over its 60 slices:
per slice and link the server scans the pairs (open + lazy preserve + scan),
closes the slice (window weights, AAT, super lists), runs the restore, the
plain estimates of the window's true super points and the learned
correction.  Inputs are resident in HBM before timing starts; the producer
keeps at most three slices per link in flight.  A paced pass after the timed
ones (a slice per link every 2 ms) gives the close latency without queueing.

Prints one JSON line: `value` is pairs per second over whole steps (Mpps),
with slice-close latency p50/p99/max, the mean relative error of the plain
and learned estimates over the true super points, the roofline of the
dominant kernel (the tiled scan launches), per-step wall times and the
single-core oracle baseline.  The realistic-link configuration, the 16-link
serving shape, a restore-list workload and the probes ride along as extra
keys.
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
LINK_WORKLOAD = ("link: 50M pairs in 10 slices of 5M, aip Zipf 1.2 over 2^22 hosts, bips from 2^26 values, "
                 "30% repeats, 371 planted log-uniform [1024, 2^18]; k=10, 2^26-AT pool (c=9,s=7,u=3,g=4096,r=4), "
                 "theta=1024")
LARGE = dict(k=60, r=4, c=10, s=6, u=4, log2g=12, theta=1024.0)
LARGE_LINKS, LARGE_SLICES, LARGE_PAIRS = 4, 60, 3_333_333
PACE_S = 0.002  # paced pass: one slice per link every 2 ms (the line rate of 100-ms slices, sped up 50x)
LARGE_WORKLOAD = ("large: 4 served links, each 200M pairs in 60 slices of 3,333,333, aip Zipf 1.1 over 2^24 hosts, "
                  "uniform 32-bit bips, 661 planted log-uniform [1024, 2^20], seeds 0-3; k=60, 2^28-AT pool per link "
                  "(c=10,s=6,u=4,g=4096,r=4; 1 GiB in all), theta=1024, learned correction and streaming server on")


def log(msg: str):
    print(msg, file=sys.stderr, flush=True)


SERVE_SHAPE = dict(r=4, c=9, s=8, u=1, log2g=12, theta=1024.0)   # 2^24 ATs per link


def serve_phase(dev, n_links: int = 16, slices: int = 200, period_scale: float = 0.25, seed: int = 0, mlp=None):
    """Streaming workload: n_links links, k drawn from {5, 10, 30}, per-slice
    pair counts lognormal (median 2M, sigma 1, clipped to [100k, 20M]), slice
    periods U[50, 200] ms times period_scale with a random phase, chunks of
    65536 pairs arriving uniformly within each slice (each link's pairs come
    from a 20M-pair stream read cyclically).  This thread submits the events
    on that schedule while the server steps on its own native thread.
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
    # every window k' <= k from one read, at this scale: the next slice closed
    # with the age histograms, then windows re-summarised from them alone
    a, b = tg.sliding_slice(shape, seed, slices, dev)
    pool.ingest(a, b)
    e0, e1 = (torch.cuda.Event(enable_timing=True) for _ in range(2))
    e0.record(stream)
    pool.close_hist(PAPER["k"])
    e1.record(stream)
    rq = {}
    for kp in (1, 10, 100, 299, 300):
        f0, f1 = (torch.cuda.Event(enable_timing=True) for _ in range(2))
        f0.record(stream)
        pool.requery(kp)
        f1.record(stream)
        rq[kp] = (f0, f1)
    torch.cuda.synchronize()
    every_window = {"hist_close_ms": e0.elapsed_time(e1),
                    "requery_ms": {str(kp): x.elapsed_time(y) for kp, (x, y) in rq.items()},
                    "histogram_bytes": pool.n_atv * PAPER["k"] * 2,
                    "note": "at_close_slice_hist reads the 8 GiB pool once and keeps 300 16-bit bins per ATV; "
                            "each at_requery_window sums the first k' bins of every row"}
    pool.destroy()
    # ACE against the timestamps at this scale (both packed at their own width)
    maint = paper_scale_maintenance(shape, seed, slices + 1, 20, dev)
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
        "every_window": every_window,
        "slice_maintenance": maint,
    }


def paper_scale_maintenance(shape, seed: int, t0: int, n: int, dev) -> dict:
    """ACE counters (9 bits) and the asynchronous timestamps (10 bits), both
    packed, on the paper's geometry, fed n slices of the sliding traffic from
    slice t0 on: per-slice maintenance and scan, event-timed."""
    import torch

    from paper_1807_01527_amd import traffic_gpu as tg
    from paper_1807_01527_amd.binding import AtCmp
    stream = torch.cuda.current_stream()
    geom = {x: v for x, v in PAPER.items() if x != "tuple_budget"}
    ace = AtCmp("ace", **geom, stream=stream)
    pat = AtCmp("at", **geom, stream=stream)
    ev = {x: [] for x in ("ace_age", "ace_set", "at_preserve", "at_set")}

    def timed(name, fn):
        e0, e1 = (torch.cuda.Event(enable_timing=True) for _ in range(2))
        e0.record(stream)
        fn()
        e1.record(stream)
        ev[name].append((e0, e1))

    for t in range(t0, t0 + n):
        a, b = tg.sliding_slice(shape, seed, t, dev)
        timed("ace_age", ace.open_slice)
        timed("ace_set", lambda: ace.ingest(a, b))
        ace.close(PAPER["k"])
        timed("at_preserve", pat.open_slice)
        timed("at_set", lambda: pat.ingest(a, b))
        pat.close(PAPER["k"])
    torch.cuda.synchronize()
    # the first slice's ACE pass has nothing to age: averages over the rest
    ms = {x: float(np.mean([p.elapsed_time(q) for p, q in v[1:]])) for x, v in ev.items()}
    same = bool(np.array_equal(ace.read_weights(), pat.read_weights()))
    out = {"slices": n, "ace": {"bits": ace.bits, "bytes": 4 * ace.n_words, "age_ms": ms["ace_age"],
                                "set_ms": ms["ace_set"]},
           "at_packed": {"bits": pat.bits, "bytes": 4 * pat.n_words, "preserve_ms": ms["at_preserve"],
                         "set_ms": ms["at_set"]},
           "maintenance_ratio": ms["ace_age"] / ms["at_preserve"], "same_weights": same,
           "note": "event-timed single launches; the counters start empty, so the timestamps' window holds only "
                   "these slices while ACE ages every counter regardless"}
    ace.destroy()
    pat.destroy()
    return out


def measured_traffic(profile: str):
    """HBM bytes per launch from a committed counter summary, or None when the
    kernel source has changed since the counters were taken."""
    import hashlib
    try:
        with open(os.path.join(ROOT, "profiles", profile)) as fh:
            rec = json.load(fh)
        with open(os.path.join(ROOT, "paper_1807_01527_amd", "csrc", "kernels.hip"), "rb") as fh:
            sha = hashlib.sha256(fh.read()).hexdigest()
    except OSError:
        return None
    if not sha.startswith(rec["kernels_hip_sha256_prefix"]):
        return None
    return rec["traffic_bytes_per_launch"]


def pct(x, q):
    return float(np.percentile(np.asarray(x), q)) if len(x) else None


# --------------------------------------------------------------- large config
def large_workload(dev):
    """Per link (seeds 0-3): device pair streams of the 60 slices and the true
    super points of the full window (exact distinct counts >= theta)."""
    from paper_1807_01527_amd import learned
    from paper_1807_01527_amd import traffic_gpu as tg
    wl = []
    for seed in range(LARGE_LINKS):
        a, b, planted = tg.link_stream(seed, LARGE_SLICES * LARGE_PAIRS, dev, **learned.LARGE_STREAM)
        hosts, counts = learned.exact_counts(a, b)
        m = counts >= LARGE["theta"]
        wl.append(dict(a=a, b=b, planted=planted, truth_h=hosts[m], truth_n=counts[m]))
    return wl


def headline(args, dev, wl, mlp) -> dict:
    import ctypes as C
    import gc

    from paper_1807_01527_amd.binding import Server
    shape = {k: v for k, v in LARGE.items() if k != "k"}
    K = LARGE["k"]
    pool_bytes = (1 << (LARGE["c"] + LARGE["u"])) * LARGE["r"] * (1 << LARGE["log2g"])
    watch_cap = 16384
    srv = Server(hbm_budget=LARGE_LINKS * (pool_bytes + (64 << 20)), max_links=LARGE_LINKS, cand_cap=2048,
                 watch_cap=watch_cap, **shape)
    if mlp is not None:
        srv.set_mlp(mlp)
    ids = []
    for li, w in enumerate(wl):
        # tuple budget 2^24: at this load every ATV is super, so a restore
        # answers AT_E_BUDGET with U instead of enumerating column tuples
        lid, adm = srv.open_link(K, li, tuple_budget=1 << 24)
        assert adm, "the four pools fit the budget"
        srv.set_watch(lid, w["truth_h"][:watch_cap])
        ids.append(lid)
    P = LARGE_PAIRS
    ptrs = [[(w["a"][t * P:].data_ptr(), w["b"][t * P:].data_ptr()) for t in range(LARGE_SLICES)] for w in wl]
    lib, h = srv.lib, srv.h
    got = {lid: [] for lid in ids}

    def drain():
        for r in srv.results():
            got[r["link"]].append(r)

    def run_pass(depth=3, period_s=0.0):
        # per link, slice t is queued (its pairs and its end in one call) once
        # slice t-depth has its result: at most `depth` slices of a link in
        # flight, so the server can close one slice and scan the next in one
        # step.  With period_s > 0 slice t is not queued before t * period_s
        # (a paced pass: the latency is then the server's, not the queue's).
        base = {lid: len(got[lid]) for lid in ids}
        nxt = [0] * len(ids)
        t0 = time.perf_counter()
        while True:
            moved = False
            for li, lid in enumerate(ids):
                t = nxt[li]
                if period_s and time.perf_counter() - t0 < t * period_s:
                    continue
                if t < LARGE_SLICES and t - (len(got[lid]) - base[lid]) < depth:
                    pa, pb = ptrs[li][t]
                    rc = lib.at_serve_submit_last(h, lid, C.c_void_p(pa), C.c_void_p(pb), P, K)
                    assert rc == 0, rc
                    nxt[li] += 1
                    moved = True
            if all(len(got[lid]) - base[lid] >= LARGE_SLICES for lid in ids):
                return
            if not moved:
                drain()
                if period_s:
                    time.sleep(1e-4)

    srv.start()
    for _ in range(args.warmup):
        run_pass()
    warm = {lid: len(got[lid]) for lid in ids}
    t_calls0 = srv.tiled_stats()
    gc.collect()
    gc.disable()
    step_ms = []
    t_start = time.perf_counter()
    for s in range(args.steps):
        s0 = time.perf_counter()
        run_pass()
        step_ms.append(1e3 * (time.perf_counter() - s0))
    elapsed = time.perf_counter() - t_start
    gc.enable()
    for s in range(args.steps):
        log(f"large step {s + 1}/{args.steps}: {step_ms[s]:.2f} ms")
    # paced pass: every link queues a slice each PACE_S, well inside what the
    # server sustains, so each close finds the server idle
    timed_end = {lid: len(got[lid]) for lid in ids}
    t_calls1 = srv.tiled_stats()
    run_pass(depth=3, period_s=PACE_S)
    srv.stop()
    drain()
    t_calls2 = srv.tiled_stats()
    st = srv.stats()
    srv.destroy()
    timed = [r for lid in ids for r in got[lid][warm[lid]:timed_end[lid]]]
    lat = [r["latency_ms"] for r in timed]
    paced = [r["latency_ms"] for lid in ids for r in got[lid][timed_end[lid]:]]
    rcs = {}
    for r in timed:
        rcs[str(r["restore_rc"])] = rcs.get(str(r["restore_rc"]), 0) + 1
    # accuracy over the true super points of the full window (last close)
    rel_p, rel_l, fb, nw = [], [], 0, 0
    for li, lid in enumerate(ids):
        last = got[lid][-1]
        n = wl[li]["truth_n"][:watch_cap].astype(np.float64)
        rel_p.append(np.abs(last["watch_plain"] - n) / n)
        rel_l.append(np.abs(last["watch_learned"] - n) / n)
        fb += int(np.count_nonzero(last["watch_flags"] & 4))
        nw += n.size
    truth_total = int(sum(w["truth_h"].size for w in wl))
    pairs = LARGE_LINKS * LARGE_SLICES * LARGE_PAIRS * args.steps
    calls = t_calls1["calls"] - t_calls0["calls"]
    tjobs = t_calls1["jobs"] - t_calls0["jobs"]
    tpairs = t_calls1["pairs"] - t_calls0["pairs"]
    tms = t_calls1["device_ms"] - t_calls0["device_ms"]
    return dict(
        value=pairs / elapsed / 1e6, elapsed=elapsed, pairs=pairs, step_ms=step_ms,
        slice_close_ms={"p50": pct(lat, 50), "p99": pct(lat, 99), "max": max(lat), "closes": len(lat),
                        "includes": "from the call that queues a slice's last pairs and its end to its result on "
                                    "the host: the scan of those pairs, the close, the restore (AT_E_BUDGET at "
                                    "this load), plain and learned estimates of the window's true super points; "
                                    "in the timed passes up to three slices per link wait in the queue"},
        slice_close_ms_paced={"p50": pct(paced, 50), "p99": pct(paced, 99), "max": max(paced), "closes": len(paced),
                              "pace_ms": 1e3 * PACE_S,
                              "includes": "the same, one pass in which each link queues a slice every pace_ms"},
        restore_rc_counts=rcs,
        mean_rel_err={"plain": float(np.mean(np.concatenate(rel_p))),
                      "learned": float(np.mean(np.concatenate(rel_l))) if mlp is not None else None,
                      "hosts": nw, "fallbacks": fb, "true_super_points": truth_total,
                      "over": "true super points of each link's full window (exact distinct count >= 1024), "
                              "at its last close"},
        tiled={"launches": calls, "jobs": tjobs, "pairs": tpairs, "device_ms": tms, "steps": st["steps"],
               "planned_ahead": t_calls1["planned_ahead"] - t_calls0["planned_ahead"]},
        tiled_paced={k: t_calls2[k] - t_calls1[k] for k in ("calls", "jobs", "pairs", "device_ms")},
        pool_bytes=pool_bytes, n_atv=pool_bytes >> LARGE["log2g"])


def probe_rate(dev, bytes_: int, a, b, n: int, r: int = 4, reps: int = 5) -> dict:
    """Uniform random byte stores (r per item) into a buffer of `bytes_`."""
    import torch

    from paper_1807_01527_amd.binding import probe_scatter
    stream = torch.cuda.current_stream()
    buf = torch.empty(bytes_, dtype=torch.uint8, device=dev)
    for _ in range(2):
        probe_scatter(buf, a, b, n, r, stream=stream)
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(reps):
        probe_scatter(buf, a, b, n, r, stream=stream)
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    del buf
    return {"buffer_bytes": bytes_, "items": n, "r": r, "avg_launch_ms": ms, "mpps": n / ms / 1e3,
            "stores_per_s": r * n / (ms / 1e3)}


# ----------------------------------------------------------- realistic link
def link_config2(args, dev, learned, Mlp) -> dict:
    """The realistic-link configuration through the single-link API (one
    tiled call per slice that opens it, fused window count)."""
    import gc

    import torch

    from paper_1807_01527_amd import traffic
    from paper_1807_01527_amd.binding import AtPool, probe_scatter
    t0 = time.perf_counter()
    tr = traffic.generate(traffic.config_link(seed=0, n_slices=args.slices, pairs_per_slice=args.pairs))
    truth_h, truth_n = traffic.window_counts(tr.aip, tr.bip, min_count=int(LINK["theta"]))
    log(f"link trace ready in {time.perf_counter() - t0:.1f}s: {tr.cfg.total_pairs} pairs, "
        f"{truth_h.size} true super points")
    aip_d = [torch.from_numpy(a.view(np.int32)).to(dev) for a in tr.aip]
    bip_d = [torch.from_numpy(b.view(np.int32)).to(dev) for b in tr.bip]
    stream = torch.cuda.current_stream()
    pool = AtPool(**LINK, stream=stream)
    weights = learned.load_weights("link")
    mlp = Mlp(weights) if weights is not None else None
    S, K, cap = tr.n_slices, LINK["k"], 1 << 20

    def step(record):
        ev, lat = [], []
        last = None

        def ingest(t):
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            pool.ingest(aip_d[t], bip_d[t])
            e1.record(stream)
            ev.append((e0, e1))

        ingest(0)
        for t in range(S):
            c0 = time.perf_counter()
            pool.close(K)
            if mlp is not None:
                pool.estimate_learned_begin(mlp, truth_h)
            rc, sip, est, fl, m = pool.restore(cap=cap)
            if mlp is None:
                e_plain, _ = pool.estimate_plain(truth_h)
                e_learn = None
            if t + 1 < S:
                ingest(t + 1)
            if mlp is not None:
                e_learn, _, e_plain = pool.estimate_learned_end()
            lat.append(time.perf_counter() - c0)
            last = (rc, m, e_plain, e_learn)
        if record is not None:
            torch.cuda.synchronize()
            record["ingest_ms"].extend(a.elapsed_time(b) for a, b in ev)
            record["close_ms"].extend(1e3 * x for x in lat)
            record["last"] = last

    for _ in range(max(1, args.link_warmup)):
        step(None)
    torch.cuda.synchronize()
    rec = {"ingest_ms": [], "close_ms": [], "last": None}
    gc.collect()
    gc.disable()
    step_ms = []
    t_start = time.perf_counter()
    for s in range(args.link_steps):
        s0 = time.perf_counter()
        step(rec)
        step_ms.append(1e3 * (time.perf_counter() - s0))
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t_start
    gc.enable()
    ingest_ms = np.array(rec["ingest_ms"])
    close_ms = np.array(rec["close_ms"])
    rc, m, e_plain, e_learn = rec["last"]
    rel = np.abs(e_plain - truth_n) / truth_n
    rel_l = np.abs(e_learn - truth_n) / truth_n if e_learn is not None else None
    per_launch = args.pairs
    avg_ingest_s = float(ingest_ms.mean()) / 1e3
    alg_pairs = (8 + LINK["r"]) * per_launch
    alg_count = pool.pool_bytes + 4 * pool.n_atv
    achieved = (alg_pairs + alg_count) / avg_ingest_s / 1e9
    out = {
        "workload": LINK_WORKLOAD, "value_mpps": tr.cfg.total_pairs * args.link_steps / elapsed / 1e6,
        "ms_per_step": 1e3 * elapsed / args.link_steps, "steps": args.link_steps,
        "step_ms": {"min": min(step_ms), "median": float(np.median(step_ms)), "max": max(step_ms)},
        "ingest_mpps": per_launch / avg_ingest_s / 1e6,
        "slice_close_ms": {"p50": pct(close_ms, 50), "p99": pct(close_ms, 99), "max": float(close_ms.max()),
                           "includes": "close + restore tuple count (AT_E_BUDGET at this load) + plain and learned "
                                       "estimates of the true super points, host wall clock"},
        "restore": {"rc": int(rc), "n_out": int(m)},
        "mean_rel_err": {"plain": float(rel.mean()), "learned": float(rel_l.mean()) if rel_l is not None else None,
                         "hosts": int(truth_h.size)},
        "roofline": {"kernel": "k_tile_count + k_tile_chunksum + k_tile_rowpre + k_tile_scatter + k_tile_apply "
                               "(one at_ingest_slice call that opens the slice)",
                     "bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": measured_traffic("ingest_link_pmc.json"),
                     "algorithmic_bytes_per_launch": {"pairs": alg_pairs, "window_count": alg_count},
                     "avg_launch_ms": float(ingest_ms.mean()), "pairs_per_launch": per_launch},
    }
    # the three scans of at_ingest_slice on the same slices
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
    # every window k' <= k from one read: the age-histogram close, then each
    # window re-summarised from the histograms alone; beside it the close of
    # 8 windows counted in one read
    hc, rq, mc = [], [], []
    wins8 = [K - j * (K - 1) // 7 for j in range(8)]
    for t in range(S):
        pool.ingest(aip_d[t], bip_d[t])
        e0, e1 = (torch.cuda.Event(enable_timing=True) for _ in range(2))
        e0.record(stream)
        pool.close_hist(K)
        e1.record(stream)
        hc.append((e0, e1))
        for kp in range(1, K + 1):
            e2, e3 = (torch.cuda.Event(enable_timing=True) for _ in range(2))
            e2.record(stream)
            pool.requery(kp)
            e3.record(stream)
            rq.append((e2, e3))
    for t in range(S):
        pool.ingest(aip_d[t], bip_d[t])
        e0, e1 = (torch.cuda.Event(enable_timing=True) for _ in range(2))
        e0.record(stream)
        pool.close_multi(wins8)
        e1.record(stream)
        mc.append((e0, e1))
    torch.cuda.synchronize()
    out["every_window"] = {
        "hist_close_ms": float(np.mean([a.elapsed_time(b) for a, b in hc])),
        "requery_ms": float(np.mean([a.elapsed_time(b) for a, b in rq])),
        "close_8_windows_ms": float(np.mean([a.elapsed_time(b) for a, b in mc])),
        "note": f"event-timed on the {pool.pool_bytes >> 20} MiB pool, k={K}: at_close_slice_hist (one read of the "
                f"pool, every ATV's {K}-bin age histogram, window k summarised), then at_requery_window for each "
                f"k' in 1..{K} (histograms only); beside it at_close_slice_multi of windows {wins8}"}
    pr = probe_rate(dev, pool.pool_bytes, aip_d[0], bip_d[0], args.pairs)
    out["scatter_probe"] = {**pr, "what": "uniform random byte stores, r per pair, into a buffer of the pool's size",
                            "ingest_frac_of_probe": (per_launch / avg_ingest_s) / (pr["mpps"] * 1e6)}
    out["slice_maintenance"] = maintenance(LINK, aip_d, bip_d, pool, args.pairs)
    pool.destroy()
    if mlp is not None:
        mlp.destroy()
    return out, tr, truth_h


def maintenance(params: dict, aip_d, bip_d, pool=None, pairs: int = 0, reps: int = 2) -> dict:
    """The paper's central claim on one geometry: ACE counters at their own
    width (every counter aged at every slice) against the asynchronous
    timestamps packed at theirs (one bit more; the lazy preserve examines 2 of
    2k blocks per ATV) and in bytes (the library's pool).  The slices go
    through all three `reps` times; every maintenance and scan step is timed
    with events on its own, over the passes after the first."""
    import torch

    from paper_1807_01527_amd.binding import AtCmp, AtPool
    stream = torch.cuda.current_stream()
    own = pool is None
    if own:
        pool = AtPool(**params, stream=stream)
    K, S = params["k"], len(aip_d)
    cmp_ace = AtCmp("ace", **params, stream=stream)
    cmp_at = AtCmp("at", **params, stream=stream)
    ev = {n: [] for n in ("ace_age", "ace_set", "at_pack_preserve", "at_pack_set", "at_byte_preserve",
                          "at_byte_scan")}

    def timed(name, fn):
        e0, e1 = (torch.cuda.Event(enable_timing=True) for _ in range(2))
        e0.record(stream)
        fn()
        e1.record(stream)
        ev[name].append((e0, e1))

    for rep in range(reps):
        for t in range(S):
            timed("ace_age", cmp_ace.open_slice)
            timed("ace_set", lambda: cmp_ace.ingest(aip_d[t], bip_d[t]))
            cmp_ace.close(K)
            timed("at_pack_preserve", cmp_at.open_slice)
            timed("at_pack_set", lambda: cmp_at.ingest(aip_d[t], bip_d[t]))
            cmp_at.close(K)
            timed("at_byte_preserve", lambda: pool.ingest(aip_d[t][:0], bip_d[t][:0], n=0))
            timed("at_byte_scan", lambda: pool.ingest(aip_d[t], bip_d[t]))
            pool.close(K)
    torch.cuda.synchronize()
    ms = {n: float(np.mean([a.elapsed_time(b) for a, b in v[S:]])) for n, v in ev.items()}
    same = bool(np.array_equal(cmp_ace.read_weights(), cmp_at.read_weights()))
    out = {
        "k": K, "ats": pool.n_atv * pool.g, "pairs_per_slice": pairs or int(aip_d[0].numel()),
        "ace": {"bits": cmp_ace.bits, "bytes": 4 * cmp_ace.n_words, "age_ms": ms["ace_age"],
                "set_ms": ms["ace_set"]},
        "at_packed": {"bits": cmp_at.bits, "bytes": 4 * cmp_at.n_words, "preserve_ms": ms["at_pack_preserve"],
                      "set_ms": ms["at_pack_set"]},
        "at_bytes": {"bits": 8 * pool.at_bytes, "bytes": pool.pool_bytes, "preserve_ms": ms["at_byte_preserve"],
                     "scan_ms": ms["at_byte_scan"]},
        "maintenance_ratio_packed": ms["ace_age"] / ms["at_pack_preserve"],
        "maintenance_ratio_bytes": ms["ace_age"] / ms["at_byte_preserve"],
        "same_weights": same,
        "note": f"event-timed single launches (launch gaps included; kernel times are in the rocprofv3 summary), "
                f"{S} slices after a first pass over them: ACE ages every counter at every slice, the timestamps "
                "preserve 2 of 2k blocks per ATV; the packed stores are 32-bit atomics (ACE one OR, a timestamp "
                "an AND and an OR), the byte pool scans through at_ingest_slice"}
    cmp_ace.destroy()
    cmp_at.destroy()
    if own:
        pool.destroy()
    return out


def maintenance_both(args, dev) -> dict:
    """maintenance() on the link geometry (its 10 slices of 5M pairs) and on
    the large one (link 0's 60 slices of 3.33M pairs)."""
    import torch

    from paper_1807_01527_amd import traffic
    from paper_1807_01527_amd import traffic_gpu as tg
    from paper_1807_01527_amd import learned
    tr = traffic.generate(traffic.config_link(seed=0, n_slices=args.slices, pairs_per_slice=args.pairs))
    a = [torch.from_numpy(x.view(np.int32)).to(dev) for x in tr.aip]
    b = [torch.from_numpy(x.view(np.int32)).to(dev) for x in tr.bip]
    out = {"link": maintenance(LINK, a, b)}
    del a, b
    la, lb, _ = tg.link_stream(0, LARGE_SLICES * LARGE_PAIRS, dev, **learned.LARGE_STREAM)
    P = LARGE_PAIRS
    a = [la[t * P:(t + 1) * P] for t in range(LARGE_SLICES)]
    b = [lb[t * P:(t + 1) * P] for t in range(LARGE_SLICES)]
    out["large"] = maintenance(dict(LARGE, seed=0), a, b)
    return out


def restore_lists(dev) -> dict:
    """Slice-close latency where the restore returns candidate lists: the small
    configuration's traffic in the (9, 7, 3, 4096) geometry at paper-like load
    (k = 4, a 2^26-AT pool), closes with restore and the candidates' estimates."""
    import torch

    from paper_1807_01527_amd import traffic
    from paper_1807_01527_amd.binding import AtPool
    tr = traffic.generate(traffic.config_small(seed=0))
    params = dict(k=4, r=4, c=9, s=7, u=3, log2g=12, theta=1024.0, seed=0)
    pool = AtPool(**params)
    aip_d = [torch.from_numpy(a.view(np.int32)).to(dev) for a in tr.aip]
    bip_d = [torch.from_numpy(b.view(np.int32)).to(dev) for b in tr.bip]
    lat, m_out, rcs = [], [], {}
    for rep in range(12):
        for t in range(tr.n_slices):
            pool.ingest(aip_d[t], bip_d[t])
            torch.cuda.synchronize()
            c0 = time.perf_counter()
            pool.close(4)
            rc, sip, est, fl, m = pool.restore(cap=1 << 20)
            el = 1e3 * (time.perf_counter() - c0)
            if rep >= 2:
                lat.append(el)
                m_out.append(m)
                rcs[str(rc)] = rcs.get(str(rc), 0) + 1
    pool.destroy()
    return {"workload": "small configuration traffic (4 x 250k pairs, 32 planted) in the (9,7,3,4096) geometry, k=4, "
                        "2^26-AT pool", "closes": len(lat), "restore_rc_counts": rcs,
            "candidates_mean": float(np.mean(m_out)),
            "slice_close_ms": {"p50": pct(lat, 50), "p99": pct(lat, 99), "max": max(lat),
                               "includes": "close + restore join and sort + estimates of every candidate, host "
                                           "wall clock, the slice's pairs already scanned"}}


def host_info() -> dict:
    model = None
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"nproc": os.cpu_count(), "affinity_cpus": len(os.sched_getaffinity(0)), "cpu_model": model}


def cpu_baseline_large(wl, budget_s: float = 20.0) -> dict:
    """The oracle as it stands, single-threaded and pinned to one host core,
    on the first slices of link 0 of the large configuration: eager preserve,
    scan, close and the estimates of the window's true super points, until
    about budget_s of work is done."""
    from oracle import oracle
    info = host_info()
    cpu = sorted(os.sched_getaffinity(0))[0]
    old = os.sched_getaffinity(0)
    os.sched_setaffinity(0, {cpu})
    try:
        w = wl[0]
        o = oracle.Oracle(**LARGE, seed=0, tuple_budget=1 << 24)
        hosts = np.ascontiguousarray(w["truth_h"])
        P = LARGE_PAIRS
        work, pairs, closes, n = 0.0, 0, [], 0
        while work <= budget_s and n < LARGE_SLICES:
            a = w["a"][n * P:(n + 1) * P].cpu().numpy().view(np.uint32)   # host copies: not oracle work
            b = w["b"][n * P:(n + 1) * P].cpu().numpy().view(np.uint32)
            s0 = time.perf_counter()
            o.ingest(a, b)
            c0 = time.perf_counter()
            o.close(LARGE["k"])
            o.tuple_count()
            o.estimate(hosts)
            c1 = time.perf_counter()
            closes.append(c1 - c0)
            work += c1 - s0
            pairs += a.size
            n += 1
        o.close_handle()
    finally:
        os.sched_setaffinity(0, old)
    return work, pairs, closes, n, info, cpu


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true", help="only the headline (large configuration)")
    ap.add_argument("--no-serve", action="store_true", help="skip the 16-link serving phase among the extras")
    ap.add_argument("--slices", type=int, default=10)
    ap.add_argument("--pairs", type=int, default=5_000_000)
    ap.add_argument("--link-steps", type=int, default=20)
    ap.add_argument("--link-warmup", type=int, default=3)
    ap.add_argument("--scatter-sweep", action="store_true",
                    help="only sweep the random byte-store probe over buffer sizes (1 MiB .. 1 GiB) and exit")
    ap.add_argument("--paper-scale", type=int, default=0, metavar="SLICES",
                    help="only run the k=300, 2^32-AT sliding shape over SLICES slices (3600 for 3300 windows) "
                         "and exit")
    ap.add_argument("--maintenance", action="store_true",
                    help="only the ACE / packed-timestamp / byte-timestamp comparison on the link and large geometries")
    ap.add_argument("--copy-probe", action="store_true",
                    help="also run a plain 256 MiB device copy (calibrates the HBM byte counters)")
    ap.add_argument("--copy-probe-only", action="store_true",
                    help="only the 256 MiB device copy, three times (the counters' calibration run)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark measures the path on one GPU; "
                                   "--gpus above 1 is not supported"}))
        sys.exit(2)
    args.warmup = max(1, args.warmup)  # the first pass fills the window: measured windows hold all 60 slices

    import torch

    if args.copy_probe_only:
        x = torch.empty(256 << 20, dtype=torch.uint8, device="cuda")
        y = torch.empty_like(x)
        for _ in range(3):
            y.copy_(x)
        torch.cuda.synchronize()
        print(json.dumps({"copy_probe_bytes": {"read": x.numel(), "write": y.numel(), "launches": 3}}), flush=True)
        return
    if args.scatter_sweep:
        scatter_sweep()
        return
    if args.paper_scale:
        print(json.dumps({"paper_scale": paper_scale(args.paper_scale)}), flush=True)
        return

    from paper_1807_01527_amd import learned
    from paper_1807_01527_amd.binding import Mlp

    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    if args.maintenance:
        print(json.dumps({"slice_maintenance": maintenance_both(args, dev)}), flush=True)
        return
    t0 = time.perf_counter()
    wl = large_workload(dev)
    torch.cuda.synchronize()
    log(f"large workload ready in {time.perf_counter() - t0:.1f}s: {LARGE_LINKS} x {LARGE_SLICES * LARGE_PAIRS} "
        f"pairs, {[w['truth_h'].size for w in wl]} true super points")
    wts = learned.load_weights("large")
    mlp = Mlp(wts) if wts is not None else None
    hl = headline(args, dev, wl, mlp)
    # the dominant kernel: the tiled scan launches of the served links (the
    # links of a step share one launch; each link's scan opens its slice and,
    # the slice's end queued with it, counts the window's weights)
    tl = hl["tiled"]
    launches = max(tl["launches"], 1)
    avg_ms = tl["device_ms"] / launches
    ppl = tl["pairs"] / launches
    jpl = tl["jobs"] / launches
    alg_pairs = (8 + LARGE["r"]) * ppl
    alg_count = jpl * (hl["pool_bytes"] + 4 * hl["n_atv"])
    achieved = (alg_pairs + alg_count) / (avg_ms / 1e3) / 1e9 if tl["launches"] else 0.0
    # the paced pass: each step's scans start with the GPU otherwise idle
    tp = hl["tiled_paced"]
    p_launch = max(tp["calls"], 1)
    p_ms = tp["device_ms"] / p_launch
    p_alg = (8 + LARGE["r"]) * tp["pairs"] / p_launch + tp["jobs"] / p_launch * (hl["pool_bytes"] + 4 * hl["n_atv"])
    p_achieved = p_alg / (p_ms / 1e3) / 1e9 if tp["calls"] else 0.0
    step_ms = hl["step_ms"]
    out = {
        "metric": "Mpps ingested + slice-close p99 ms; mean rel. error plain vs learned at θ=1024",
        "value": hl["value"],
        "unit": "Mpps",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * hl["elapsed"] / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u8",
        "data": "synthetic",
        "config": {"workload": LARGE_WORKLOAD, "links": LARGE_LINKS, "slices": LARGE_SLICES,
                   "pairs_per_slice": LARGE_PAIRS, "k": LARGE["k"], "pool_ats_per_link": hl["pool_bytes"],
                   "learned": mlp is not None, "parallelism": "single GPU"},
        "step_ms": {"min": min(step_ms), "median": float(np.median(step_ms)), "max": max(step_ms),
                    "all": [round(x, 3) for x in step_ms]},
        "slice_close_ms": hl["slice_close_ms"],
        "slice_close_ms_paced": hl["slice_close_ms_paced"],
        "restore_rc_counts": hl["restore_rc_counts"],
        "mean_rel_err": hl["mean_rel_err"],
        "roofline": {"kernel": "tiled scan launch of a step's served links (one grid row per link in every "
                               "pass): k_tile_count + k_tile_chunksum + k_tile_rowpre + k_tile_scatter + "
                               "k_tile_apply (stores grouped per 64 KiB tile and applied in LDS; the opening "
                               "preserve and the window count run in k_tile_apply)",
                     "bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": measured_traffic("ingest_large_pmc.json"),
                     "traffic_of": "the six kernels of one launch, rocprofv3 FETCH_SIZE + WRITE_SIZE, each scaled "
                                   "by its count for a plain device copy",
                     "bytes_per_pair": 8 + LARGE["r"],
                     "algorithmic_bytes_per_launch": {"pairs": alg_pairs, "window_count": alg_count},
                     "avg_launch_ms": avg_ms, "pairs_per_launch": ppl, "links_per_launch": jpl,
                     "launches_timed": tl["launches"], "steps_planned_ahead": tl["planned_ahead"],
                     "timing": "HIP events around each launch's two halves (record passes on their own stream, "
                               "beside the previous step's close graph; the tile pass behind that graph), summed",
                     "uncontended": {"avg_launch_ms": p_ms, "achieved": p_achieved, "frac": p_achieved / HBM_PEAK_GBS,
                                     "launches": tp["calls"], "links_per_launch": tp["jobs"] / p_launch,
                                     "what": "the paced pass's launches: a slice per link every 2 ms, so no step "
                                             "is queued ahead and each launch has the GPU to itself"}},
        "tiled_share_of_pairs": tl["pairs"] / hl["pairs"] if hl["pairs"] else None,
    }
    # random-store roofline at the headline's total pool size (1 GiB) and at one pool
    a0 = wl[0]["a"][:LARGE_PAIRS // 4 * 4]
    b0 = wl[0]["b"][:LARGE_PAIRS // 4 * 4]
    pr_all = probe_rate(dev, LARGE_LINKS * hl["pool_bytes"], a0, b0, LARGE_PAIRS // 4 * 4)
    pr_one = probe_rate(dev, hl["pool_bytes"], a0, b0, LARGE_PAIRS // 4 * 4)
    scan_mpps = ppl / (avg_ms / 1e3) / 1e6 if tl["launches"] else None
    out["scatter_probe"] = {"what": "uniform random byte stores, 4 per pair of link 0's first slice",
                            "all_pools_1GiB": pr_all, "one_pool_256MiB": pr_one,
                            "tiled_scan_mpps": scan_mpps,
                            "tiled_scan_over_probe_at_1GiB": scan_mpps / pr_all["mpps"] if scan_mpps else None}
    if not args.no_extras:
        log("realistic-link configuration ...")
        link, tr, truth_h = link_config2(args, dev, learned, Mlp)
        out["link_config"] = link
        if not args.no_serve:
            log("streaming-server phase (16 links) ...")
            out["serving_16_links"] = serve_phase(dev)
        log("restore-list latency ...")
        out["restore_lists"] = restore_lists(dev)
    if args.copy_probe:
        x = torch.empty(256 << 20, dtype=torch.uint8, device=dev)
        y = torch.empty_like(x)
        for _ in range(3):
            y.copy_(x)
        torch.cuda.synchronize()
        out["copy_probe_bytes"] = {"read": x.numel(), "write": y.numel(), "launches": 3}
        del x, y
    if not args.no_cpu_baseline:
        log("timing the oracle on one host core ...")
        el, pairs, closes, n, info, cpu = cpu_baseline_large(wl)
        out["cpu_baseline"] = {"value": pairs / el / 1e6, "unit": "Mpps", "cores": 1, "kind": "oracle",
                               "sample": f"the first {n} slices of link 0 of the large configuration ({pairs} "
                                         f"pairs): eager preserve + scan + close + estimates of its "
                                         f"{wl[0]['truth_h'].size} true super points, single thread pinned to "
                                         f"CPU {cpu}",
                               "slice_close_ms_mean": 1e3 * float(np.mean(closes)), "seconds": el, **info}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
