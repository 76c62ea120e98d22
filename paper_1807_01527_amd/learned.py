"""Learned correction of the plain estimate: training set, training and evaluation.

Everything on the path runs in the HIP library:
- the traces are ingested by at_ingest_slice / at_close_slice;
- the features come from at_features;
- training gathers its batches and targets with at_mlp_gather_batch and runs
  at_mlp_train_step (bf16 matrix-core forward/backward + Adam);
- inference runs at_estimate_learned.

This module only orchestrates.  Labels are the exact distinct counts of the
synthetic traces.

    python -m paper_1807_01527_amd.learned --geom small --samples 1000000 --out weights/small.npy
    python -m paper_1807_01527_amd.learned --geom large --samples 500000 --eval-seeds 4 --out weights/large.npy
"""
from __future__ import annotations

import argparse
import dataclasses
import math
import os
import sys
import time
from typing import Dict, Optional

import numpy as np

from . import traffic
from .binding import MLP_NPARAM, AtPool, Mlp

GEOMS = {
    # the small configuration's literal pool: 2^20 ATs, k = 4
    "small": dict(k=4, r=4, c=9, s=8, u=0, log2g=9, theta=1024.0),
    # the realistic link's pool: 2^26 ATs, k = 10
    "link": dict(k=10, r=4, c=9, s=7, u=3, log2g=12, theta=1024.0),
    # the serving links' pools: 2^24 ATs, k from {5, 10, 30} (one network for all)
    "serve": dict(k=30, r=4, c=9, s=8, u=1, log2g=12, theta=1024.0),
}
KS = {"serve": (5, 10, 30)}

# Traffic-shaped training sets: whole traces of a configuration's own traffic
# law through its own geometry (one window per trace), sampled over the
# label range.  "large": the large configuration, 60 slices of 3,333,333
# pairs, k = 60, a 2^28-AT pool, aip Zipf 1.1 over 2^24 hosts, 661 planted
# hosts log-uniform over [1024, 2^20].  "serve_mix": the serving links' pools
# (2^24 ATs) with k from {5, 10, 30}, lognormal slices (median 2M, sigma 1,
# clipped to [100k, 20M]) of small-configuration content.
STREAM_GEOMS = {
    "large": dict(k=60, r=4, c=10, s=6, u=4, log2g=12, theta=1024.0),
    "serve_mix": dict(k=30, r=4, c=9, s=8, u=1, log2g=12, theta=1024.0),
}
LARGE_STREAM = dict(hosts=1 << 24, zipf_s=1.1, planted=661, lo=1024, hi=1 << 20, card_dist="loguniform")
LARGE_SLICES, LARGE_PAIRS = 60, 3_333_333


def stream_trace(name: str, seed: int, dev):
    """One trace of a traffic-shaped family: (k, per-slice (aip, bip) device
    views, aip and bip of the whole window as device tensors)."""
    from . import traffic_gpu as tg
    if name == "large":
        n = LARGE_SLICES * LARGE_PAIRS
        a, b, _ = tg.link_stream(seed, n, dev, **LARGE_STREAM)
        bounds = [t * LARGE_PAIRS for t in range(LARGE_SLICES + 1)]
        k = STREAM_GEOMS[name]["k"]
    else:
        k = (5, 10, 30)[seed % 3]
        rng = np.random.default_rng(seed)
        sizes = np.clip(np.exp(np.log(2e6) + rng.standard_normal(k)), 1e5, 2e7).astype(np.int64)
        bounds = np.concatenate([[0], np.cumsum(sizes)]).tolist()
        a, b, _ = tg.link_stream(seed, int(bounds[-1]), dev)
    slices = [(a[lo:hi], b[lo:hi]) for lo, hi in zip(bounds[:-1], bounds[1:])]
    return k, slices, a, b


def exact_counts(a, b):
    """Exact distinct bips per aip over the given pairs (device tensors of
    int32 holding 32-bit words): (hosts uint32, counts int64) on the host."""
    import torch
    from .traffic_gpu import _srl
    keys = torch.unique(((a.to(torch.int64) & 0xFFFFFFFF) << 32) | (b.to(torch.int64) & 0xFFFFFFFF))
    hosts, counts = torch.unique(_srl(keys, 32), return_counts=True)
    return hosts.cpu().numpy().astype(np.uint32), counts.cpu().numpy().astype(np.int64)


def build_dataset_stream(name: str, n_samples: int, seed: int = 1, log=print, per_trace: int = 40000):
    """(features, ln n) from whole traces of the family `name`: every host of
    the window with at least theta distinct bips, and as many hosts with 16 to
    theta - 1 sampled uniformly, until n_samples are collected.  Trace seeds
    start at 1000 * seed + 100, away from the evaluation seeds."""
    import torch
    geom = STREAM_GEOMS[name]
    dev = torch.device("cuda", torch.cuda.current_device())
    X, T = [], []
    have, tr = 0, 0
    t0 = time.perf_counter()
    while have < n_samples:
        ts = 1000 * seed + 100 + tr
        k, slices, a, b = stream_trace(name, ts, dev)
        pool = AtPool(**{**geom, "k": k}, seed=ts)
        for sa, sb in slices:
            pool.ingest(sa, sb)
            pool.close(k)
        hosts, counts = exact_counts(a, b)
        big = np.nonzero(counts >= geom["theta"])[0]
        small = np.nonzero((counts >= 16) & (counts < geom["theta"]))[0]
        rng = np.random.default_rng(ts)
        take = min(small.size, big.size)
        sel = np.concatenate([big, rng.choice(small, take, replace=False)])[:per_trace]
        hd = torch.from_numpy(hosts[sel].view(np.int32)).to(dev)
        feat = torch.empty((sel.size, 64), dtype=torch.float32, device=dev)
        pool.features(hd, feat)
        X.append(feat)
        T.append(torch.from_numpy(np.log(counts[sel].astype(np.float64)).astype(np.float32)).to(dev))
        have += sel.size
        pool.destroy()
        del a, b, slices
        tr += 1
        log(f"  dataset {name}: {tr} traces, {have} samples, {time.perf_counter() - t0:.1f}s")
    torch.cuda.synchronize()
    return torch.cat(X)[:n_samples].contiguous(), torch.cat(T)[:n_samples].contiguous()


def evaluate_stream(name: str, mlp: Optional[Mlp], seeds=range(2)) -> Dict[str, float]:
    """Mean relative error of the plain and learned estimates over the true
    super points (exact count >= theta) of whole traces of the family, at
    the seeds given (the large configuration's own links are seeds 0-3)."""
    import torch
    geom = STREAM_GEOMS[name]
    dev = torch.device("cuda", torch.cuda.current_device())
    rel_p, rel_l, fb = [], [], 0
    for sd in seeds:
        k, slices, a, b = stream_trace(name, sd, dev)
        pool = AtPool(**{**geom, "k": k}, seed=sd)
        for sa, sb in slices:
            pool.ingest(sa, sb)
            pool.close(k)
        hosts, counts = exact_counts(a, b)
        m = counts >= geom["theta"]
        h, n = hosts[m], counts[m]
        if mlp is not None:
            est_l, fl, plain = pool.estimate_learned(mlp, h)
            rel_l.append(np.abs(est_l - n) / n)
            fb += int(np.count_nonzero(fl & 4))
        else:
            plain, _ = pool.estimate_plain(h)
        rel_p.append(np.abs(plain - n) / n)
        pool.destroy()
    out = {"plain": float(np.mean(np.concatenate(rel_p))), "hosts": int(sum(x.size for x in rel_p))}
    if mlp is not None:
        out["learned"] = float(np.mean(np.concatenate(rel_l)))
        out["fallbacks"] = fb
    return out


WEIGHTS_DIR = os.path.join(os.path.dirname(os.path.abspath(__file__)), "weights")


def pool_ats(geom: dict) -> int:
    return (1 << (geom["c"] + geom["u"])) * geom["r"] * (1 << geom["log2g"])


def trace_shape(name: str):
    from .traffic_gpu import TraceShape
    g = GEOMS[name]
    if name == "small":
        return TraceShape(slices=g["k"], pool_ats=pool_ats(g), rows=g["r"], hosts=1 << 16, zipf_s=1.1)
    if name == "serve":
        return TraceShape(slices=g["k"], pool_ats=pool_ats(g), rows=g["r"], hosts=1 << 16, zipf_s=1.1,
                          max_planted=200, bg_samples=400)
    return TraceShape(slices=g["k"], pool_ats=pool_ats(g), rows=g["r"], hosts=1 << 22, zipf_s=1.2,
                      lam_lo=0.3, lam_hi=3.0, max_planted=400, bg_samples=3000, hi=1 << 18)


def init_params(seed: int) -> np.ndarray:
    """He-uniform weights, zero biases; a small output layer so the network
    starts near the plain estimate."""
    rng = np.random.default_rng(seed)
    lim = math.sqrt(6.0 / 64)
    W1 = rng.uniform(-lim, lim, (64, 64))
    W2 = rng.uniform(-lim, lim, (64, 64))
    w3 = rng.uniform(-lim, lim, 64) * 0.1
    return np.concatenate([W1.ravel(), np.zeros(64), W2.ravel(), np.zeros(64), w3, [0.0]]).astype(np.float32)


def build_dataset(name: str, n_samples: int, seed: int = 1, log=print):
    """(features [N, 64] float32, ln n [N] float32) as device tensors."""
    import torch
    from .traffic_gpu import make_trace
    geom = GEOMS[name]
    shape = trace_shape(name)
    dev = torch.device("cuda", torch.cuda.current_device())
    X, T = [], []
    have = 0
    trace = 0
    t0 = time.perf_counter()
    while have < n_samples:
        k = KS[name][trace % len(KS[name])] if name in KS else geom["k"]
        aips, bips, hosts, counts = make_trace(dataclasses.replace(shape, slices=k), seed, trace, dev)
        pool = AtPool(**{**geom, "k": k}, seed=seed * 100003 + trace)
        for t in range(k):
            if aips[t].numel():
                pool.ingest(aips[t], bips[t])
            pool.close(k)
        if hosts.size:
            hd = torch.from_numpy(hosts.view(np.int32)).to(dev)
            feat = torch.empty((hosts.size, 64), dtype=torch.float32, device=dev)
            pool.features(hd, feat)
            X.append(feat)
            T.append(torch.from_numpy(np.log(counts.astype(np.float64)).astype(np.float32)).to(dev))
            have += hosts.size
        pool.destroy()
        trace += 1
        if trace % 200 == 0:
            log(f"  dataset {name}: {trace} traces, {have} samples, {time.perf_counter() - t0:.1f}s")
    torch.cuda.synchronize()
    return torch.cat(X)[:n_samples].contiguous(), torch.cat(T)[:n_samples].contiguous()


def train(mlp: Mlp, X, T, epochs: int = 40, batch: int = 4096, lr: float = 2e-3, seed: int = 0, log=print):
    """T holds ln n; the network is fit to its residual over 16*f[61].  The
    batch order is a seeded permutation drawn on the host; the library
    gathers each batch and its targets on the device."""
    import torch
    n = X.shape[0]
    g = torch.Generator(device="cpu").manual_seed(seed)
    xb = torch.empty((batch, 64), dtype=torch.float32, device=X.device)
    tb = torch.empty(batch, dtype=torch.float32, device=X.device)
    losses = []
    for ep in range(epochs):
        perm = torch.randperm(n, generator=g).to(X.device)
        lr_ep = lr * (0.5 * (1 + math.cos(math.pi * ep / epochs)) * 0.95 + 0.05)
        tot, cnt = 0.0, 0
        for s in range(0, n - batch + 1, batch):
            mlp.gather_batch(X, T, perm[s:s + batch], xb, tb)
            want = (s // batch) % 50 == 0
            loss = mlp.train_step(xb, tb, lr_ep, want_loss=want)
            if want:
                tot += loss
                cnt += 1
        losses.append(tot / max(cnt, 1))
        log(f"  epoch {ep + 1}/{epochs}: loss {losses[-1]:.5f} (lr {lr_ep:.2e})")
    return losses


def evaluate(name: str, mlp: Optional[Mlp], seeds=range(10)) -> Dict[str, float]:
    """Mean relative error over the true super points (exact count >= theta
    in the window) of the plain and the learned estimates, on traces of the
    configuration's own traffic shape."""
    import torch
    geom = GEOMS[name]
    dev = torch.device("cuda", torch.cuda.current_device())
    rel_p, rel_l, fb = [], [], 0
    for sd in seeds:
        k = KS[name][sd % len(KS[name])] if name in KS else geom["k"]
        if name == "small":
            tr = traffic.generate(traffic.config_small(seed=sd))
        elif name == "serve":
            cfg = traffic.config_small(seed=sd)
            cfg.n_slices, cfg.pairs_per_slice = k, 1_000_000 // k * 4 // 4
            tr = traffic.generate(cfg)
        else:
            tr = traffic.generate(traffic.config_link(seed=sd))
        pool = AtPool(**{**geom, "k": k}, seed=sd)
        for t in range(tr.n_slices):
            pool.ingest(torch.from_numpy(tr.aip[t].view(np.int32)).to(dev),
                        torch.from_numpy(tr.bip[t].view(np.int32)).to(dev))
            pool.close(k)
        lo = max(0, tr.n_slices - k)
        h, n = traffic.window_counts(tr.aip[lo:], tr.bip[lo:], min_count=int(geom["theta"]))
        if mlp is not None:
            est_l, fl, plain = pool.estimate_learned(mlp, h)
            rel_l.append(np.abs(est_l - n) / n)
            fb += int(np.count_nonzero(fl & 4))
        else:
            plain, _ = pool.estimate_plain(h)
        rel_p.append(np.abs(plain - n) / n)
        pool.destroy()
    out = {"plain": float(np.mean(np.concatenate(rel_p))), "hosts": int(sum(x.size for x in rel_p))}
    if mlp is not None:
        out["learned"] = float(np.mean(np.concatenate(rel_l)))
        out["fallbacks"] = fb
    return out


def load_weights(name: str) -> Optional[np.ndarray]:
    path = os.path.join(WEIGHTS_DIR, f"{name}.npy")
    if not os.path.exists(path):
        return None
    p = np.load(path, allow_pickle=False).astype(np.float32)
    return p if p.size == MLP_NPARAM else None


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--geom", choices=sorted(GEOMS) + sorted(STREAM_GEOMS), default="small")
    ap.add_argument("--samples", type=int, default=1_000_000)
    ap.add_argument("--epochs", type=int, default=40)
    ap.add_argument("--seed", type=int, default=1)
    ap.add_argument("--eval-seeds", type=int, default=10)
    ap.add_argument("--out", default=None)
    args = ap.parse_args(argv)
    import torch
    torch.cuda.set_device(0)
    log = lambda m: print(m, flush=True)  # noqa: E731
    t0 = time.perf_counter()
    stream = args.geom in STREAM_GEOMS
    if stream:
        X, T = build_dataset_stream(args.geom, args.samples, seed=args.seed, log=log)
    else:
        X, T = build_dataset(args.geom, args.samples, seed=args.seed, log=log)
    log(f"dataset: {X.shape[0]} samples in {time.perf_counter() - t0:.1f}s")
    mlp = Mlp(init_params(args.seed))
    t1 = time.perf_counter()
    train(mlp, X, T, epochs=args.epochs, log=log)
    torch.cuda.synchronize()
    log(f"training: {time.perf_counter() - t1:.1f}s")
    if args.out:
        os.makedirs(os.path.dirname(os.path.abspath(args.out)), exist_ok=True)
        np.save(args.out, mlp.get_params())
    if stream:
        res = evaluate_stream(args.geom, mlp, seeds=range(args.eval_seeds))
    else:
        res = evaluate(args.geom, mlp, seeds=range(args.eval_seeds))
    log(f"evaluation ({args.geom} traffic, seeds 0..{args.eval_seeds - 1}): {res}")
    return res


if __name__ == "__main__":
    sys.exit(0 if main() else 1)
