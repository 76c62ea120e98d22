"""Seeded synthetic (aip, bip) traffic for the sliding-window super-point workloads.

This module produces *inputs only*: packet pairs per time slice and the exact
per-host distinct counts of a window (the plain definition of cardinality,
Section 2.2, used as ground truth).  It holds none of the estimation method's
arithmetic (no mangling, no column extraction, no timestamps), so both the HIP
path and the CPU oracle may consume what it produces.

Randomness is counter based: value(stream, i) = mix64(key(stream) + (i+1)*G),
with mix64 the SplitMix64 finaliser (Steele, Lea, Flood, "Fast splittable
pseudorandom number generators", OOPSLA 2014) and G = 0x9E3779B97F4A7C15.
Host addresses are a seeded bijective 32-bit mix of a host rank (the MurmurHash3
fmix32 finaliser, which is a bijection of 32-bit words), so distinct ranks give
distinct addresses, and planted hosts (ranks above the background range) never
collide with background hosts.

The paper measured on CAIDA backbone traces that are not available here; these
generators stand in for them with the shapes of the benchmark configurations
(Zipf host popularity, uniform opposite hosts, planted super points with stated
cardinality laws, optional repeat pairs).
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional, Sequence, Tuple

import numpy as np

_G = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)


def _mix64(z: np.ndarray) -> np.ndarray:
    z = z.astype(np.uint64, copy=True)
    with np.errstate(over="ignore"):
        z ^= z >> np.uint64(30)
        z *= _M1
        z ^= z >> np.uint64(27)
        z *= _M2
        z ^= z >> np.uint64(31)
    return z


def stream_key(seed: int, stream: int) -> np.uint64:
    """Key of an independent substream (seed, stream)."""
    s = np.array([(seed * 0x100000001B3 + stream * 0xD1B54A32D192ED03) & 0xFFFFFFFFFFFFFFFF],
                 dtype=np.uint64)
    return _mix64(s)[0]


def rand_u64(seed: int, stream: int, start: int, n: int) -> np.ndarray:
    """n raw 64-bit values at counters [start, start+n) of substream (seed, stream)."""
    key = stream_key(seed, stream)
    ctr = np.arange(start + 1, start + n + 1, dtype=np.uint64)
    with np.errstate(over="ignore"):
        return _mix64(key + ctr * _G)


def rand_u32(seed: int, stream: int, start: int, n: int) -> np.ndarray:
    return (rand_u64(seed, stream, start, n) >> np.uint64(32)).astype(np.uint32)


def rand_unit(seed: int, stream: int, start: int, n: int) -> np.ndarray:
    """Uniform doubles in [0,1) with 53 random bits."""
    return (rand_u64(seed, stream, start, n) >> np.uint64(11)).astype(np.float64) * (2.0 ** -53)


def fmix32(x: np.ndarray) -> np.ndarray:
    """MurmurHash3 32-bit finaliser: a bijection on 32-bit words."""
    x = np.asarray(x, dtype=np.uint32).copy()
    with np.errstate(over="ignore"):
        x ^= x >> np.uint32(16)
        x *= np.uint32(0x85EBCA6B)
        x ^= x >> np.uint32(13)
        x *= np.uint32(0xC2B2AE35)
        x ^= x >> np.uint32(16)
    return x


def host_address(rank: np.ndarray, seed: int) -> np.ndarray:
    """Address of host `rank` (distinct ranks -> distinct addresses)."""
    key = np.uint32(int(rand_u32(seed, 0xA11CE, 0, 1)[0]))
    return fmix32(np.asarray(rank, dtype=np.uint32) ^ key)


@dataclasses.dataclass
class TraceConfig:
    """Shape of a synthetic trace.

    pairs_per_slice: total pairs in each slice (background + planted + repeats).
    hosts / zipf_s: background aip popularity, Zipf(s) over `hosts` ranks.
    bip_space: None -> uniform 32-bit opposite hosts; else uniform over a fixed
      set of that many distinct values.
    planted: number of planted hosts; their cardinalities follow `planted_law`
      ("uniform" integer U[lo,hi] or "loguniform" over [lo,hi]); each planted
      host's distinct opposite hosts are split evenly over the slices
      (remainder to the earliest slices) and each appears once.
    repeat_frac: fraction of each slice's pairs that re-emit a uniformly chosen
      earlier (fresh) pair of the same slice.
    """
    name: str
    n_slices: int
    pairs_per_slice: int
    hosts: int
    zipf_s: float
    bip_space: Optional[int] = None
    planted: int = 0
    planted_lo: int = 1024
    planted_hi: int = 8000
    planted_law: str = "uniform"
    repeat_frac: float = 0.0
    seed: int = 0

    @property
    def total_pairs(self) -> int:
        return self.n_slices * self.pairs_per_slice


@dataclasses.dataclass
class Trace:
    cfg: TraceConfig
    aip: List[np.ndarray]          # per slice, uint32
    bip: List[np.ndarray]          # per slice, uint32
    planted_hosts: np.ndarray      # uint32 addresses
    planted_card: np.ndarray       # int64 cardinalities over the whole trace

    @property
    def n_slices(self) -> int:
        return len(self.aip)


def planted_cardinalities(cfg: TraceConfig) -> np.ndarray:
    u = rand_unit(cfg.seed, 0xCA4D, 0, cfg.planted)
    if cfg.planted_law == "uniform":
        n = cfg.planted_lo + np.floor(u * (cfg.planted_hi - cfg.planted_lo + 1))
    elif cfg.planted_law == "loguniform":
        lo, hi = math.log(cfg.planted_lo), math.log(cfg.planted_hi)
        n = np.floor(np.exp(lo + u * (hi - lo)))
    else:
        raise ValueError(cfg.planted_law)
    return np.clip(n, cfg.planted_lo, cfg.planted_hi).astype(np.int64)


_ZIPF_CACHE: dict = {}


def _zipf_cdf(hosts: int, s: float) -> np.ndarray:
    key = (hosts, s)
    if key not in _ZIPF_CACHE:
        w = np.arange(1, hosts + 1, dtype=np.float64) ** (-s)
        c = np.cumsum(w)
        c /= c[-1]
        _ZIPF_CACHE.clear()
        _ZIPF_CACHE[key] = c
    return _ZIPF_CACHE[key]


def zipf_ranks(hosts: int, s: float, u: np.ndarray) -> np.ndarray:
    """Ranks 1..hosts by inverse CDF of Zipf(s) at uniforms u."""
    cdf = _zipf_cdf(hosts, s)
    r = np.searchsorted(cdf, u, side="right") + 1
    return np.minimum(r, hosts).astype(np.uint32)


def _shuffle(a: np.ndarray, b: np.ndarray, seed: int, stream: int) -> Tuple[np.ndarray, np.ndarray]:
    perm = np.argsort(rand_u64(seed, stream, 0, a.size), kind="stable")
    return a[perm], b[perm]


def generate(cfg: TraceConfig) -> Trace:
    S = cfg.n_slices
    card = planted_cardinalities(cfg) if cfg.planted else np.zeros(0, np.int64)
    p_ranks = np.arange(cfg.hosts + 1, cfg.hosts + 1 + cfg.planted, dtype=np.uint32)
    p_addr = host_address(p_ranks, cfg.seed)
    p_keys = rand_u32(cfg.seed, 0xB1B, 0, cfg.planted)
    bip_key = np.uint32(int(rand_u32(cfg.seed, 0xB1C, 0, 1)[0]))
    base = card // S
    rem = card % S
    aips, bips = [], []
    n_rep = int(round(cfg.repeat_frac * cfg.pairs_per_slice))
    for t in range(S):
        cnt = base + (t < rem)
        start = base * t + np.minimum(t, rem)
        tot_planted = int(cnt.sum())
        n_bg = cfg.pairs_per_slice - tot_planted - n_rep
        if n_bg < 0:
            raise ValueError(f"{cfg.name}: planted+repeat pairs exceed the slice size")
        # planted pairs: host h uses counters [start_h, start_h+cnt_h) of its own bijection
        pa = np.repeat(p_addr, cnt)
        offs = np.arange(tot_planted, dtype=np.int64) - np.repeat(np.cumsum(cnt) - cnt, cnt)
        ctr = (np.repeat(start, cnt) + offs).astype(np.uint32)
        pb = fmix32(ctr ^ np.repeat(p_keys, cnt))
        # background pairs
        st = 0x100 + 4 * t
        ranks = zipf_ranks(cfg.hosts, cfg.zipf_s, rand_unit(cfg.seed, st, 0, n_bg))
        ba = host_address(ranks, cfg.seed)
        if cfg.bip_space is None:
            bb = rand_u32(cfg.seed, st + 1, 0, n_bg)
        else:
            idx = (rand_u64(cfg.seed, st + 1, 0, n_bg) % np.uint64(cfg.bip_space)).astype(np.uint32)
            bb = fmix32(idx ^ bip_key)
        fa = np.concatenate([pa, ba]).astype(np.uint32)
        fb = np.concatenate([pb, bb]).astype(np.uint32)
        if n_rep:
            pick = (rand_u64(cfg.seed, st + 2, 0, n_rep) % np.uint64(fa.size)).astype(np.int64)
            fa = np.concatenate([fa, fa[pick]])
            fb = np.concatenate([fb, fb[pick]])
        fa, fb = _shuffle(fa, fb, cfg.seed, st + 3)
        aips.append(np.ascontiguousarray(fa))
        bips.append(np.ascontiguousarray(fb))
    return Trace(cfg, aips, bips, p_addr.astype(np.uint32), card)


def window_counts(aip_slices: Sequence[np.ndarray], bip_slices: Sequence[np.ndarray],
                  min_count: int = 1) -> Tuple[np.ndarray, np.ndarray]:
    """Exact distinct-bip count per aip over the union of the given slices.

    Returns (hosts ascending, counts) restricted to counts >= min_count.  This is
    the plain definition of a host's cardinality in a window (Section 2.2)."""
    if len(aip_slices) == 0:
        return np.zeros(0, np.uint32), np.zeros(0, np.int64)
    a = np.concatenate([np.asarray(x, np.uint64) for x in aip_slices])
    b = np.concatenate([np.asarray(x, np.uint64) for x in bip_slices])
    keys = np.unique((a << np.uint64(32)) | b)
    hosts = (keys >> np.uint64(32)).astype(np.uint32)
    h, c = np.unique(hosts, return_counts=True)
    keep = c >= min_count
    return h[keep], c[keep].astype(np.int64)


# ---------------------------------------------------------------------------
# Benchmark workload shapes (sizes from the configurations the path is quoted on)
# ---------------------------------------------------------------------------

def config_small(seed: int = 0) -> TraceConfig:
    """1M pairs in 4 slices of 250k, Zipf 1.1 over 2^16 hosts, uniform 32-bit
    bips, 32 planted hosts with U[1500,8000] distinct bips."""
    return TraceConfig("small", 4, 250_000, 1 << 16, 1.1, None, 32, 1500, 8000, "uniform", 0.0, seed)


def config_link(seed: int = 0, n_slices: int = 10, pairs_per_slice: int = 5_000_000,
                planted: int = 371) -> TraceConfig:
    """Realistic link: 10 slices of 5M pairs, Zipf 1.2 over 2^22 hosts, bips from a
    fixed set of 2^26 values, 30% repeat pairs, planted hosts log-uniform over
    [1024, 2^18] (count capped so planted pairs stay within half the distinct-pair
    budget)."""
    return TraceConfig("link", n_slices, pairs_per_slice, 1 << 22, 1.2, 1 << 26, planted,
                       1024, 1 << 18, "loguniform", 0.30, seed)


def config_large(seed: int = 0, n_slices: int = 60, pairs_per_slice: int = 3_333_333,
                 planted: int = 661) -> TraceConfig:
    return TraceConfig("large", n_slices, pairs_per_slice, 1 << 24, 1.1, None, planted,
                       1024, 1 << 20, "loguniform", 0.0, seed)


def config_tiny(seed: int = 0, n_slices: int = 6, pairs_per_slice: int = 20_000,
                hosts: int = 1 << 12, planted: int = 4, lo: int = 300, hi: int = 2000) -> TraceConfig:
    """Small traces for parity tests."""
    return TraceConfig("tiny", n_slices, pairs_per_slice, hosts, 1.1, None, planted, lo, hi,
                       "uniform", 0.1, seed)
