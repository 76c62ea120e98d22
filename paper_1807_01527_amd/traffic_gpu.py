"""Seeded synthetic traces generated on the GPU (torch), for the learned
correction's training and evaluation sets.

Inputs only, like `traffic`: counter-based randomness (the SplitMix64
finaliser over (seed, stream, index), computed with int64 tensor arithmetic),
host addresses from the fmix32 bijection of a rank, Zipf background by
inverse CDF, planted hosts with distinct opposite hosts, and exact per-host
distinct counts (the plain definition of cardinality).  None of the
estimation method's arithmetic lives here.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Tuple

import numpy as np
import torch

_M64 = (1 << 64) - 1


def _s64(v: int) -> int:
    v &= _M64
    return v - (1 << 64) if v >= (1 << 63) else v


_G = _s64(0x9E3779B97F4A7C15)
_M1 = _s64(0xBF58476D1CE4E5B9)
_M2 = _s64(0x94D049BB133111EB)


def _srl(z: torch.Tensor, s: int) -> torch.Tensor:
    """Logical right shift of int64 lanes holding 64-bit words."""
    return (z >> s) & ((1 << (64 - s)) - 1)


def mix64(z: torch.Tensor) -> torch.Tensor:
    z = (z ^ _srl(z, 30)) * _M1
    z = (z ^ _srl(z, 27)) * _M2
    return z ^ _srl(z, 31)


def _key(seed: int, stream: int) -> int:
    v = (seed * 0x100000001B3 + stream * 0xD1B54A32D192ED03) & _M64
    z = torch.tensor([_s64(v)], dtype=torch.int64)
    return int(mix64(z)[0])


def rand_u64(seed: int, stream: int, n: int, device) -> torch.Tensor:
    ctr = torch.arange(1, n + 1, dtype=torch.int64, device=device)
    return mix64(ctr * _G + _key(seed, stream))


def rand_unit(seed: int, stream: int, n: int, device) -> torch.Tensor:
    return _srl(rand_u64(seed, stream, n, device), 11).to(torch.float64) * (2.0 ** -53)


def rand_u32(seed: int, stream: int, n: int, device) -> torch.Tensor:
    return _srl(rand_u64(seed, stream, n, device), 32)


def fmix32(x: torch.Tensor) -> torch.Tensor:
    """MurmurHash3 fmix32 on int64 lanes holding 32-bit words (a bijection)."""
    m = 0xFFFFFFFF
    x = x & m
    x = x ^ (x >> 16)
    x = (x * 0x85EBCA6B) & m
    x = x ^ (x >> 13)
    x = (x * 0xC2B2AE35) & m
    return x ^ (x >> 16)


def as_u32_device(x: torch.Tensor) -> torch.Tensor:
    """int64 lanes holding 32-bit words -> contiguous int32 tensor with the same bits."""
    return (x & 0xFFFFFFFF).to(torch.int64).sub_((x & 0x80000000) << 1).to(torch.int32).contiguous()


@dataclasses.dataclass
class TraceShape:
    """A family of training traces.  Each trace has `slices` slices; its
    distinct-pair count D is set from a row load drawn uniformly in
    [lam_lo, lam_hi] (lambda = r*D/P for a pool of P ATs and r rows); planted
    hosts with log-uniform cardinality in [lo, hi] take up to `planted_share`
    of D, the rest is Zipf(zipf_s) background over `hosts` ranks."""
    slices: int
    pool_ats: int
    rows: int
    hosts: int = 1 << 16
    zipf_s: float = 1.1
    lam_lo: float = 0.05
    lam_hi: float = 4.0
    lo: int = 16
    hi: int = 1 << 18
    max_planted: int = 48
    planted_share: float = 0.6
    bg_samples: int = 24
    min_count: int = 16


_CDF = {}


def _zipf_cdf(hosts: int, s: float, device) -> torch.Tensor:
    """Zipf(s) CDF over ranks 1..hosts.  The prefix sums run on the host in
    rank order: a device scan may associate its float additions differently
    from run to run, and a last-bit change moves the rank a uniform draw maps
    to, so a trace would no longer be the same in every process."""
    key = (hosts, s, str(device))
    if key not in _CDF:
        c = np.cumsum(np.arange(1, hosts + 1, dtype=np.float64) ** -s)
        _CDF.clear()
        _CDF[key] = torch.from_numpy(c / c[-1]).to(device)
    return _CDF[key]


def make_trace(shape: TraceShape, seed: int, trace: int, device) -> Tuple[List[torch.Tensor], List[torch.Tensor],
                                                                           np.ndarray, np.ndarray]:
    """One trace: per-slice (aip, bip) int32 device tensors, plus the sample
    hosts (uint32) and their exact distinct counts over the whole trace."""
    base = 0x7000 + 64 * trace
    u = rand_unit(seed, base, 2, device).cpu().numpy()
    lam = shape.lam_lo + u[0] * (shape.lam_hi - shape.lam_lo)
    D = int(lam * shape.pool_ats / shape.rows)
    # planted cardinalities, log-uniform, until the planted share is reached
    lu = rand_unit(seed, base + 1, shape.max_planted, device).cpu().numpy()
    card = np.floor(np.exp(math.log(shape.lo) + lu * (math.log(shape.hi) - math.log(shape.lo)))).astype(np.int64)
    keep = np.cumsum(card) <= max(shape.planted_share * D, card[0])
    card = card[keep]
    n_pl = int(card.sum())
    n_bg = max(D - n_pl, 0)
    # planted pairs: host rank hosts+1+h, bip = fmix32(counter ^ key_h)
    hid = torch.repeat_interleave(torch.arange(card.size, device=device), torch.from_numpy(card).to(device))
    first = torch.from_numpy(np.concatenate([[0], np.cumsum(card)[:-1]])).to(device)
    ctr = torch.arange(n_pl, device=device, dtype=torch.int64) - first[hid]
    hkey = rand_u32(seed, base + 2, card.size, device)
    addr_key = int(rand_u32(seed, 0xA11CE, 1, device)[0])
    p_addr = fmix32((torch.arange(card.size, device=device, dtype=torch.int64) + shape.hosts + 1) ^ addr_key)
    pa = p_addr[hid]
    pb = fmix32(ctr ^ hkey[hid])
    pslice = ctr % shape.slices
    # background pairs
    cdf = _zipf_cdf(shape.hosts, shape.zipf_s, device)
    ranks = torch.searchsorted(cdf, rand_unit(seed, base + 3, n_bg, device), right=True).clamp_(max=shape.hosts - 1) + 1
    ba = fmix32(ranks ^ addr_key)
    bb = rand_u32(seed, base + 4, n_bg, device)
    bslice = _srl(rand_u64(seed, base + 5, n_bg, device), 40) % shape.slices
    a = torch.cat([pa, ba])
    b = torch.cat([pb, bb])
    sl = torch.cat([pslice, bslice])
    perm = torch.argsort(rand_u64(seed, base + 6, a.numel(), device))
    a, b, sl = a[perm], b[perm], sl[perm]
    aips, bips = [], []
    for t in range(shape.slices):
        mk = sl == t
        aips.append(as_u32_device(a[mk]))
        bips.append(as_u32_device(b[mk]))
    # exact distinct counts per host over the trace
    keys = torch.unique((a << 32) | b)
    hosts, counts = torch.unique(_srl(keys, 32), return_counts=True)
    counts_np = counts.cpu().numpy()
    hosts_np = hosts.cpu().numpy().astype(np.uint32)
    p_np = p_addr.cpu().numpy().astype(np.uint32)
    is_pl = np.isin(hosts_np, p_np)
    bg_idx = np.nonzero(~is_pl & (counts_np >= shape.min_count))[0]
    if bg_idx.size > shape.bg_samples:
        pick = (rand_u64(seed, base + 7, shape.bg_samples, device).cpu().numpy().view(np.uint64)
                % np.uint64(bg_idx.size)).astype(np.int64)
        bg_idx = np.unique(bg_idx[pick])
    sel = np.concatenate([np.nonzero(is_pl & (counts_np >= shape.min_count))[0], bg_idx])
    return aips, bips, hosts_np[sel], counts_np[sel].astype(np.int64)


def link_stream(seed: int, n_pairs: int, device, hosts: int = 1 << 16, zipf_s: float = 1.1, planted: int = 32,
                lo: int = 1500, hi: int = 8000, card_dist: str = "uniform") -> Tuple[torch.Tensor, torch.Tensor,
                                                                                     np.ndarray]:
    """A long pair stream of one link (by default small-configuration content:
    Zipf background, uniform 32-bit bips, planted hosts with U[lo, hi]
    distinct bips spread uniformly over the stream; card_dist="loguniform"
    draws the planted cardinalities log-uniformly over [lo, hi]).  Returns
    int32 aip and bip device tensors and the planted hosts.  Consecutive
    sub-ranges serve as slices."""
    base = 0x9000
    u = rand_unit(seed, base, planted, device).cpu().numpy()
    if card_dist == "loguniform":
        card = np.floor(np.exp(math.log(lo) + u * (math.log(hi) - math.log(lo)))).astype(np.int64)
    else:
        card = (lo + np.floor(u * (hi - lo + 1))).astype(np.int64)
    n_pl = int(card.sum())
    n_bg = max(n_pairs - n_pl, 0)
    hid = torch.repeat_interleave(torch.arange(planted, device=device), torch.from_numpy(card).to(device))
    first = torch.from_numpy(np.concatenate([[0], np.cumsum(card)[:-1]])).to(device)
    ctr = torch.arange(n_pl, device=device, dtype=torch.int64) - first[hid]
    hkey = rand_u32(seed, base + 1, planted, device)
    addr_key = int(rand_u32(seed, 0xA11CE, 1, device)[0])
    p_addr = fmix32((torch.arange(planted, device=device, dtype=torch.int64) + hosts + 1) ^ addr_key)
    cdf = _zipf_cdf(hosts, zipf_s, device)
    ranks = torch.searchsorted(cdf, rand_unit(seed, base + 2, n_bg, device), right=True).clamp_(max=hosts - 1) + 1
    a = torch.cat([p_addr[hid], fmix32(ranks ^ addr_key)])
    b = torch.cat([fmix32(ctr ^ hkey[hid]), rand_u32(seed, base + 3, n_bg, device)])
    perm = torch.argsort(rand_u64(seed, base + 4, a.numel(), device))
    return as_u32_device(a[perm]), as_u32_device(b[perm]), p_addr.cpu().numpy().astype(np.uint32)


@dataclasses.dataclass
class SlidingShape:
    """Sliding-window traffic at the scale of the paper's own run (1-s slices,
    a window of k slices).  Every slice carries `distinct` fresh background
    pairs (aip Zipf(zipf_s) over `hosts` ranks, uniform 32-bit bips), each
    sent `repeat` times, plus `planted` hosts whose cardinality over any full
    window is k * m_h with m_h = floor(card_h / k) and card_h log-uniform in
    [lo, hi]: host h adds m_h fresh bips in every slice."""
    k: int = 300
    distinct: int = 100_000
    repeat: int = 10
    hosts: int = 1 << 22
    zipf_s: float = 1.1
    planted: int = 1000
    lo: int = 1024
    hi: int = 1 << 18


def sliding_planted(shape: SlidingShape, seed: int, device) -> Tuple[np.ndarray, np.ndarray]:
    """Planted host addresses (uint32) and their per-slice fresh bips m_h."""
    u = rand_unit(seed, 0xB000, shape.planted, device).cpu().numpy()
    card = np.floor(np.exp(math.log(shape.lo) + u * (math.log(shape.hi) - math.log(shape.lo)))).astype(np.int64)
    m = card // shape.k
    addr_key = int(rand_u32(seed, 0xA11CE, 1, device)[0])
    ranks = torch.arange(shape.planted, device=device, dtype=torch.int64) + shape.hosts + 1
    return fmix32(ranks ^ addr_key).cpu().numpy().astype(np.uint32), m


def sliding_slice(shape: SlidingShape, seed: int, t: int, device) -> Tuple[torch.Tensor, torch.Tensor]:
    """Pairs of slice t as int32 device tensors (shuffled)."""
    addr_key = int(rand_u32(seed, 0xA11CE, 1, device)[0])
    base = 0xC000 + 8 * t
    cdf = _zipf_cdf(shape.hosts, shape.zipf_s, device)
    ranks = torch.searchsorted(cdf, rand_unit(seed, base, shape.distinct, device), right=True)
    ranks = ranks.clamp_(max=shape.hosts - 1) + 1
    ba = fmix32(ranks ^ addr_key)
    bb = rand_u32(seed, base + 1, shape.distinct, device)
    ba, bb = ba.repeat(shape.repeat), bb.repeat(shape.repeat)
    p_addr, m = sliding_planted(shape, seed, device)
    mt = torch.from_numpy(m).to(device)
    hid = torch.repeat_interleave(torch.arange(m.size, device=device), mt)
    first = torch.from_numpy(np.concatenate([[0], np.cumsum(m)[:-1]])).to(device)
    ctr = torch.arange(int(m.sum()), device=device, dtype=torch.int64) - first[hid]
    hkey = rand_u32(seed, 0xB001, m.size, device)
    pa = torch.from_numpy(p_addr.astype(np.int64)).to(device)[hid]
    pb = fmix32((ctr + t * mt[hid]) ^ hkey[hid])           # fresh bips: counters never repeat
    a = torch.cat([ba, pa])
    b = torch.cat([bb, pb])
    perm = torch.argsort(rand_u64(seed, base + 2, a.numel(), device))
    return as_u32_device(a[perm]), as_u32_device(b[perm])
