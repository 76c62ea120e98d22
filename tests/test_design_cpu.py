"""CPU measurements that design decisions rest on.

Wave-level merging of duplicate stores (a ballot or match over a wave's
targets before the stores) was considered for the Zipf-heavy scans.  A wave
of 64 pairs makes 64*r stores; merging can save at most the stores whose AT
another store of the same wave already targets.  On the configurations'
traffic that share stays below 0.3%: a heavy host's pairs share its r ATVs
but spread over the g positions by BH(bip), and the slices are shuffled, so
repeated pairs rarely meet in one wave.  So no merging is built."""
import numpy as np
import pytest

from paper_1807_01527_amd import traffic


def _wave_duplicate_share(o, aip, bip, wave):
    c = o.constants()
    alpha, beta = np.uint64(c["alpha"]), np.uint64(c["beta"])
    hosts, inv = np.unique(aip, return_inverse=True)
    ncol = 1 << o.c
    atv = np.zeros((hosts.size, o.r), np.int64)
    for q, h in enumerate(hosts.tolist()):
        z, x = o.rrh(h)
        atv[q] = [(z * o.r + j) * ncol + int(x[j]) for j in range(o.r)]
    with np.errstate(over="ignore"):
        i = ((alpha * bip.astype(np.uint64) + beta) >> np.uint64(64 - o.log2g)).astype(np.int64)
    tgt = atv[inv] * o.g + i[:, None]
    n = aip.size // wave * wave
    w = np.sort(tgt[:n].reshape(-1, wave * o.r), axis=1)
    top = np.bincount(inv).max() / aip.size
    return float((w[:, 1:] == w[:, :-1]).sum() / w.size), float(top)


@pytest.mark.parametrize("name,cfg,geom", [
    ("small", traffic.config_small(0), dict(k=4, r=4, c=8, s=8, u=1, log2g=9)),
    ("link", traffic.config_link(0, n_slices=1, pairs_per_slice=1_000_000, planted=0),
     dict(k=10, r=4, c=9, s=7, u=3, log2g=12)),
    ("large", traffic.config_large(0, n_slices=1, pairs_per_slice=1_000_000, planted=0),
     dict(k=60, r=4, c=10, s=6, u=4, log2g=12)),
])
def test_duplicate_stores_within_a_wave_are_rare(oracle_lib, name, cfg, geom):
    tr = traffic.generate(cfg)
    o = oracle_lib.Oracle(**geom, seed=0)
    share, top = _wave_duplicate_share(o, tr.aip[0], tr.bip[0], 64)
    assert top > 0.1, (name, top)         # the traffic is Zipf-heavy: one host holds over 10% of the pairs
    assert share < 0.003, (name, share)   # yet under 0.3% of a wave's stores repeat a target of that wave
