"""at_ingest_slice_noalloc (the ingest entry point that allocates nothing:
its tiled-scan scratch lives in a fixed device array) against
at_ingest_slice on the same pairs: pool bytes, weights and AAT identical
after every close, over two calls in a row, the second with fewer pairs, on
pools that take the tiled scan (the worst-case scratch layout included) and
on one that does not tile (direct scan, no scratch)."""
import numpy as np
import pytest

from ._parity import compare_summary, to_dev

pytestmark = pytest.mark.gpu

GEOMS = [
    # 64 MiB pool, 1024 tiles, k = 10
    dict(k=10, r=4, c=9, s=7, u=3, log2g=12, theta=1024.0, seed=3),
    # r = 8 on 4096 tiles: the largest records and tables a call can need
    dict(k=6, r=8, c=10, s=3, u=3, log2g=12, theta=1024.0, seed=5),
    # 16-bit ATs (k = 300) on 32 tiles
    dict(k=300, r=4, c=9, s=8, u=0, log2g=9, theta=256.0, seed=7),
    # a pool smaller than one tile (32 KiB): the direct scan, no scratch
    dict(k=4, r=4, c=9, s=8, u=0, log2g=4, theta=12.0, seed=9),
]


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1807_01527_amd import binding
    binding.load()
    return torch


def _pairs(n, seed):
    rng = np.random.default_rng(seed)
    hosts = rng.integers(0, 2**32, 5000, dtype=np.uint64).astype(np.uint32)
    a = hosts[np.minimum(rng.zipf(1.2, n), hosts.size) - 1]
    b = rng.integers(0, 2**32, n, dtype=np.uint64).astype(np.uint32)
    return a, b


@pytest.mark.parametrize("geom", GEOMS)
def test_noalloc_ingest_equals_ingest(torch_cuda, geom):
    from paper_1807_01527_amd.binding import AT_E_INVAL, NOALLOC_MAX_PAIRS, AtPool
    ref, na = AtPool(**geom), AtPool(**geom)
    tiles = ref.pool_bytes % (1 << 16) == 0 and ref.pool_bytes >> 16 <= 4096
    if tiles:
        ref.set_scan_mode(3)
        na.set_scan_mode(3)
    sizes = [NOALLOC_MAX_PAIRS, 300_001, 0, 77]
    for t, n in enumerate(sizes):
        a, b = _pairs(n, 100 * geom["seed"] + t)
        da, db = to_dev(a), to_dev(b)
        ref.ingest(da, db, n=n)
        assert na.ingest_noalloc(da, db, n) == 0
        kq = geom["k"] if t % 2 == 0 else max(1, geom["k"] // 2)
        ref.close(kq)
        na.close(kq)
        assert ref.clock() == na.clock()
        assert np.array_equal(ref.read_pool(), na.read_pool()), f"slice {t} ({n} pairs): pool differs"
        w_r, aat_r = ref.read_summary()
        w_n, aat_n = na.read_summary()
        assert np.array_equal(w_r, w_n) and np.array_equal(aat_r, aat_n), f"slice {t}: summary differs"
    # beyond the maximum: rejected on the host, nothing done
    big = to_dev(np.zeros(NOALLOC_MAX_PAIRS + 1, np.uint32))
    before = na.read_pool()
    assert na.ingest_noalloc(big, big) == AT_E_INVAL
    assert na.clock()["open"] == 0 and np.array_equal(na.read_pool(), before)
    ref.destroy()
    na.destroy()


def test_noalloc_slice_over_several_calls(torch_cuda, oracle_lib):
    """One slice split over several no-alloc calls (the first opens it, the
    next add to it) equals the oracle fed the whole slice."""
    from paper_1807_01527_amd.binding import AtPool
    geom = GEOMS[0]
    g, o = AtPool(**geom), oracle_lib.Oracle(**geom)
    g.set_scan_mode(3)
    for t in range(3):
        a, b = _pairs(2_500_000, 900 + t)
        da, db = to_dev(a), to_dev(b)
        for lo in range(0, a.size, 1 << 20):
            hi = min(a.size, lo + (1 << 20))
            assert g.ingest_noalloc(da[lo:hi], db[lo:hi]) == 0
        o.ingest(a, b)
        g.close(geom["k"])
        o.close(geom["k"])
        assert np.array_equal(g.read_pool(), o.pool()), f"slice {t}: pool differs from the oracle"
        compare_summary(g, o, f"slice {t}")
    g.destroy()
