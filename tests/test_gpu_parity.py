"""HIP path vs CPU oracle, element by element, through the C ABI.

AT pool bytes, clock, per-ATV weights, AAT, NAT, flags and restore lists must
be identical; FP64 estimates agree to 1e-12 relative.  Sizes span several
tiles/workgroups with ragged tails; the literal-size workloads are covered in
test_gpu_fullsize.py.
"""
import numpy as np
import pytest

from paper_1807_01527_amd import traffic

from ._parity import compare_estimates, compare_restore, compare_state, compare_summary, make_pair, run_trace, to_dev

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1807_01527_amd import binding
    binding.load()
    return torch


def _tiny(seed=0, **kw):
    return traffic.generate(traffic.config_tiny(seed=seed, **kw))


def test_constants_match(cuda, oracle_lib):
    for seed in (0, 1, 99, 2**64 - 1):
        params = dict(k=4, r=4, c=9, s=8, u=0, log2g=9, seed=seed)
        g, o = make_pair(params, oracle_lib)
        assert g.constants() == o.constants()


@pytest.mark.parametrize("geom", [
    dict(k=3, r=4, c=8, s=8, u=1, log2g=6),        # several blocks per ATV
    dict(k=13, r=4, c=8, s=8, u=1, log2g=4),       # g < 2k: every AT in the last block
    dict(k=1, r=4, c=8, s=8, u=1, log2g=5),        # discrete window
    dict(k=5, r=3, c=11, s=10, u=3, log2g=7),      # r = 3, 8 frames
    dict(k=7, r=5, c=8, s=6, u=2, log2g=8),        # r = 5
    dict(k=4, r=2, c=16, s=16, u=2, log2g=4),      # r = 2
])
def test_small_geometries(cuda, oracle_lib, geom):
    tr = _tiny(seed=geom["k"], n_slices=2 * geom["k"] + 5, pairs_per_slice=3001, hosts=1 << 9, planted=3,
               lo=100, hi=700)
    aip = list(tr.aip)
    bip = list(tr.bip)
    aip[3] = aip[3][:0]  # an empty slice
    bip[3] = bip[3][:0]
    g, o = make_pair(dict(**geom, theta=64.0, seed=5), oracle_lib)
    kps = list(range(1, geom["k"] + 1))
    run_trace(g, o, aip, bip, kprimes=kps, batches=4, seed=1, query_hosts=tr.planted_hosts)


def test_unaligned_and_tiny_batches(cuda, oracle_lib):
    tr = _tiny(seed=3, n_slices=5, pairs_per_slice=4099)
    g, o = make_pair(dict(k=2, r=4, c=8, s=8, u=1, log2g=6, theta=100.0, seed=2), oracle_lib)
    run_trace(g, o, tr.aip, tr.bip, batches=7, seed=3, query_hosts=tr.planted_hosts, unaligned=True)


def test_small_config_literal(cuda, oracle_lib):
    """1M pairs in 4 slices of 250k into the 2^20-AT literal pool: pool bytes
    after every slice; restore exceeds the tuple budget on both sides."""
    tr = traffic.generate(traffic.config_small(seed=0))
    g, o = make_pair(dict(k=4, r=4, c=9, s=8, u=0, log2g=9, theta=1024.0, seed=0, tuple_budget=10**7), oracle_lib)
    h, cnt = traffic.window_counts(tr.aip, tr.bip, min_count=800)
    run_trace(g, o, tr.aip, tr.bip, batches=3, seed=4, query_hosts=h, cap=1 << 16)


def test_small_config_companion(cuda, oracle_lib):
    """Same traffic at paper-like load (2^26 ATs): the restored list equals the
    oracle's and contains the true super points."""
    tr = traffic.generate(traffic.config_small(seed=1))
    g, o = make_pair(dict(k=4, r=4, c=9, s=7, u=3, log2g=12, theta=1024.0, seed=1), oracle_lib)
    h, cnt = traffic.window_counts(tr.aip, tr.bip, min_count=1024)
    run_trace(g, o, tr.aip, tr.bip, batches=2, seed=5, query_hosts=h, check_pool_every=False)
    compare_state(g, o, "final")
    rc, cs, m = compare_restore(g, o)
    assert rc == 0 and m > 0
    assert np.isin(h[cnt >= 2048], cs).all()


def test_order_split_and_repeats_invariant(cuda, oracle_lib):
    """Shuffled order, other batch splits and repeated pairs give the same pool."""
    tr = _tiny(seed=9, n_slices=4, pairs_per_slice=20000)
    params = dict(k=3, r=4, c=8, s=8, u=1, log2g=6, seed=7)
    from paper_1807_01527_amd.binding import AtPool
    pools = []
    rng = np.random.default_rng(0)
    for variant in range(3):
        g = AtPool(**params)
        for a, b in zip(tr.aip, tr.bip):
            if variant == 1:
                p = rng.permutation(a.size)
                a, b = a[p], b[p]
            if variant == 2:
                a = np.concatenate([a, a[::3]])
                b = np.concatenate([b, b[::3]])
            da, db = to_dev(a), to_dev(b)
            step = [a.size, 777, 5000][variant]
            for lo in range(0, a.size, step):
                g.ingest(da[lo:lo + step], db[lo:lo + step])
            g.close(3)
        pools.append(g.read_pool())
    assert np.array_equal(pools[0], pools[1]) and np.array_equal(pools[0], pools[2])


def test_error_paths(cuda, oracle_lib):
    from paper_1807_01527_amd import binding
    from paper_1807_01527_amd.binding import AtError, AtPool
    bad = [dict(k=4, r=4, c=9, s=7, u=0, log2g=9), dict(k=0, r=4, c=9, s=8, u=0, log2g=9),
           dict(k=32768, r=4, c=9, s=8, u=0, log2g=9), dict(k=4, r=4, c=7, s=7, u=4, log2g=9),
           dict(k=4, r=4, c=9, s=8, u=0, log2g=9, theta=0.0)]
    for p in bad:
        assert AtPool.try_create(**p) == binding.AT_E_INVAL
        assert oracle_lib.Oracle.try_create(**p) == oracle_lib.E_INVAL
    g = AtPool(k=3, r=4, c=8, s=8, u=1, log2g=6)
    with pytest.raises(AtError) as e:
        g.estimate(np.array([1], np.uint32))
    assert e.value.rc == binding.AT_E_STATE
    with pytest.raises(AtError) as e:
        g.close(4)
    assert e.value.rc == binding.AT_E_INVAL
    host = np.zeros(16, np.uint32)
    rc = g.ingest_raw(host.ctypes.data, host.ctypes.data, 16)
    assert rc == binding.AT_E_INVAL
    g.close(3)
    e_, f_, n_ = g.estimate(np.array([1, 2, 3], np.uint32))
    assert (n_ == 0).all()
    g.ingest(to_dev(np.array([1], np.uint32)), to_dev(np.array([2], np.uint32)))
    with pytest.raises(AtError) as e:
        g.estimate(np.array([1], np.uint32))
    assert e.value.rc == binding.AT_E_STATE
    g.destroy()


def test_restore_cap_and_budget(cuda, oracle_lib):
    tr = _tiny(seed=8, n_slices=2, pairs_per_slice=20000, hosts=1 << 10, planted=2, lo=2000, hi=3000)
    p = dict(k=2, r=4, c=8, s=8, u=1, log2g=10, theta=128.0, seed=2)
    g, o = make_pair({**p, "tuple_budget": 10}, oracle_lib)
    run_trace(g, o, tr.aip, tr.bip, restore=False)
    compare_restore(g, o)
    g2, o2 = make_pair(p, oracle_lib)
    run_trace(g2, o2, tr.aip, tr.bip, restore=False)
    rc, cs, m = compare_restore(g2, o2)
    assert rc == 0 and m > 1
    compare_restore(g2, o2, cap=m - 1)
    assert g2.tuple_count() == o2.tuple_count()


@pytest.mark.parametrize("mode", [1, 2, 3])
@pytest.mark.parametrize("geom", [
    dict(k=3, r=4, c=8, s=8, u=1, log2g=6),       # fewer frames than bins; two 64 KiB tiles
    dict(k=5, r=3, c=11, s=10, u=3, log2g=7),
    dict(k=4, r=4, c=9, s=7, u=3, log2g=12),      # the companion geometry (64 MiB)
    dict(k=7, r=5, c=8, s=6, u=4, log2g=8),       # 16 frames: two frames per bin
])
def test_scan_modes(cuda, oracle_lib, geom, mode):
    """The direct, the binned and the tiled scan give the oracle's pool, with
    ragged batches (including ones larger than a workgroup's share and tiny
    ones)."""
    tr = _tiny(seed=11 + geom["k"], n_slices=5, pairs_per_slice=70001, hosts=1 << 10)
    g, o = make_pair(dict(**geom, theta=64.0, seed=9), oracle_lib)
    g.set_scan_mode(mode)
    run_trace(g, o, tr.aip, tr.bip, batches=5, seed=2, query_hosts=tr.planted_hosts, restore=False)


@pytest.mark.parametrize("geom", [
    dict(k=3, r=4, c=8, s=8, u=1, log2g=6),      # ACE 2 bits (16 per word), timestamps 3 bits (10 per word)
    dict(k=10, r=4, c=8, s=8, u=1, log2g=7),     # 4 and 5 bits
    dict(k=60, r=4, c=9, s=7, u=3, log2g=4),     # 6 and 7 bits; g = 16 < 2k, a ragged last word per ATV
    dict(k=100, r=4, c=8, s=8, u=1, log2g=8),    # 7 and 8 bits
    dict(k=300, r=4, c=8, s=8, u=1, log2g=9),    # 9 and 10 bits, the paper's k
])
def test_comparator_pools_match_oracle(cuda, oracle_lib, geom):
    """ACE counters and the asynchronous timestamps, each packed at its own
    width, set and aged on the same slices: the ACE fields equal the oracle's
    ACE counters, the timestamp fields equal the oracle's ATs, and the
    k'-weights of both equal the oracle's (the same ATs active)."""
    import math

    from paper_1807_01527_amd.binding import AtCmp
    k = geom["k"]
    n_slices = 2 * k + 5 if k <= 60 else k + 15
    tr = _tiny(seed=41 + k, n_slices=n_slices, pairs_per_slice=2001, hosts=1 << 9, planted=3, lo=100, hi=700)
    ace = AtCmp("ace", **geom, seed=7)
    pat = AtCmp("at", **geom, seed=7)
    o = oracle_lib.Oracle(**geom, seed=7)
    a = oracle_lib.AceOracle(**geom, seed=7)
    assert ace.bits == a.bits == math.ceil(math.log2(k + 1))
    assert pat.bits == ace.bits + 1 == math.ceil(math.log2(2 * k + 1))
    assert ace.F == 32 // ace.bits and pat.wv == -(-o.g // pat.F)
    rng = np.random.default_rng(k)
    for t in range(n_slices):
        aip, bip = tr.aip[t], tr.bip[t]
        if t % 9 == 4:
            aip, bip = aip[:0], bip[:0]
        if t % 4 == 1:
            ace.open_slice()
            pat.open_slice()
        cut = int(rng.integers(0, aip.size + 1))
        for lo, hi in ((0, cut), (cut, aip.size)):
            if hi > lo:
                ace.ingest(to_dev(aip[lo:hi]), to_dev(bip[lo:hi]))
                pat.ingest(to_dev(aip[lo:hi]), to_dev(bip[lo:hi]))
        o.ingest(aip, bip)
        a.ingest(aip, bip)
        kq = 1 + (t * 5) % k
        ace.close(kq)
        pat.close(kq)
        o.close(kq)
        a.close(kq)
        if k > 60 and t % 10 and t != n_slices - 1:
            continue
        where = f"slice {t} window {kq}"
        assert np.array_equal(ace.unpack(ace.read_words()), a.counters()), where
        assert np.array_equal(pat.unpack(pat.read_words()), o.pool()), where
        w = o.weights()
        assert np.array_equal(a.weights(), w), where
        assert np.array_equal(ace.read_weights(), w), where
        assert np.array_equal(pat.read_weights(), w), where
    ace.destroy()
    pat.destroy()


@pytest.mark.parametrize("geom", [
    dict(k=6, r=4, c=8, s=8, u=1, log2g=7),
    dict(k=10, r=4, c=9, s=7, u=3, log2g=10),
    dict(k=150, r=4, c=8, s=8, u=1, log2g=9),     # 16-bit ATs
])
def test_close_multi_windows(cuda, oracle_lib, geom):
    """One close summarising several windows k' (Section 3: every k' <= k is
    answerable from the same state) equals the oracle re-summarised for each
    k', and leaves the pool and clock as a single-window close does."""
    from paper_1807_01527_amd import binding
    from paper_1807_01527_amd.binding import AtError
    k = geom["k"]
    per_slice = 9001 if k <= 10 else 1200
    tr = _tiny(seed=21 + k, n_slices=k + 4, pairs_per_slice=per_slice, hosts=1 << 10, planted=4, lo=300, hi=2000)
    # the budget keeps the oracle's tuple enumeration short; both sides apply it
    g, o = make_pair(dict(**geom, theta=256.0, seed=4, tuple_budget=1 << 22), oracle_lib)
    wins = sorted({1, 2, k // 2, k - 1, k})[:8]
    for t in range(tr.n_slices):
        g.ingest(to_dev(tr.aip[t]), to_dev(tr.bip[t]))
        o.ingest(tr.aip[t], tr.bip[t])
        order = wins[::-1] if t % 2 else wins
        g.close_multi(order)
        o.close(order[0])
        compare_state(g, o, f"slice {t}")
        if t < k - 1 and t != tr.n_slices - 1:
            continue
        hosts = np.unique(np.concatenate([tr.planted_hosts, tr.aip[t][:64]]))
        for kp in order[1:] + order[:1]:
            g.select_window(kp)
            assert o.requery(kp) == 0
            where = f"slice {t} window {kp}"
            compare_state(g, o, where, pool=False)
            compare_summary(g, o, where)
            compare_estimates(g, o, hosts, where)
            compare_restore(g, o, where=where)
    with pytest.raises(AtError) as e:
        g.select_window(k + 1 if k + 1 not in wins else 99)
    assert e.value.rc == binding.AT_E_INVAL
    for bad in ([], [k + 1], [0], list(range(1, 10))):
        with pytest.raises(AtError) as e:
            g.close_multi(bad)
        assert e.value.rc == binding.AT_E_INVAL
    g.ingest(to_dev(tr.aip[0][:10]), to_dev(tr.bip[0][:10]))
    with pytest.raises(AtError) as e:
        g.select_window(k)
    assert e.value.rc == binding.AT_E_STATE
    g.destroy()


@pytest.mark.parametrize("geom", [
    dict(k=6, r=4, c=8, s=8, u=1, log2g=7),
    dict(k=60, r=4, c=9, s=7, u=3, log2g=10),     # the large configuration's k
    dict(k=13, r=4, c=8, s=8, u=1, log2g=4),      # g < 2k: empty blocks
    dict(k=300, r=4, c=8, s=8, u=1, log2g=9),     # 16-bit ATs, the paper's k
])
def test_close_hist_every_window(cuda, oracle_lib, geom):
    """at_close_slice_hist reads the pool once and keeps every ATV's age
    histogram: it equals the oracle's, and every window k' <= k summarised
    from it alone (at_requery_window) equals the oracle re-summarised for
    that k' -- weights, AAT, estimates and the restore list."""
    from paper_1807_01527_amd import binding
    from paper_1807_01527_amd.binding import AtError
    k = geom["k"]
    n_slices = min(k, 40) + 4
    per_slice = 9001 if k <= 13 else 2500
    tr = _tiny(seed=31 + k, n_slices=n_slices, pairs_per_slice=per_slice, hosts=1 << 10, planted=4, lo=300,
               hi=2000)
    g, o = make_pair(dict(**geom, theta=256.0, seed=6, tuple_budget=1 << 22), oracle_lib)
    # before any histogram close there is nothing to requery
    g.ingest(to_dev(tr.aip[0]), to_dev(tr.bip[0]))
    o.ingest(tr.aip[0], tr.bip[0])
    g.close(k)
    o.close(k)
    with pytest.raises(AtError) as e:
        g.requery(1)
    assert e.value.rc == binding.AT_E_STATE
    checks = {3, n_slices - 1}
    for t in range(1, n_slices):
        g.ingest(to_dev(tr.aip[t]), to_dev(tr.bip[t]))
        o.ingest(tr.aip[t], tr.bip[t])
        kq = 1 + (t * 7) % k
        g.close_hist(kq)
        o.close(kq)
        compare_state(g, o, f"slice {t}")
        compare_summary(g, o, f"slice {t}")
        if t not in checks:
            continue
        assert np.array_equal(g.read_age_hist().astype(np.uint32), o.age_hist()), f"slice {t}"
        hosts = np.unique(np.concatenate([tr.planted_hosts, tr.aip[t][:64]]))
        wins = range(1, k + 1) if k <= 60 else sorted({1, 2, 3, k // 3, k // 2, k - 1, k})
        for kp in wins:
            g.requery(kp)
            assert o.requery(kp) == 0
            where = f"slice {t} window {kp}"
            compare_state(g, o, where, pool=False)
            compare_summary(g, o, where)
            if kp in (1, k // 2, k) or kp % 17 == 0:
                compare_estimates(g, o, hosts, where)
                compare_restore(g, o, where=where)
    for bad in (0, k + 1):
        with pytest.raises(AtError) as e:
            g.requery(bad)
        assert e.value.rc == binding.AT_E_INVAL
    # a new slice makes the histograms stale
    g.ingest(to_dev(tr.aip[0][:10]), to_dev(tr.bip[0][:10]))
    for call in (lambda: g.requery(1), g.read_age_hist):
        with pytest.raises(AtError) as e:
            call()
        assert e.value.rc == binding.AT_E_STATE
    g.destroy()


def test_close_hist_rejects_long_windows(cuda, oracle_lib):
    """The histogram close keeps k bins per wave in LDS: k above
    AT_HIST_MAX_K is refused before any work, and the handle stays usable."""
    from paper_1807_01527_amd import binding
    from paper_1807_01527_amd.binding import AtError
    g, o = make_pair(dict(k=binding.AT_HIST_MAX_K + 1, r=4, c=8, s=8, u=1, log2g=5, seed=2), oracle_lib)
    with pytest.raises(AtError) as e:
        g.close_hist()
    assert e.value.rc == binding.AT_E_INVAL
    g.close()
    o.close()
    compare_state(g, o, "after the refused close")
    g.destroy()


@pytest.mark.parametrize("mode", [1, 2, 3])
@pytest.mark.parametrize("geom,slices", [
    (dict(k=150, r=4, c=8, s=8, u=1, log2g=9), 310),    # blocks of 1 AT and a 213-AT last block
    (dict(k=300, r=4, c=8, s=8, u=3, log2g=4), 610),    # the paper's k; g < 2k: one block holds every AT
    (dict(k=200, r=4, c=9, s=8, u=3, log2g=8), 40),     # 8 frames, a larger pool, no wrap
    (dict(k=20000, r=4, c=8, s=8, u=1, log2g=5), 12),   # 4k > 2^16: the unpacked form of Alg 1
])
def test_wide_ats(cuda, oracle_lib, geom, slices, mode):
    """k > 127 needs 2k+1 > 256 AT values: 16-bit ATs.  The two long runs go
    past a full turn of the block clock (2k slices), with empty slices and a
    cycle of windows k'; both scans; pool, summaries, estimates and restore
    after every slice."""
    k = geom["k"]
    tr = _tiny(seed=k + mode, n_slices=slices, pairs_per_slice=1500, hosts=1 << 9, planted=3, lo=200, hi=900)
    aip, bip = list(tr.aip), list(tr.bip)
    for t in range(5, slices, 37):
        aip[t], bip[t] = aip[t][:0], bip[t][:0]
    g, o = make_pair(dict(**geom, theta=64.0, seed=7, tuple_budget=1 << 22), oracle_lib)
    assert g.at_bytes == 2 and g.pool_bytes == 2 * o.pool_size
    g.set_scan_mode(mode)
    run_trace(g, o, aip, bip, kprimes=[k, 1, k // 2, k - 1, 7], batches=3, seed=3, query_hosts=tr.planted_hosts)


def test_tiled_mode_needs_whole_tiles(cuda):
    """The tiled scan needs a pool of whole 64 KiB tiles, at most 4096."""
    from paper_1807_01527_amd import binding
    from paper_1807_01527_amd.binding import AtError, AtPool
    g = AtPool(k=13, r=4, c=8, s=8, u=1, log2g=4)          # 32 KiB pool
    with pytest.raises(AtError) as e:
        g.set_scan_mode(3)
    assert e.value.rc == binding.AT_E_INVAL
    g.destroy()
    g = AtPool(k=4, r=4, c=14, s=6, u=4, log2g=12)         # 4 GiB pool: 65536 tiles
    with pytest.raises(AtError) as e:
        g.set_scan_mode(3)
    assert e.value.rc == binding.AT_E_INVAL
    g.destroy()


@pytest.mark.parametrize("geom", [
    dict(k=3, r=4, c=8, s=8, u=1, log2g=6),       # 1024 ATVs per 64 KiB tile, 4 chunks per ATV
    dict(k=5, r=3, c=10, s=10, u=3, log2g=12),    # 256 chunks per ATV
    dict(k=150, r=4, c=8, s=8, u=1, log2g=9),     # 16-bit ATs
])
def test_tiled_single_call_slices(cuda, oracle_lib, geom):
    """One tiled call per slice: the call opens the slice, runs the opening
    preserve in its tile pass and writes the full window's weights there, so
    a close with k' = k reads no pool.  Closes alternate k' = k and other
    windows (which take the close kernel), and one slice gets a second call
    (which makes the fused weights stale)."""
    k = geom["k"]
    tr = _tiny(seed=31 + k, n_slices=12, pairs_per_slice=20001, hosts=1 << 10, planted=3, lo=300, hi=3000)
    g, o = make_pair(dict(**geom, theta=128.0, seed=6, tuple_budget=1 << 22), oracle_lib)
    g.set_scan_mode(3)
    for t in range(tr.n_slices):
        a, b = tr.aip[t], tr.bip[t]
        if t == 5:
            half = a.size // 2
            g.ingest(to_dev(a[:half]), to_dev(b[:half]))
            g.ingest(to_dev(a[half:]), to_dev(b[half:]))
        else:
            g.ingest(to_dev(a), to_dev(b))
        o.ingest(a, b)
        kp = k if t % 3 != 2 else max(1, k // 2)
        g.close(kp)
        o.close(kp)
        where = f"slice {t} k'={kp}"
        compare_state(g, o, where)
        compare_summary(g, o, where)
        compare_estimates(g, o, np.unique(np.concatenate([tr.planted_hosts, a[:64]])), where)
    g.destroy()


@pytest.mark.parametrize("geom", [
    dict(k=5, r=2, c=11, s=9, u=12, log2g=4),   # a host's two rows in one tile; 4096 tiles
    dict(k=5, r=4, c=10, s=9, u=2, log2g=12),   # four rows in four tiles
])
def test_tiled_one_host_fills_blocks(cuda, oracle_lib, geom):
    """Every pair of a slice from one host, so that all stores of a block of
    the tiled scan land in the tiles of that host's r ATVs.  With r = 2 and
    both rows in one tile, that tile takes all 16384 stores of every block:
    the largest count the 16-bit per-block count table has to hold.  Then the
    host with half the pairs among random others, then the host and one
    other.  Pools, summaries and estimates equal the oracle's after every
    slice."""
    r = geom["r"]
    geom = dict(**geom, theta=64.0, seed=9, tuple_budget=1 << 22)
    rng = np.random.default_rng(40 + r)
    n = 100_003
    heavy, other = np.uint32(0x9E3779B9), np.uint32(12345)
    rand = rng.integers(0, 2**32, n, dtype=np.uint64).astype(np.uint32)
    slices = [np.full(n, heavy, np.uint32),
              np.where(rng.random(n) < 0.5, heavy, rand).astype(np.uint32),
              np.where(rng.random(n) < 0.5, heavy, other).astype(np.uint32)]
    g, o = make_pair(geom, oracle_lib)
    g.set_scan_mode(3)
    hosts = np.array([heavy, other, *rand[:32]], np.uint32)
    for t, a in enumerate(slices):
        b = rng.integers(0, 2**32, n, dtype=np.uint64).astype(np.uint32)
        g.ingest(to_dev(a), to_dev(b))
        o.ingest(a, b)
        g.close(5)
        o.close(5)
        where = f"r={r} slice {t}"
        compare_state(g, o, where)
        compare_summary(g, o, where)
        compare_estimates(g, o, hosts, where)
    g.destroy()


def test_calls_larger_than_one_batch(cuda, oracle_lib):
    """Calls of more than 8Mi pairs are cut into batches by every scan (the
    tiled call then leaves the window count to the close).  Two slices of
    9M pairs, each in one call, on a small pool: all three scans give the
    oracle's pool and summaries."""
    from paper_1807_01527_amd.binding import AtPool
    geom = dict(k=4, r=4, c=8, s=8, u=3, log2g=6, theta=256.0, seed=12)
    rng = np.random.default_rng(12)
    n = 9_000_001
    slices = []
    for _ in range(2):
        a = (rng.zipf(1.3, n) % (1 << 16)).astype(np.uint32) * np.uint32(2654435761)
        b = rng.integers(0, 2**32, n, dtype=np.uint64).astype(np.uint32)
        slices.append((a, b))
    o = oracle_lib.Oracle(**geom)
    for a, b in slices:
        o.ingest(a, b)
        o.close(4)
    want_pool, want_w, want_aat = o.pool(), o.weights(), o.aat()
    for mode in (1, 2, 3):
        g = AtPool(**geom)
        g.set_scan_mode(mode)
        for a, b in slices:
            g.ingest(to_dev(a), to_dev(b))
            g.close(4)
        assert np.array_equal(g.read_pool(), want_pool), f"mode {mode}: pool differs"
        w, aat = g.read_summary()
        assert np.array_equal(w, want_w) and np.array_equal(aat, want_aat), f"mode {mode}: summaries differ"
        g.destroy()


def test_eq4_edge_branches_match_oracle(cuda, oracle_lib):
    """Windows built so that Eq 4 takes each of its edge branches on both
    sides: a heavy frame (UP ~ 0.41) with unseen hosts (negative estimates,
    AT_F_NEG), a host with every AT position active (NAT = g clamped, AT_F_SAT),
    and a frame with every AT active (UP = 1: +inf, AT_F_SAT).  Pools,
    summaries, NAT, flags and estimates must match, and the flags must occur."""
    from ._scenarios import CLAMP, FULL, LOADED, clamp_hosts, full_frame, loaded_frames, unseen_hosts
    # heavy frame, unseen hosts and targets
    g, o = make_pair(dict(**LOADED, seed=7), oracle_lib)
    aip, bip, targets, *_ = loaded_frames(o, 3)
    g.ingest(to_dev(aip), to_dev(bip))
    o.ingest(aip, bip)
    g.close(1)
    o.close(1)
    compare_state(g, o, "loaded frames")
    compare_summary(g, o, "loaded frames")
    hosts = np.concatenate([unseen_hosts(o, 3), targets])
    _, fl, _ = compare_estimates(g, o, hosts, "loaded frames")
    assert (fl & 2).any() and ((fl & 2) == 0).any()
    g.destroy()
    # NAT = g clamped
    g, o = make_pair(dict(**CLAMP, seed=4), oracle_lib)
    aip, bip, h_all, h_most, _ = clamp_hosts(o)
    g.ingest(to_dev(aip), to_dev(bip))
    o.ingest(aip, bip)
    g.close(CLAMP["k"])
    o.close(CLAMP["k"])
    compare_state(g, o, "clamp")
    e, fl, nat = compare_estimates(g, o, np.array([h_all, h_most], np.uint32), "clamp")
    assert nat.tolist() == [1 << CLAMP["log2g"], (1 << CLAMP["log2g"]) - 1]
    assert fl[0] & 1 and not fl[1] & 1 and e[0] == e[1]
    g.destroy()
    # UP = 1
    g, o = make_pair(dict(**FULL, seed=2), oracle_lib)
    aip, bip, probe = full_frame()
    g.ingest(to_dev(aip), to_dev(bip))
    o.ingest(aip, bip)
    g.close(FULL["k"])
    o.close(FULL["k"])
    compare_state(g, o, "full frame")
    compare_summary(g, o, "full frame")
    e, fl, _ = compare_estimates(g, o, probe, "full frame")
    assert np.isinf(e).all() and ((fl & 1) != 0).all()
    g.destroy()
