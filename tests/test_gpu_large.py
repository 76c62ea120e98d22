"""Full-size parity on the large configuration and on the serving shape.

Large configuration: 200M pairs in 60 slices of 3,333,333, k = 60 (7-bit
ATs), r = 4, (c, s, u, g) = (10, 6, 4, 4096): a 2^28-AT pool (256 MiB).  aip
Zipf 1.1 over 2^24 hosts, uniform 32-bit bips, 661 planted hosts with
log-uniform cardinality over [1024, 2^20].

- One link through the single-link API as a caller drives it (an opening
  call, then one scan launch per slice on the automatic scan path) against
  the oracle on the same pairs: weights and AAT after every slice, the whole
  pool every tenth slice, then the NAT, flags and FP64 estimates of the
  planted hosts and a host sample, and the restore outcome.
- Four such links (seeds 0-3) served together with the learned correction
  on: every closed slice of every link equals that link run through the
  single-link API.

Serving shape: 16 links with 2^24-AT pools, (c, s, u, g) = (9, 8, 1, 4096),
k in {5, 10, 30}, lognormal slice sizes (median 2M) cut into 64Ki-pair
chunks: the served results equal the single-link API's.
"""
import numpy as np
import pytest

from oracle import mlp as ref

from ._parity import (compare_estimates, compare_restore, compare_serve_results, compare_serve_with_oracle,
                      compare_state, compare_summary, make_pair, oracle_link_run)

pytestmark = [pytest.mark.gpu, pytest.mark.slow]

LARGE = dict(k=60, r=4, c=10, s=6, u=4, log2g=12, theta=1024.0)
LARGE_SLICES = 60
LARGE_PAIRS = 3_333_333
SERVE = dict(r=4, c=9, s=8, u=1, log2g=12, theta=1024.0)
CAND_CAP = 2048
WATCH_CAP = 64
BUDGET = 1 << 24


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1807_01527_amd import binding
    binding.load()
    return torch


def _large_stream(seed: int):
    from paper_1807_01527_amd import traffic_gpu as tg
    return tg.link_stream(seed, LARGE_SLICES * LARGE_PAIRS, "cuda", hosts=1 << 24, zipf_s=1.1, planted=661,
                          lo=1024, hi=1 << 20, card_dist="loguniform")


def _slice(x, t):
    return x[t * LARGE_PAIRS:(t + 1) * LARGE_PAIRS]


@pytest.mark.timeout(900)
def test_large_single_link_vs_oracle(torch_cuda, oracle_lib):
    a, b, planted = _large_stream(0)
    g, o = make_pair(dict(**LARGE, seed=0, tuple_budget=BUDGET), oracle_lib)
    for t in range(LARGE_SLICES):
        da, db = _slice(a, t), _slice(b, t)
        g.ingest(da[:0], db[:0], n=0)
        g.ingest(da, db)
        o.ingest(da.cpu().numpy().view(np.uint32), db.cpu().numpy().view(np.uint32))
        g.close(LARGE["k"])
        o.close(LARGE["k"])
        full = t % 10 == 9
        compare_state(g, o, f"slice {t}", pool=full)
        compare_summary(g, o, f"slice {t}")
        print(f"slice {t}: weights and AAT identical{', pool identical' if full else ''}", flush=True)
    rng = np.random.default_rng(0)
    last = _slice(a, LARGE_SLICES - 1).cpu().numpy().view(np.uint32)
    sample = np.unique(np.concatenate([planted, last[rng.integers(0, last.size, 4000)],
                                       rng.integers(0, 2**32, 2000, dtype=np.uint64).astype(np.uint32)]))
    compare_estimates(g, o, sample, "final window")
    rc, _, U = compare_restore(g, o, cap=CAND_CAP, where="final window")
    print(f"restore rc={rc} U/m={U}", flush=True)
    g.destroy()


def _single_link(k, seed, a, b, slices, net, watch, params):
    """The single-link API, eagerly, slice by slice."""
    from paper_1807_01527_amd.binding import AtPool
    g = AtPool(k=k, seed=seed, tuple_budget=BUDGET, **params)
    out = []
    for lo, hi in slices:
        if hi > lo:
            g.ingest(a[lo:hi], b[lo:hi])
        g.close(k)
        rc, cand, _, _, m = g.restore(cap=CAND_CAP)
        rec = dict(restore_rc=rc, n_out=m, cand=cand if rc == 0 else np.zeros(0, np.uint32))
        if rc == 0 and cand.size:
            rec["cand_learned"], rec["cand_flags"], rec["cand_plain"] = g.estimate_learned(net, cand)
        else:
            rec["cand_learned"] = rec["cand_plain"] = np.zeros(0)
            rec["cand_flags"] = np.zeros(0, np.uint8)
        rec["watch_learned"], rec["watch_flags"], rec["watch_plain"] = g.estimate_learned(net, watch)
        out.append(rec)
    pool = g.read_pool()
    g.destroy()
    return out, pool


def _serve(links, net, params, chunk=65536):
    """All links through one server stepped by its native thread; chunks of
    the links interleaved round robin."""
    from paper_1807_01527_amd.binding import Server
    pool_bytes = (1 << (params["c"] + params["u"])) * params["r"] * (1 << params["log2g"])
    srv = Server(hbm_budget=len(links) * (pool_bytes + (16 << 20)), max_links=len(links), cand_cap=CAND_CAP,
                 watch_cap=WATCH_CAP, **params)
    srv.set_mlp(net)
    ids = []
    for ln in links:
        lid, adm = srv.open_link(ln["k"], ln["seed"], tuple_budget=BUDGET)
        assert adm
        srv.set_watch(lid, ln["watch"])
        ids.append(lid)
    # per link: its event list (chunks, then the slice end)
    evs = []
    for ln in links:
        e = []
        for lo, hi in ln["slices"]:
            for c0 in range(lo, hi, chunk):
                e.append(("chunk", c0, min(hi, c0 + chunk)))
            e.append(("end",))
        evs.append(e)
    srv.start()
    cur = [0] * len(links)
    while any(c < len(e) for c, e in zip(cur, evs)):
        for i, (ln, e) in enumerate(zip(links, evs)):
            if cur[i] >= len(e):
                continue
            ev = e[cur[i]]
            cur[i] += 1
            if ev[0] == "chunk":
                assert srv.submit(ids[i], ln["a"][ev[1]:ev[2]], ln["b"][ev[1]:ev[2]]) == 0
            else:
                assert srv.end_slice(ids[i], ln["k"]) == 0
    srv.stop()
    results = {lid: [] for lid in ids}
    for r in srv.results():
        results[r["link"]].append(r)
    pools = {lid: srv.read_pool(lid) for lid in ids}
    srv.destroy()
    return ids, results, pools


def _oracle_events(a, b, slices, k):
    """Host copies of a link's slices as oracle events (a whole slice per
    chunk: the state does not depend on how a slice is split)."""
    ah = a.cpu().numpy().view(np.uint32)
    bh = b.cpu().numpy().view(np.uint32)
    ev = []
    for lo, hi in slices:
        if hi > lo:
            ev.append(("chunk", ah[lo:hi], bh[lo:hi]))
        ev.append(("end", k))
    return ev


@pytest.mark.timeout(900)
def test_large_four_links_served_equal_single_link(torch_cuda, oracle_lib):
    """Four served links of the large configuration with the learned
    correction on: every close equals the CPU oracle fed the same pairs
    (restore outcome, plain estimates of the watch hosts, flags, final pool;
    the oracles run in threads while the GPU works) and the single-link API."""
    from concurrent.futures import ThreadPoolExecutor

    from paper_1807_01527_amd.binding import Mlp
    net = Mlp(ref.init_params(7).astype(np.float32) * np.float32(0.5))
    links = []
    for seed in range(4):
        a, b, planted = _large_stream(seed)
        slices = [(t * LARGE_PAIRS, (t + 1) * LARGE_PAIRS) for t in range(LARGE_SLICES)]
        links.append(dict(k=LARGE["k"], seed=seed, a=a, b=b, slices=slices, watch=planted[:WATCH_CAP]))
    params = {k: v for k, v in LARGE.items() if k != "k"}
    ex = ThreadPoolExecutor(max_workers=4)
    futs = [ex.submit(oracle_link_run, oracle_lib, params, ln["k"], ln["seed"],
                      _oracle_events(ln["a"], ln["b"], ln["slices"], ln["k"]), ln["watch"], CAND_CAP, BUDGET)
            for ln in links]
    ids, res, pools = _serve(links, net, params)
    for i, (lid, ln) in enumerate(zip(ids, links)):
        want, pool = _single_link(ln["k"], ln["seed"], ln["a"], ln["b"], ln["slices"], net, ln["watch"], params)
        compare_serve_results(res[lid], want, f"large link {i}")
        assert np.array_equal(pools[lid], pool), f"large link {i}: pool differs"
        print(f"large link {i}: {len(want)} slices identical served and alone", flush=True)
    for i, (lid, f) in enumerate(zip(ids, futs)):
        want, pool = f.result()
        compare_serve_with_oracle(res[lid], want, f"large link {i} vs oracle")
        assert np.array_equal(pools[lid], pool), f"large link {i}: pool differs from the oracle"
        print(f"large link {i}: {len(want)} slices identical served and in the oracle", flush=True)
    ex.shutdown()


@pytest.mark.timeout(900)
def test_serving_shape_sixteen_links(torch_cuda, oracle_lib):
    from paper_1807_01527_amd import traffic_gpu as tg
    from paper_1807_01527_amd.binding import Mlp
    rng = np.random.default_rng(5)
    net = Mlp(ref.init_params(9).astype(np.float32) * np.float32(0.5))
    n_slices = 5
    links = []
    for i in range(16):
        sizes = np.clip(np.exp(np.log(2e6) + rng.standard_normal(n_slices)), 1e5, 2e7).astype(np.int64)
        sizes[rng.integers(0, n_slices)] = 0 if i % 5 == 0 else sizes[0]   # some links have an empty slice
        bounds = np.concatenate([[0], np.cumsum(sizes)])
        a, b, planted = tg.link_stream(500 + i, int(bounds[-1]), "cuda")
        links.append(dict(k=int([5, 10, 30][i % 3]), seed=500 + i, a=a, b=b,
                          slices=list(zip(bounds[:-1].tolist(), bounds[1:].tolist())), watch=planted[:WATCH_CAP]))
    from concurrent.futures import ThreadPoolExecutor
    ex = ThreadPoolExecutor(max_workers=8)
    futs = [ex.submit(oracle_link_run, oracle_lib, SERVE, ln["k"], ln["seed"],
                      _oracle_events(ln["a"], ln["b"], ln["slices"], ln["k"]), ln["watch"], CAND_CAP, BUDGET)
            for ln in links]
    ids, res, pools = _serve(links, net, SERVE)
    for i, (lid, ln) in enumerate(zip(ids, links)):
        want, pool = _single_link(ln["k"], ln["seed"], ln["a"], ln["b"], ln["slices"], net, ln["watch"], SERVE)
        compare_serve_results(res[lid], want, f"serving-shape link {i}")
        assert np.array_equal(pools[lid], pool), f"serving-shape link {i}: pool differs"
    for i, (lid, f) in enumerate(zip(ids, futs)):
        want, pool = f.result()
        compare_serve_with_oracle(res[lid], want, f"serving-shape link {i} vs oracle")
        assert np.array_equal(pools[lid], pool), f"serving-shape link {i}: pool differs from the oracle"
    ex.shutdown()


PAPER = dict(k=300, r=4, c=14, s=6, u=4, log2g=12, theta=1024.0, seed=0, tuple_budget=1 << 40)


@pytest.mark.timeout(900)
def test_paper_geometry_16bit_vs_oracle(torch_cuda, oracle_lib):
    """The paper's own sliding shape (Section 5.2 and the geometry of 5.1):
    k = 300 (10-bit ATs, held in 16-bit words), (c, s, u, g) = (14, 6, 4,
    4096), r = 4: 2^32 ATs, an 8 GiB pool whose byte offsets pass 2^32.
    Three one-second slices of the synthetic sliding traffic (100k fresh
    background pairs sent 10 times each, 1000 planted hosts) against the
    oracle: weights and AAT after every slice, the whole pool after the last,
    then the estimates of the planted hosts and a sample, and the restore."""
    from paper_1807_01527_amd import traffic_gpu as tg
    shape = tg.SlidingShape(k=PAPER["k"])
    planted, _ = tg.sliding_planted(shape, 0, "cuda")
    g, o = make_pair(PAPER, oracle_lib)
    assert g.pool_bytes == 2 * (1 << 32)
    last = None
    for t in range(3):
        a, b = tg.sliding_slice(shape, 0, t, "cuda")
        g.ingest(a, b)
        last = a.cpu().numpy().view(np.uint32)
        o.ingest(last, b.cpu().numpy().view(np.uint32))
        g.close(PAPER["k"])
        o.close(PAPER["k"])
        compare_state(g, o, f"paper geometry slice {t}", pool=(t == 2))
        compare_summary(g, o, f"paper geometry slice {t}")
        print(f"paper geometry slice {t}: {a.numel()} pairs, state identical", flush=True)
    rng = np.random.default_rng(1)
    sample = np.unique(np.concatenate([planted, last[rng.integers(0, last.size, 3000)]]))
    compare_estimates(g, o, sample, "paper geometry")
    rc, _, m = compare_restore(g, o, cap=1 << 22, where="paper geometry")
    print(f"paper geometry: restore rc={rc} m={m}", flush=True)
    g.destroy()
