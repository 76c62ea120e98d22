"""Helpers that drive the HIP path and the CPU oracle over the same seeded
pairs and compare them (pool bytes, clock, window summaries, estimates and
restore lists)."""
from __future__ import annotations

import numpy as np

EST_RTOL = 1e-12  # FP64 estimates: same operation order, libm log vs device log


def to_dev(a: np.ndarray):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a, np.uint32).view(np.int32)).to("cuda")


def make_pair(params: dict, oracle_mod):
    from paper_1807_01527_amd.binding import AtPool
    return AtPool(**params), oracle_mod.Oracle(**params)


def splits(n: int, parts: int, rng) -> list:
    if parts <= 1 or n == 0:
        return [0, n]
    cuts = np.sort(rng.integers(0, n + 1, parts - 1))
    return [0, *cuts.tolist(), n]


def compare_estimates(gpu, orc, hosts: np.ndarray, where: str = ""):
    e_g, f_g, n_g = gpu.estimate(hosts)
    e_o, f_o, n_o = orc.estimate(hosts)
    assert np.array_equal(n_g, n_o), f"{where}: NAT differs"
    assert np.array_equal(f_g, f_o), f"{where}: flags differ"
    fin = np.isfinite(e_o)
    assert np.array_equal(np.isfinite(e_g), fin), f"{where}: finiteness differs"
    assert np.array_equal(e_g[~fin], e_o[~fin])
    den = np.maximum(np.abs(e_o[fin]), 1e-300)
    rel = np.abs(e_g[fin] - e_o[fin]) / den
    assert rel.max(initial=0.0) <= EST_RTOL, f"{where}: max rel err {rel.max()}"
    return e_g, f_g, n_g


def compare_state(gpu, orc, where: str = "", pool: bool = True):
    assert gpu.clock() == orc.clock(), f"{where}: clock differs"
    if pool:
        pg, po = gpu.read_pool(), orc.pool()
        if not np.array_equal(pg, po):
            bad = np.nonzero(pg != po)[0]
            raise AssertionError(f"{where}: {bad.size} pool bytes differ, first at {bad[0]}: "
                                 f"gpu={pg[bad[0]]} oracle={po[bad[0]]}")


def compare_summary(gpu, orc, where: str = ""):
    w_g, aat_g = gpu.read_summary()
    assert np.array_equal(w_g, orc.weights()), f"{where}: weights differ"
    assert np.array_equal(aat_g, orc.aat()), f"{where}: AAT differs"


def compare_restore(gpu, orc, cap: int = 1 << 20, where: str = ""):
    rc_o, cs_o, m_o = orc.restore(cap=cap)
    rc_g, cs_g, est_g, fl_g, m_g = gpu.restore(cap=cap)
    assert rc_g == rc_o, f"{where}: restore rc gpu={rc_g} oracle={rc_o}"
    assert m_g == m_o, f"{where}: restore count gpu={m_g} oracle={m_o}"
    if rc_o == 0:
        assert np.array_equal(cs_g, cs_o), f"{where}: candidate lists differ"
        if m_o:
            e_o, f_o, _ = orc.estimate(cs_o)
            assert np.array_equal(fl_g, f_o)
            fin = np.isfinite(e_o)
            rel = np.abs(est_g[fin] - e_o[fin]) / np.maximum(np.abs(e_o[fin]), 1e-300)
            assert rel.max(initial=0.0) <= EST_RTOL
    return rc_o, cs_o, m_o


def run_trace(gpu, orc, aip_slices, bip_slices, kprimes=None, batches=3, seed=0, check_pool_every=True,
              query_hosts=None, restore=True, cap=1 << 20, unaligned=False):
    """Feed the same slices to both sides (GPU in ragged batches) and compare
    after every close."""
    rng = np.random.default_rng(seed)
    k = orc.k
    for t, (a, b) in enumerate(zip(aip_slices, bip_slices)):
        if a.size:
            da, db = to_dev(a), to_dev(b)
            cuts = splits(a.size, batches, rng)
            for lo, hi in zip(cuts[:-1], cuts[1:]):
                if unaligned and hi - lo > 1 and lo % 4 == 0:
                    gpu.ingest(da[lo:lo + 1], db[lo:lo + 1])
                    lo += 1
                gpu.ingest(da[lo:hi], db[lo:hi], n=hi - lo)
            orc.ingest(a, b)
        kp = k if kprimes is None else kprimes[t % len(kprimes)]
        gpu.close(kp)
        orc.close(kp)
        where = f"slice {t} k'={kp}"
        compare_state(gpu, orc, where, pool=check_pool_every)
        compare_summary(gpu, orc, where)
        if query_hosts is not None:
            hosts = np.unique(np.concatenate([query_hosts, a[:64]]))
            compare_estimates(gpu, orc, hosts, where)
        if restore:
            compare_restore(gpu, orc, cap=cap, where=where)


def compare_serve_results(got, want, where):
    """Per closed slice: a served link's results against the single-link API's."""
    assert len(got) == len(want), where
    for s, (g, w) in enumerate(zip(got, want)):
        tag = f"{where} slice {s}"
        assert g["slice"] == s, tag
        assert g["restore_rc"] == w["restore_rc"], tag
        assert g["n_out"] == w["n_out"], tag
        assert np.array_equal(g["cand"], w["cand"]), tag
        for key in ("cand_plain", "cand_learned", "watch_plain", "watch_learned"):
            a, b = np.asarray(g[key]), np.asarray(w[key])
            assert a.shape == b.shape, (tag, key)
            assert np.array_equal(np.isfinite(a), np.isfinite(b)), (tag, key)
            fin = np.isfinite(b)
            assert np.all(np.abs(a[fin] - b[fin]) <= 1e-12 * np.abs(b[fin])), (tag, key)
        assert np.array_equal(g["cand_flags"], w["cand_flags"]), tag
        assert np.array_equal(g["watch_flags"], w["watch_flags"]), tag
        assert g["latency_ms"] > 0


def oracle_link_run(oracle_mod, params: dict, k: int, seed: int, events, watch: np.ndarray, cand_cap: int,
                    tuple_budget: int = 0):
    """The CPU oracle driven like a served link: events are ("chunk", aip, bip)
    host arrays and ("end", k') slice ends.  Per close: restore outcome
    (cap = cand_cap), candidates, plain estimates and SAT/NEG flags of the
    candidates and the watch hosts.  Returns (records, final pool)."""
    o = oracle_mod.Oracle(k=k, seed=seed, tuple_budget=tuple_budget, **params)
    out = []
    for ev in events:
        if ev[0] == "chunk":
            o.ingest(ev[1], ev[2])
            continue
        o.close(ev[1])
        rc, cand, m = o.restore(cap=cand_cap)
        rec = dict(restore_rc=rc, n_out=m, cand=cand if rc == 0 else np.zeros(0, np.uint32))
        if rc == 0 and cand.size:
            rec["cand_plain"], rec["cand_flags"], _ = o.estimate(cand)
        else:
            rec["cand_plain"], rec["cand_flags"] = np.zeros(0), np.zeros(0, np.uint8)
        rec["watch_plain"], rec["watch_flags"], _ = o.estimate(np.asarray(watch, np.uint32))
        out.append(rec)
    pool = o.pool()
    o.close_handle()
    return out, pool


def oracle_link_runs(oracle_mod, jobs, workers: int = 8):
    """oracle_link_run over several links at once (the oracle's calls release
    the interpreter lock, so threads run the links in parallel)."""
    from concurrent.futures import ThreadPoolExecutor
    with ThreadPoolExecutor(max_workers=max(1, min(workers, len(jobs)))) as ex:
        futs = [ex.submit(oracle_link_run, oracle_mod, *job) for job in jobs]
        return [f.result() for f in futs]


def compare_serve_with_oracle(got, want, where):
    """Per closed slice: a served link's results against the oracle's: restore
    outcome and count, candidate list, plain FP64 estimates to EST_RTOL, and
    the flags of the plain estimate (AT_F_SAT, AT_F_NEG)."""
    assert len(got) == len(want), f"{where}: {len(got)} closes served, {len(want)} in the oracle"
    for s, (g, w) in enumerate(zip(got, want)):
        tag = f"{where} slice {s}"
        assert g["restore_rc"] == w["restore_rc"], (tag, g["restore_rc"], w["restore_rc"])
        assert g["n_out"] == w["n_out"], (tag, g["n_out"], w["n_out"])
        assert np.array_equal(g["cand"], w["cand"]), tag
        for key, fkey in (("cand_plain", "cand_flags"), ("watch_plain", "watch_flags")):
            a, b = np.asarray(g[key]), np.asarray(w[key])
            assert a.shape == b.shape, (tag, key)
            assert np.array_equal(np.isfinite(a), np.isfinite(b)), (tag, key)
            fin = np.isfinite(b)
            assert np.array_equal(a[~fin], b[~fin]), (tag, key)
            assert np.all(np.abs(a[fin] - b[fin]) <= EST_RTOL * np.abs(b[fin])), (tag, key)
            assert np.array_equal(np.asarray(g[fkey]) & 3, np.asarray(w[fkey]) & 3), (tag, fkey)
