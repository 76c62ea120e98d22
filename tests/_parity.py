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
