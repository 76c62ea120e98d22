"""Parity at the benchmark's full size and launch configuration.

The realistic-link workload (10 slices of 5M pairs, k = 10, 2^26-AT pool)
goes through the HIP path exactly as bench.py issues it: one at_ingest_slice
call per slice, which opens the slice and scans its pairs (on the automatic
path; at this size the tiled scan, with the opening preserve in its tile
pass).  A second pool takes the same slices with a separate opening call
first.  The oracle follows on the same pairs.  After every
slice, the whole pool, the weights and the AAT are compared.  After the last
slice, the estimates of every true super point and of a host sample are
compared, along with the restore outcome (AT_E_BUDGET with the same U).
"""
import numpy as np
import pytest

from paper_1807_01527_amd import traffic

from ._parity import compare_estimates, compare_restore, compare_state, compare_summary, make_pair, to_dev

pytestmark = pytest.mark.gpu

LINK = dict(k=10, r=4, c=9, s=7, u=3, log2g=12, theta=1024.0, seed=0)


@pytest.fixture(scope="module")
def link_trace():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return traffic.generate(traffic.config_link(seed=0))


def test_link_workload_full_size(oracle_lib, link_trace):
    from paper_1807_01527_amd.binding import AtPool
    tr = link_trace
    g, o = make_pair(LINK, oracle_lib)
    g2 = AtPool(**LINK)
    for t in range(tr.n_slices):
        da, db = to_dev(tr.aip[t]), to_dev(tr.bip[t])
        g.ingest(da, db)
        g2.ingest(da[:0], db[:0], n=0)
        g2.ingest(da, db)
        o.ingest(tr.aip[t], tr.bip[t])
        g.close(10)
        g2.close(10)
        o.close(10)
        compare_state(g, o, f"slice {t}")
        compare_summary(g, o, f"slice {t}")
        assert np.array_equal(g2.read_pool(), g.read_pool()), f"slice {t}: separate opening call differs"
        print(f"slice {t}: pool, weights and AAT identical", flush=True)
    h, n = traffic.window_counts(tr.aip, tr.bip, min_count=1024)
    rng = np.random.default_rng(0)
    sample = np.unique(np.concatenate([h, tr.aip[-1][rng.integers(0, tr.aip[-1].size, 4000)],
                                       rng.integers(0, 2**32, 2000, dtype=np.uint64).astype(np.uint32)]))
    compare_estimates(g, o, sample, "final window")
    rc, _, U = compare_restore(g, o, cap=1 << 20, where="final window")
    assert rc == -6 and U > 2**32
