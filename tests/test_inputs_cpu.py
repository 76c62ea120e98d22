"""The seeded input generators that run on the GPU in the benchmark and the
full-size tests, exercised on the CPU (torch's CPU device): exact planted
cardinalities, determinism, the Zipf background's skew, disjoint planted and
background addresses.  They hold none of the method's arithmetic."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from paper_1807_01527_amd import traffic_gpu as tg  # noqa: E402


def _u32(t):
    return t.numpy().view(np.uint32)


def test_sliding_shape_planted_counts_are_exact_per_window():
    sh = tg.SlidingShape(k=6, distinct=3000, repeat=3, hosts=1 << 12, planted=12, lo=200, hi=5000)
    planted, m = tg.sliding_planted(sh, 7, "cpu")
    assert planted.size == 12 and np.unique(planted).size == 12
    slices = [tg.sliding_slice(sh, 7, t, "cpu") for t in range(9)]
    for t0 in range(0, 4):                       # every full window of k slices
        keys = set()
        for a, b in slices[t0:t0 + sh.k]:
            keys.update(zip(_u32(a).tolist(), _u32(b).tolist()))
        per = {}
        for a, _ in keys:
            per[a] = per.get(a, 0) + 1
        assert [per.get(int(h), 0) for h in planted] == (sh.k * m).tolist()
    # background pairs appear `repeat` times; sizes add up
    a, b = slices[0]
    assert a.numel() == sh.distinct * sh.repeat + int(m.sum())
    # deterministic
    a2, b2 = tg.sliding_slice(sh, 7, 0, "cpu")
    assert torch.equal(a, a2) and torch.equal(b, b2)


def test_link_stream_loguniform_planted_and_zipf_background():
    a, b, planted = tg.link_stream(3, 200_000, "cpu", hosts=1 << 14, zipf_s=1.2, planted=20, lo=1000, hi=20000,
                                   card_dist="loguniform")
    au, bu = _u32(a), _u32(b)
    assert a.numel() >= 200_000
    pairs = np.unique(au.astype(np.uint64) << np.uint64(32) | bu.astype(np.uint64))
    hosts, counts = np.unique((pairs >> np.uint64(32)).astype(np.uint32), return_counts=True)
    c = dict(zip(hosts.tolist(), counts.tolist()))
    card = [c.get(int(h), 0) for h in planted]
    assert min(card) >= 1000 and max(card) <= 20000
    # log-uniform: about as many below the geometric midpoint as above it
    mid = np.sqrt(1000 * 20000)
    assert 3 <= sum(x < mid for x in card) <= 17
    # background: Zipf 1.2, the top host carries far more pairs than the median host
    bg = np.isin(au, planted, invert=True)
    _, bc = np.unique(au[bg], return_counts=True)
    assert bc.max() > 50 * np.median(bc)
    # the uniform law is unchanged by the new option
    a1, _, p1 = tg.link_stream(3, 50_000, "cpu")
    a2, _, p2 = tg.link_stream(3, 50_000, "cpu", card_dist="uniform")
    assert torch.equal(a1, a2) and np.array_equal(p1, p2)
