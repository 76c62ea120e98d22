"""Pins of the CPU oracle to facts fixed by the paper and by mathematics.

Each test checks the oracle against something other than itself: a worked
example printed in the paper (tests/golden), a closed form, an exhaustive
enumeration, an independent plain definition (exact timestamps, raw-pair
window replay, hash-set counts) or a textbook special case.
"""
import math
import os

import numpy as np
import pytest

from paper_1807_01527_amd import traffic

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _golden_rows(name):
    rows = []
    with open(os.path.join(GOLDEN, name)) as fh:
        for line in fh:
            line = line.strip()
            if line and not line.startswith("#"):
                rows.append(line.split())
    return rows


# --------------------------------------------------------------------------
# Section 4.1: the prime of the mangling and its inverse
# --------------------------------------------------------------------------

def _is_prime_mr(n):
    """Deterministic Miller-Rabin for n < 3.3e24 (bases up to 37)."""
    if n < 2:
        return False
    small = [2, 3, 5, 7, 11, 13, 17, 19, 23, 29, 31, 37]
    for q in small:
        if n % q == 0:
            return n == q
    d, s = n - 1, 0
    while d % 2 == 0:
        d //= 2
        s += 1
    for a in small:
        x = pow(a, d, n)
        if x in (1, n - 1):
            continue
        for _ in range(s - 1):
            x = x * x % n
            if x == n - 1:
                break
        else:
            return False
    return True


def test_prime_is_largest_32bit_prime(oracle_lib):
    o = oracle_lib.Oracle(k=4, r=4, c=9, s=8, u=0, log2g=9)
    p = o.constants()["p"]
    assert p == 2**32 - 5
    assert _is_prime_mr(p)
    assert not any(_is_prime_mr(q) for q in range(p + 1, 2**32))


@pytest.mark.parametrize("seed", [0, 1, 2, 7, 12345, 2**63 + 11])
def test_inverse_multiplier(oracle_lib, seed):
    o = oracle_lib.Oracle(k=4, r=4, c=9, s=8, u=0, log2g=9, seed=seed)
    cst = o.constants()
    p, A, Ainv = cst["p"], cst["A"], cst["Ainv"]
    assert 2**31 <= A < p
    assert (A * Ainv) % p == 1
    assert cst["alpha"] % 2 == 1


@pytest.mark.slow
def test_mangle_is_a_bijection_exhaustive(oracle_lib):
    """f^-1(f(a)) == a for all 2^32 addresses, hence f is a permutation."""
    o = oracle_lib.Oracle(k=10, r=4, c=9, s=7, u=3, log2g=12, seed=3)
    bad, first = o.pin_bijection()
    assert bad == 0, f"first failing address {first}"


def test_mangle_fixed_points_and_samples(oracle_lib):
    o = oracle_lib.Oracle(k=4, r=4, c=9, s=8, u=0, log2g=9, seed=5)
    cst = o.constants()
    for a in range(cst["p"], 2**32):
        assert o.mangle(a) == a and o.unmangle(a) == a
    rng = np.random.default_rng(0)
    for a in rng.integers(0, cst["p"], 2000):
        a = int(a)
        y = o.mangle(a)
        assert y < cst["p"]
        assert (y * pow(cst["A"], -1, cst["p"])) % cst["p"] == a
    assert o.mangle(0) == 0


# --------------------------------------------------------------------------
# Section 4.1: column extraction, worked example, completeness, duplicates
# --------------------------------------------------------------------------

def test_rrh_worked_example(oracle_lib):
    rows = {r[0]: r[1:] for r in _golden_rows("rrh_worked_example.txt") if r[0] != "wrap"}
    wraps = [tuple(map(int, r[1:])) for r in _golden_rows("rrh_worked_example.txt") if r[0] == "wrap"]
    r, s, u, c = (int(rows[k][0]) for k in ("r", "s", "u", "c"))
    o = oracle_lib.Oracle(k=1, r=r, c=c, s=s, u=u, log2g=4)
    W = 32 - u
    dup = []
    for b in range(W):
        cover = sum(1 for x in o.columns_of_L(1 << b) if x != 0)
        assert cover >= 1, "completeness: every LBS bit appears in some column"
        if cover >= 2:
            dup.append(b)
    assert dup == [int(v) for v in rows["duplicates"]]
    for j, n, pos in wraps:
        x = o.columns_of_L(1 << pos)
        assert x[j] == (1 << n)


GEOMS = [  # (r, c, s, u): the small-config, link-config, serving-config,
    (4, 9, 8, 0),  # large-config and paper geometries, plus a 16-bit one
    (4, 9, 7, 3),
    (4, 9, 8, 1),
    (4, 10, 6, 4),
    (4, 14, 6, 4),
    (4, 6, 4, 16),
    (3, 12, 10, 4),
]


@pytest.mark.parametrize("geom", GEOMS)
def test_columns_round_trip(oracle_lib, geom):
    r, c, s, u = geom
    o = oracle_lib.Oracle(k=2, r=r, c=c, s=s, u=u, log2g=4)
    W = 32 - u
    rng = np.random.default_rng(1)
    Ls = range(1 << W) if W <= 16 else rng.integers(0, 1 << W, 3000)
    for L in Ls:
        L = int(L)
        x = o.columns_of_L(L)
        assert all(int(v) < (1 << c) for v in x)
        assert o.tuple_to_L(x) == L
        assert o.tuple_dupcheck(x)


@pytest.mark.parametrize("geom", GEOMS)
def test_dupcheck_matches_round_trip(oracle_lib, geom):
    """Alg 4's consecutive-row duplicate check accepts exactly the tuples that
    some LBS produces."""
    r, c, s, u = geom
    o = oracle_lib.Oracle(k=2, r=r, c=c, s=s, u=u, log2g=4)
    rng = np.random.default_rng(2)
    W = 32 - u
    hits = 0
    for _ in range(3000):
        if rng.random() < 0.5:
            x = o.columns_of_L(int(rng.integers(0, 1 << W)))
            j = int(rng.integers(0, r))
            x[j] ^= np.uint32(1 << int(rng.integers(0, c))) if rng.random() < 0.5 else 0
        else:
            x = rng.integers(0, 1 << c, r).astype(np.uint32)
        a = o.tuple_to_L(x) is not None
        b = o.tuple_dupcheck(x)
        assert a == b
        hits += a
    assert hits > 100


def test_rejects_invalid_geometry(oracle_lib):
    Or = oracle_lib.Oracle
    ok = dict(k=4, r=4, c=9, s=8, u=0, log2g=9)
    assert Or.try_create(**ok) == 0
    assert Or.try_create(**{**ok, "s": 7}) == oracle_lib.E_INVAL      # not complete
    assert Or.try_create(**{**ok, "u": 4, "c": 7, "s": 7}) == oracle_lib.E_INVAL  # c*r <= W
    assert Or.try_create(**{**ok, "k": 0}) == oracle_lib.E_INVAL
    assert Or.try_create(**{**ok, "k": 32768}) == oracle_lib.E_INVAL   # 2k must fit a 16-bit AT
    assert Or.try_create(**{**ok, "k": 32767}) == 0
    assert Or.try_create(**{**ok, "s": 10}) == oracle_lib.E_INVAL     # s > c
    assert Or.try_create(**{**ok, "log2g": 0}) == oracle_lib.E_INVAL
    assert Or.try_create(**{**ok, "theta": 0.0}) == oracle_lib.E_INVAL


def test_bh_range_and_uniformity(oracle_lib):
    o = oracle_lib.Oracle(k=4, r=4, c=9, s=8, u=0, log2g=9, seed=9)
    rng = np.random.default_rng(3)
    vals = np.array([o.bh(int(b)) for b in rng.integers(0, 2**32, 40000)])
    assert vals.min() >= 0 and vals.max() < 512
    counts = np.bincount(vals, minlength=512)
    chi2 = ((counts - 40000 / 512) ** 2 / (40000 / 512)).sum()
    assert chi2 < 511 + 6 * math.sqrt(2 * 511)


# --------------------------------------------------------------------------
# Section 3: asynchronous timestamps
# --------------------------------------------------------------------------

def test_at_bit_width_claim():
    """An AT holds 2k+1 values, i.e. ceil(log2(2k+1)) bits, which is one bit
    more than the ceil(log2(k+1)) of an aging counter, for every k."""
    for k in range(1, (1 << 20) + 1):
        w_at = (2 * k).bit_length()            # ceil(log2(2k+1)): 2k+1 is never a power of 2
        w_ac = k.bit_length() if (k + 1) & k else (k + 1).bit_length() - 1
        assert w_at == w_ac + 1
        assert 2 * k < (1 << w_at)
    widths = {k: (2 * k).bit_length() for k in (4, 5, 10, 30, 60, 127, 300)}
    assert widths == {4: 4, 5: 4, 10: 5, 30: 6, 60: 7, 127: 8, 300: 10}


def test_preserve_k9_worked_example(oracle_lib):
    for act, v, e in _golden_rows("at_k9_preserve.txt"):
        assert oracle_lib.preserve_at(9, int(act), int(v)) == int(e), (act, v)


def test_checkat_active_distance(oracle_lib):
    """Alg 1 on the k = 9 circle: an AT set at ACT a is active for window k'
    exactly while the ACT has advanced by less than k'."""
    k = 9
    for a in range(2 * k):
        for adv in range(2 * k):
            act = (a + adv) % (2 * k)
            for kp in range(1, k + 1):
                assert oracle_lib.check_at(k, act, a, kp) == (adv < kp)
    for act in range(2 * k):
        assert not oracle_lib.check_at(k, act, 2 * k, k)


def _positions(o, aip, bip):
    """ATV index and AT index touched by each pair, through the oracle's hash."""
    ncol = 1 << o.c
    out = []
    for a, b in zip(aip.tolist(), bip.tolist()):
        z, x = o.rrh(a)
        i = o.bh(b)
        for j in range(o.r):
            out.append(((z * o.r + j) * ncol + int(x[j]), i))
    return out


@pytest.mark.parametrize("k,log2g", [(1, 4), (2, 4), (3, 4), (5, 4), (9, 5), (13, 4), (4, 3), (150, 9), (300, 4)])
def test_lazy_timestamps_match_exact_timestamps(oracle_lib, k, log2g):
    """After every slice, checkAT(at, k') for every AT and every k' <= k equals
    'set within the last k' slices' from 64-bit exact timestamps (a timestamp
    vector).  Slices include empty ones and run past several ACT wraps; k=13 with
    g=16 and k=9/g=32 cover g < 2k.  k = 150 and the paper's k = 300 need ATs
    wider than a byte (2k >= 256); for them one wrap is run and a spread of
    k' values is checked."""
    o = oracle_lib.Oracle(k=k, r=4, c=8, s=8, u=1, log2g=log2g, seed=k)
    g = 1 << log2g
    ts = np.full(o.pool_size, -(10**9), np.int64)
    rng = np.random.default_rng(k * 100 + log2g)
    hosts = rng.integers(0, 2**32, 6, dtype=np.uint64).astype(np.uint32)
    blocks = np.array([o.block_of(i) for i in range(g)])
    wide = k > 20
    kps = sorted({1, 2, k // 3, k // 2, k - 1, k}) if wide else range(1, k + 1)
    for t in range(2 * k + 25 if wide else 5 * k + 7):
        n = 0 if t % 4 == 3 else int(rng.integers(1, 40))
        if n:
            aip = hosts[rng.integers(0, hosts.size, n)]
            bip = rng.integers(0, 2**32, n, dtype=np.uint64).astype(np.uint32)
            assert o.ingest(aip, bip) == 0
            for atv, i in _positions(o, aip, bip):
                ts[atv * g + i] = t
        assert o.close(k) == 0
        pool = o.pool()
        c0 = t % (2 * k)
        act = (c0 + blocks) % (2 * k)
        touched = np.nonzero(ts > t - 2 * k - 2)[0]
        if wide and touched.size > 300:
            touched = touched[rng.integers(0, touched.size, 300)]
        sample = np.unique(np.concatenate([touched, rng.integers(0, o.pool_size, 200)]))
        for idx in sample.tolist():
            a = int(act[idx % g])
            for kp in kps:
                assert oracle_lib.check_at(k, a, int(pool[idx]), kp) == (ts[idx] >= t - kp + 1), \
                    (t, idx, kp, int(pool[idx]), int(ts[idx]))
        w = o.weights()
        w_exact = (ts.reshape(-1, g) >= t - k + 1).sum(axis=1)
        assert np.array_equal(w, w_exact)


# --------------------------------------------------------------------------
# Window replay: w, AAT and NAT from raw pairs, without any timestamp
# --------------------------------------------------------------------------

def test_window_replay_matches_oracle(oracle_lib):
    cfg = traffic.config_tiny(seed=4, n_slices=7, pairs_per_slice=6000, hosts=1 << 10, planted=3,
                              lo=200, hi=900)
    tr = traffic.generate(cfg)
    k = 3
    o = oracle_lib.Oracle(k=k, r=4, c=8, s=8, u=1, log2g=6, theta=128.0, seed=11)
    g, ncol = o.g, 1 << o.c
    per_slice_pos = []
    for t in range(tr.n_slices):
        o.ingest(tr.aip[t], tr.bip[t])
        per_slice_pos.append(set(_positions(o, tr.aip[t], tr.bip[t])))
        kp = 1 + t % k
        o.close(kp)
        window = set().union(*per_slice_pos[max(0, t - kp + 1): t + 1])
        w_direct = np.zeros(o.n_atv, np.int64)
        for atv, _i in window:
            w_direct[atv] += 1
        assert np.array_equal(o.weights(), w_direct), t
        aat_direct = w_direct.reshape((1 << o.u) * o.r, ncol).sum(axis=1)
        assert np.array_equal(o.aat(), aat_direct)
        hosts = np.unique(np.concatenate([tr.aip[t][:50], tr.planted_hosts]))
        _, _, nat = o.estimate(hosts)
        for a, n_o in zip(hosts.tolist(), nat.tolist()):
            z, x = o.rrh(a)
            rows = [(z * o.r + j) * ncol + int(x[j]) for j in range(o.r)]
            n_d = sum(1 for i in range(g) if all((rw, i) in window for rw in rows))
            assert n_o == n_d


def test_super_threshold_closed_form(oracle_lib):
    for g, theta, T in _golden_rows("super_threshold.txt"):
        o = oracle_lib.Oracle(k=4, r=4, c=9, s=8, u=0, log2g=int(g).bit_length() - 1, theta=float(theta))
        assert o.constants()["T"] == int(T)


# --------------------------------------------------------------------------
# Eq 2 / Eq 4 reduce to the linear estimator for a host alone in the cube
# --------------------------------------------------------------------------

def test_single_host_reduces_to_linear_estimator(oracle_lib):
    g = 1024
    n = 1024
    trials = 120
    est, occ = [], []
    for seed in range(trials):
        o = oracle_lib.Oracle(k=1, r=4, c=9, s=8, u=0, log2g=10, theta=1024.0, seed=seed + 1)
        a = np.array([0x0A000001 + seed], np.uint32)
        b = traffic.fmix32(np.arange(n, dtype=np.uint32) ^ np.uint32(seed * 7919))
        o.ingest(np.repeat(a, n), b)
        o.close(1)
        e, fl, nat = o.estimate(a)
        occ.append(int(nat[0]))
        est.append(float(e[0]))
        # with one host, the other ATVs are empty and every row holds the same
        # positions, so NAT equals the host's weight in every row
        z, x = o.rrh(int(a[0]))
        w = o.weights()
        assert all(w[(z * 4 + j) * 512 + int(x[j])] == nat[0] for j in range(4))
    t = n / g
    occ_mean = np.mean(occ)
    occ_exp = g - g * math.exp(-t)                      # Section 3: E|BIdx|
    occ_sd = math.sqrt(g * math.exp(-t) * (1 - (1 + t) * math.exp(-t)))
    assert abs(occ_mean - occ_exp) < 4 * occ_sd / math.sqrt(trials)
    rel = np.array(est) / n
    se = math.sqrt(math.exp(t) - t - 1) / (t * math.sqrt(g))  # Whang et al. std error
    assert abs(rel.mean() - 1) < 4 * se / math.sqrt(trials) + 2e-3
    assert 0.5 * se < rel.std() < 1.5 * se


# --------------------------------------------------------------------------
# Alg 4: restore set equals the brute-force definition over all 2^32 addresses
# --------------------------------------------------------------------------

@pytest.mark.slow
def test_restore_equals_bruteforce(oracle_lib):
    cfg = traffic.config_tiny(seed=6, n_slices=5, pairs_per_slice=30000, hosts=1 << 11, planted=5,
                              lo=1500, hi=3000)
    tr = traffic.generate(cfg)
    o = oracle_lib.Oracle(k=3, r=4, c=8, s=8, u=1, log2g=10, theta=256.0, seed=21)
    for t in range(tr.n_slices):
        o.ingest(tr.aip[t], tr.bip[t])
        o.close(3)
    U = o.tuple_count()
    assert 0 < U < 5_000_000
    rc, cs, m = o.restore(cap=1 << 20)
    assert rc == 0
    n_bf, bf = o.pin_restore_bruteforce(cap=1 << 20)
    assert n_bf == m
    assert np.array_equal(cs, bf)
    assert np.all(np.diff(cs.astype(np.int64)) > 0)
    # planted hosts far above the threshold in the window are restored
    h, cnt = traffic.window_counts(tr.aip[2:], tr.bip[2:])
    big = h[cnt >= 1000]
    assert big.size > 0 and np.isin(big, cs).all()


def test_restore_budget_and_cap(oracle_lib):
    cfg = traffic.config_tiny(seed=8, n_slices=2, pairs_per_slice=20000, hosts=1 << 10, planted=2,
                              lo=2000, hi=3000)
    tr = traffic.generate(cfg)
    o = oracle_lib.Oracle(k=2, r=4, c=8, s=8, u=1, log2g=10, theta=128.0, seed=2, tuple_budget=10)
    assert o.estimate.__self__ is o
    for t in range(2):
        o.ingest(tr.aip[t], tr.bip[t])
        o.close(2)
    U = o.tuple_count()
    assert U > 10
    rc, _, n = o.restore(cap=1 << 20)
    assert rc == oracle_lib.E_BUDGET and n == U
    o2 = oracle_lib.Oracle(k=2, r=4, c=8, s=8, u=1, log2g=10, theta=128.0, seed=2)
    for t in range(2):
        o2.ingest(tr.aip[t], tr.bip[t])
        o2.close(2)
    rc, cs, m = o2.restore(cap=1 << 20)
    assert rc == 0 and m > 0
    rc, _, n = o2.restore(cap=m - 1)
    assert rc == oracle_lib.E_OVERFLOW and n == m


def test_state_machine(oracle_lib):
    o = oracle_lib.Oracle(k=3, r=4, c=8, s=8, u=1, log2g=6)
    with pytest.raises(RuntimeError):
        o.estimate(np.array([1], np.uint32))
    assert o.close(0) == oracle_lib.E_INVAL
    assert o.close(4) == oracle_lib.E_INVAL
    assert o.close(3) == 0                     # an empty slice still slides the window
    assert o.clock()["t"] == 1
    e, fl, nat = o.estimate(np.array([1, 2], np.uint32))
    assert (nat == 0).all()
    o.ingest(np.array([1], np.uint32), np.array([5], np.uint32))
    with pytest.raises(RuntimeError):          # the closed window is gone once a slice opens
        o.estimate(np.array([1], np.uint32))


# --------------------------------------------------------------------------
# Ground truth: exact distinct counts and the synthetic planted hosts
# --------------------------------------------------------------------------

def test_window_counts_exact():
    cfg = traffic.config_tiny(seed=1, n_slices=3, pairs_per_slice=5000, hosts=300, planted=2,
                              lo=100, hi=400)
    tr = traffic.generate(cfg)
    h, c = traffic.window_counts(tr.aip, tr.bip)
    sets = {}
    for a_s, b_s in zip(tr.aip, tr.bip):
        for a, b in zip(a_s.tolist(), b_s.tolist()):
            sets.setdefault(a, set()).add(b)
    assert sorted(sets) == h.tolist()
    assert [len(sets[a]) for a in h.tolist()] == c.tolist()
    for a, n in zip(tr.planted_hosts.tolist(), tr.planted_card.tolist()):
        assert len(sets[a]) == n


def test_generator_shapes():
    cfg = traffic.config_small(seed=0)
    tr = traffic.generate(cfg)
    assert tr.n_slices == 4
    assert all(a.size == 250_000 and a.dtype == np.uint32 for a in tr.aip)
    assert tr.planted_hosts.size == 32
    assert tr.planted_card.min() >= 1500 and tr.planted_card.max() <= 8000
    tr2 = traffic.generate(cfg)
    assert all(np.array_equal(a, b) for a, b in zip(tr.aip, tr2.aip))
    h, c = traffic.window_counts(tr.aip, tr.bip)
    d = dict(zip(h.tolist(), c.tolist()))
    assert [d[a] for a in tr.planted_hosts.tolist()] == tr.planted_card.tolist()


@pytest.mark.parametrize("k", [3, 5, 10, 60])
def test_ace_oracle_matches_exact_timestamps_and_the_timestamps_windows(oracle_lib, k):
    """The aging counters the paper compares against (ACE, Section 2.3), in the
    oracle: ceil(log2(k+1))-bit counters, set to c = 2^bits - 1 when visited,
    decreased at every slice after the first.  After every close each counter
    equals max(c - age, 0) from exact 64-bit timestamps (0 if never set); the
    k'-weights ACE reports (at least c - k' + 1) equal the asynchronous
    timestamps' for the k' of that close, one k' per slice in turn; and ACE
    rewrites every live counter at every slice while the timestamps' preserve
    examines two blocks of 2k per ATV: about k times fewer."""
    geom = dict(k=k, r=4, c=8, s=8, u=1, log2g=6, seed=k)
    o = oracle_lib.Oracle(**geom)
    a = oracle_lib.AceOracle(**geom)
    assert a.bits == math.ceil(math.log2(k + 1)) and a.cmax == (1 << a.bits) - 1
    g = o.g
    ts = np.full(o.pool_size, -(10**9), np.int64)
    rng = np.random.default_rng(k)
    hosts = rng.integers(0, 2**32, 5, dtype=np.uint64).astype(np.uint32)
    blocks = np.array([o.block_of(i) for i in range(g)])
    touched, aged = [], []
    prev = np.zeros(o.pool_size, np.int64)
    for t in range(2 * k + 7):
        n = 0 if t % 7 == 6 else 30
        aip = hosts[rng.integers(0, hosts.size, n)]
        bip = rng.integers(0, 2**32, n, dtype=np.uint64).astype(np.uint32)
        o.ingest(aip, bip)
        assert a.ingest(aip, bip) == 0
        for atv, i in _positions(o, aip, bip):
            ts[atv * g + i] = t
        kp = 1 + t % k
        o.close(kp)
        assert a.close(kp) == 0
        cnt = a.counters().astype(np.int64)
        expect = np.where(ts >= 0, np.maximum(a.cmax - (t - ts), 0), 0)
        assert np.array_equal(cnt, expect), t
        assert np.array_equal(a.weights(), o.weights()), (t, kp)
        if t > 0:
            aged.append(int(np.count_nonzero(prev)))
        prev = cnt
        c0 = t % (2 * k)
        due = {(2 * k - c0) % (2 * k), (3 * k - c0) % (2 * k)}
        touched.append(int(np.isin(blocks, list(due)).sum()) * o.n_atv)
    assert abs(np.mean(touched) / o.pool_size - 1.0 / k) < 0.5 / k
    assert np.mean(aged) > 0


def test_requery_equals_close_with_that_window(oracle_lib):
    """Re-summarising the closed window for k' gives what closing with k'
    would have given (two oracles fed the same pairs)."""
    tr = traffic.generate(traffic.config_tiny(seed=12, n_slices=6, pairs_per_slice=4000, hosts=1 << 9))
    k = 5
    for kp in range(1, k + 1):
        a = oracle_lib.Oracle(k=k, r=4, c=8, s=8, u=1, log2g=6, seed=1)
        b = oracle_lib.Oracle(k=k, r=4, c=8, s=8, u=1, log2g=6, seed=1)
        for t in range(tr.n_slices):
            a.ingest(tr.aip[t], tr.bip[t])
            b.ingest(tr.aip[t], tr.bip[t])
            a.close(k)
            b.close(kp)
        assert a.requery(kp) == 0
        assert np.array_equal(a.weights(), b.weights()) and np.array_equal(a.aat(), b.aat())
        hosts = np.unique(tr.aip[-1][:200])
        ea, fa, na = a.estimate(hosts)
        eb, fb, nb = b.estimate(hosts)
        assert np.array_equal(na, nb) and np.array_equal(fa, fb) and np.array_equal(ea, eb)
    assert a.requery(0) == oracle_lib.E_INVAL and a.requery(k + 1) == oracle_lib.E_INVAL


# --------------------------------------------------------------------------
# Eq 3 / Eq 4 under load: the bias term UP (product of the rows' P_j)
# --------------------------------------------------------------------------

def test_eq3_expected_nat_and_unbiased_estimate_under_load(oracle_lib):
    """Eq 3: with background load, a position outside the host's BIdx is
    active in all r of its ATVs with probability UP = prod_j P_j, so
    E[NAT] = |BIdx| + UP * (g - |BIdx|), and Eq 4 then estimates n without
    bias.  Two frames with different loads (UP ~ 0.41 and ~ 0.03), hosts of
    80, 160 and 320 distinct bips, 120 seeds.  |BIdx| is the exact count of
    distinct BH values of the host's bips; P_j comes from AAT, which the
    window-replay pin ties to raw pairs.  A sum of the P_j in place of their
    product, a dropped (1 - UP), UP over fewer rows or another frame's AAT
    each moves the mean estimate by at least 40%."""
    from ._scenarios import LOADED, frames_of, loaded_frames  # noqa: F401
    g = 1 << LOADED["log2g"]
    ncol = 1 << LOADED["c"]
    rows = []
    for seed in range(120):
        o = oracle_lib.Oracle(**LOADED, seed=seed + 100)
        aip, bip, targets, tframes, tn, tb = loaded_frames(o, seed)
        o.ingest(aip, bip)
        o.close(1)
        est, fl, nat = o.estimate(targets)
        P = o.aat().astype(np.float64) / (g * ncol)
        for q in range(targets.size):
            z = int(tframes[q])
            assert frames_of(o, targets[q:q + 1])[0] == z
            up = float(np.prod(P[z * o.r:(z + 1) * o.r]))
            bidx = len({o.bh(int(b)) for b in tb[q]})
            rows.append((z, int(tn[q]), int(nat[q]), bidx, up, float(est[q]), int(fl[q])))
    rows = np.array(rows, dtype=np.float64)
    heavy_up = rows[rows[:, 0] == 0, 4].mean()
    assert 0.3 < heavy_up < 0.55 and rows[rows[:, 0] == 1, 4].mean() < 0.06
    for z in (0, 1):
        for n in (80, 160, 320):
            r = rows[(rows[:, 0] == z) & (rows[:, 1] == n)]
            dev = r[:, 2] - (r[:, 3] + r[:, 4] * (g - r[:, 3]))
            assert abs(dev.mean()) < 4 * dev.std() / math.sqrt(len(r)) + 0.5, (z, n, dev.mean())
            rel = r[:, 5] / n
            assert np.isfinite(rel).all()
            assert abs(rel.mean() - 1.0) < 4 * rel.std() / math.sqrt(len(r)) + 0.02, (z, n, rel.mean())
            assert (r[:, 6] == 0).all()          # no SAT / NEG / SUPER flag at these sizes (theta 1024)


def test_eq4_unseen_hosts_estimate_zero_and_flag_negatives(oracle_lib):
    """A host never seen has n = 0; at heavy load its NAT counts only
    false-active positions, so Eq 4 is zero on average and negative whenever
    NAT < g * UP, which then carries AT_F_NEG (reading of the undefined edge)."""
    from ._scenarios import LOADED, loaded_frames, unseen_hosts
    g = 1 << LOADED["log2g"]
    o = oracle_lib.Oracle(**LOADED, seed=7)
    aip, bip, *_ = loaded_frames(o, 3)
    o.ingest(aip, bip)
    o.close(1)
    hosts = unseen_hosts(o, 3)
    assert hosts.size == 2000 and not np.isin(hosts, aip).any()
    est, fl, nat = o.estimate(hosts)
    up = float(np.prod(o.aat()[:o.r].astype(np.float64) / (g << o.c)))
    sd = math.sqrt(g * up / (1 - up))
    assert abs(est.mean()) < 4 * sd / math.sqrt(hosts.size) + 1.0
    neg = (fl & oracle_lib.F_NEG) != 0
    assert 0.3 < neg.mean() < 0.7
    assert np.array_equal(neg, est < 0)
    assert not (fl & oracle_lib.F_SAT).any()


def test_eq4_saturated_host_is_clamped_to_g_minus_one(oracle_lib):
    """A host whose every AT position is active (NAT = g) makes Eq 4's
    logarithm infinite; it is estimated as if NAT were g - 1 and flagged
    AT_F_SAT.  A second host of the same frame with exactly g - 1 active
    positions must get the same estimate without the flag."""
    from ._scenarios import CLAMP, clamp_hosts
    o = oracle_lib.Oracle(**CLAMP, seed=4)
    aip, bip, h_all, h_most, _ = clamp_hosts(o)
    o.ingest(aip, bip)
    o.close(CLAMP["k"])
    est, fl, nat = o.estimate(np.array([h_all, h_most], np.uint32))
    g = 1 << CLAMP["log2g"]
    assert nat.tolist() == [g, g - 1]
    assert fl[0] & oracle_lib.F_SAT and not fl[1] & oracle_lib.F_SAT
    assert np.isfinite(est).all() and est[0] == est[1] and est[0] > 0


def test_eq4_full_frame_gives_infinity(oracle_lib):
    """When every AT of every row of the frame is active, P_j = 1 for all rows,
    UP = 1 and Eq 4's denominator g * (1 - UP) is zero: +inf with AT_F_SAT."""
    from ._scenarios import FULL, full_frame
    o = oracle_lib.Oracle(**FULL, seed=2)
    aip, bip, probe = full_frame()
    o.ingest(aip, bip)
    o.close(FULL["k"])
    g = 1 << FULL["log2g"]
    assert (o.pool() < 2 * FULL["k"]).all()          # every AT set in this slice
    assert (o.aat() == g << FULL["c"]).all()
    est, fl, nat = o.estimate(probe)
    assert np.isinf(est).all() and (est > 0).all()
    assert ((fl & oracle_lib.F_SAT) != 0).all() and ((fl & oracle_lib.F_SUPER) != 0).all()
    assert (nat == g).all()


# --------------------------------------------------------------------------
# Features of the learned correction against exact per-pair timestamps
# --------------------------------------------------------------------------

@pytest.mark.parametrize("k,log2g", [(5, 6), (12, 5), (3, 7)])
def test_features_age_histogram_matches_exact_timestamps(oracle_lib, k, log2g):
    """e_i = the largest age over a host's r ATs at position i when all r were
    set within the last k slices: with 64-bit exact timestamps of every AT
    (last slice in which some pair touched it) the histogram of e_i over
    positions must equal feat[d] * g, its prefix sums NAT(k') of Alg 5 for
    every k' <= k, feat[62] = k/64, feat[63] the mean P_j of the frame and
    feat[61] the clipped log of the plain estimate."""
    o = oracle_lib.Oracle(k=k, r=4, c=8, s=8, u=1, log2g=log2g, seed=30 + k)
    g, ncol = o.g, 1 << o.c
    ts = np.full(o.pool_size, -(10**9), np.int64)
    rng = np.random.default_rng(k)
    hosts = rng.integers(0, 2**32, 8, dtype=np.uint64).astype(np.uint32)
    # background hosts share the targets' ATVs, so a position's r ATs are set
    # in different slices and the largest age differs from the others
    bg = rng.integers(0, 2**32, 3000, dtype=np.uint64).astype(np.uint32)
    T = 3 * k + 4
    for t in range(T):
        n = 0 if t % 5 == 4 else int(rng.integers(20, 4 * g))
        if n:
            aip = np.concatenate([hosts[rng.integers(0, hosts.size, n)], bg[rng.integers(0, bg.size, 8 * n)]])
            bip = rng.integers(0, 2**32, aip.size, dtype=np.uint64).astype(np.uint32)
            o.ingest(aip, bip)
            for atv, i in _positions(o, aip, bip):
                ts[atv * g + i] = t
        o.close(k)
    t = T - 1
    feat = o.features(hosts)
    est, _, _ = o.estimate(hosts)
    aat = o.aat().astype(np.float64) / (g * ncol)
    for q, a in enumerate(hosts.tolist()):
        z, x = o.rrh(a)
        rows = [(z * o.r + j) * ncol + int(x[j]) for j in range(o.r)]
        last = np.stack([ts[rw * g:(rw + 1) * g] for rw in rows])      # r x g last-set slices
        ages = t - last
        live = (ages < k).all(axis=0)
        e = ages.max(axis=0)[live]
        hist = np.bincount(e, minlength=k)[:k]
        assert np.array_equal((feat[q, :min(k, 61)] * g).astype(np.int64), hist[:61]), (a, hist)
        assert (feat[q, min(k, 61):61] == 0).all()
        assert feat[q, 62] == np.float32(k / 64)
        assert feat[q, 63] == np.float32(aat[z * o.r:(z + 1) * o.r].sum() / o.r)
        lp = min(math.log1p(max(float(est[q]), 0.0)), 20.0) / 16
        assert abs(float(feat[q, 61]) - lp) <= 1e-6 * max(lp, 1e-30) + 1e-7
    for kp in range(1, k + 1):
        o.requery(kp)
        _, _, nat = o.estimate(hosts)
        pref = np.rint(feat[:, :kp].astype(np.float64) * g).sum(axis=1)
        assert np.array_equal(pref.astype(np.int64), nat.astype(np.int64)), kp


# --------------------------------------------------------------------------
# Per-ATV age histograms (one read of the pool serves every window k' <= k)
# --------------------------------------------------------------------------

@pytest.mark.parametrize("k,log2g", [(5, 6), (12, 5), (40, 4)])
def test_atv_age_histograms_match_exact_timestamps(oracle_lib, k, log2g):
    """Bin a of an ATV's histogram counts its ATs last set exactly a slices
    before the close (a < k): checked against exact 64-bit timestamps of
    every AT, at a close inside the first 2k slices and at the last.  Its
    prefix sums are the k'-weights and AAT that oat_requery computes with
    Alg 1 for every k' <= k (g = 16 < 2k in the last case, where some blocks
    are empty)."""
    o = oracle_lib.Oracle(k=k, r=4, c=8, s=8, u=1, log2g=log2g, seed=50 + k)
    g, ncol = o.g, 1 << o.c
    ts = np.full(o.pool_size, -(10**9), np.int64)
    rng = np.random.default_rng(100 + k)
    hosts = rng.integers(0, 2**32, 300, dtype=np.uint64).astype(np.uint32)
    T = 2 * k + 7
    checks = {k + 2, T - 1}
    for t in range(T):
        n = 0 if t % 5 == 4 else int(rng.integers(10, 2 * g))
        if n:
            aip = hosts[rng.integers(0, hosts.size, n)]
            bip = rng.integers(0, 2**32, n, dtype=np.uint64).astype(np.uint32)
            o.ingest(aip, bip)
            for atv, i in _positions(o, aip, bip):
                ts[atv * g + i] = t
        o.close(k)
        if t not in checks:
            continue
        ages = (t - ts).reshape(o.n_atv, g)
        exact = np.stack([(ages == a).sum(axis=1) for a in range(k)], axis=1)
        h = o.age_hist()
        assert h.shape == (o.n_atv, k)
        assert np.array_equal(h, exact), t
        assert h.sum() > 0
        for kp in range(1, k + 1):
            assert o.requery(kp) == 0
            w = o.weights()
            assert np.array_equal(w, exact[:, :kp].sum(axis=1)), (t, kp)
            assert np.array_equal(o.aat(), w.reshape(-1, ncol).sum(axis=1).astype(np.uint64)), (t, kp)
        assert o.requery(k) == 0
