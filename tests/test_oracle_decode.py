"""Pins for the oracle's decode (Algorithm 3 and Algorithm 2).

The oracle decodes from the definition: the k smallest keys
(-m(x), c*(x), id).  Here that is pinned against brute force of what
Algorithm 3 does: the sequence of (cell, point) visits in the relaxation's
order (cells by descending count, ties by ascending cell id, points by
ascending id) fixes each point's completion position, the position of its
R-th visit; the reported points are the first k by completion position,
each scored with the count of the cell it completed in.  Further pins from
the paper's statements: Algorithm 3 equals Algorithm 2 run with decreasing
thresholds, always returns min(k, N) distinct points, and, with tests of
true positive rate p, reports a positive point with probability p^R
(Lemma 1)."""
import math

import numpy as np
import pytest


def _grid(orc, rng, N, R, B, L):
    g = orc.groups(N, R, B, int(rng.integers(0, 2**31)))
    cnt = rng.integers(0, L + 1, R * B).astype(np.uint8)
    # plant ties and zeros
    if rng.random() < 0.5:
        cnt[rng.random(R * B) < 0.5] = 0
    return g, cnt


def brute_relaxation(cnt, g, B, k):
    """Completion order of every point under the relaxation's visit sequence
    (numpy; no keys): ids and scores of the first k, padded."""
    R, N = g.shape
    cell_of = (np.arange(R)[:, None] * B + g).ravel()     # visit (r, x) -> cell
    point_of = np.tile(np.arange(N), R)
    # visit order: count descending, cell ascending, point ascending
    order = np.lexsort((point_of, cell_of, -cnt[cell_of].astype(np.int64)))
    seen = np.zeros(N, dtype=np.int64)
    done_at = np.full(N, -1, dtype=np.int64)
    for pos, v in enumerate(order):
        x = point_of[v]
        seen[x] += 1
        if seen[x] == R:
            done_at[x] = pos
    first = np.argsort(done_at, kind="stable")[:k]
    ids = np.full(k, 0xFFFFFFFF, dtype=np.uint32)
    sc = np.zeros(k, dtype=np.uint32)
    ids[:len(first)] = first
    sc[:len(first)] = cnt[cell_of[order[done_at[first]]]]
    return ids, sc


def test_decode_equals_brute_relaxation_random(orc):
    rng = np.random.default_rng(123)
    for _ in range(1500):
        N = int(rng.integers(1, 40))
        R = int(rng.integers(1, 5))
        B = int(rng.integers(1, min(N, 6) + 1))
        L = int(rng.integers(1, 6))
        k = int(rng.integers(1, N + 4))
        g, cnt = _grid(orc, rng, N, R, B, L)
        a = orc.decode(cnt, g, B, k)
        b = brute_relaxation(cnt, g, B, k)
        assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])
        n = min(k, N)
        assert len(set(a[0][:n].tolist())) == n and np.all(a[0][:n] < N)
        assert np.all(a[0][n:] == 0xFFFFFFFF) and np.all(a[1][n:] == 0)
        assert np.all(np.diff(a[1][:n].astype(int)) <= 0)


def test_decode_equals_brute_relaxation_larger(orc):
    rng = np.random.default_rng(7)
    for _ in range(40):
        N, R, B, L = 3000, int(rng.integers(2, 6)), int(rng.integers(20, 300)), 16
        g = orc.groups(N, R, B, int(rng.integers(0, 2**31)))
        cnt = np.minimum(rng.poisson(1.0, R * B), L).astype(np.uint8)
        for k in (1, 10, 100):
            a = orc.decode(cnt, g, B, k)
            b = brute_relaxation(cnt, g, B, k)
            assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])


def test_query_many_equals_per_query_decode(orc):
    """The batched oracle query (counts through the reverse index, then the
    decode, queries spread over threads) equals counts + decode query by
    query, with one thread and with several."""
    rng = np.random.default_rng(44)
    N, L, R, B, nbits = 500, 6, 3, 20, 5
    codes = rng.integers(0, 1 << nbits, (N, L)).astype(np.uint32)
    g = orc.groups(N, R, B, 9)
    offs, cells = orc.build_lists(codes, g, B, nbits)
    qc = rng.integers(0, 1 << nbits, (64, L)).astype(np.uint32)
    cnt = orc.counts(offs, cells, qc, R * B, nbits)
    want = [orc.decode(cnt[i], g, B, 12) for i in range(64)]
    ix = orc.OracleIndex.__new__(orc.OracleIndex)
    ix.offsets, ix.cells, ix.g, ix.L, ix.nbits, ix.N, ix.R, ix.B = offs, cells, g, L, nbits, N, R, B
    before = orc.get_threads()
    try:
        for th in (1, 4):
            orc.set_threads(th)
            ids, sc = ix.query_codes(qc, 12)
            for i in range(64):
                assert np.array_equal(ids[i], want[i][0]) and np.array_equal(sc[i], want[i][1])
    finally:
        orc.set_threads(before)


def test_alg3_is_alg2_with_decreasing_threshold(orc):
    """For every threshold t whose Algorithm-2 output has at most k points,
    those points are exactly the reported points with score >= t."""
    rng = np.random.default_rng(5)
    for _ in range(200):
        N, R, B, L = int(rng.integers(10, 200)), int(rng.integers(1, 4)), int(rng.integers(2, 9)), 6
        g, cnt = _grid(orc, rng, N, R, B, L)
        k = int(rng.integers(1, N + 1))
        ids, sc = orc.decode(cnt, g, B, k)
        for t in range(L + 1):
            rep = set(np.nonzero(orc.query_fixed_t(cnt, g, B, t))[0].tolist())
            if len(rep) <= k:
                got = {int(i) for i, s in zip(ids, sc) if s >= t and i != 0xFFFFFFFF}
                assert got == rep


def test_prefix_property(orc):
    rng = np.random.default_rng(9)
    for _ in range(100):
        N, R, B, L = int(rng.integers(5, 60)), int(rng.integers(1, 4)), int(rng.integers(1, 6)), 4
        g, cnt = _grid(orc, rng, N, R, B, L)
        full = orc.decode(cnt, g, B, N)
        for k in range(1, N + 1, 3):
            a = orc.decode(cnt, g, B, k)
            assert np.array_equal(a[0], full[0][:k])


def test_special_cases(orc):
    rng = np.random.default_rng(2)
    # B = 1: every point is in the single cell of every repetition -> ids 0..k-1
    N, R = 30, 3
    g = orc.groups(N, R, 1, 1)
    cnt = rng.integers(0, 5, R).astype(np.uint8)
    ids, sc = orc.decode(cnt, g, 1, 7)
    assert ids.tolist() == list(range(7)) and np.all(sc == cnt.min())
    # R = 1: cells in (count desc, id asc) order, members ascending
    N, B = 50, 6
    g = orc.groups(N, 1, B, 3)
    cnt = np.array([2, 5, 2, 0, 5, 1], dtype=np.uint8)
    ids, sc = orc.decode(cnt, g, B, N)
    expect = []
    for b in sorted(range(B), key=lambda b: (-int(cnt[b]), b)):
        expect += sorted(np.nonzero(g[0] == b)[0].tolist())
    assert ids.tolist() == expect
    # k > N pads
    ids, sc = orc.decode(cnt, g, B, N + 3)
    assert ids[-3:].tolist() == [0xFFFFFFFF] * 3


def test_lemma1_true_positive_rate(orc):
    """Lemma 1: with i.i.d. tests of true positive rate p, Algorithm 2 reports a
    positive point with probability p^R (exactly, for a lone positive)."""
    rng = np.random.default_rng(31)
    N, R, B, p, q = 400, 3, 20, 0.8, 0.05
    hits = 0
    trials = 3000
    fp = 0
    for it in range(trials):
        g = orc.groups(N, R, B, it)
        pos = 17
        cnt = (rng.random(R * B) < q).astype(np.uint8)
        for r in range(R):
            cnt[r * B + g[r, pos]] = 1 if rng.random() < p else 0
        rep = orc.query_fixed_t(cnt, g, B, 1)
        hits += rep[pos]
        fp += rep[:pos].sum() + rep[pos + 1:].sum()
    rate = hits / trials
    assert abs(rate - p**R) < 5 * math.sqrt(p**R * (1 - p**R) / trials)
    # false report bound of Lemma 1 for |K| = 1
    Kn = 1
    bound = (q * (math.e * N * (B - 1) / (B * (N - 1))) ** Kn
             + p * (1 - (N * (B - 1) / (math.e * B * (N - 1))) ** Kn)) ** R
    assert fp / (trials * (N - 1)) <= bound
