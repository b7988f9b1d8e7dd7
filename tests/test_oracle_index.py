"""Pins for the oracle's reverse index and cell counts: counts through the
reverse index equal the distance-sensitive Bloom filter definition computed
without any index; an indexed point queried as itself scores L in all R of its
cells; per-repetition count sums equal the number of distinct groups per
matching bucket."""
import numpy as np
import pytest

from workloads import synth


def _rand_codes(rng, N, L, nbits, spread):
    return rng.integers(0, min(1 << nbits, spread), (N, L)).astype(np.uint32)


@pytest.mark.parametrize("N,L,R,B,nbits", [(50, 3, 2, 5, 3), (300, 6, 3, 17, 4),
                                           (1000, 4, 4, 64, 8), (7, 2, 3, 7, 2)])
def test_counts_index_equals_definition(orc, N, L, R, B, nbits):
    rng = np.random.default_rng(N + L)
    codes = _rand_codes(rng, N, L, nbits, 1 << nbits)
    g = orc.groups(N, R, B, 4)
    offs, cells = orc.build_lists(codes, g, B, nbits)
    q = np.concatenate([codes[:5], _rand_codes(rng, 10, L, nbits, 1 << nbits)])
    c1 = orc.counts(offs, cells, q, R * B, nbits)
    c2 = orc.counts_brute(codes, g, B, q)
    assert np.array_equal(c1, c2)
    assert c1.max() <= L
    # a query equal to an indexed point: all R of its cells count L
    for i in range(5):
        for r in range(R):
            assert c1[i, r * B + g[r, i]] == L
    # per-repetition sums: distinct groups among points in each matching bucket
    for i in range(q.shape[0]):
        for r in range(R):
            tot = 0
            for t in range(L):
                pts = np.nonzero(codes[:, t] == q[i, t])[0]
                tot += len(np.unique(g[r, pts]))
            assert c1[i, r * B:(r + 1) * B].sum() == tot


def test_lists_sorted_distinct(orc):
    rng = np.random.default_rng(1)
    N, L, R, B, nbits = 500, 4, 3, 20, 5
    codes = _rand_codes(rng, N, L, nbits, 6)
    g = orc.groups(N, R, B, 8)
    offs, cells = orc.build_lists(codes, g, B, nbits)
    for t in range(L):
        for h in range(1 << nbits):
            seg = cells[offs[t, h]:offs[t, h + 1]].astype(np.int64)
            assert np.all(np.diff(seg) > 0)
            expect = set()
            for x in np.nonzero(codes[:, t] == h)[0]:
                for r in range(R):
                    expect.add(r * B + int(g[r, x]))
            assert set(seg.tolist()) == expect


def test_end_to_end_identical_query_is_returned(orc):
    """A query identical to an indexed point has all its groups positive at
    the top count and is returned (dense SRP and MinHash)."""
    X, _, _ = synth.dense_gmm(N=2000, d=32, n_centres=40, nq=1)
    idx = orc.OracleIndex(orc.SRP_F32, X, 8, 6, 3, 40, seed=5)
    Q = X[[3, 99, 1500]]
    ids, sc = idx.query(Q, 10)
    for i, x in enumerate([3, 99, 1500]):
        assert x in ids[i] and sc[i][list(ids[i]).index(x)] == 6
    it, of, _, _, _ = synth.genome(n_base=500, nq=1)
    idx = orc.OracleIndex(orc.MINHASH_U64, (it, of), 2, 8, 3, 30, seed=2,
                          bucket_bits=16)
    sel = [0, 10, 777]
    qit = np.concatenate([it[of[s]:of[s + 1]] for s in sel])
    qof = np.zeros(4, dtype=np.uint64)
    qof[1:] = np.cumsum([of[s + 1] - of[s] for s in sel])
    ids, sc = idx.query((qit, qof), 5)
    for i, x in enumerate(sel):
        assert x in ids[i] and sc[i][list(ids[i]).index(x)] == 8


def test_recall_sanity_tiny(orc):
    """On a tiny well-separated mixture FLINNG's top-10 holds the exact nearest
    neighbour for most queries (recall sanity, not parity)."""
    from workloads import truth
    X, Q, _ = synth.dense_gmm(N=3000, d=64, n_centres=300, sigma=0.05, nq=50)
    idx = orc.OracleIndex(orc.SRP_F32, X, 10, 16, 3, 100, seed=1)
    ids, _ = idx.query(Q, 10)
    ti, _ = truth.cosine_topk(X, Q, 1)
    assert truth.recall_at(ids, ti[:, 0]) >= 0.8
