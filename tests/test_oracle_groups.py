"""Pins for the oracle's group design (Algorithm 1): each repetition is a
random permutation, point x joins group P_r(x) mod B, so every point is in
exactly one group per repetition and groups hold floor(N/B) or ceil(N/B)."""
import numpy as np
import pytest


@pytest.mark.parametrize("N", [1, 2, 3, 4, 5, 17, 64, 65, 1000, 4097])
def test_permutation_is_bijection(orc, N):
    for r in range(3):
        img = sorted(orc.permute(N, r, 77, x) for x in range(N))
        assert img == list(range(N))


@pytest.mark.parametrize("N,B", [(10, 1), (10, 3), (1000, 7), (4097, 64), (100, 100)])
def test_groups_balanced_and_partition(orc, N, B):
    R = 4
    g = orc.groups(N, R, B, 12)
    assert g.shape == (R, N) and g.max() < B
    for r in range(R):
        sizes = np.bincount(g[r], minlength=B)
        assert sizes.min() >= N // B and sizes.max() <= -(-N // B)
        # exact sizes: group b has ceil for b < N mod B (positions b, b+B, ...)
        expect = np.array([N // B + (1 if b < N % B else 0) for b in range(B)])
        assert np.array_equal(sizes, expect)
    off, mem = orc.members(g, B)
    for r in range(R):
        assert sorted(mem[r].tolist()) == list(range(N))
        for b in range(B):
            seg = mem[r, off[r, b]:off[r, b + 1]]
            assert np.all(np.diff(seg.astype(np.int64)) > 0)
            assert np.all(g[r, seg] == b)


def test_repetitions_independent(orc):
    """Different repetitions use different permutations: the joint histogram of
    (g_0(x), g_1(x)) is close to uniform (chi-square), as independent random
    assignments would give."""
    N, B = 40000, 20
    g = orc.groups(N, 2, B, 3)
    assert not np.array_equal(g[0], g[1])
    joint = np.bincount(g[0] * B + g[1], minlength=B * B).astype(float)
    exp = N / (B * B)
    chi2 = ((joint - exp) ** 2 / exp).sum()
    assert chi2 < (B * B) + 6 * np.sqrt(2 * B * B)


@pytest.mark.parametrize("N0,B", [(10, 1), (10, 3), (1000, 7), (4097, 64), (300, 300)])
def test_stream_groups_blocks(orc, N0, B):
    """Points arriving after the build: every complete block of B arrivals
    puts exactly one point into each group of each repetition, so group sizes
    stay within two of each other whatever the number of arrivals; the
    assignment of a point does not depend on how arrivals are batched."""
    R, seed = 3, 21
    g0 = orc.groups(N0, R, B, seed)
    n = 5 * B + (B // 2)
    g1 = orc.stream_groups(N0, R, B, seed, N0, n)
    assert g1.shape == (R, n) and g1.max() < B
    for r in range(R):
        for j in range(n // B):
            assert sorted(g1[r, j * B:(j + 1) * B].tolist()) == list(range(B))
        for m in range(0, n + 1, max(1, B // 3)):
            sizes = np.bincount(np.concatenate([g0[r], g1[r, :m]]), minlength=B)
            assert sizes.max() - sizes.min() <= 2
    # the same points in two batches get the same groups
    a = orc.stream_groups(N0, R, B, seed, N0, n // 3)
    b = orc.stream_groups(N0, R, B, seed, N0 + n // 3, n - n // 3)
    assert np.array_equal(np.concatenate([a, b], axis=1), g1)


def test_stream_groups_independent_across_repetitions_and_blocks(orc):
    """The permutations differ between repetitions and between blocks: the
    joint histogram of (g_0(x), g_1(x)) over many blocks is close to uniform
    (chi-square), and consecutive blocks are not the same permutation."""
    B, nblk = 20, 2000
    g = orc.stream_groups(0, 2, B, 8, 0, B * nblk)
    assert not np.array_equal(g[0, :B], g[0, B:2 * B])
    joint = np.bincount(g[0] * B + g[1], minlength=B * B).astype(float)
    exp = B * nblk / (B * B)
    chi2 = ((joint - exp) ** 2 / exp).sum()
    assert chi2 < (B * B) + 6 * np.sqrt(2 * B * B)


def test_oracle_insert_equals_groups_of_stream(orc):
    """OracleIndex.insert: the first N0 points keep Algorithm 1's groups, the
    arrivals take the stream groups, and the reverse index equals the one
    built from the codes and groups of all points."""
    rng = np.random.default_rng(4)
    X = rng.standard_normal((700, 16)).astype(np.float32)
    oi = orc.OracleIndex(orc.SRP_F32, X[:500], 6, 5, 3, 25, 9)
    g_before = oi.g.copy()
    oi.insert(X[500:620])
    oi.insert(X[620:])
    assert oi.N == 700 and np.array_equal(oi.g[:, :500], g_before)
    assert np.array_equal(oi.g[:, 500:], orc.stream_groups(500, 3, 25, 9, 500, 200))
    codes = orc.srp_codes(X.astype(np.float64), 9, 6, 5)
    offs, cells = orc.build_lists(codes, oi.g, 25, 6)
    assert np.array_equal(offs, oi.offsets) and np.array_equal(cells, oi.cells)
