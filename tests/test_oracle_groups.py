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
