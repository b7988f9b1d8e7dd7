"""Pins for the oracle's generator and LSH functions (CPU only).

Nothing here retypes the oracle's formulas: the generator is pinned by
published known-answer values, SRP bits by exact rational arithmetic
(fractions) and by the sign-geometry of projections, and both hash families by
their collision statistics (1 - theta/pi per SRP bit, Jaccard per MinHash,
the property the paper's analysis assumes of an LSH family)."""
import math
import os
from fractions import Fraction

import numpy as np
import pytest

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def test_splitmix64_known_answers(orc):
    vals = [int(l, 16) for l in open(os.path.join(GOLDEN, "splitmix64_seed0.txt"))
            if l.strip() and not l.startswith("#")]
    assert [orc.sm64(0, i) for i in range(3)] == vals


def test_mix64_is_a_bijection_on_samples(orc):
    rng = np.random.default_rng(5)
    xs = [int(v) for v in rng.integers(0, 2**63, 2000, dtype=np.int64)]
    ys = {orc.mix64(x) for x in xs}
    assert len(ys) == len(set(xs))


def test_hyperplane_entries_binomial(orc):
    """Entries are (Binomial(64, 1/2) - 32) / 4: a chi-square test against the
    exact binomial pmf, plus exact representability in bf16."""
    w = orc.hyperplanes(7, 64, 512).ravel()
    k = np.round(w * 4 + 32).astype(int)
    assert np.all(w * 4 == np.round(w * 4)) and np.all(np.abs(w) <= 8)
    obs = np.bincount(k, minlength=65).astype(float)
    pmf = np.array([math.comb(64, i) for i in range(65)], dtype=float) / 2.0**64
    exp = pmf * w.size
    m = exp > 5
    chi2 = (((obs[m] - exp[m]) ** 2) / exp[m]).sum()
    assert chi2 < 2.0 * m.sum() + 30  # far in the tail only if wrong
    # bf16 round trip: value * 2^16 bits fit in 8 significant bits
    f32 = w.astype(np.float32)
    bits = f32.view(np.uint32)
    assert np.all((bits & 0xFFFF) == 0)


def _exact_sign(x, w):
    s = sum(Fraction(float(a)) * Fraction(float(b)) for a, b in zip(x, w))
    return (s > 0) - (s < 0)


def test_exact_dot_sign_cancellation(orc):
    big = 2.0**60
    assert orc.exact_dot_sign([big, 1.0, -big], [1.0, 1.0, 1.0]) == 1
    assert orc.exact_dot_sign([big, -1.0, -big], [1.0, 1.0, 1.0]) == -1
    assert orc.exact_dot_sign([big, 2.0**-60, -big], [1.0, 1.0, 1.0]) == 1
    assert orc.exact_dot_sign([1.0, -1.0], [3.0, 3.0]) == 0
    assert orc.exact_dot_sign([0.0, 0.0], [1.0, -1.0]) == 0


def test_exact_dot_sign_random_vs_fractions(orc):
    rng = np.random.default_rng(11)
    for _ in range(300):
        n = int(rng.integers(1, 12))
        e = rng.integers(-70, 70, n)
        x = rng.choice([-1, 1], n) * np.ldexp(rng.integers(1, 2**24, n).astype(float), e - 24)
        w = rng.integers(-32, 33, n) / 4.0
        # plant exact cancellations (inputs stay fp32-representable, as the
        # stored data always is, so every product is exact in FP64)
        if n >= 2 and rng.random() < 0.5:
            x[1], w[1] = -x[0], w[0]
        assert orc.exact_dot_sign(x, w) == _exact_sign(x, w)


def test_srp_bits_are_exact_signs(orc):
    """Codes of random fp32 rows equal the exact rational sign of every
    projection, including rows built to project exactly onto 0 and onto
    +-2^-60."""
    rng = np.random.default_rng(3)
    K, L, d, seed = 4, 3, 24, 99
    w = orc.hyperplanes(seed, K * L, d)
    x = rng.standard_normal((20, d)).astype(np.float32).astype(np.float64)
    # exact zero on hyperplane 0: x = w1 * e0 - w0 * e1 style construction
    h = 5
    i, j = np.nonzero(w[h])[0][:2]
    x[0] = 0.0
    x[0, i], x[0, j] = w[h, j], -w[h, i]
    # a projection of exactly +2^-60 (w entries are multiples of 1/4)
    x[1] = x[0]
    k_ = [q for q in np.nonzero(w[h])[0] if q not in (i, j)][0]
    x[1, k_] = 2.0**-60 / w[h, k_]
    x[2] = -x[1]
    codes = orc.srp_codes(x, seed, K, L, w=w)
    for r in range(x.shape[0]):
        for t in range(L):
            for b in range(K):
                s = _exact_sign(x[r], w[t * K + b])
                assert ((codes[r, t] >> b) & 1) == (1 if s > 0 else 0)
    assert (codes[0, h // K] >> (h % K)) & 1 == 0
    assert (codes[1, h // K] >> (h % K)) & 1 == 1
    assert (codes[2, h // K] >> (h % K)) & 1 == 0


def test_srp_scale_and_negation(orc):
    rng = np.random.default_rng(4)
    K, L, d, seed = 8, 4, 64, 5
    w = orc.hyperplanes(seed, K * L, d)
    x = rng.standard_normal((50, d)).astype(np.float32).astype(np.float64)
    c = orc.srp_codes(x, seed, K, L, w=w)
    assert np.array_equal(c, orc.srp_codes(x * 2.0**40, seed, K, L, w=w))
    assert np.array_equal(c, orc.srp_codes(x * 2.0**-40, seed, K, L, w=w))
    neg = orc.srp_codes(-x, seed, K, L, w=w)
    # random data: no projection is exactly zero, so negation flips every bit
    assert np.array_equal(neg, (~c) & ((1 << K) - 1))
    zero = orc.srp_codes(np.zeros((1, d)), seed, K, L, w=w)
    assert np.all(zero == 0)


def test_srp_collision_rate_is_one_minus_angle_over_pi(orc):
    """Per-bit collision probability of signed random projections is
    1 - theta/pi (the 'collision probability equals similarity' property)."""
    rng = np.random.default_rng(8)
    d, H = 96, 8192
    w = orc.hyperplanes(17, H, d)
    for theta in (0.3, 0.9, 1.6, 2.4):
        u = rng.standard_normal(d)
        u /= np.linalg.norm(u)
        v = rng.standard_normal(d)
        v -= v.dot(u) * u
        v /= np.linalg.norm(v)
        y = np.cos(theta) * u + np.sin(theta) * v
        cx = orc.srp_codes(u[None, :], 17, 1, H, w=w)
        cy = orc.srp_codes(y[None, :], 17, 1, H, w=w)
        rate = np.mean(cx == cy)
        p = 1 - theta / math.pi
        sd = math.sqrt(p * (1 - p) / H)
        assert abs(rate - p) < 5 * sd + 0.01, (theta, rate, p)


def _mh(orc, sets, K, L, b, seed=1):
    offs = np.zeros(len(sets) + 1, dtype=np.uint64)
    offs[1:] = np.cumsum([len(s) for s in sets])
    items = np.concatenate([np.asarray(s, dtype=np.uint64) for s in sets]) if offs[-1] else np.zeros(0, np.uint64)
    return orc.minhash_codes(items, offs, seed, K, L, b)


def test_minhash_set_semantics(orc):
    rng = np.random.default_rng(2)
    s = rng.integers(0, 2**63, 50, dtype=np.int64).astype(np.uint64)
    perm = rng.permutation(s)
    dup = np.concatenate([s, s[:17]])
    c = _mh(orc, [s, perm, dup, s[:49], [], []], 3, 16, 20)
    assert np.array_equal(c[0], c[1]) and np.array_equal(c[0], c[2])
    assert not np.array_equal(c[0], c[3])
    assert np.array_equal(c[4], c[5])          # empty sets agree
    assert np.all(c < (1 << 20))


@pytest.mark.parametrize("K", [1, 2])
def test_minhash_collision_rate_is_jaccard_power(orc, K):
    """Per table, two sets collide with probability J^K (MinHash collision
    probability J, concatenated K times) up to a 2^-b fold collision term."""
    rng = np.random.default_rng(9 + K)
    pool = rng.choice(2**40, 400, replace=False).astype(np.uint64)
    a, b = pool[:200], pool[100:300]          # |A & B| = 100, |A | B| = 300
    J = 100 / 300
    L = 6000
    c = _mh(orc, [a, b], K, L, 32, seed=21)
    rate = np.mean(c[0] == c[1])
    p = J ** K
    sd = math.sqrt(p * (1 - p) / L)
    assert abs(rate - p) < 5 * sd, (rate, p)
