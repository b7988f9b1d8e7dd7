"""GPU parity: the HIP library, called through its C ABI, against the CPU
oracle on the same seeded inputs, layer by layer and bit-exact: hash codes,
the exported index (groups and reverse-index lists), per-cell counts, and the
decoded ids and scores.  Sizes span several tiles and ragged tails."""
import numpy as np
import pytest

import oracle
from gpu_common import build_both, log, oracle_query, random_sets, scaled, subset_sets
from workloads import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def fl():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a ROCm device"
    import paper_2106_11565_amd as flinng
    flinng.lib()
    return flinng


# --------------------------------------------------------------------------
# hash codes

@pytest.mark.parametrize("family", [0, 1])
@pytest.mark.parametrize("n,d,K,L", [(1, 1, 1, 1), (77, 7, 5, 3), (300, 33, 13, 7),
                                     (513, 130, 8, 4), (1000, 256, 16, 9)])
def test_srp_codes_random_shapes(fl, family, n, d, K, L):
    log("srp codes", family, n, d, K, L)
    rng = np.random.default_rng(n * 131 + d)
    x = rng.standard_normal((n, d)).astype(np.float32)
    if family == 1:
        x = synth.f32_to_bf16(x)
    B = max(1, n // 4)
    gi = fl.Index(x, family, K, L, 2, B, seed=1234)
    w = oracle.hyperplanes(1234, K * L, d)
    xd = oracle.bf16_to_f64(x) if family == 1 else x.astype(np.float64)
    want = oracle.srp_codes(xd, 1234, K, L, w=w)
    got = gi.debug_hash(x)
    assert np.array_equal(got, want)


def test_srp_exact_zero_and_tiny_projections(fl):
    """Rows built so that some projections are exactly 0 or +-2^-60: the GPU
    flags them (|P| under its bound), rechecks in FP64 and falls back to the
    exact sum; the bits must equal the exact rational signs."""
    K, L, d, seed = 8, 4, 64, 77
    w = oracle.hyperplanes(seed, K * L, d)
    rng = np.random.default_rng(5)
    rows = [rng.standard_normal(d).astype(np.float32) for _ in range(40)]
    for h in range(K * L):
        nz = np.nonzero(w[h])[0]
        i, j, k_ = nz[0], nz[1], nz[2]
        z = np.zeros(d, dtype=np.float32)
        z[i], z[j] = w[h, j], -w[h, i]        # exactly orthogonal to w[h]
        rows.append(z.copy())
        t = z.copy()
        t[k_] = np.float32(2.0**-60 / w[h, k_])   # projection exactly +2^-60
        rows.append(t)
        rows.append(-t)
    x = np.stack(rows).astype(np.float32)
    want = oracle.srp_codes(x.astype(np.float64), seed, K, L, w=w)
    gi = fl.Index(x, 0, K, L, 3, 10, seed=seed)
    assert np.array_equal(gi.debug_hash(x), want)
    assert gi.info.srp_rechecked > 0 and gi.info.srp_exact > 0
    log("rechecked", gi.info.srp_rechecked, "exact", gi.info.srp_exact)


def _cancelling_rows(w, rng, nrand, boost=2.0**6, tiny=2.0**-20):
    """Random rows, then for each hyperplane h a row exactly orthogonal to it
    whose products with w[h] are all positive on the first half of the
    coordinates and all negative on the second half (pairs (i, j) of equal
    hyperplane sign with x_i = w[h, j], x_j = -w[h, i]), so partial sums grow
    far from the exact total 0; and that row plus / minus `tiny` at a free
    coordinate (projection exactly +-tiny * w[h, k]).  Values are
    quarter-integers times powers of two: exact in bf16."""
    H, d = w.shape
    rows = [rng.standard_normal(d) for _ in range(nrand)]
    half = d // 2
    for h in range(H):
        wh = w[h]
        z = np.zeros(d)
        for sgn in (1, -1):
            a = [i for i in range(half) if np.sign(wh[i]) == sgn]
            b = [i for i in range(half, d) if np.sign(wh[i]) == sgn]
            for i, j in zip(a, b):
                z[i], z[j] = wh[j], -wh[i]
        z *= boost
        rows.append(z.copy())
        free = [i for i in range(d) if z[i] == 0 and wh[i] != 0]
        if free:
            t = z.copy()
            t[free[0]] = tiny
            rows.append(t)
            rows.append(-t)
    return np.stack(rows)


@pytest.mark.parametrize("n,d,K,L", [(1, 1024, 13, 40), (17, 2080, 24, 12), (300, 2080, 7, 41),
                                     (1000, 1024, 16, 19), (2500, 4064, 5, 60), (129, 4064, 24, 13)])
def test_srp_bf16_k_groups_and_table_groups(fl, n, d, K, L):
    """bf16 rows through the fused SRP kernel's k-split and table-group
    paths: d = 1024 (8 chunks of 128), 2080 (16 chunks and a final half
    step of 32) and 4064 (a final chunk of 96), K*L above 288 so a row tile
    spans several groups of whole tables (the last one ragged), and ragged
    row counts; codes equal the oracle's."""
    log("srp bf16 k groups", n, d, K, L)
    rng = np.random.default_rng(n * 7 + d + K * L)
    x = synth.f32_to_bf16(rng.standard_normal((n, d)).astype(np.float32))
    gi = fl.Index(x, 1, K, L, 2, max(1, n // 4), seed=4321)
    w = oracle.hyperplanes(4321, K * L, d)
    want = oracle.srp_codes(oracle.bf16_to_f64(x), 4321, K, L, w=w)
    assert np.array_equal(gi.debug_hash(x), want)


@pytest.mark.parametrize("n,d,K,L", [(2048, 4096, 24, 12), (3000, 256, 16, 7), (4000, 512, 24, 12),
                                     (700, 96, 24, 5), (600, 100, 24, 5), (1500, 64, 3, 33)])
def test_srp_bf16_rechecks_only_near_zero(fl, n, d, K, L):
    """bf16 rows with no projection near zero (Gaussian rows): the projection
    stage may flag only projections within its error bound of zero, so every
    flagged one has |v| <= tau + gamma |x| |w| (v the exact value, tau =
    gamma |x| |w| + tau_abs), and only those FP64 cannot certify take the
    exact-sum fallback.  Flags
    outside the hyperplanes a workgroup covers (hyperplane groups whose count
    is an odd number of 16) would show up as extra rechecks and exact sums."""
    log("srp bf16 recheck count", n, d, K, L)
    rng = np.random.default_rng(n + 7 * d + K)
    x = synth.f32_to_bf16(rng.standard_normal((n, d)).astype(np.float32))
    gi = fl.Index(x, 1, K, L, 2, max(1, n // 4), seed=99)
    w = oracle.hyperplanes(99, K * L, d)
    xd = oracle.bf16_to_f64(x)
    v = xd @ w.T
    _, (gam, tabs) = gi.debug_projections(x[:1])
    tau = gam * np.sqrt((xd * xd).sum(1))[:, None] * np.sqrt((w * w).sum(1))[None, :] + tabs
    near = int((np.abs(v) <= 2.1 * tau).sum())
    # FP64 certifies a sign unless |v| <= 2 d 2^-53 sum|x_i w_i| (exact zeros
    # among them): only those may take the exact sum
    uncert = int((np.abs(v) <= 2 * d * 2.0**-53 * (np.abs(xd) @ np.abs(w).T)).sum())
    log("rechecked", gi.info.srp_rechecked, "exact", gi.info.srp_exact, "near zero", near,
        "uncertifiable", uncert)
    assert gi.info.srp_exact <= uncert
    assert gi.info.srp_rechecked <= near
    m = min(n, 400)
    assert np.array_equal(gi.debug_hash(x[:m]), oracle.srp_codes(xd[:m], 99, K, L, w=w))


@pytest.mark.parametrize("family,d", [(0, 64), (0, 100), (1, 128), (1, 100)])
def test_srp_extreme_scales_and_cancellations(fl, family, d):
    """Rows scaled by 2^0, 2^-70, 2^-80 and 2^-100 (fp32 sums of their
    squares underflow from 2^-80 on), including exactly cancelling and
    +-tiny projections: codes equal the oracle's and are the same at every
    scale (SRP bits are scale invariant).  bf16 rows with d a multiple of 32
    take the in-place recheck kernel, ragged d the general one; both reach
    the exact-sum fallback (srp_exact > 0)."""
    log("srp scales", family, d)
    K, L, seed = 8, 4, 77
    w = oracle.hyperplanes(seed, K * L, d)
    X = _cancelling_rows(w, np.random.default_rng(d + family), 24)
    n0 = X.shape[0]
    x = np.concatenate([X * 2.0**-e for e in (0, 70, 80, 100)]).astype(np.float32)
    xs = synth.f32_to_bf16(x) if family == 1 else x
    xd = oracle.bf16_to_f64(xs) if family == 1 else x.astype(np.float64)
    for b in range(1, 4):   # power-of-two scaling stayed exact in storage
        assert np.array_equal(xd[b * n0:(b + 1) * n0] * 2.0**[0, 70, 80, 100][b], xd[:n0])
    want = oracle.srp_codes(xd, seed, K, L, w=w)
    for b in range(1, 4):
        assert np.array_equal(want[b * n0:(b + 1) * n0], want[:n0])
    gi = fl.Index(xs, family, K, L, 3, 10, seed=seed)
    got = gi.debug_hash(xs)
    bad = np.nonzero(np.any(got != want, axis=1))[0]
    assert len(bad) == 0, (bad[:8], got[bad[:2]], want[bad[:2]])
    log("rechecked", gi.info.srp_rechecked, "exact", gi.info.srp_exact)
    assert gi.info.srp_rechecked > 0 and gi.info.srp_exact > 0


def test_mfma_projection_error_within_bound(fl):
    """The accuracy the sign certificate assumes of the bf16 matrix cores:
    on ReLU-embedding rows (d = 4096, 1024 hyperplanes) every fp32
    projection is within half the certified bound of the FP64 value,
    |v32 - v| < gamma / 2 * |x| |w|, and every trusted sign is right."""
    cfg, X, Q, _ = scaled("c3", 0.002, 1500)
    gi = fl.Index(X, 1, cfg["K"], cfg["L"], 2, 16, seed=21)
    w = oracle.hyperplanes(21, cfg["K"] * cfg["L"], cfg["d"])
    wn = np.sqrt((w * w).sum(axis=1))
    worst = 0.0
    for rows in (Q, X[:1500]):
        proj, (gamma, tau_abs) = gi.debug_projections(rows)
        xd = oracle.bf16_to_f64(rows)
        v = xd @ w.T
        scale = np.sqrt((xd * xd).sum(axis=1))[:, None] * wn[None, :]
        err = np.abs(proj.astype(np.float64) - v)
        ratio = np.max(err / np.maximum(scale, 1e-300))
        worst = max(worst, float(ratio))
        trusted = np.abs(proj) > gamma * scale + tau_abs
        assert np.all(np.sign(proj[trusted]) == np.sign(v[trusted]))
        log("mfma error: max ratio", ratio, "gamma", gamma, "trusted", trusted.mean())
    assert worst < gamma / 2, (worst, gamma)


@pytest.mark.parametrize("family", [2, 3])
@pytest.mark.parametrize("K,L,b,mean", [(1, 1, 1, 3), (2, 32, 20, 81), (3, 48, 22, 68),
                                        (4, 5, 12, 300), (1, 200, 16, 10), (7, 3, 24, 1000)])
def test_minhash_codes_random(fl, family, K, L, b, mean):
    log("minhash codes", family, K, L, b, mean)
    rng = np.random.default_rng(K * 1000 + L + b)
    dt = np.uint64 if family == 3 else np.uint32
    items, offs = random_sets(rng, 150, mean, dt)
    gi = fl.Index((items, offs), family, K, L, 2, 10, seed=99, bucket_bits=b)
    want = oracle.minhash_codes(items.astype(np.uint64), offs, 99, K, L, b)
    assert np.array_equal(gi.debug_hash((items, offs)), want)


# --------------------------------------------------------------------------
# whole pipeline on the workloads (scaled where the oracle needs it)

def _check_all(fl, family, data, q, K, L, R, B, seed, bucket_bits, ks=(1, 10, 37, 64, 65, 200)):
    gi, oi = build_both(fl, family, data, K, L, R, B, seed, bucket_bits)
    log("built", family, "N", oi.N, "entries", gi.info.list_entries)
    # index
    offs, cells, groups = gi.export()
    assert np.array_equal(groups, oi.g)
    assert np.array_equal(offs, oi.offsets)
    assert np.array_equal(cells, oi.cells)
    # codes and counts
    assert np.array_equal(gi.debug_hash(q), oi.hash(q))
    cnt = gi.debug_counts(q)
    assert np.array_equal(cnt, oi.counts(oi.hash(q)))
    # ids and scores, one workgroup per query and persistent
    for k in ks:
        want_i, want_s = oracle_query(oi, q, k)
        for pers in (False, True):
            got_i, got_s = gi.query(q, k, persistent=pers)
            bad = np.nonzero(np.any(got_i != want_i, axis=1))[0]
            assert len(bad) == 0, (k, pers, bad[:5], got_i[bad[:2]], want_i[bad[:2]],
                                   got_s[bad[:2]], want_s[bad[:2]])
            assert np.array_equal(got_s, want_s)
    return gi, oi


def test_c1_dense_gmm_full(fl):
    cfg, X, Q, _ = scaled("c1", 1.0, 100)
    _check_all(fl, 0, X, Q, cfg["K"], cfg["L"], cfg["R"], cfg["B"], 5, 0)


def test_c2_genome_scaled(fl):
    cfg, (it, of), (qit, qof), _ = scaled("c2", 0.01, 120)
    _check_all(fl, 3, (it, of), (qit, qof), cfg["K"], cfg["L"], cfg["R"], cfg["B"], 6,
               cfg["bucket_bits"])


def test_c3_relu_scaled(fl):
    cfg, X, Q, _ = scaled("c3", 0.006, 60)
    _check_all(fl, 1, X, Q, cfg["K"], cfg["L"], cfg["R"], cfg["B"], 7, 0, ks=(1, 10))


def test_c4_url_scaled(fl):
    cfg, (it, of), (qit, qof), _ = scaled("c4", 0.002, 150)
    _check_all(fl, 2, (it, of), (qit, qof), cfg["K"], cfg["L"], cfg["R"], cfg["B"], 8, 18)


# --------------------------------------------------------------------------
# degenerate cases of the method

@pytest.mark.parametrize("R,B,L,k", [(3, 1, 4, 7), (1, 9, 3, 50), (4, 5, 1, 12),
                                     (2, 50, 6, 500), (16, 7, 2, 3)])
def test_degenerate_grids(fl, R, B, L, k):
    log("degenerate", R, B, L, k)
    X, Q, _ = synth.dense_gmm(N=300, d=24, n_centres=12, nq=40)
    _check_all(fl, 0, X, Q, 6, L, R, B, 11, 0, ks=(k,))


def test_skewed_codes_and_mostly_empty_buckets(fl):
    """Nine points in ten are the same set, so before deduplication one
    bucket of every table holds most of the table's keys, and the tables
    have 2^20 buckets, nearly all empty: the build's merge of the bucket
    numbers with the sorted keys then has workgroups that see only keys of
    one bucket and workgroups that see only empty buckets.  The offsets,
    lists and query results must equal the oracle's."""
    rng = np.random.default_rng(41)
    n = 12000
    items, offs = random_sets(rng, n, 40, np.uint32)
    common = rng.integers(0, 2**32, 40, dtype=np.int64).astype(np.uint32)
    same = rng.random(n) < 0.9
    parts = [common if same[i] else items[offs[i]:offs[i + 1]] for i in range(n)]
    o = np.zeros(n + 1, dtype=np.uint64)
    o[1:] = np.cumsum([len(p) for p in parts])
    it = np.concatenate(parts).astype(np.uint32)
    sel = np.concatenate([np.nonzero(same)[0][:5], np.nonzero(~same)[0][:45]])
    q = subset_sets(it, o, sel)
    log("skewed", int(same.sum()), "of", n, "points share one set")
    gi, oi = _check_all(fl, 2, (it, o), q, 2, 4, 4, 50, 19, 20, ks=(10, 200))
    assert gi.info.list_entries == oi.cells.size


def test_identical_queries_returned_with_full_score(fl):
    X, _, _ = synth.dense_gmm(N=5000, d=64, n_centres=200, sigma=0.05, nq=1)
    gi = fl.Index(X, 0, 12, 16, 3, 250, seed=3)
    sel = np.arange(0, 5000, 97)
    ids, sc = gi.query(X[sel], 10)
    for i, x in enumerate(sel):
        row = list(ids[i])
        assert x in row and sc[i][row.index(x)] == 16


def test_large_k_and_ragged(fl):
    cfg, (it, of), (qit, qof), _ = scaled("c2", 0.002, 33)
    gi, oi = build_both(fl, 3, (it, of), 2, 8, 3, 17, 13, 12)
    for k in (1000, oi.N, oi.N + 5):
        if k > 4096:
            continue
        want = oracle_query(oi, (qit, qof), k)
        got = gi.query((qit, qof), k)
        assert np.array_equal(got[0], want[0]) and np.array_equal(got[1], want[1])


def test_errors(fl):
    X, _, _ = synth.dense_gmm(N=50, d=8, n_centres=3, nq=1)
    with pytest.raises(fl.FlinngError) as e:
        fl.Index(X, 0, 4, 3, 2, 51, seed=1)      # B > N
    assert e.value.code == fl.EINVAL
    with pytest.raises(fl.FlinngError):
        fl.Index(X, 0, 0, 3, 2, 5, seed=1)       # K = 0
    with pytest.raises(fl.FlinngError):
        fl.Index(X, 0, 4, 256, 2, 5, seed=1)     # L > 255
    gi = fl.Index(X, 0, 4, 3, 2, 5, seed=1)
    with pytest.raises(fl.FlinngError):
        gi.query(X[:3], 0)
    with pytest.raises(fl.FlinngError):
        gi.query(X[:3], 5000)
    # on_device = 2 (device items, host offsets) is a serving-only placement
    import ctypes
    inp, keep = fl.make_input(X[:3], 0)
    inp.on_device = 2
    ids = np.empty((3, 5), dtype=np.uint32)
    rc = fl.lib().flinng_query(gi.handle, ctypes.byref(inp), 5, ids.ctypes.data, None, 0, 0, None)
    assert rc == fl.EINVAL
    # the theory helper and the projections export reject what they cannot do
    with pytest.raises(fl.FlinngError):
        fl.theory_params(100, 0.9, 0.5, 0.1)
    it, of, qit, qof, _ = synth.genome(n_base=60, nq=4)
    si = fl.Index((it, of), fl.MINHASH_U64, 1, 4, 2, 5, seed=1, bucket_bits=10)
    with pytest.raises(fl.FlinngError):
        si.debug_projections((qit, qof))


@pytest.mark.parametrize("name,scale,nq,fam", [("c1", 1.0, 100, 0), ("c2", 0.01, 80, 3),
                                                ("c3", 0.006, 40, 1), ("c4", 0.002, 80, 2)])
def test_fixed_threshold_equals_oracle(fl, name, scale, nq, fam):
    """flinng_query_threshold (Algorithm 2 at a fixed t) returns exactly the
    oracle's {x : every repetition's cell of x has count >= t}, for t from 0
    (every point) to L + 1 (none); the counts are exact even when fewer id
    slots are given, and the truncated ids are a prefix of the full answer."""
    cfg, data, q, _ = scaled(name, scale, nq)
    bb = {0: 0, 1: 0, 3: cfg["bucket_bits"], 2: 18}[fam]
    gi, oi = build_both(fl, fam, data, cfg["K"], cfg["L"], cfg["R"], cfg["B"], 31, bb)
    cnt = oi.counts(oi.hash(q))
    L = cfg["L"]
    for t in sorted({0, 1, 2, max(1, L // 2), L - 1, L, L + 1}):
        want = [np.nonzero(oracle.query_fixed_t(cnt[i], oi.g, oi.B, t))[0] for i in range(nq)]
        M = max(1, max(len(w) for w in want))
        ids, counts = gi.query_threshold(q, t, M)
        log("threshold", name, "t", t, "largest answer", M)
        for i in range(nq):
            assert counts[i] == len(want[i]), (t, i)
            assert np.array_equal(np.sort(ids[i][:counts[i]]), want[i]), (t, i)
            assert np.all(ids[i][counts[i]:] == 0xFFFFFFFF)
        small = max(1, M // 3)
        ids2, counts2 = gi.query_threshold(q, t, small)
        assert np.array_equal(counts2, counts)
        for i in range(nq):
            n = min(small, int(counts[i]))
            assert np.array_equal(ids2[i][:n], ids[i][:n]), (t, i)
        _, counts0 = gi.query_threshold(q, t, 0)
        assert np.array_equal(counts0, counts)


def test_c4_grid_u32_cells_large_lds(fl):
    """R*B = 131072 cells: 32-bit cell ids and 128 KiB of LDS counters per
    workgroup, the URL workload's grid, on a small dataset."""
    X, Q, _ = synth.dense_gmm(N=40000, d=16, n_centres=400, sigma=0.05, nq=80)
    gi, oi = build_both(fl, 0, X, 6, 5, 8, 16384, 21, 0)
    assert gi.info.cell_id_bytes == 4
    offs, cells, groups = gi.export()
    assert np.array_equal(groups, oi.g) and np.array_equal(cells, oi.cells)
    assert np.array_equal(gi.debug_counts(Q), oi.counts(oi.hash(Q)))
    for k in (1, 10, 64, 65):
        want = oracle_query(oi, Q, k)
        for pers in (False, True):
            got = gi.query(Q, k, persistent=pers)
            assert np.array_equal(got[0], want[0]) and np.array_equal(got[1], want[1]), (k, pers)


def test_c2_genome_hashed_filter(fl):
    """N = 40 000 (over 2^15 points, B = 164): larger cells than the other
    scaled genome index, so a decode pass streams several 256-member chunks
    per cell and the per-lane sorted insertion sees long runs of members."""
    cfg, (it, of), (qit, qof), _ = scaled("c2", 0.04, 100)
    _check_all(fl, 3, (it, of), (qit, qof), cfg["K"], cfg["L"], cfg["R"], cfg["B"], 9,
               cfg["bucket_bits"], ks=(1, 10, 64))


@pytest.mark.parametrize("R", [2, 5])
def test_many_positive_cells_chunked(fl, R):
    """One 1-bit table: about half of all cells are positive, more than the
    decode's positive-cell list holds in one round, so a pass collects and
    streams the cells of its repetition in several rounds."""
    X, Q, _ = synth.dense_gmm(N=20000, d=8, n_centres=50, nq=40)
    gi, oi = build_both(fl, 0, X, 1, 1, R, 2000, 23, 0)
    for k in (1, 10, 64):
        want = oracle_query(oi, Q, k)
        got = gi.query(Q, k)
        assert np.array_equal(got[0], want[0]) and np.array_equal(got[1], want[1]), k


def test_query_streams_and_threads(fl):
    """flinng_query keeps one codes region per stream: batches queried from
    several host threads on several streams (two threads sharing one
    stream), and a later larger batch that grows a region, give the same
    ids and scores as the oracle."""
    import threading

    import torch
    cfg, (it, of), (qit, qof), _ = scaled("c2", 0.01, 120)
    gi, oi = build_both(fl, 3, (it, of), cfg["K"], cfg["L"], cfg["R"], cfg["B"], 21,
                        cfg["bucket_bits"])
    want_i, want_s = oracle_query(oi, (qit, qof), 10)

    def dev(a):
        a = np.ascontiguousarray(a)
        return torch.from_numpy(a.view(np.int64)).cuda()

    q_d = (dev(qit), dev(qof))
    nq = len(qof) - 1
    streams = [torch.cuda.Stream(), torch.cuda.Stream(), torch.cuda.Stream()]
    results, errors = {}, []

    def worker(t, s):
        try:
            ids = torch.empty((nq, 10), dtype=torch.int32, device="cuda")
            sc = torch.empty((nq, 10), dtype=torch.int32, device="cuda")
            for _ in range(5):
                gi.query(q_d, 10, stream=s, out=(ids, sc))
            s.synchronize()
            results[t] = (ids.cpu().numpy().view(np.uint32), sc.cpu().numpy().view(np.uint32))
        except Exception as e:  # noqa: BLE001
            errors.append(repr(e))

    stream_of = [0, 1, 2, 0]  # threads 0 and 3 share a stream
    threads = [threading.Thread(target=worker, args=(t, streams[stream_of[t]])) for t in range(4)]
    for th in threads:
        th.start()
    for th in threads:
        th.join()
    assert not errors, errors
    for t, (gi_, gs_) in results.items():
        assert np.array_equal(gi_, want_i) and np.array_equal(gs_, want_s), t
    # a larger batch on a stream whose region was sized for the smaller one
    big_it = np.concatenate([qit, qit])
    big_of = np.concatenate([qof, qof[1:] + qof[-1]])
    got_i, got_s = gi.query((dev(big_it), dev(big_of)), 10, stream=streams[0])
    assert np.array_equal(got_i[:nq], want_i) and np.array_equal(got_i[nq:], want_i)
    assert np.array_equal(got_s[:nq], want_s) and np.array_equal(got_s[nq:], want_s)


def test_sparse_counting_touched_list_overflow(fl):
    """Sparse queries (list entries at most the counter words) note the cells
    they touch in a 256-entry list; a query touching more cells builds its
    positive-cell lists by scanning instead.  Short MinHash buckets over a
    small grid give sparse queries on both sides of that limit and a few
    dense ones in one batch; the answers equal the oracle's in both launch
    modes."""
    rng = np.random.default_rng(5)
    pool = rng.integers(0, 2**32, 20000, dtype=np.uint64).astype(np.uint32)
    it, of = random_sets(rng, 4096, 20, np.uint32, pool=pool)
    qit, qof = random_sets(rng, 96, 20, np.uint32, pool=pool)
    K, L, R, B, bits = 1, 4, 4, 1024, 8
    gi, oi = build_both(fl, 2, (it, of), K, L, R, B, 31, bits)
    codes = oi.hash((qit, qof))
    cnt = oi.counts(codes)
    nent = np.array([sum(int(oi.offsets[t, c + 1] - oi.offsets[t, c]) for t, c in enumerate(row))
                     for row in codes])
    words = ((R * ((B + 3) & ~3)) // 4 + 3) & ~3
    touched = (cnt > 0).sum(axis=1)
    sparse = nent <= words
    log("entries", nent.min(), nent.max(), "touched", touched.min(), touched.max(), "words", words)
    # sparse queries on both sides of the list's capacity, and dense ones
    assert np.any(sparse & (touched > 256)) and np.any(sparse & (touched <= 256))
    assert np.any(~sparse)
    for k in (1, 10, 64, 65):
        want_i, want_s = oracle_query(oi, (qit, qof), k)
        for pers in (False, True):
            got_i, got_s = gi.query((qit, qof), k, persistent=pers)
            assert np.array_equal(got_i, want_i) and np.array_equal(got_s, want_s), (k, pers)


@pytest.mark.parametrize("B", [4600, 5200])
def test_one_query_kernel_register_budgets(fl, B):
    """Per-query states of about 21 and 24 KiB: the launcher picks the
    one-query kernel built for seven (B = 4600) and six (B = 5200)
    wavefronts per SIMD, the most the LDS allows; both equal the oracle."""
    X, Q, _ = synth.dense_gmm(N=12000, d=16, n_centres=40, nq=48)
    gi, oi = build_both(fl, 0, X, 2, 4, 4, B, 41, 0)
    for k in (1, 10, 64):
        want = oracle_query(oi, Q, k)
        got = gi.query(Q, k)
        assert np.array_equal(got[0], want[0]) and np.array_equal(got[1], want[1]), k
