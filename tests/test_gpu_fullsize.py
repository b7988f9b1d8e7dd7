"""Parity at the workloads' full sizes, in the launch configuration the
benchmark times (data and queries resident on the device, one workgroup per
query, k = 10).

Genome reads (1M sets): the oracle builds the whole index, so every one of
the 10 000 queries is compared with the oracle's Algorithm 3 (threshold
relaxation), at the configured (K, L) and at the tuned one.

ReLU embeddings (1M x 4096) and URL strings (5M sets): the oracle cannot
build these indexes in test time, so the check is a chain over samples, each
link against the oracle or a property that holds at any size:
  1. bucket codes of sampled queries and points equal the oracle's;
  2. the groups of all N points equal the oracle's permutation (Algorithm 1);
  3. every sampled point's cell is in its bucket's list in every table, and
     every list touched is strictly ascending (deduplicated);
  4. the GPU's per-cell counts of sampled queries equal counts recomputed
     from the exported lists by their definition;
  5. the GPU's ids and scores equal the oracle's Algorithm 3 over those
     counts (with the oracle's groups);
  6. a query identical to an indexed point finds all its cells at count L
     (every group test positive) and is returned.
"""
import numpy as np
import pytest

import oracle
from gpu_common import log
from workloads import configs

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def env():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a ROCm device"
    import paper_2106_11565_amd as flinng
    flinng.lib()
    return torch, flinng


def _dev(torch, a):
    a = np.ascontiguousarray(a)
    view = {np.dtype(np.uint64): np.int64, np.dtype(np.uint32): np.int32,
            np.dtype(np.uint16): np.int16}.get(a.dtype)
    return torch.from_numpy(a.view(view) if view else a).cuda()


def _query_dev(torch, fl, gi, q_d, nq, k=10, persistent=False):
    ids = torch.empty((nq, k), dtype=torch.int32, device="cuda")
    sc = torch.empty((nq, k), dtype=torch.int32, device="cuda")
    gi.query(q_d, k, persistent=persistent, out=(ids, sc))
    torch.cuda.synchronize()
    return ids.cpu().numpy().view(np.uint32), sc.cpu().numpy().view(np.uint32)


def _sets_subset(items, offs, sel):
    parts = [items[int(offs[s]):int(offs[s + 1])] for s in sel]
    o = np.zeros(len(sel) + 1, dtype=np.uint64)
    o[1:] = np.cumsum([len(p) for p in parts])
    return np.concatenate(parts), o


@pytest.mark.parametrize("which", ["configured", "tuned"])
def test_genome_full_all_queries(env, which):
    torch, fl = env
    cfg, (it, of), (qit, qof), _ = configs.make("c2")
    K, L = (cfg["K"], cfg["L"]) if which == "configured" else (cfg["tuned"]["K"], cfg["tuned"]["L"])
    data_d = (_dev(torch, it), _dev(torch, of))
    gi = fl.Index(data_d, fl.MINHASH_U64, K, L, cfg["R"], cfg["B"], configs.INDEX_SEED,
                  bucket_bits=cfg["bucket_bits"])
    oi = oracle.OracleIndex(oracle.MINHASH_U64, (it, of), K, L, cfg["R"], cfg["B"],
                            configs.INDEX_SEED, bucket_bits=cfg["bucket_bits"])
    log("genome", which, "K", K, "L", L, "entries", gi.info.list_entries)
    assert gi.info.list_entries == len(oi.cells)
    nq = len(qof) - 1
    got_i, got_s = _query_dev(torch, fl, gi, (_dev(torch, qit), _dev(torch, qof)), nq)
    want_i, want_s = oi.query((qit, qof), 10)
    bad = np.nonzero(np.any(got_i != want_i, axis=1) | np.any(got_s != want_s, axis=1))[0]
    assert len(bad) == 0, (len(bad), bad[:5])
    # the persistent launch gives the same answers
    p_i, p_s = _query_dev(torch, fl, gi, (_dev(torch, qit), _dev(torch, qof)), nq, persistent=True)
    assert np.array_equal(p_i, got_i) and np.array_equal(p_s, got_s)


def _sampled_chain(torch, fl, family, data, queries, cfg, nsample, dense):
    K, L, R, B = cfg["K"], cfg["L"], cfg["R"], cfg["B"]
    seed = configs.INDEX_SEED
    rng = np.random.default_rng(11)
    if dense:
        N, nq = data.shape[0], queries.shape[0]
        data_d, q_d = _dev(torch, data), _dev(torch, queries)
        bits = K
    else:
        N, nq = len(data[1]) - 1, len(queries[1]) - 1
        data_d = (_dev(torch, data[0]), _dev(torch, data[1]))
        q_d = (_dev(torch, queries[0]), _dev(torch, queries[1]))
        bits = cfg["bucket_bits"]
    gi = fl.Index(data_d, family, K, L, R, B, seed, bucket_bits=0 if dense else bits)
    log("built", cfg["name"], "entries", gi.info.list_entries)
    qs = np.sort(rng.choice(nq, nsample, replace=False))
    ps = np.sort(rng.choice(N, nsample, replace=False))
    if dense:
        qsub, psub = queries[qs], data[ps]
        w = oracle.hyperplanes(seed, K * L, data.shape[1])
        to64 = oracle.bf16_to_f64 if family == fl.SRP_BF16 else (lambda a: a.astype(np.float64))
        ohash = lambda a: oracle.srp_codes(to64(a), seed, K, L, w=w)  # noqa: E731
    else:
        qsub, psub = _sets_subset(*queries, qs), _sets_subset(*data, ps)
        ohash = lambda a: oracle.minhash_codes(a[0], a[1], seed, K, L, bits)  # noqa: E731
    # 1. codes
    qcodes, pcodes = ohash(qsub), ohash(psub)
    assert np.array_equal(gi.debug_hash(qsub), qcodes)
    assert np.array_equal(gi.debug_hash(psub), pcodes)
    # 2. groups
    offs, cells, groups = gi.export()
    g = oracle.groups(N, R, B, seed)
    assert np.array_equal(groups, g)
    del groups
    # 3. lists: structure, membership of sampled points, strictly ascending
    assert offs.shape == (L, (1 << bits) + 1)
    assert np.all(np.diff(offs.astype(np.int64), axis=1) >= 0)
    assert int(offs[-1, -1]) == len(cells) == gi.info.list_entries
    touched = set()
    for i, p in enumerate(ps):
        for t in range(L):
            b = int(pcodes[i, t])
            lst = cells[int(offs[t, b]):int(offs[t, b + 1])]
            want = (np.arange(R, dtype=np.int64) * B + g[:, p]).astype(np.uint32)
            assert np.all(np.isin(want, lst)), (p, t)
            touched.add((t, b))
    for i in range(len(qs)):
        for t in range(L):
            touched.add((t, int(qcodes[i, t])))
    for t, b in touched:
        lst = cells[int(offs[t, b]):int(offs[t, b + 1])].astype(np.int64)
        assert np.all(np.diff(lst) > 0), (t, b)
        assert len(lst) == 0 or (lst[0] >= 0 and lst[-1] < R * B)
    # 4. counts by definition over the exported lists
    cnt = gi.debug_counts(qsub)
    want_cnt = oracle.counts(offs, cells, qcodes, R * B, bits)
    assert np.array_equal(cnt, want_cnt)
    del cells
    # 5. decode of the full batch in the benchmark's launch, sampled rows
    got_i, got_s = _query_dev(torch, fl, gi, q_d, nq)
    for j, q in enumerate(qs):
        wi, ws = oracle.decode(want_cnt[j], g, B, 10)
        assert np.array_equal(got_i[q], wi) and np.array_equal(got_s[q], ws), q
    # 6. an indexed point as the query: all its group tests positive, returned
    pcnt = gi.debug_counts(psub)
    cells_p = (np.arange(R)[None, :] * B + g[:, ps].T)
    assert np.all(np.take_along_axis(pcnt, cells_p, axis=1) == L)
    pi, psc = gi.query(psub, 10)
    for i, p in enumerate(ps):
        assert psc[i, 0] == L
        # returned, unless more than 10 points tie at the top score
        assert p in pi[i] or np.all(psc[i] == L), p
    return gi, qs, got_i


def test_relu_full_sampled(env):
    torch, fl = env
    cfg, X, Q, _ = configs.make("c3")
    _sampled_chain(torch, fl, fl.SRP_BF16, X, Q, cfg, 48, dense=True)


def test_url_full_sampled(env):
    torch, fl = env
    cfg, data, queries, _ = configs.make("c4")
    gi, qs, got_i = _sampled_chain(torch, fl, fl.MINHASH_U32, data, queries, cfg, 48, dense=False)
    # the configuration's single persistent launch over uneven groups gives
    # the same answers as one workgroup per query
    q_d = (_dev(torch, queries[0]), _dev(torch, queries[1]))
    p_i, _ = _query_dev(torch, fl, gi, q_d, len(queries[1]) - 1, persistent=True)
    assert np.array_equal(p_i, got_i)


def test_relu_tuned_hash_every_batch_plan(env):
    """The SRP stage at the benchmark's tuned (K, L) = (24, 12), d = 4096,
    for the batch sizes whose kernel plans the benchmark runs: a full
    10,000-query batch, an 8,192-row index-build chunk, served batches of
    2,900 and 2,048, small ones of 512, 128 and 1.  Each batch is hashed
    on the device in one call; 40 sampled rows of each must equal the
    oracle's codes (FP64 / exact signs)."""
    torch, fl = env
    from workloads import synth
    X, Q, _ = synth.dense_relu(N=20000, d=4096, n_centres=200, nq=10000)
    assert Q.shape[0] == 10000
    K, L, seed = 24, 12, configs.INDEX_SEED
    gi = fl.Index(X[:4000], fl.SRP_BF16, K, L, 4, 100, seed)
    w = oracle.hyperplanes(seed, K * L, 4096)
    rng = np.random.default_rng(3)
    q_d = _dev(torch, Q)
    for n in (10000, 8192, 2900, 2048, 512, 128, 1):
        codes = gi.debug_hash(q_d[:n].contiguous())
        codes = codes.cpu().numpy() if hasattr(codes, "cpu") else np.asarray(codes)
        rows = np.sort(rng.choice(n, min(n, 40), replace=False))
        want = oracle.srp_codes(oracle.bf16_to_f64(Q[rows]), seed, K, L, w=w)
        log("tuned hash", n, "rows checked", len(rows))
        assert np.array_equal(codes.reshape(n, L)[rows].astype(np.uint32), want.astype(np.uint32)), n
