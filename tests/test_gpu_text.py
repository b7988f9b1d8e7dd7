"""Device-side n-gram extraction (flinng_build_text, flinng_query_text,
flinng_serve_submit_text) against the oracle: genome reads (20-grams over 4
bases, 64-bit items) and URL-like strings (3-grams over 40 symbols, 32-bit
items) given as raw symbol sequences.  The index built from text equals the
oracle's index over the oracle's own n-gram items; text queries equal the
oracle's answers, from host and device memory, plain and served; and an
index built from the generator's item sets answers text queries exactly as
it answers the same queries given as item sets."""
import numpy as np
import pytest

import oracle
from gpu_common import log, oracle_query
from workloads import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def fl():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a ROCm device"
    import paper_2106_11565_amd as flinng
    flinng.lib()
    return flinng


def _dev_text(torch, seqs):
    sym, off = seqs
    return (torch.from_numpy(np.ascontiguousarray(sym).view(np.int8)).cuda(),
            torch.from_numpy(np.ascontiguousarray(off).view(np.int64)).cuda())


def _workload(kind):
    if kind == "genome":
        it, of, qit, qof, _, ex = synth.genome(n_base=3000, nq=150, text=True)
        return (it, of), (qit, qof), ex, 3, 64, dict(K=1, L=12, R=4, B=60, b=18)
    it, of, qit, qof, _, sizes, ex = synth.url(n_templates=1500, nq=150, text=True)
    return (it, of), (qit, qof), ex, 2, 32, dict(K=3, L=16, R=8, B=75, b=18)


def _slice(seqs, a, b):
    sym, off = seqs
    o = off[a:b + 1]
    return sym[int(o[0]):int(o[-1])], (o - o[0]).astype(np.uint64)


@pytest.mark.parametrize("kind", ["genome", "url"])
def test_text_index_and_queries_equal_oracle(fl, kind):
    import torch
    data, queries, ex, fam, bits, p = _workload(kind)
    txt = (ex["gram"], ex["radix"], ex["key"])
    gi = fl.Index(ex["data"], fam, p["K"], p["L"], p["R"], p["B"], seed=5,
                  bucket_bits=p["b"], text=txt)
    oit, oof = oracle.text_items(*ex["data"], *txt, bits)
    oi = oracle.OracleIndex(fam, (oit, oof), p["K"], p["L"], p["R"], p["B"], 5, bucket_bits=p["b"])
    offs, cells, groups = gi.export()
    assert np.array_equal(groups, oi.g) and np.array_equal(offs, oi.offsets)
    assert np.array_equal(cells, oi.cells)
    qit, qof = oracle.text_items(*ex["queries"], *txt, bits)
    for k in (1, 10, 70):
        want = oracle_query(oi, (qit, qof), k)
        got = gi.query_text(ex["queries"], txt, k)
        assert np.array_equal(got[0], want[0]) and np.array_equal(got[1], want[1]), k
    # device text, device results, persistent launch
    nq = len(ex["queries"][1]) - 1
    ids = torch.empty((nq, 10), dtype=torch.int32, device="cuda")
    sc = torch.empty((nq, 10), dtype=torch.int32, device="cuda")
    gi.query_text(_dev_text(torch, ex["queries"]), txt, 10, persistent=True, out=(ids, sc))
    torch.cuda.synchronize()
    want = oracle_query(oi, (qit, qof), 10)
    assert np.array_equal(ids.cpu().numpy().view(np.uint32), want[0])
    assert np.array_equal(sc.cpu().numpy().view(np.uint32), want[1])
    # an index built from the generator's item sets answers text queries as
    # it answers the item sets (the items agree)
    gs = fl.Index(data, fam, p["K"], p["L"], p["R"], p["B"], seed=5, bucket_bits=p["b"])
    a = gs.query_text(ex["queries"], txt, 10)
    b = gs.query(queries, 10)
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])
    log("text", kind, "entries", gi.info.list_entries)


def test_served_text_requests_equal_oracle(fl):
    """Text requests through the server (host text copied, device text
    borrowed; results to the host or into device buffers), in a burst mixed
    with item-set requests for the same index."""
    import torch
    data, queries, ex, fam, bits, p = _workload("genome")
    txt = (ex["gram"], ex["radix"], ex["key"])
    gi = fl.Index(data, fam, p["K"], p["L"], p["R"], p["B"], seed=5, bucket_bits=p["b"])
    qit, qof = oracle.text_items(*ex["queries"], *txt, bits)
    oi = oracle.OracleIndex(fam, data, p["K"], p["L"], p["R"], p["B"], 5, bucket_bits=p["b"])
    want = oracle_query(oi, (qit, qof), 10)
    srv = fl.Server([gi], mem_budget=1 << 30, max_inflight=3, max_batch=256)
    nq = len(ex["queries"][1]) - 1
    try:
        reqs, pos, i = [], 0, 0
        while pos < nq:
            n = min(nq - pos, 1 + (7 * i) % 40)
            mode = i % 4
            seqs = _slice(ex["queries"], pos, pos + n)
            if mode == 0:      # host text, host results
                reqs.append((mode, pos, n, srv.submit_text(0, seqs, txt, 10), None))
            elif mode == 1:    # device text, device results
                out = (torch.empty((n, 10), dtype=torch.int32, device="cuda"),
                       torch.empty((n, 10), dtype=torch.int32, device="cuda"))
                d = _dev_text(torch, seqs)
                torch.cuda.synchronize()
                reqs.append((mode, pos, n, srv.submit_text(0, d, txt, 10, out=out), (out, d)))
            else:              # item sets of the same queries
                o = qof[pos:pos + n + 1]
                q = (qit[int(o[0]):int(o[-1])], (o - o[0]).astype(np.uint64))
                reqs.append((mode, pos, n, srv.submit(0, q, 10), None))
            pos += n
            i += 1
        for mode, pos, n, (t, _), keep in reqs:
            if mode == 1:
                srv.wait_done(t)
                (ids, sc), _ = keep
                got = (ids.cpu().numpy().view(np.uint32), sc.cpu().numpy().view(np.uint32))
            else:
                got = srv.wait(t, n, 10)
            assert np.array_equal(got[0], want[0][pos:pos + n]), (mode, pos)
            assert np.array_equal(got[1], want[1][pos:pos + n]), (mode, pos)
        log("served text", srv.stats())
    finally:
        srv.close()


def test_text_errors(fl):
    it, of, qit, qof, _, ex = synth.genome(n_base=100, nq=5, text=True)
    for gram, radix in ((0, 4), (20, 1), (20, 300), (40, 4)):
        with pytest.raises(fl.FlinngError) as e:
            fl.Index(ex["data"], fl.MINHASH_U64, 1, 4, 2, 10, seed=1, bucket_bits=12,
                     text=(gram, radix, 7))
        assert e.value.code == fl.EINVAL, (gram, radix)
    X, _, _ = synth.dense_gmm(N=50, d=8, n_centres=3, nq=1)
    gd = fl.Index(X, fl.SRP_F32, 4, 3, 2, 5, seed=1)
    with pytest.raises(fl.FlinngError):
        gd.query_text(ex["queries"], (20, 4, 7), 5)
