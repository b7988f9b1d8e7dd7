"""GPU tests of the continuous-batching server (flinng_serve_*): every
request's ids and scores equal the CPU oracle's (Algorithm 3 on the oracle's
own index) for its queries, whether the request runs alone, in a mixed burst
over two resident indexes of different hash families, under linger, or
through the persistent launch; a URL-shaped index serves the uneven groups
(log-uniform sizes 1..4096) of its query stream; admission by device memory;
error paths.
"""
import numpy as np
import pytest

import oracle
from gpu_common import log, oracle_query, scaled
from workloads import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def fl():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a ROCm device"
    import paper_2106_11565_amd as flinng
    flinng.lib()
    return flinng


@pytest.fixture(scope="module")
def two_indexes(fl):
    X, Q, _ = synth.dense_relu(N=6000, d=512, n_centres=60, nq=700)
    dense = fl.Index(X, fl.SRP_BF16, 12, 16, 4, 60, seed=3)
    it, of, qit, qof, _ = synth.genome(n_base=4000, nq=700)
    sets = fl.Index((it, of), fl.MINHASH_U64, 2, 16, 4, 80, seed=4, bucket_bits=18)
    return dense, Q, sets, (qit, qof)


@pytest.fixture(scope="module")
def oracles(two_indexes):
    """The oracle's own indexes over the same data and parameters."""
    X, _, _ = synth.dense_relu(N=6000, d=512, n_centres=60, nq=700)
    od = oracle.OracleIndex(oracle.SRP_BF16, X, 12, 16, 4, 60, 3)
    it, of, _, _, _ = synth.genome(n_base=4000, nq=700)
    os_ = oracle.OracleIndex(oracle.MINHASH_U64, (it, of), 2, 16, 4, 80, 4, bucket_bits=18)
    return od, os_


def _want(oracles, fam, q, k):
    return oracle_query(oracles[fam], q, k)


def _same(got, want):
    return np.array_equal(got[0], want[0]) and np.array_equal(got[1], want[1])


def _requests(Q, S, rng, n):
    reqs = []
    qpos = [0, 0]
    for _ in range(n):
        fam = int(rng.integers(0, 2))
        # small payloads are packed into one staging run, those of 64 KiB and
        # more (about 64 dense rows or 100 read sets here) travel from pooled
        # pinned blocks; mix both in one batch
        sz = int(rng.integers(1, 40)) if rng.random() < 0.7 else int(rng.integers(64, 160))
        p = qpos[fam]
        if fam == 0:
            if p + sz > Q.shape[0]:
                p = 0
            q = Q[p:p + sz]
        else:
            it, of = S
            nq = len(of) - 1
            if p + sz > nq:
                p = 0
            o = of[p:p + sz + 1]
            q = (it[int(o[0]):int(o[-1])], (o - o[0]).astype(np.uint64))
        qpos[fam] = p + sz
        reqs.append((fam, sz, q, int(rng.integers(1, 20))))
    return reqs


@pytest.mark.parametrize("persistent", [False, True])
def test_results_equal_oracle_alone_and_in_mix(fl, two_indexes, oracles, persistent):
    dense, Q, sets, S = two_indexes
    rng = np.random.default_rng(1)
    reqs = _requests(Q, S, rng, 120)
    # reference: the oracle's Algorithm 3 for each request's queries
    want = [_want(oracles, fam, q, k) for fam, sz, q, k in reqs]
    # the plain batched path agrees with it as well
    for (fam, sz, q, k), ref in zip(reqs[:10], want[:10]):
        assert _same((dense if fam == 0 else sets).query(q, k), ref)
    srv = fl.Server([dense, sets], mem_budget=1 << 30, max_inflight=3, max_batch=256,
                    persistent=persistent)
    try:
        # alone through the server (one at a time)
        for i, ((fam, sz, q, k), ref) in enumerate(zip(reqs[:20], want[:20])):
            t, n = srv.submit(fam, q, k)
            assert _same(srv.wait(t, n, k), ref), ("alone", i)
        # mixed burst: everything submitted before anything is waited on
        tickets = [srv.submit(fam, q, k) for fam, sz, q, k in reqs]
        for i, ((fam, sz, q, k), ref, (t, n)) in enumerate(zip(reqs, want, tickets)):
            assert _same(srv.wait(t, n, k), ref), ("mixed", i)
        st = srv.stats()
        log("serve stats", st)
        assert st["completed"] == 140 and st["batches"] >= 2
        assert st["p99_ms"] >= st["p50_ms"] > 0
    finally:
        srv.close()


def test_url_uneven_groups_persistent(fl):
    """A URL-shaped index (3-gram sets, K=3, L=48, R=8, 32-bit cell ids) serves
    its query stream split into uneven groups with log-uniform sizes in
    [1, 4096], each batch one persistent launch; every group equals the
    oracle, and so does the whole stream queried as one persistent batch."""
    cfg, (it, of), (qit, qof), _ = scaled("c4", 0.002, 6000)
    # B * R above 2^16, as in the full-size URL index: 32-bit cell ids
    K, L, R, B, b = cfg["K"], cfg["L"], cfg["R"], 9000, 18
    gi = fl.Index((it, of), fl.MINHASH_U32, K, L, R, B, seed=13, bucket_bits=b)
    oi = oracle.OracleIndex(oracle.MINHASH_U32, (it, of), K, L, R, B, 13, bucket_bits=b)
    assert gi.info.cell_id_bytes == 4
    sizes = cfg["group_sizes"]
    assert sizes.sum() == len(qof) - 1 and sizes.max() > 1000 and sizes.min() >= 1
    want = oracle_query(oi, (qit, qof), 10)
    got = gi.query((qit, qof), 10, persistent=True)
    assert _same(got, want)
    srv = fl.Server([gi], mem_budget=1 << 30, max_inflight=2, max_batch=4096, persistent=True)
    try:
        tickets, pos = [], 0
        for sz in sizes:
            o = qof[pos:pos + sz + 1]
            tickets.append((srv.submit(0, (qit[int(o[0]):int(o[-1])], o - o[0]), 10), pos))
            pos += int(sz)
        for (t, n), p in tickets:
            g = srv.wait(t, n, 10)
            assert _same(g, (want[0][p:p + n], want[1][p:p + n])), p
        log("url groups", len(sizes), srv.stats())
    finally:
        srv.close()


def test_admission_by_memory(fl, two_indexes, oracles):
    dense, Q, sets, S = two_indexes
    # a budget too small for one request: refused with EBUSY
    srv = fl.Server([dense], mem_budget=1024, max_inflight=2)
    try:
        t, rc = srv.try_submit(0, Q[:5], 10)
        assert t is None and rc == fl.EBUSY
        assert srv.stats()["rejected"] == 1
    finally:
        srv.close()
    # a budget that fits one small request at a time: all complete, in order
    one = _want(oracles, 0, Q[:8], 10)
    srv = fl.Server([dense], mem_budget=1 << 20, max_inflight=4, max_batch=8)
    try:
        tickets = [srv.submit(0, Q[:8], 10) for _ in range(12)]
        for t, n in tickets:
            assert _same(srv.wait(t, n, 10), one)
        st = srv.stats()
        assert st["completed"] == 12 and st["peak_mem_bytes"] <= (1 << 20)
    finally:
        srv.close()


def test_serve_errors_and_shutdown(fl, two_indexes):
    dense, Q, sets, S = two_indexes
    srv = fl.Server([dense, sets], mem_budget=1 << 30)
    with pytest.raises(fl.FlinngError) as e:
        srv.wait(12345, 1, 10)
    assert e.value.code == fl.ESTATE
    with pytest.raises(fl.FlinngError):
        srv.submit(5, Q[:2], 10)       # bad slot
    with pytest.raises(fl.FlinngError):
        srv.submit(0, Q[:2], 0)        # bad k
    # poll reaches 1 once done
    t, n = srv.submit(0, Q[:3], 5)
    import time
    for _ in range(2000):
        if srv.poll(t):
            break
        time.sleep(0.001)
    assert srv.poll(t)
    srv.wait(t, n, 5)
    srv.reset_stats()
    st = srv.stats()
    assert st["completed"] == 0 and st["submitted"] == 0 and st["batches"] == 0
    # destroy with requests in flight and queued: drains, no hang
    for _ in range(30):
        srv.submit(0, Q[:30], 10)
    srv.close()


def test_linger_coalesces(fl, two_indexes, oracles):
    dense, Q, sets, S = two_indexes
    ref = _want(oracles, 0, Q[:40], 7)
    # a long linger holds the first request until the rest have arrived
    srv = fl.Server([dense], mem_budget=1 << 30, max_inflight=2, linger_ns=200_000_000)
    try:
        tickets = [srv.submit(0, Q[4 * i:4 * i + 4], 7) for i in range(10)]
        for i, (t, n) in enumerate(tickets):
            got = srv.wait(t, n, 7)
            assert np.array_equal(got[0], ref[0][4 * i:4 * i + 4])
            assert np.array_equal(got[1], ref[1][4 * i:4 * i + 4])
        st = srv.stats()
        assert st["completed"] == 10 and st["batches"] <= 2, st
    finally:
        srv.close()
    # a full batch does not wait for the linger
    srv = fl.Server([dense], mem_budget=1 << 30, max_batch=4, linger_ns=10_000_000_000)
    try:
        t, n = srv.submit(0, Q[:4], 7)
        got = srv.wait(t, n, 7, timeout_ns=5_000_000_000)
        assert _same(got, (ref[0][:4], ref[1][:4]))
    finally:
        srv.close()


def test_device_requests_equal_oracle(fl, two_indexes, oracles):
    """Requests whose queries are already in device memory: results written
    straight into device buffers (submit_to), or returned to the host
    (submit with a device input), equal the oracle's, in a mixed burst; set
    requests give their offsets on the device or, in every third request,
    on the host beside device items."""
    import torch
    dense, Q, sets, S = two_indexes
    rng = np.random.default_rng(7)
    reqs = _requests(Q, S, rng, 60)

    def dev(q):
        if isinstance(q, tuple):
            it, of = q
            return (torch.from_numpy(np.ascontiguousarray(it).view(np.int64)).cuda(),
                    torch.from_numpy(np.ascontiguousarray(of).view(np.int64)).cuda())
        return torch.from_numpy(np.ascontiguousarray(q).view(np.int16)).cuda()

    dq = [dev(q) for _, _, q, _ in reqs]
    for i, (fam, _, q, _) in enumerate(reqs):
        if fam == 1 and i % 3 == 1:
            dq[i] = (dq[i][0], np.ascontiguousarray(q[1], dtype=np.uint64))
    outs = [(torch.full((sz, k), -1, dtype=torch.int32, device="cuda"),
             torch.full((sz, k), -1, dtype=torch.int32, device="cuda"))
            for _, sz, _, k in reqs]
    torch.cuda.synchronize()
    srv = fl.Server([dense, sets], mem_budget=1 << 30, max_inflight=4, max_batch=512)
    try:
        tickets = []
        for i, ((fam, sz, q, k), d) in enumerate(zip(reqs, dq)):
            if i % 3 == 2:
                tickets.append(("host",) + srv.submit(fam, d, k))
            else:
                tickets.append(("dev",) + srv.submit_to(fam, d, k, outs[i]))
        for i, ((fam, sz, q, k), tk) in enumerate(zip(reqs, tickets)):
            want = _want(oracles, fam, q, k)
            if tk[0] == "host":
                got = srv.wait(tk[1], tk[2], k)
            else:
                srv.wait_done(tk[1])
                got = (outs[i][0].cpu().numpy().view(np.uint32),
                       outs[i][1].cpu().numpy().view(np.uint32))
            assert _same(got, want), (i, tk[0])
        log("device requests", srv.stats())
    finally:
        srv.close()
