"""GPU tests of the continuous-batching server (flinng_serve_*): results of
every request are identical alone and in a mixed burst over two resident
indexes of different hash families; admission by device memory; error paths.
"""
import numpy as np
import pytest

from gpu_common import log
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


def test_results_identical_alone_and_in_mix(fl, two_indexes):
    dense, Q, sets, S = two_indexes
    rng = np.random.default_rng(1)
    reqs = _requests(Q, S, rng, 120)
    # reference: each request alone through the plain batched path
    alone = [(dense if fam == 0 else sets).query(q, k) for fam, sz, q, k in reqs]
    srv = fl.Server([dense, sets], mem_budget=1 << 30, max_inflight=3, max_batch=256)
    try:
        # alone through the server (one at a time)
        for (fam, sz, q, k), ref in zip(reqs[:20], alone[:20]):
            t, n = srv.submit(fam, q, k)
            got = srv.wait(t, n, k)
            assert np.array_equal(got[0], ref[0]) and np.array_equal(got[1], ref[1])
        # mixed burst: everything submitted before anything is waited on
        tickets = [srv.submit(fam, q, k) for fam, sz, q, k in reqs]
        for (fam, sz, q, k), ref, (t, n) in zip(reqs, alone, tickets):
            got = srv.wait(t, n, k)
            assert np.array_equal(got[0], ref[0]) and np.array_equal(got[1], ref[1])
        st = srv.stats()
        log("serve stats", st)
        assert st["completed"] == 140 and st["batches"] >= 2
        assert st["p99_ms"] >= st["p50_ms"] > 0
    finally:
        srv.close()


def test_admission_by_memory(fl, two_indexes):
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
    one = dense.query(Q[:8], 10)
    srv = fl.Server([dense], mem_budget=1 << 20, max_inflight=4, max_batch=8)
    try:
        tickets = [srv.submit(0, Q[:8], 10) for _ in range(12)]
        for t, n in tickets:
            got = srv.wait(t, n, 10)
            assert np.array_equal(got[0], one[0])
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


def test_linger_coalesces(fl, two_indexes):
    dense, Q, sets, S = two_indexes
    ref = dense.query(Q[:40], 7)
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
        assert np.array_equal(got[0], ref[0][:4])
    finally:
        srv.close()
