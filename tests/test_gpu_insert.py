"""Streaming insert (flinng_index_insert) on the GPU against the oracle's
index built under the same reading: the first N0 points take Algorithm 1's
groups, the arrivals the block rule (blocks of B arrivals, a keyed
permutation of the groups per block and repetition), and the reverse index
holds the cells of all points.  After every insert the exported index
(groups, offsets, lists), the per-cell counts and the ids and scores of both
launch modes equal the oracle's, bit for bit.  Batches cross block
boundaries and make cells outgrow their member stride.  While a server keeps
serving, every request's answer equals the oracle's answer for one version
of the index (before or after each insert), and versions never go back."""
import threading
import time

import numpy as np
import pytest

import oracle
from gpu_common import fam_oracle, log, oracle_query
from workloads import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def fl():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a ROCm device"
    import paper_2106_11565_amd as flinng
    flinng.lib()
    return flinng


def _rows(data, a, b):
    if isinstance(data, tuple):
        it, of = data
        o = of[a:b + 1]
        return it[int(o[0]):int(o[-1])], (o - o[0]).astype(np.uint64)
    return data[a:b]


def _check(gi, oi, q, ks=(1, 10, 65)):
    offs, cells, groups = gi.export()
    assert gi.info.N == oi.N
    assert np.array_equal(groups, oi.g)
    assert np.array_equal(offs, oi.offsets)
    assert np.array_equal(cells, oi.cells)
    assert np.array_equal(gi.debug_counts(q), oi.counts(oi.hash(q)))
    for k in ks:
        want = oracle_query(oi, q, k)
        for pers in (False, True):
            got = gi.query(q, k, persistent=pers)
            bad = np.nonzero(np.any(got[0] != want[0], axis=1))[0]
            assert len(bad) == 0, (k, pers, bad[:5])
            assert np.array_equal(got[1], want[1]), (k, pers)


def _case(kind):
    if kind == "bf16":
        X, Q, _ = synth.dense_relu(N=6000, d=512, n_centres=60, nq=120)
        return X, Q, 1, 12, 16, 4, 60, 0, 4000
    if kind == "sets":
        it, of, qit, qof, _ = synth.genome(n_base=3000, nq=120)
        return (it, of), (qit, qof), 3, 2, 16, 4, 80, 18, 4000
    # fp32 rows, R * B > 2^16 cells: 32-bit cell ids, 128 KiB of counters
    X, Q, _ = synth.dense_gmm(N=60000, d=16, n_centres=400, sigma=0.05, nq=60)
    return X, Q, 0, 6, 5, 8, 16384, 0, 40000


@pytest.mark.parametrize("kind", ["bf16", "sets", "fp32_u32_cells"])
def test_insert_equals_oracle(fl, kind):
    import torch
    data, Q, fam, K, L, R, B, bb, N0 = _case(kind)
    N = len(data[1]) - 1 if isinstance(data, tuple) else data.shape[0]
    gi = fl.Index(_rows(data, 0, N0), fam, K, L, R, B, seed=29, bucket_bits=bb)
    oi = oracle.OracleIndex(fam_oracle(fam), _rows(data, 0, N0), K, L, R, B, 29,
                            bucket_bits=bb if bb else None)
    _check(gi, oi, Q)
    # batches: one point, a partial block, a run over several blocks, the rest
    cuts = [N0, N0 + 1, N0 + B - 1, min(N, N0 + 3 * B + 5), N]
    for i, (a, b) in enumerate(zip(cuts[:-1], cuts[1:])):
        if b <= a:
            continue
        part = _rows(data, a, b)
        if i == 2:  # device input for one batch
            if isinstance(part, tuple):
                part = (torch.from_numpy(part[0].view(np.int64)).cuda(),
                        torch.from_numpy(part[1].view(np.int64)).cuda())
            else:
                view = np.int16 if part.dtype == np.uint16 else np.float32
                part = torch.from_numpy(np.ascontiguousarray(part).view(view)).cuda()
            torch.cuda.synchronize()
        gi.insert(part)
        oi.insert(_rows(data, a, b))
        log("insert", kind, a, b, "N", gi.info.N, "bytes", gi.info.device_bytes)
        _check(gi, oi, Q)
    sizes = np.stack([np.bincount(oi.g[r], minlength=B) for r in range(R)])
    stride0 = (-(-N0 // B) + 3) // 4 * 4
    assert sizes.max() > stride0, "the inserts should outgrow the build's member stride"
    assert sizes.max() - sizes.min() <= 2
    # the fixed-threshold query reads the same cells
    cnt = oi.counts(oi.hash(Q))
    t = max(1, L // 2)
    ids, counts = gi.query_threshold(Q, t, N)
    for j in range(len(cnt)):
        want = np.nonzero(oracle.query_fixed_t(cnt[j], oi.g, B, t))[0]
        assert counts[j] == len(want) and np.array_equal(np.sort(ids[j][:counts[j]]), want)


def test_insert_while_serving(fl):
    """A client keeps submitting the same requests while two inserts land:
    each answer is the oracle's answer before the first insert, between the
    two, or after the second, and a later request never sees an older
    version."""
    X, Q, _ = synth.dense_relu(N=5000, d=256, n_centres=50, nq=160)
    N0, cuts = 3000, [3000, 4100, 5000]
    gi = fl.Index(X[:N0], fl.SRP_BF16, 12, 12, 4, 50, seed=41)
    oi = oracle.OracleIndex(oracle.SRP_BF16, X[:N0], 12, 12, 4, 50, 41)
    versions = [oracle_query(oi, Q, 10)]
    for a, b in zip(cuts[:-1], cuts[1:]):
        oi.insert(X[a:b])
        versions.append(oracle_query(oi, Q, 10))
    assert not np.array_equal(versions[0][0], versions[-1][0])
    srv = fl.Server([gi], mem_budget=1 << 30, max_inflight=3, max_batch=64)
    seen, stop, errors = [], threading.Event(), []

    def client():
        try:
            while not stop.is_set():
                tickets = [(srv.submit(0, Q[p:p + 40], 10), p) for p in range(0, 160, 40)]
                for (t, n), p in tickets:
                    ids, sc = srv.wait(t, n, 10)
                    v = [i for i, (wi, ws) in enumerate(versions)
                         if np.array_equal(ids, wi[p:p + n]) and np.array_equal(sc, ws[p:p + n])]
                    seen.append((p, v))
        except Exception as e:  # noqa: BLE001
            errors.append(e)

    th = threading.Thread(target=client)
    th.start()
    try:
        time.sleep(0.2)
        for a, b in zip(cuts[:-1], cuts[1:]):
            gi.insert(X[a:b])
            time.sleep(0.2)
    finally:
        stop.set()
        th.join()
        srv.close()
    assert not errors, errors
    assert seen and all(v for _, v in seen), [s for s in seen if not s[1]][:3]
    # versions only move forward (the smallest version consistent with each
    # answer is nondecreasing; answers that several versions share allow any)
    lo = 0
    for _, v in seen:
        assert max(v) >= lo
        lo = max(lo, min(v))
    log("served", len(seen), "requests across", len(versions), "index versions")
