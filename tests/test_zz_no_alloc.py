"""flinng_query_noalloc, the allocation-free batched query, against
flinng_query through the C ABI: ids and scores equal bit for bit on two
calls in a row, the second with a smaller batch (and another k), for a
bf16 dense index (rows projected in place), an fp32 dense index (operand
planes in the scratch array) and a set index, with one workgroup per query
and with the persistent grid; host inputs and a batch whose scratch would
exceed the array are refused with EINVAL."""
import ctypes

import numpy as np
import pytest

from gpu_common import log
from workloads import synth

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
            np.dtype(np.uint16): np.int16, np.dtype(np.float32): np.float32}[a.dtype]
    return torch.from_numpy(a.view(view)).cuda()


def _noalloc(env, gi, q_d, nq, k, persistent):
    torch, fl = env
    inp, keep = fl.make_input(q_d, gi.family)
    ids = torch.full((nq, k), -1, dtype=torch.int32, device="cuda")
    sc = torch.full((nq, k), -1, dtype=torch.int32, device="cuda")
    torch.cuda.synchronize()
    rc = fl.lib().flinng_query_noalloc(gi.handle, ctypes.byref(inp), k, ids.data_ptr(),
                                       sc.data_ptr(), int(persistent), fl.current_stream())
    fl.check(rc)
    torch.cuda.synchronize()
    return ids.cpu().numpy().view(np.uint32), sc.cpu().numpy().view(np.uint32)


def _cases():
    X, Q, _ = synth.dense_relu(N=6000, d=512, n_centres=60, nq=700)
    G, P, _ = synth.dense_gmm(N=3000, d=96, n_centres=60, nq=300)
    it, of, qit, qof, _ = synth.genome(n_base=4000, nq=700)
    return {"bf16": (X, Q, 1, 12, 16, 4, 60, 0), "fp32": (G, P, 0, 8, 6, 3, 60, 0),
            "sets": ((it, of), (qit, qof), 3, 2, 16, 4, 80, 18)}


CASES = _cases()


def _subset(q, a, b):
    if isinstance(q, tuple):
        it, of = q
        o = of[a:b + 1]
        return it[int(o[0]):int(o[-1])], (o - o[0]).astype(np.uint64)
    return q[a:b]


def _to_dev(torch, q):
    if isinstance(q, tuple):
        return (_dev(torch, q[0]), _dev(torch, q[1]))
    return _dev(torch, q)


@pytest.mark.parametrize("kind", ["bf16", "fp32", "sets"])
@pytest.mark.parametrize("persistent", [False, True])
def test_noalloc_equals_query(env, kind, persistent):
    torch, fl = env
    data, Q, fam, K, L, R, B, bb = CASES[kind]
    gi = fl.Index(data, fam, K, L, R, B, seed=17, bucket_bits=bb)
    nq = len(Q[1]) - 1 if isinstance(Q, tuple) else Q.shape[0]
    # first call: the whole batch, k = 10; second call: a smaller, different
    # batch and k = 7, so that nothing may carry over from the first
    for (a, b), k in (((0, nq), 10), ((nq - 123, nq), 7)):
        q = _subset(Q, a, b)
        log("noalloc", kind, "persistent", persistent, "queries", b - a, "k", k)
        want = gi.query(q, k, persistent=persistent)
        got = _noalloc(env, gi, _to_dev(torch, q), b - a, k, persistent)
        bad = np.nonzero(np.any(got[0] != want[0], axis=1))[0]
        assert len(bad) == 0, (kind, a, b, bad[:5])
        assert np.array_equal(got[1], want[1])


def test_noalloc_refuses_host_inputs_and_oversized_batches(env):
    torch, fl = env
    data, Q, fam, K, L, R, B, bb = CASES["fp32"]
    gi = fl.Index(data, fam, K, L, R, B, seed=17)
    inp, keep = fl.make_input(Q[:4], fam)  # host input
    ids = torch.empty((4, 10), dtype=torch.int32, device="cuda")
    rc = fl.lib().flinng_query_noalloc(gi.handle, ctypes.byref(inp), 10, ids.data_ptr(), None, 0,
                                       fl.current_stream())
    assert rc == fl.EINVAL
    # fp32 rows of d = 4096 need three bf16 planes of 8 KiB each per row:
    # 3000 rows exceed the 64 MiB array
    big = torch.zeros((3000, 4096), dtype=torch.float32, device="cuda")
    gb = fl.Index(np.random.default_rng(0).standard_normal((64, 4096)).astype(np.float32),
                  fam, 4, 2, 1, 4, seed=3)
    inp, keep = fl.make_input(big, fam)
    ids = torch.empty((3000, 10), dtype=torch.int32, device="cuda")
    rc = fl.lib().flinng_query_noalloc(gb.handle, ctypes.byref(inp), 10, ids.data_ptr(), None, 0,
                                       fl.current_stream())
    assert rc == fl.EINVAL
    assert b"split the batch" in fl.lib().flinng_last_error()
