"""FLINNG (group-testing near-neighbour search) on AMD MI355X / gfx950.

Python face of the C ABI in include/flinng.h: build an index on the GPU,
query it in batches, and serve mixed query streams with continuous batching.
All computation runs in the HIP library (libflinng.so); this package only
marshals arguments.
"""
import ctypes

import numpy as np

from ._lib import (  # noqa: F401
    SRP_F32, SRP_BF16, MINHASH_U32, MINHASH_U64, FlinngError, Params, Input,
    IndexInfo, ServeConfig, ServeStats, Theory, Text, check, lib, make_input, make_text,
    current_stream,
    EBUSY, EINVAL, ENOMEM, ETIMEDOUT, ESTATE,
)


def theory_params(N, s_k, s_k1, delta):
    """flinng_theory_params: the design the paper's analysis gives for N
    points, neighbour similarities s_k > s_k1 and failure probability delta
    (B, R, K hashes per table, L tables, threshold t, and the rates)."""
    th = Theory()
    check(lib().flinng_theory_params(int(N), float(s_k), float(s_k1), float(delta),
                                     ctypes.byref(th)))
    return {f: getattr(th, f) for f, _ in Theory._fields_}


def _stream(stream):
    if stream is None:
        return current_stream()
    if isinstance(stream, ctypes.c_void_p):
        return stream
    return ctypes.c_void_p(getattr(stream, "cuda_stream", stream))


class Index:
    """A FLINNG index resident on the current HIP device (flinng_build).
    text=(gram, radix, key): `data` is (symbols, offsets) of symbol
    sequences read as n-gram sets (flinng_build_text)."""

    def __init__(self, data, family, K, L, R, B, seed, dim=None, bucket_bits=0,
                 stream=None, text=None):
        self.family = family
        p = Params(family=family, K=K, L=L, R=R, B=B, bucket_bits=bucket_bits,
                   reserved=0, seed=seed)
        if family in (SRP_F32, SRP_BF16):
            p.dim = dim if dim is not None else data.shape[1]
        h = ctypes.c_void_p()
        if text is not None:
            t, keep = make_text(data, *text)
            check(lib().flinng_build_text(ctypes.byref(p), ctypes.byref(t), _stream(stream),
                                          ctypes.byref(h)))
        else:
            inp, keep = make_input(data, family)
            check(lib().flinng_build(ctypes.byref(p), ctypes.byref(inp), _stream(stream),
                                     ctypes.byref(h)))
        self._h = h
        del keep

    @property
    def handle(self):
        return self._h

    @property
    def info(self):
        return self.get_info()

    def insert(self, data, stream=None):
        """flinng_index_insert: add points (ids N, N+1, ...) to the index."""
        inp, keep = make_input(data, self.family)
        check(lib().flinng_index_insert(self._h, ctypes.byref(inp), _stream(stream)))
        del keep

    def get_info(self):
        info = IndexInfo()
        check(lib().flinng_index_get_info(self._h, ctypes.byref(info)))
        return info

    def query(self, q, k, persistent=False, stream=None, out=None):
        """flinng_query.  Host inputs/outputs: returns numpy (ids, scores).
        Device: pass out=(ids_tensor, scores_tensor or None) (uint32 as
        torch.int32 storage) and the call only enqueues work."""
        inp, keep = make_input(q, self.family)
        nq = inp.count
        if out is not None:
            ids_t, sc_t = out
            check(lib().flinng_query(self._h, ctypes.byref(inp), k, ids_t.data_ptr(),
                                     sc_t.data_ptr() if sc_t is not None else None,
                                     1, int(persistent), _stream(stream)))
            return out
        ids = np.empty((nq, k), dtype=np.uint32)
        sc = np.empty((nq, k), dtype=np.uint32)
        check(lib().flinng_query(self._h, ctypes.byref(inp), k, ids.ctypes.data,
                                 sc.ctypes.data, 0, int(persistent), _stream(stream)))
        del keep
        return ids, sc

    def query_text(self, seqs, text, k, persistent=False, stream=None, out=None):
        """flinng_query_text: queries given as symbol sequences (symbols,
        offsets) with text=(gram, radix, key); host results unless out=(ids,
        scores) device tensors are given."""
        t, keep = make_text(seqs, *text)
        nq = t.count
        if out is not None:
            ids_t, sc_t = out
            check(lib().flinng_query_text(self._h, ctypes.byref(t), k, ids_t.data_ptr(),
                                          sc_t.data_ptr() if sc_t is not None else None, 1,
                                          int(persistent), _stream(stream)))
            return out
        ids = np.empty((nq, k), dtype=np.uint32)
        sc = np.empty((nq, k), dtype=np.uint32)
        check(lib().flinng_query_text(self._h, ctypes.byref(t), k, ids.ctypes.data, sc.ctypes.data,
                                      0, int(persistent), _stream(stream)))
        del keep
        return ids, sc

    def query_threshold(self, q, t, max_per_query, stream=None, out=None):
        """flinng_query_threshold (Algorithm 2 at threshold t), host outputs:
        (ids [nq, max_per_query] uint32 padded with 0xFFFFFFFF, counts [nq]);
        out=(ids, counts) device tensors: the call only enqueues work."""
        inp, keep = make_input(q, self.family)
        nq = inp.count
        if out is not None:
            check(lib().flinng_query_threshold(self._h, ctypes.byref(inp), t, max_per_query,
                                               out[0].data_ptr(), out[1].data_ptr(), 1,
                                               _stream(stream)))
            return out
        ids = np.empty((nq, max(max_per_query, 1)), dtype=np.uint32)
        cnt = np.empty(nq, dtype=np.uint32)
        check(lib().flinng_query_threshold(self._h, ctypes.byref(inp), t, max_per_query,
                                           ids.ctypes.data, cnt.ctypes.data, 0, _stream(stream)))
        return ids[:, :max_per_query], cnt

    def debug_hash(self, q, stream=None):
        inp, keep = make_input(q, self.family)
        codes = np.empty((inp.count, self.info.L), dtype=np.uint32)
        check(lib().flinng_debug_hash(self._h, ctypes.byref(inp), codes.ctypes.data, 0,
                                      _stream(stream)))
        return codes

    def debug_projections(self, q, stream=None):
        """(proj [n, L*K] float32 before any recheck, (gamma, tau_abs)):
        the matrix-core projections and the bound under which their signs
        are not trusted (dense indexes)."""
        inp, keep = make_input(q, self.family)
        i = self.info
        proj = np.empty((inp.count, i.L * i.K), dtype=np.float32)
        bound = (ctypes.c_double * 2)()
        check(lib().flinng_debug_projections(self._h, ctypes.byref(inp), proj.ctypes.data,
                                             bound, 0, _stream(stream)))
        return proj, (bound[0], bound[1])

    def debug_counts(self, q, stream=None):
        inp, keep = make_input(q, self.family)
        c = np.empty((inp.count, self.info.R * self.info.B), dtype=np.uint8)
        check(lib().flinng_debug_counts(self._h, ctypes.byref(inp), c.ctypes.data, 0,
                                        _stream(stream)))
        return c

    def export(self, stream=None):
        """(offsets [L, 2^bits+1] uint64, cells uint32, groups [R, N] uint32)."""
        i = self.info
        offs = np.empty((i.L, (1 << i.bucket_bits) + 1), dtype=np.uint64)
        cells = np.empty(max(i.list_entries, 1), dtype=np.uint32)
        groups = np.empty((i.R, i.N), dtype=np.uint32)
        check(lib().flinng_index_export(self._h, offs.ctypes.data, cells.ctypes.data,
                                        groups.ctypes.data, _stream(stream)))
        return offs, cells[:i.list_entries], groups

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            lib().flinng_index_free(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Server:
    """Continuous-batching server over resident indexes (flinng_serve_*)."""

    def __init__(self, indexes, mem_budget=1 << 30, max_inflight=4, max_batch=4096,
                 max_queue=1 << 20, persistent=False, linger_ns=0):
        self._indexes = list(indexes)
        arr = (ctypes.c_void_p * len(self._indexes))(*[ix.handle.value for ix in self._indexes])
        cfg = ServeConfig(mem_budget=mem_budget, max_inflight=max_inflight,
                          max_batch=max_batch, max_queue=max_queue,
                          persistent=int(persistent), linger_ns=linger_ns)
        h = ctypes.c_void_p()
        check(lib().flinng_serve_create(arr, len(self._indexes), ctypes.byref(cfg),
                                        ctypes.byref(h)))
        self._h = h

    def _family(self, slot):
        # an out-of-range slot is marshalled as slot 0's family so that the
        # library itself rejects it
        ok = isinstance(slot, int) and 0 <= slot < len(self._indexes)
        return self._indexes[slot if ok else 0].family

    def submit(self, slot, q, k):
        inp, keep = make_input(q, self._family(slot))
        t = ctypes.c_uint64()
        check(lib().flinng_serve_submit(self._h, slot, ctypes.byref(inp), k, ctypes.byref(t)))
        return t.value, int(inp.count)

    def submit_to(self, slot, q, k, out):
        """Device request: q on the device (torch tensors, borrowed until
        the request completes) and out = (ids, scores or None) device
        tensors the batch writes into.  Complete it with wait_done."""
        inp, keep = make_input(q, self._family(slot))
        ids_t, sc_t = out
        t = ctypes.c_uint64()
        check(lib().flinng_serve_submit_to(self._h, slot, ctypes.byref(inp), k, ids_t.data_ptr(),
                                           sc_t.data_ptr() if sc_t is not None else None,
                                           ctypes.byref(t)))
        return t.value, int(inp.count)

    def submit_text(self, slot, seqs, text, k, out=None):
        """flinng_serve_submit_text: symbol sequences with text=(gram, radix,
        key); results into out=(ids, scores) device tensors (then complete
        with wait_done) or, without out, taken with wait."""
        t, keep = make_text(seqs, *text)
        tk = ctypes.c_uint64()
        ip = sp = None
        if out is not None:
            ip = out[0].data_ptr()
            sp = out[1].data_ptr() if out[1] is not None else None
        check(lib().flinng_serve_submit_text(self._h, slot, ctypes.byref(t), k, ip, sp,
                                             ctypes.byref(tk)))
        return tk.value, int(t.count)

    def wait_done(self, ticket, timeout_ns=-1):
        """Wait for a request submitted with submit_to."""
        check(lib().flinng_serve_wait(self._h, ticket, None, None, timeout_ns))

    def try_submit(self, slot, q, k):
        """Like submit, but returns (None, rc) instead of raising on refusal."""
        inp, keep = make_input(q, self._family(slot))
        t = ctypes.c_uint64()
        rc = lib().flinng_serve_submit(self._h, slot, ctypes.byref(inp), k, ctypes.byref(t))
        return (t.value if rc == 0 else None), rc

    def wait(self, ticket, nq, k, timeout_ns=-1):
        ids = np.empty((nq, k), dtype=np.uint32)
        sc = np.empty((nq, k), dtype=np.uint32)
        check(lib().flinng_serve_wait(self._h, ticket, ids.ctypes.data, sc.ctypes.data,
                                      timeout_ns))
        return ids, sc

    def poll(self, ticket):
        rc = lib().flinng_serve_poll(self._h, ticket)
        if rc < 0:
            check(rc)
        return rc == 1

    def stats(self):
        st = ServeStats()
        check(lib().flinng_serve_stats_get(self._h, ctypes.byref(st)))
        return {f: getattr(st, f) for f, _ in ServeStats._fields_}

    def reset_stats(self):
        check(lib().flinng_serve_stats_reset(self._h))

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            lib().flinng_serve_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
