"""ctypes driver for the C oracle (test infrastructure only; see __init__)."""
import ctypes
import os
import subprocess
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "flinng_oracle.c")
_SO = os.path.join(_HERE, "liboracle.so")

SRP_F32, SRP_BF16, MINHASH_U32, MINHASH_U64 = 0, 1, 2, 3

_lock = threading.Lock()
_lib = None


def build_lib(force=True):
    """Compile the oracle with gcc (plain -O2, no fast-math, no FMA contraction:
    the exact-sum fallback relies on IEEE round-to-nearest Two-Sum)."""
    cmd = ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-fopenmp",
           "-ffp-contract=off", "-fno-fast-math", "-o", _SO + ".tmp", _SRC, "-lm"]
    if force or not os.path.exists(_SO):
        subprocess.check_call(cmd)
        os.replace(_SO + ".tmp", _SO)
    return _SO


def lib():
    global _lib
    with _lock:
        if _lib is None:
            if not os.path.exists(_SO):
                build_lib(force=True)
            _lib = _bind(ctypes.CDLL(_SO))
    return _lib


def _bind(L):
    u64, u32, i64, dbl, vp = (ctypes.c_uint64, ctypes.c_uint32, ctypes.c_int64,
                              ctypes.c_double, ctypes.c_void_p)
    sig = {
        "or_sm64": (u64, [u64, u64]),
        "or_mix64_public": (u64, [u64]),
        "or_hyperplane_entry": (dbl, [u64, u64, u32, u32]),
        "or_hyperplanes": (None, [u64, u32, u32, vp]),
        "or_srp_codes": (u64, [vp, u64, u32, vp, u32, u32, vp]),
        "or_exact_dot_sign": (ctypes.c_int, [vp, vp, u32]),
        "or_minhash_codes": (None, [vp, vp, u64, u64, u32, u32, u32, vp]),
        "or_text_items": (u64, [vp, vp, u64, u32, u32, u64, u32, vp, vp]),
        "or_permute": (u64, [u64, u32, u64, u64]),
        "or_groups": (None, [u64, u32, u32, u64, vp]),
        "or_members": (None, [vp, u64, u32, u32, vp, vp]),
        "or_stream_groups": (None, [u64, u32, u32, u64, u64, u64, vp]),
        "or_build_lists": (i64, [vp, vp, u64, u32, u32, u32, u32, vp, vp, u64]),
        "or_counts": (None, [vp, vp, u32, u32, u32, vp, u64, vp]),
        "or_counts_brute": (None, [vp, vp, u64, u32, u32, u32, vp, u64, vp]),
        "or_decode": (None, [vp, vp, u64, u32, u32, u32, vp, vp]),
        "or_query_many": (None, [vp, vp, u32, u32, vp, u64, u32, u32, vp, u64, u32, vp, vp]),
        "or_set_threads": (None, [ctypes.c_int]),
        "or_get_threads": (ctypes.c_int, []),
        "or_query_fixed_t": (None, [vp, vp, u64, u32, u32, u32, vp]),
    }
    for name, (res, args) in sig.items():
        f = getattr(L, name)
        f.restype = res
        f.argtypes = args
    return L


def _p(a):
    return a.ctypes.data_as(ctypes.c_void_p)


def sm64(s, i):
    """i-th output of SplitMix64 started at state s (counter-based)."""
    return int(lib().or_sm64(int(s) & (2**64 - 1), int(i) & (2**64 - 1)))


def mix64(z):
    return int(lib().or_mix64_public(int(z) & (2**64 - 1)))


def bf16_to_f64(u16):
    """Exact value of stored bf16 bit patterns, as FP64."""
    u16 = np.ascontiguousarray(u16, dtype=np.uint16)
    return (u16.astype(np.uint32) << 16).view(np.float32).astype(np.float64)


def hyperplanes(seed, H, d):
    """SRP hyperplanes: H x d FP64, entries (popcount(sm64) - 32) / 4."""
    w = np.empty((H, d), dtype=np.float64)
    lib().or_hyperplanes(seed, H, d, _p(w))
    return w


def srp_codes(x, seed, K, L, w=None, return_exact_count=False):
    """Bucket codes of dense rows x (FP64 view of the stored values): bit j of
    table t is the exact sign of x . w[t*K + j] (> 0 gives 1)."""
    x = np.ascontiguousarray(x, dtype=np.float64)
    n, d = x.shape
    if w is None:
        w = hyperplanes(seed, K * L, d)
    w = np.ascontiguousarray(w, dtype=np.float64)
    codes = np.empty((n, L), dtype=np.uint32)
    nex = lib().or_srp_codes(_p(x), n, d, _p(w), K, L, _p(codes))
    return (codes, int(nex)) if return_exact_count else codes


def exact_dot_sign(x, w):
    x = np.ascontiguousarray(x, dtype=np.float64)
    w = np.ascontiguousarray(w, dtype=np.float64)
    assert x.shape == w.shape and x.ndim == 1
    return int(lib().or_exact_dot_sign(_p(x), _p(w), x.shape[0]))


def minhash_codes(items, offsets, seed, K, L, b):
    """Bucket codes of item sets (CSR): per table, fold of K MinHash values to
    the top b bits of a 64-bit mix."""
    items = np.ascontiguousarray(items).astype(np.uint64, copy=False)
    offsets = np.ascontiguousarray(offsets, dtype=np.uint64)
    n = offsets.shape[0] - 1
    codes = np.empty((n, L), dtype=np.uint32)
    if items.size == 0:
        items = np.zeros(1, dtype=np.uint64)
    lib().or_minhash_codes(_p(items), _p(offsets), n, seed, K, L, b, _p(codes))
    return codes


def text_items(symbols, offsets, gram, radix, key, item_bits):
    """Item sets (CSR, uint64 / uint32 per item_bits) of symbol sequences read
    as n-grams: each window's base-radix value mixed with the key."""
    sym = np.ascontiguousarray(symbols, dtype=np.uint8)
    off = np.ascontiguousarray(offsets, dtype=np.uint64)
    n = off.shape[0] - 1
    cap = max(1, int(off[-1] - off[0]) if n else 1)
    items = np.empty(cap, dtype=np.uint64)
    ioff = np.empty(n + 1, dtype=np.uint64)
    if sym.size == 0:
        sym = np.zeros(1, dtype=np.uint8)
    m = lib().or_text_items(_p(sym), _p(off), n, gram, radix, int(key) & (2**64 - 1), item_bits,
                            _p(items), _p(ioff))
    items = items[:m].copy()
    return (items if item_bits == 64 else items.astype(np.uint32)), ioff


def permute(N, r, seed, x):
    return int(lib().or_permute(N, r, seed, x))


def groups(N, R, B, seed):
    """g[r, x] = P_r(x) mod B (Algorithm 1)."""
    g = np.empty((R, N), dtype=np.uint32)
    lib().or_groups(N, R, B, seed, _p(g))
    return g


def stream_groups(N0, R, B, seed, x0, n):
    """Groups (R x n) of the points x0 .. x0+n-1 that arrive after the first
    N0: blocks of B arrivals, each a keyed permutation of the B groups."""
    g = np.empty((R, n), dtype=np.uint32)
    if n:
        lib().or_stream_groups(N0, R, B, seed, x0, n, _p(g))
    return g


def members(g, B):
    R, N = g.shape
    g = np.ascontiguousarray(g, dtype=np.uint32)
    off = np.empty((R, B + 1), dtype=np.uint64)
    mem = np.empty((R, N), dtype=np.uint32)
    lib().or_members(_p(g), N, R, B, _p(off), _p(mem))
    return off, mem


def build_lists(codes, g, B, nbits):
    """Reverse index: per table, bucket -> ascending distinct cell ids."""
    codes = np.ascontiguousarray(codes, dtype=np.uint32)
    g = np.ascontiguousarray(g, dtype=np.uint32)
    N, L = codes.shape
    R = g.shape[0]
    offsets = np.empty((L, (1 << nbits) + 1), dtype=np.uint64)
    cap = N * L * R
    cells = np.empty(max(cap, 1), dtype=np.uint32)
    n = lib().or_build_lists(_p(codes), _p(g), N, L, R, B, nbits, _p(offsets),
                             _p(cells), cap)
    assert n >= 0
    return offsets, cells[:n].copy()


def counts(offsets, cells, qcodes, ncells, nbits):
    qcodes = np.ascontiguousarray(qcodes, dtype=np.uint32)
    nq, L = qcodes.shape
    out = np.empty((nq, ncells), dtype=np.uint8)
    cells = np.ascontiguousarray(cells, dtype=np.uint32)
    if cells.size == 0:
        cells = np.zeros(1, dtype=np.uint32)
    lib().or_counts(_p(offsets), _p(cells), L, nbits, ncells, _p(qcodes), nq,
                    _p(out))
    return out


def counts_brute(codes, g, B, qcodes):
    codes = np.ascontiguousarray(codes, dtype=np.uint32)
    g = np.ascontiguousarray(g, dtype=np.uint32)
    qcodes = np.ascontiguousarray(qcodes, dtype=np.uint32)
    N, L = codes.shape
    R = g.shape[0]
    nq = qcodes.shape[0]
    out = np.empty((nq, R * B), dtype=np.uint8)
    lib().or_counts_brute(_p(codes), _p(g), N, L, R, B, _p(qcodes), nq, _p(out))
    return out


def decode(cnt, g, B, k):
    """Algorithm 3 (threshold relaxation) of one query's cell counts: the k
    smallest keys (-m(x), c*(x), x), ids and scores (m(x))."""
    cnt = np.ascontiguousarray(cnt, dtype=np.uint8)
    g = np.ascontiguousarray(g, dtype=np.uint32)
    R, N = g.shape
    ids = np.empty(k, dtype=np.uint32)
    sc = np.empty(k, dtype=np.uint32)
    lib().or_decode(_p(cnt), _p(g), N, R, B, k, _p(ids), _p(sc))
    return ids, sc


def set_threads(n):
    """Threads of the oracle's parallel loops (1 for a one-core baseline)."""
    lib().or_set_threads(int(n))


def get_threads():
    return int(lib().or_get_threads())


def query_fixed_t(cnt, g, B, t):
    """Algorithm 2 at fixed threshold t: boolean mask of reported points."""
    cnt = np.ascontiguousarray(cnt, dtype=np.uint8)
    g = np.ascontiguousarray(g, dtype=np.uint32)
    R, N = g.shape
    out = np.empty(N, dtype=np.uint8)
    lib().or_query_fixed_t(_p(cnt), _p(g), N, R, B, t, _p(out))
    return out.astype(bool)


class OracleIndex:
    """A whole FLINNG index built by the oracle (Algorithm 1 + reverse index).

    family: SRP_F32 / SRP_BF16 (dense rows; data given as the stored fp32
    array or bf16 bit patterns) or MINHASH_U32 / MINHASH_U64 (CSR item sets,
    data = (items, offsets)).
    """

    def __init__(self, family, data, K, L, R, B, seed, bucket_bits=None):
        self.family, self.K, self.L, self.R, self.B = family, K, L, R, B
        self.seed = seed
        if family in (SRP_F32, SRP_BF16):
            self.nbits = K
            x = self._dense(data)
            self.N, self.d = x.shape
            self.w = hyperplanes(seed, K * L, self.d)
            self.codes = srp_codes(x, seed, K, L, w=self.w)
        else:
            self.nbits = bucket_bits
            items, offs = data
            self.N = len(offs) - 1
            self.codes = minhash_codes(items, offs, seed, K, L, bucket_bits)
        self.g = groups(self.N, R, B, seed)
        self.N0 = self.N
        self.offsets, self.cells = build_lists(self.codes, self.g, B, self.nbits)

    def insert(self, data):
        """Points arriving after the build (ids N, N+1, ...): hashed with the
        same functions, grouped by stream_groups, and the reverse index
        rebuilt over all points."""
        codes = self.hash(data)
        n = codes.shape[0]
        g = stream_groups(self.N0, self.R, self.B, self.seed, self.N, n)
        self.codes = np.concatenate([self.codes, codes])
        self.g = np.concatenate([self.g, g], axis=1)
        self.N += n
        self.offsets, self.cells = build_lists(self.codes, self.g, self.B, self.nbits)

    def _dense(self, data):
        if self.family == SRP_BF16:
            return bf16_to_f64(data)
        return np.asarray(data, dtype=np.float32).astype(np.float64)

    def hash(self, q):
        if self.family in (SRP_F32, SRP_BF16):
            return srp_codes(self._dense(q), self.seed, self.K, self.L, w=self.w)
        items, offs = q
        return minhash_codes(items, offs, self.seed, self.K, self.L, self.nbits)

    def counts(self, qcodes):
        return counts(self.offsets, self.cells, qcodes, self.R * self.B,
                      self.nbits)

    def query(self, q, k):
        """Full query: hash, count through the reverse index, relax
        (Algorithm 3), queries spread over the oracle's threads."""
        return self.query_codes(self.hash(q), k)

    def query_codes(self, qc, k):
        qc = np.ascontiguousarray(qc, dtype=np.uint32)
        nq = qc.shape[0]
        ids = np.empty((nq, k), dtype=np.uint32)
        sc = np.empty((nq, k), dtype=np.uint32)
        cells = self.cells if self.cells.size else np.zeros(1, dtype=np.uint32)
        g = np.ascontiguousarray(self.g, dtype=np.uint32)
        lib().or_query_many(_p(self.offsets), _p(cells), self.L, self.nbits, _p(g), self.N,
                            self.R, self.B, _p(qc), nq, k, _p(ids), _p(sc))
        return ids, sc
