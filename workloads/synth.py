"""Seeded synthetic workloads shaped like the paper's datasets.

This module only produces inputs (and their exact ground-truth neighbours in
``truth.py``).  It holds none of FLINNG's arithmetic: the hashing, grouping,
counting and decoding live in the HIP library and, independently, in the
oracle.  Item ids of n-gram sets are made with MurmurHash3's 64-/32-bit
finalisers (Appleby, public domain), which FLINNG itself never uses.

The paper's datasets are not available; these generators stand in for their
shapes (Table 1): genome reads as sets of 20-gram ids (PromethION/RefSeq
shaped), URL-like strings as sets of character 3-gram ids (URL shaped) and
dense non-negative CNN-like embeddings (YFCC100M shaped), plus a small
Gaussian mixture.
"""
import os
from concurrent.futures import ThreadPoolExecutor

import numpy as np

M64 = np.uint64(0xFFFFFFFFFFFFFFFF)


def _workers():
    return max(1, min(16, os.cpu_count() or 1))


def fmix64(k):
    """MurmurHash3 64-bit finaliser, vectorised over uint64."""
    k = np.asarray(k, dtype=np.uint64).copy()
    with np.errstate(over="ignore"):
        k ^= k >> np.uint64(33)
        k *= np.uint64(0xFF51AFD7ED558CCD)
        k ^= k >> np.uint64(33)
        k *= np.uint64(0xC4CEB9FE1A85EC53)
        k ^= k >> np.uint64(33)
    return k


def fmix32(h):
    """MurmurHash3 32-bit finaliser, vectorised over uint32."""
    h = np.asarray(h, dtype=np.uint32).copy()
    with np.errstate(over="ignore"):
        h ^= h >> np.uint32(16)
        h *= np.uint32(0x85EBCA6B)
        h ^= h >> np.uint32(13)
        h *= np.uint32(0xC2B2AE35)
        h ^= h >> np.uint32(16)
    return h


def f32_to_bf16(x):
    """Round float32 values to bf16 (round to nearest even); returns the bf16
    bit patterns as uint16.  Inputs are finite."""
    u = np.ascontiguousarray(x, dtype=np.float32).view(np.uint32)
    r = (u + np.uint32(0x7FFF) + ((u >> np.uint32(16)) & np.uint32(1))) >> np.uint32(16)
    return r.astype(np.uint16)


def bf16_to_f32(u16):
    return (np.asarray(u16, dtype=np.uint16).astype(np.uint32) << np.uint32(16)).view(np.float32)


# --------------------------------------------------------------------------
# Dense: Gaussian mixture (small "plain FLINNG" case)

def dense_gmm(N=10000, d=128, n_centres=100, sigma=0.1, seed=0, nq=100,
              q_sigma=0.05, q_seed=1):
    """Centres ~ N(0, I_d); point i = centre[a_i] + sigma * z, a_i ~ U{centres};
    computed in FP64, stored as fp32 (round to nearest).  Queries: nq distinct
    dataset points + q_sigma * z, stored as fp32.
    Returns (X fp32 [N,d], Q fp32 [nq,d], qbase int64 [nq])."""
    rng = np.random.default_rng(seed)
    centres = rng.standard_normal((n_centres, d))
    a = rng.integers(0, n_centres, N)
    X = (centres[a] + sigma * rng.standard_normal((N, d))).astype(np.float32)
    rq = np.random.default_rng(q_seed)
    qbase = rq.choice(N, size=min(nq, N), replace=False)
    Q = (X[qbase].astype(np.float64) + q_sigma * rq.standard_normal((len(qbase), d))).astype(np.float32)
    return X, Q, qbase


# --------------------------------------------------------------------------
# Dense: non-negative ReLU-like embeddings (CNN-embedding shaped)

def _relu_centres(n_centres, d, p_zero, seed):
    rng = np.random.default_rng([seed, 0])
    mask = rng.random((n_centres, d), dtype=np.float32) >= p_zero
    vals = np.abs(rng.standard_normal((n_centres, d), dtype=np.float32))
    return np.where(mask, vals, np.float32(0.0)), mask


def dense_relu(N=1_000_000, d=4096, n_centres=10000, p_zero=0.6, sigma=0.1,
               seed=0, nq=10000, q_sigma=0.05, q_seed=1, chunk=16384):
    """Centres: each coordinate is 0 w.p. p_zero, else |N(0,1)|.  A point picks
    a centre uniformly and is max(0, c + sigma*z) on the centre's support, 0
    elsewhere (about 60% zeros).  Queries are nq distinct dataset points
    perturbed the same way with q_sigma.  Values are computed in float32 and
    stored as bf16 (round to nearest even).  Chunk j of the data uses its own
    stream (seed, 1, j), so any row range can be regenerated independently.
    Returns (X bf16-bits uint16 [N,d], Q uint16 [nq,d], qbase int64 [nq])."""
    centres, mask = _relu_centres(n_centres, d, p_zero, seed)
    X = np.empty((N, d), dtype=np.uint16)
    assign = np.empty(N, dtype=np.int64)

    def fill(j):
        s = j * chunk
        e = min(N, s + chunk)
        rng = np.random.default_rng([seed, 1, j])
        a = rng.integers(0, n_centres, e - s)
        z = rng.standard_normal((e - s, d), dtype=np.float32)
        v = np.maximum(centres[a] + np.float32(sigma) * z, np.float32(0.0))
        v = np.where(mask[a], v, np.float32(0.0))
        X[s:e] = f32_to_bf16(v)
        assign[s:e] = a

    with ThreadPoolExecutor(_workers()) as ex:
        list(ex.map(fill, range((N + chunk - 1) // chunk)))
    rq = np.random.default_rng([q_seed, 2])
    qbase = rq.choice(N, size=min(nq, N), replace=False)
    z = rq.standard_normal((len(qbase), d), dtype=np.float32)
    xb = bf16_to_f32(X[qbase])
    v = np.maximum(xb + np.float32(q_sigma) * z, np.float32(0.0))
    v = np.where(mask[assign[qbase]], v, np.float32(0.0))
    Q = f32_to_bf16(v)
    return X, Q, qbase


# --------------------------------------------------------------------------
# Sets: genome reads as sets of 20-gram ids

def _grams_2bit(A, n):
    """2-bit packed n-grams of rows of A (uint8 bases 0..3)."""
    rows, length = A.shape
    w = length - n + 1
    G = np.zeros((rows, w), dtype=np.uint64)
    for j in range(n):
        G |= A[:, j:j + w].astype(np.uint64) << np.uint64(2 * (n - 1 - j))
    return G


def _csr_unique_rows(V):
    """Per-row sorted distinct values of a 2-D array -> (items, offsets)."""
    S = np.sort(V, axis=1)
    keep = np.ones(S.shape, dtype=bool)
    keep[:, 1:] = S[:, 1:] != S[:, :-1]
    cnt = keep.sum(axis=1)
    offsets = np.zeros(S.shape[0] + 1, dtype=np.uint64)
    np.cumsum(cnt, out=offsets[1:])
    return S[keep], offsets


def _substitute(A, s, rng, alphabet):
    """s[i] substitutions at distinct positions of row i, each to a different
    symbol."""
    rows, length = A.shape
    A = A.copy()
    smax = int(s.max()) if rows else 0
    pos = np.argsort(rng.random((rows, length)), axis=1)[:, :smax]
    delta = rng.integers(1, alphabet, (rows, smax))
    for e in range(smax):
        sel = s > e
        r = np.nonzero(sel)[0]
        p = pos[sel, e]
        A[r, p] = (A[r, p].astype(np.int64) + delta[sel, e]) % alphabet
    return A


def _genome_items(A, gram, key, chunk=65536):
    items, offs = [], [np.zeros(1, dtype=np.uint64)]
    base = np.uint64(0)
    for s in range(0, A.shape[0], chunk):
        G = _grams_2bit(A[s:s + chunk], gram)
        it, of = _csr_unique_rows(fmix64(G ^ key))
        items.append(it)
        offs.append(of[1:] + base)
        base = base + of[-1]
    return np.concatenate(items), np.concatenate(offs)


def _text_of_rows(A, lens=None):
    """Symbol sequences (uint8 symbols, offsets) of the rows of A (the first
    lens[i] symbols of row i, or whole rows)."""
    if lens is None:
        return (np.ascontiguousarray(A, dtype=np.uint8).ravel(),
                np.arange(0, A.shape[0] * A.shape[1] + 1, A.shape[1], dtype=np.uint64))
    keep = np.arange(A.shape[1])[None, :] < np.asarray(lens)[:, None]
    offs = np.zeros(A.shape[0] + 1, dtype=np.uint64)
    np.cumsum(np.asarray(lens, dtype=np.uint64), out=offs[1:])
    return A[keep].astype(np.uint8), offs


def genome(n_base=500_000, read_len=100, gram=20, seed=0, nq=10000, q_seed=2,
           max_sub=5, text=False):
    """n_base random reads over {A,C,G,T} plus one mutated copy of each (1..5
    substitutions at distinct positions, each to a different base): ids
    0..n_base-1 are the base reads, n_base+i is the copy of read i.  Each read
    is the set of its 20-gram ids, 20-grams 2-bit packed then hashed to 64 bits
    with the MurmurHash3 finaliser under a seeded key.  Queries: nq distinct
    base reads, freshly mutated the same way.
    Returns (items u64, offsets u64 [N+1], q_items, q_offsets, qbase)."""
    rng = np.random.default_rng([seed, 10])
    key = np.uint64(rng.integers(0, 2**63, dtype=np.int64)) | np.uint64(1)
    A = rng.integers(0, 4, (n_base, read_len), dtype=np.uint8)
    s = rng.integers(1, max_sub + 1, n_base)
    C = _substitute(A, s, rng, 4)
    items, offs = _genome_items(np.concatenate([A, C]), gram, key)
    rq = np.random.default_rng([q_seed, 11])
    qbase = rq.choice(n_base, size=min(nq, n_base), replace=False)
    sq = rq.integers(1, max_sub + 1, len(qbase))
    QA = _substitute(A[qbase], sq, rq, 4)
    qitems, qoffs = _genome_items(QA, gram, key)
    if text:
        # the reads themselves (bases 0..3), which the items are the 2-bit
        # packed n-grams of, mixed with the key
        extra = {"data": _text_of_rows(np.concatenate([A, C])), "queries": _text_of_rows(QA),
                 "gram": gram, "radix": 4, "key": int(key)}
        return items, offs, qitems, qoffs, qbase, extra
    return items, offs, qitems, qoffs, qbase


# --------------------------------------------------------------------------
# Sets: URL-like strings as sets of character 3-gram ids

def _edit(A, lens, nedit, rng, alphabet):
    """Apply nedit[i] uniform random edits (insert / delete / substitute) to
    row i of the padded symbol array A (padding -1)."""
    A = A.copy()
    lens = lens.copy()
    rows, W = A.shape
    cols = np.arange(W)[None, :]
    for e in range(int(nedit.max()) if rows else 0):
        act = nedit > e
        op = rng.integers(0, 3, rows)
        u = rng.random(rows)
        sym = rng.integers(0, alphabet, rows)
        dsub = rng.integers(1, alphabet, rows)
        # insert
        ins = act & (op == 0)
        p = np.minimum((u * (lens + 1)).astype(np.int64), lens)
        if ins.any():
            src = np.where(cols < p[:, None], cols, cols - 1).clip(0, W - 1)
            B = np.take_along_axis(A, src, axis=1)
            B[np.arange(rows), np.minimum(p, W - 1)] = sym
            A = np.where(ins[:, None], B, A)
            lens = np.where(ins, lens + 1, lens)
        # delete
        dl = act & (op == 1) & (lens > 3)
        p = np.minimum((u * lens).astype(np.int64), lens - 1)
        if dl.any():
            src = np.where(cols < p[:, None], cols, cols + 1).clip(0, W - 1)
            B = np.take_along_axis(A, src, axis=1)
            B[np.arange(rows), lens - 1] = -1
            A = np.where(dl[:, None], B, A)
            lens = np.where(dl, lens - 1, lens)
        # substitute
        sb = act & (op == 2)
        p = np.minimum((u * lens).astype(np.int64), lens - 1)
        if sb.any():
            r = np.nonzero(sb)[0]
            A[r, p[r]] = (A[r, p[r]].astype(np.int64) + dsub[r]) % alphabet
    return A, lens


def _url_items(A, lens, key32):
    rows, W = A.shape
    A64 = A.astype(np.int64)
    P = A64[:, :-2] * 1600 + A64[:, 1:-1] * 40 + A64[:, 2:]
    valid = np.arange(W - 2)[None, :] < (lens - 2)[:, None]
    H = fmix32((P.astype(np.uint32)) ^ key32)
    # push invalid positions to a sentinel above every id, then drop them
    H64 = np.where(valid, H.astype(np.uint64), np.uint64(1) << np.uint64(40))
    S = np.sort(H64, axis=1)
    keep = np.ones(S.shape, dtype=bool)
    keep[:, 1:] = S[:, 1:] != S[:, :-1]
    keep &= S < (np.uint64(1) << np.uint64(40))
    cnt = keep.sum(axis=1)
    offsets = np.zeros(rows + 1, dtype=np.uint64)
    np.cumsum(cnt, out=offsets[1:])
    return S[keep].astype(np.uint32), offsets


def url(n_templates=1_000_000, dups=4, min_len=20, max_len=120, alphabet=40,
        max_edit=5, seed=0, nq=10000, q_seed=3, chunk=131072, text=False):
    """n_templates strings of length U[min_len, max_len] over a 40-symbol
    alphabet, each followed by `dups` near-duplicates made by 1..5 uniform
    random edits: id t*(dups+1) is template t, the next `dups` ids are its
    copies.  Each string is the set of its character 3-gram ids (packed to
    18 bits, hashed to 32 bits by the MurmurHash3 32-bit finaliser under a
    seeded key).  Queries: nq fresh edits of random templates, split into
    uneven groups whose sizes are log-uniform in [1, 4096].
    Returns (items u32, offsets, q_items, q_offsets, qbase, group_sizes)."""
    W = max_len + max_edit + 1
    rng0 = np.random.default_rng([seed, 20])
    key32 = np.uint32(rng0.integers(0, 2**32, dtype=np.uint64)) | np.uint32(1)
    def block(j):
        s = j * chunk
        n = min(chunk, n_templates - s)
        rng = np.random.default_rng([seed, 21, j])
        lens = rng.integers(min_len, max_len + 1, n)
        A = rng.integers(0, alphabet, (n, W)).astype(np.int16)
        A[np.arange(W)[None, :] >= lens[:, None]] = -1
        blocks_A = [A]
        blocks_L = [lens]
        for c in range(dups):
            ne = rng.integers(1, max_edit + 1, n)
            Ac, Lc = _edit(A, lens, ne, rng, alphabet)
            blocks_A.append(Ac)
            blocks_L.append(Lc)
        # interleave: template, then its copies
        SA = np.stack(blocks_A, axis=1).reshape(n * (dups + 1), W)
        SL = np.stack(blocks_L, axis=1).reshape(n * (dups + 1))
        it, of = _url_items(SA, SL, key32)
        return A, lens, it, of, (_text_of_rows(SA, SL) if text else None)

    with ThreadPoolExecutor(_workers()) as ex:
        parts = list(ex.map(block, range((n_templates + chunk - 1) // chunk)))
    items_l, offs_l, base = [], [np.zeros(1, dtype=np.uint64)], np.uint64(0)
    T_all_A, T_all_len = [], []
    for A, lens, it, of, _ in parts:
        T_all_A.append(A)
        T_all_len.append(lens)
        items_l.append(it)
        offs_l.append(of[1:] + base)
        base = base + of[-1]
    items = np.concatenate(items_l)
    offs = np.concatenate(offs_l)
    TA = np.concatenate(T_all_A)
    TL = np.concatenate(T_all_len)
    rq = np.random.default_rng([q_seed, 22])
    qt = rq.integers(0, n_templates, nq)
    ne = rq.integers(1, max_edit + 1, nq)
    QA, QL = _edit(TA[qt], TL[qt], ne, rq, alphabet)
    qitems, qoffs = _url_items(QA, QL, key32)
    sizes = []
    tot = 0
    while tot < nq:
        sz = int(np.exp(rq.uniform(0.0, np.log(4096.0))))
        sz = max(1, min(sz, nq - tot))
        sizes.append(sz)
        tot += sz
    sizes = np.array(sizes, dtype=np.int64)
    if text:
        syms = [p[4][0] for p in parts]
        base, offl = np.uint64(0), [np.zeros(1, dtype=np.uint64)]
        for p in parts:
            offl.append(p[4][1][1:] + base)
            base = base + p[4][1][-1]
        extra = {"data": (np.concatenate(syms), np.concatenate(offl)),
                 "queries": _text_of_rows(QA, QL), "gram": 3, "radix": alphabet,
                 "key": int(key32)}
        return items, offs, qitems, qoffs, qt * (dups + 1), sizes, extra
    return items, offs, qitems, qoffs, qt * (dups + 1), sizes
