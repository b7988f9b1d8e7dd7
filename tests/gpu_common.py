"""Shared helpers for the GPU parity tests (HIP library vs CPU oracle)."""
import sys

import numpy as np

import oracle
from workloads import configs, synth


def log(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def fam_oracle(family):
    return {0: oracle.SRP_F32, 1: oracle.SRP_BF16, 2: oracle.MINHASH_U32,
            3: oracle.MINHASH_U64}[family]


def build_both(flinng, family, data, K, L, R, B, seed, bucket_bits=0):
    """GPU index and oracle index over the same data."""
    gi = flinng.Index(data, family, K, L, R, B, seed, bucket_bits=bucket_bits)
    oi = oracle.OracleIndex(fam_oracle(family), data, K, L, R, B, seed,
                            bucket_bits=bucket_bits if bucket_bits else None)
    return gi, oi


def oracle_query(oi, q, k):
    return oi.query(q, k)


def scaled(name, scale, nq, **over):
    cfg, data, q, qb = configs.make(name, scale=scale, nq=nq)
    cfg.update(over)
    return cfg, data, q, qb


def subset_sets(items, offs, sel):
    sel = np.asarray(sel)
    parts = [items[offs[s]:offs[s + 1]] for s in sel]
    o = np.zeros(len(sel) + 1, dtype=np.uint64)
    o[1:] = np.cumsum([len(p) for p in parts])
    it = np.concatenate(parts) if len(parts) else items[:0]
    return it, o


def random_sets(rng, n, mean, dtype, pool=None):
    sizes = rng.poisson(mean, n)
    sizes[rng.random(n) < 0.05] = 0
    o = np.zeros(n + 1, dtype=np.uint64)
    o[1:] = np.cumsum(sizes)
    hi = 2**32 if dtype == np.uint32 else 2**63
    if pool is None:
        it = rng.integers(0, hi, int(o[-1]), dtype=np.uint64 if dtype == np.uint64 else np.int64)
    else:
        it = rng.choice(pool, int(o[-1]))
    return it.astype(dtype), o
