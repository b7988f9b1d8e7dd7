"""The five workloads (sizes and FLINNG parameters) and scaled-down variants
used by the parity tests.  Family ids match the C ABI's FLINNG_* values.

Parameters follow the paper's notation mapped to the library's: L = number of
LSH tables (the paper's m), K = hashes concatenated per table (the paper's L),
R repetitions, B groups per repetition, k neighbours.
"""
from . import synth

SRP_F32, SRP_BF16, MINHASH_U32, MINHASH_U64 = 0, 1, 2, 3
INDEX_SEED = 0x5EEDF1A7

CONFIGS = {
    "c1": dict(name="dense_gmm_10k_d128", family=SRP_F32, N=10_000, d=128,
               n_centres=100, K=8, L=4, R=3, B=100, bucket_bits=8, k=10,
               nq=100),
    # tuned: a (K, L) of a sweep at this R, B whose R1@10 on 3000 queries
    # clears 0.9 by well over two standard errors: K=1, L=12 reaches 0.936
    # (8 s.e.).  L=10 (0.919) and L=9 (0.913) also clear it and run 8-13%
    # faster, but with the decode kernel under half the HBM peak; L=8 (0.904)
    # is within one s.e.; the configured K=2, L=32 reaches 0.79
    "c2": dict(name="genome_reads_1M_minhash", family=MINHASH_U64,
               n_base=500_000, N=1_000_000, K=2, L=32, R=4, B=4096,
               bucket_bits=20, k=10, nq=10_000, tuned=dict(K=1, L=12)),
    # tuned: the fastest (K, L) of the sweep at this R, B reaching
    # R1@10 >= 0.9 (K=24, L=12: 0.960 on 1000 queries; 24 is the largest
    # SRP K the library takes); the configured K=16, L=64 reaches 1.000
    "c3": dict(name="relu_embed_1M_d4096_bf16", family=SRP_BF16, N=1_000_000,
               d=4096, n_centres=10_000, K=16, L=64, R=8, B=8192,
               bucket_bits=16, k=10, nq=10_000, tuned=dict(K=24, L=12)),
    "c4": dict(name="url_strings_5M_minhash", family=MINHASH_U32,
               n_templates=1_000_000, N=5_000_000, K=3, L=48, R=8, B=16384,
               bucket_bits=22, k=10, nq=10_000),
}


def params(cfg):
    return dict(family=cfg["family"], K=cfg["K"], L=cfg["L"], R=cfg["R"],
                B=cfg["B"], bucket_bits=cfg["bucket_bits"], seed=INDEX_SEED)


def make(name, scale=1.0, nq=None):
    """Generate the data of config `name`, optionally scaled down in N (and
    B scaled with N so groups keep their size).  Returns (cfg, data, queries,
    qbase) where data/queries are an array (dense) or (items, offsets)."""
    cfg = dict(CONFIGS[name])
    nq = cfg["nq"] if nq is None else nq
    cfg["nq"] = nq
    if scale != 1.0:
        cfg["B"] = max(1, int(round(cfg["B"] * scale)))
    if name == "c1":
        N = max(2, int(cfg["N"] * scale))
        X, Q, qb = synth.dense_gmm(N=N, d=cfg["d"],
                                   n_centres=max(1, int(cfg["n_centres"] * scale)),
                                   nq=nq)
        cfg["N"] = N
        return cfg, X, Q, qb
    if name == "c2":
        nb = max(1, int(cfg["n_base"] * scale))
        it, of, qit, qof, qb, text = synth.genome(n_base=nb, nq=nq, text=True)
        cfg["N"] = 2 * nb
        cfg["text"] = text   # the reads as symbol sequences, and their n-gram item map
        return cfg, (it, of), (qit, qof), qb
    if name == "c3":
        N = max(2, int(cfg["N"] * scale))
        X, Q, qb = synth.dense_relu(N=N, d=cfg["d"],
                                    n_centres=max(1, int(cfg["n_centres"] * scale)),
                                    nq=nq)
        cfg["N"] = N
        return cfg, X, Q, qb
    if name == "c4":
        nt = max(1, int(cfg["n_templates"] * scale))
        it, of, qit, qof, qb, sizes = synth.url(n_templates=nt, nq=nq)
        cfg["N"] = 5 * nt
        cfg["group_sizes"] = sizes
        return cfg, (it, of), (qit, qof), qb
    raise KeyError(name)
