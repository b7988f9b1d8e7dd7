/*
 * flinng.h -- C ABI of the MI355X (gfx950) FLINNG library.
 *
 * FLINNG (Filters to Identify Near-Neighbor Groups; Engels, Coleman and
 * Shrivastava, "Practical Near Neighbor Search via Group Testing", 2021)
 * answers randomized nearest-neighbour queries (Definition 1) with a B x R
 * grid of group tests.  Each repetition r spreads the N points evenly over B
 * groups by a random permutation (Algorithm 1).  Each group's test is a
 * distance-sensitive Bloom filter (Section 3, Theorem 1) built from L shared
 * LSH functions, each the concatenation of K hashes (Section 3, concatenation
 * trick).  The filters are stored as one reverse index per LSH function:
 * bucket value -> list of cells (Section 6, Implementation).  A query counts,
 * for every cell, in how many tables it collides, then decodes by threshold
 * relaxation (Algorithm 3, equivalent to Algorithm 2 at decreasing
 * thresholds) and returns k point ids.
 *
 * Notation in this header: L = number of LSH tables (the paper's m),
 * K = hashes concatenated per table (the paper's L), R repetitions, B groups
 * per repetition, cell id c = r*B + b.
 *
 * Conventions for every entry point:
 *  - Returns FLINNG_OK (0) or a negative error code; on error a message is
 *    available from flinng_last_error() (thread-local) and no output is
 *    guaranteed.  No C++ exception crosses this boundary.
 *  - `stream` is a hipStream_t (NULL = the null stream).  All device work is
 *    enqueued on it.  Entry points that return host results synchronize the
 *    stream before returning; entry points whose outputs are device pointers
 *    return as soon as the work is enqueued.
 *  - Pointers flagged "device" must be device (or managed) memory of the
 *    current HIP device; "host" pointers are ordinary host memory.
 *  - The library never keeps a pointer to caller memory after the call's
 *    stream work has completed.
 */
#ifndef FLINNG_H
#define FLINNG_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- error codes (negative errno values) ------------------------------ */
#define FLINNG_OK 0
#define FLINNG_EINVAL (-22)    /* invalid argument or parameter            */
#define FLINNG_ENOMEM (-12)    /* device or host allocation failed          */
#define FLINNG_EDEVICE (-5)    /* HIP runtime / kernel launch error         */
#define FLINNG_EBUSY (-16)     /* serving: admission refused                */
#define FLINNG_ETIMEDOUT (-110)/* serving: wait timed out                   */
#define FLINNG_ESTATE (-77)    /* serving: server shut down / bad ticket    */

/* ---- hash families ----------------------------------------------------- */
/* Dense rows hashed by signed random projections: bit j of table t is 1 iff
 * the exact dot product of the row with hyperplane t*K+j is > 0; the bucket
 * of table t is sum_j bit_j 2^j (K bits).  Item sets hashed by MinHash: K
 * 32-bit minima per table folded to `bucket_bits` bits. */
enum flinng_family {
    FLINNG_SRP_F32 = 0,     /* dense, values fp32, row-major count x dim     */
    FLINNG_SRP_BF16 = 1,    /* dense, values bf16 bit patterns (uint16_t)    */
    FLINNG_MINHASH_U32 = 2, /* sets of uint32_t items, CSR offsets           */
    FLINNG_MINHASH_U64 = 3  /* sets of uint64_t items, CSR offsets           */
};

/* Index parameters (Appendix "Hyperparameters": R, B, m, L of the paper). */
typedef struct flinng_params {
    uint32_t family;      /* enum flinng_family                               */
    uint32_t dim;         /* dense: row length d >= 1; sets: ignored           */
    uint32_t K;           /* hashes per table: SRP bits 1..24, MinHash 1..32  */
    uint32_t L;           /* tables (the paper's m): 1..255                   */
    uint32_t R;           /* repetitions: 1..16                               */
    uint32_t B;           /* groups per repetition: 1..65536, B <= N          */
    uint32_t bucket_bits; /* sets: bucket width 1..24; dense: must be 0 or K  */
    uint32_t reserved;    /* must be 0                                        */
    uint64_t seed;        /* seeds the hyperplanes, MinHash keys and groups   */
} flinng_params;

/* A batch of points or queries. */
typedef struct flinng_input {
    const void *values;       /* dense: count*dim elements, row-major;
                                 sets: concatenated items                     */
    const uint64_t *offsets;  /* sets: count+1 nondecreasing offsets into
                                 values (offsets[0] = 0); dense: NULL         */
    uint64_t count;           /* number of rows / sets                        */
    uint32_t on_device;       /* 0: host pointers; 1: values and offsets are
                                 device pointers; 2 (serving only): values on
                                 the device, offsets on the host              */
    uint32_t reserved;        /* must be 0                                    */
} flinng_input;

/* A batch of symbol sequences to be read as sets of n-grams (the paper
 * hashes genome reads and URLs as n-gram sets, Section 7, Datasets).  The
 * item set of a sequence is, for every window of `gram` consecutive symbols,
 * the window's base-`radix` value v = sum_i s_{p+i} radix^(gram-1-i) mixed
 * with `key`: MurmurHash3's 64-bit finaliser of (v XOR key) for an index of
 * 64-bit items, its 32-bit finaliser of (low 32 bits of v) XOR (low 32 bits
 * of key) for 32-bit items.  A sequence shorter than `gram` is the empty
 * set.  Symbols must be below `radix`. */
typedef struct flinng_text {
    const uint8_t *symbols;   /* concatenated sequences, one symbol per byte  */
    const uint64_t *offsets;  /* count+1 nondecreasing offsets into symbols   */
    uint64_t count;           /* number of sequences                          */
    uint64_t key;             /* item key                                     */
    uint32_t gram;            /* n-gram length >= 1, radix^gram <= 2^64        */
    uint32_t radix;           /* alphabet size, 2..256                        */
    uint32_t on_device;       /* 1: symbols and offsets are device pointers   */
    uint32_t reserved;        /* must be 0                                    */
} flinng_text;

typedef struct flinng_index flinng_index;

/* Facts about a built index (sizes in elements unless noted). */
typedef struct flinng_index_info {
    uint64_t N;               /* indexed points                               */
    uint64_t list_entries;    /* total reverse-index list entries             */
    uint64_t device_bytes;    /* device memory held by the index              */
    uint32_t family, dim, K, L, R, B, bucket_bits;
    uint32_t cell_id_bytes;   /* 2 when R*B <= 65536, else 4                  */
    uint64_t srp_rechecked;   /* build: projections recomputed in FP64        */
    uint64_t srp_exact;       /* build: of those, decided by the exact sum    */
} flinng_index_info;

/*
 * flinng_build -- one-pass index construction (Algorithm 1 plus the reverse
 * index of Section 6).
 *  p      (host)  parameters; validated (FLINNG_EINVAL on any violation,
 *                 including B > N, dense dim mismatch, L*K*dim overflow).
 *  data   (host struct) the N points; values/offsets on host or device per
 *                 data->on_device.  Borrowed for the duration of the call;
 *                 the library does not store the data (no vectors are kept).
 *  out    (host)  receives the new index; the library owns all its device
 *                 memory until flinng_index_free.
 * The call synchronizes `stream` before returning.
 */
int flinng_build(const flinng_params *p, const flinng_input *data,
                 void *stream, flinng_index **out);

/*
 * flinng_query -- batched query: hash, count per cell through the reverse
 * index (Section 6), decode by threshold relaxation (Algorithm 3).
 *  q        (host struct) nq = q->count queries of the index's family.
 *  k        neighbours per query, 1..4096.
 *  ids      (host or device per out_on_device) nq*k uint32, row-major:
 *           point ids in the order Algorithm 3 reports them (cells by
 *           descending count, ties by ascending cell id; points within a cell
 *           by ascending id).  Padded with 0xFFFFFFFF when k > N.
 *  scores   same layout: the count of the cell that completed each point,
 *           i.e. the relaxed threshold at which it is reported; 0 for pads.
 *           May be NULL.
 *  persistent  0: one workgroup per query; 1: a persistent grid that pulls
 *           queries from a device counter (for uneven batches in one launch).
 * Device outputs: the call returns once the work is enqueued on `stream`.
 * Host outputs: the call synchronizes `stream`.  Queries only read the index,
 * so concurrent calls (from any threads, on any streams) are allowed, also
 * beside flinng_index_insert (each call sees one version of the index).  The batch's codes go to a device region the index keeps for
 * each stream it is queried on (up to 8 streams; allocated on first use,
 * grown synchronously for a larger batch, freed by flinng_index_free).
 */
int flinng_query(const flinng_index *idx, const flinng_input *q, uint32_t k,
                 uint32_t *ids, uint32_t *scores, uint32_t out_on_device,
                 uint32_t persistent, void *stream);

/*
 * flinng_build_text / flinng_query_text -- flinng_build and flinng_query
 * for MinHash indexes whose points and queries arrive as symbol sequences
 * (flinng_text): the n-gram items are extracted and mixed on the device,
 * then hashed, indexed and queried exactly as the same items given as sets
 * (an index built from sets answers text queries and vice versa, when the
 * items agree).  For device text the calls read two offsets back to size
 * the item buffer.  FLINNG_EINVAL for a dense index, radix outside 2..256,
 * gram 0, radix^gram above 2^64, or what flinng_build / flinng_query reject.
 */
int flinng_build_text(const flinng_params *p, const flinng_text *data,
                      void *stream, flinng_index **out);
int flinng_query_text(const flinng_index *idx, const flinng_text *q, uint32_t k,
                      uint32_t *ids, uint32_t *scores, uint32_t out_on_device,
                      uint32_t persistent, void *stream);

/*
 * flinng_query_codes -- the count + threshold + decode stage alone, for
 * bucket codes already on the device (as flinng_debug_hash produces them).
 *  codes   (device) nq*L uint32, row-major, each < 2^bucket_bits; a code
 *          outside that range matches no bucket, so its table adds nothing.
 *  ids, scores  (device) nq*k uint32 as in flinng_query (scores may be NULL).
 *  stats   (device, optional) 5 uint64 that the launch adds to: reverse-index
 *          list entries read, cell members walked over all decode passes,
 *          cell members walked in the final passes (each costs a 4-byte read:
 *          its id, or its filter word where the pass filters), decode passes,
 *          and candidate group rows gathered in the final passes (every
 *          walked member, or the filter's survivors).  The caller zeroes them.
 * Returns once the work is enqueued on `stream`.
 */
int flinng_query_codes(const flinng_index *idx, const uint32_t *codes, uint64_t nq,
                       uint32_t k, uint32_t *ids, uint32_t *scores,
                       uint32_t persistent, uint64_t *stats, void *stream);

/*
 * flinng_query_threshold -- Algorithm 2 (Index Query) at a fixed threshold:
 * a cell's group test is positive when at least t of the L tables collide
 * with the query (count >= t, the Section 3 filter rule), and a point is
 * reported when its cell is positive in all R repetitions, i.e. the set
 * {x : min_r C[r, g_r(x)] >= t}.  (flinng_query relaxes t per query instead,
 * Algorithm 3; its output is this set at decreasing t.)
 *  q        (host struct) nq = q->count queries of the index's family.
 *  t        threshold, any value: 0 reports every point, t > L none.
 *  max_per_query  id slots per query (may be 0: sizes only).
 *  ids      (host or device per out_on_device) nq*max_per_query uint32,
 *           row-major: each query's reported ids, as many as fit, unused
 *           slots 0xFFFFFFFF.  They come grouped by the cells of one
 *           repetition (ascending cell, then ascending id); compare them as
 *           a set.  May be NULL when max_per_query is 0.
 *  counts   (same placement) nq uint32: the size of each query's answer,
 *           also when it exceeds max_per_query (query again with more slots
 *           for the rest).
 * Device outputs: returns once the work is enqueued; host outputs
 * synchronize `stream`.  FLINNG_EINVAL for a bad input or when the B*R
 * counters do not fit a workgroup's LDS.
 */
int flinng_query_threshold(const flinng_index *idx, const flinng_input *q, uint32_t t,
                           uint32_t max_per_query, uint32_t *ids, uint32_t *counts,
                           uint32_t out_on_device, void *stream);

/*
 * flinng_query_noalloc -- flinng_query for callers that cannot allocate
 * (code under HIP graph capture, tight serving loops, harnesses that forbid
 * allocation): the same kernels and results, but every piece of scratch
 * (the batch's bucket codes, the SRP stage's counters, operand planes and,
 * for fp32 rows, norms and sign/flag words, the persistent grid's counter)
 * comes from one 64 MiB device
 * array that the library holds per GPU until the process ends; nothing is
 * allocated or freed, and nothing is cleared with a memset call.
 *  q        device input only (q->on_device = 1), as in flinng_query.
 *  ids, scores  device outputs, nq*k uint32 as in flinng_query (scores may
 *           be NULL).
 * Returns once the work is enqueued on `stream`.  FLINNG_EINVAL when the
 * batch needs more scratch than the array holds (about nq*L*4 bytes plus,
 * for bf16 rows, one operand plane of nq*dim*2 bytes unless dim is a
 * multiple of 32 and the rows are used in place, and for fp32 rows three
 * planes of nq*dim*2 bytes and nq*(4 + 8*ceil(K*L/32)) bytes of norms and
 * sign/flag words): split the batch.
 * Calls that overlap on one GPU share the array and race: serialize them
 * (one stream, or events).
 */
int flinng_query_noalloc(const flinng_index *idx, const flinng_input *q, uint32_t k,
                         uint32_t *ids, uint32_t *scores, uint32_t persistent, void *stream);

/*
 * flinng_index_insert -- add points to a built, resident index (the index is
 * built in one pass over the data, so later points join the same way).
 *  data   (host struct) data->count points of the index's family, host or
 *         device per data->on_device (0 or 1); borrowed for the call.  They
 *         get ids N, N+1, ... in order (N = the index's size before).
 * Each point is hashed with the index's functions and joins one group per
 * repetition.  Algorithm 1's permutation is drawn for the N0 points of the
 * build, so the arrivals follow their own rule: in arrival order they form
 * blocks of B, and block j places its u-th point in group pi_{r,j}(u), a
 * keyed random permutation of the B groups of repetition r.  Every complete
 * block adds one point to each group, so group sizes stay within two of
 * each other.  The point's cell then enters the reverse-index list of its
 * bucket in every table (lists stay deduplicated sets, members ascending).
 * New arrays are built beside the old ones (the index's memory transiently
 * doubles) and swapped in while no query is being enqueued: queries and
 * served batches in flight or queued see the index either before or after
 * the insert, never a mix.  The call synchronizes the device.  One insert
 * runs at a time per index; FLINNG_EINVAL past 2^32 - 2 points.
 */
int flinng_index_insert(flinng_index *idx, const flinng_input *data, void *stream);

/* Release an index and all its device memory (NULL is allowed). */
void flinng_index_free(flinng_index *idx);

/* Index facts (host struct). */
int flinng_index_get_info(const flinng_index *idx, flinng_index_info *info);

/* Last error message of the calling thread ("" if none). */
const char *flinng_last_error(void);

/* ---- layered parity hooks ---------------------------------------------- */
/* Bucket codes of a batch: codes[count*L] (host or device), row-major. */
int flinng_debug_hash(const flinng_index *idx, const flinng_input *q,
                      uint32_t *codes, uint32_t out_on_device, void *stream);

/*
 * The matrix-core projections of a dense batch, before any recheck (the
 * hashing layer of Section 3: bit j of table t is the sign of x . w_{t*K+j}).
 *  proj   (host or device per out_on_device, may be NULL) count*L*K float,
 *         row-major: the fp32 value the BF16 MFMA stage computed for
 *         x . w_h, h = t*K + j.  Its sign is trusted (no FP64 recheck) only
 *         when |proj| > gamma * |x|_2 * |w_h|_2 + tau_abs.
 *  bound  (host, may be NULL) 2 doubles: gamma and tau_abs of that rule.
 *         gamma = m u / (1 - m u) * (1 + 2^-6), u = 2^-23, with m the
 *         roundings a product passes through (bf16 rows: min(128, dpad) +
 *         ceil(dpad / 128); fp32 rows: 3 * dpad; dpad = dim rounded up to
 *         32); tau_abs = (1 or 3) * dpad * 2^-100.
 * FLINNG_EINVAL for MinHash indexes.
 */
int flinng_debug_projections(const flinng_index *idx, const flinng_input *q, float *proj,
                             double *bound, uint32_t out_on_device, void *stream);

/* Per-cell collision counts of a batch: counts[count*R*B] uint8 (host or
 * device), cell id c = r*B + b. */
int flinng_debug_counts(const flinng_index *idx, const flinng_input *q,
                        uint8_t *counts, uint32_t out_on_device, void *stream);

/*
 * Export the index to host arrays (tests; small indexes).
 *  offsets  L*(2^bits + 1) uint64: absolute positions into cells of each
 *           table's bucket lists (bits = K for dense, bucket_bits for sets).
 *  cells    list_entries uint32 cell ids, each bucket's list ascending.
 *  groups   R*N uint32, repetition-major: group of point x in repetition r.
 * Any pointer may be NULL to skip it.  Synchronizes `stream`.
 */
int flinng_index_export(const flinng_index *idx, uint64_t *offsets,
                        uint32_t *cells, uint32_t *groups, void *stream);

/* ---- parameters from the theory (Section 5 and its proofs) ------------- */
/* Host arithmetic only (no device is touched).  Our notation: K hashes per
 * table = the paper's L, L tables = the paper's m. */
typedef struct flinng_theory {
    uint32_t B;             /* groups per repetition, 2 sqrt(N) rounded        */
    uint32_t R;             /* repetitions: the cellwise rate bound, rounded up */
    uint32_t K;             /* hashes per table: smallest with
                               s_k^K >= 2 (N/B) s_k1^K                           */
    uint32_t L;             /* tables: smallest with alpha <= min(q, 1 - p)     */
    uint32_t t;             /* threshold for flinng_query_threshold: ceil(t_real) */
    uint32_t conditions_met;/* 1 when N >= 150 and R_real >= 10 ln N (the
                               footnote of the bound)                           */
    double R_real;          /* ln(1/delta) / (ln(4.80 sqrt N) -
                               ln(2 e^2 + 3.44 sqrt N))                         */
    double p, q;            /* test true / false positive rates required:
                               p = 1 - delta / (2R), q = N^-1/2                 */
    double one_minus_p;     /* delta / (2R), exact where p rounds to 1          */
    double gamma;           /* the query's stability ln s_k / (ln s_k1 - ln s_k) */
    double m_paper;         /* the closed form -8 ln(min(q, 1-p)) N^gamma       */
    double t_real;          /* L * (t_over_m_low + t_over_m_high) / 2           */
    double t_over_m_low;    /* (N/B) s_k1^K: negative groups' collision rate    */
    double t_over_m_high;   /* s_k^K: positive groups' collision rate           */
    double alpha;           /* filter error bound on either side at (K, L, t)   */
} flinng_theory;

/*
 * flinng_theory_params -- the group-test design (B, R, and the rates p, q a
 * test must reach; Lemma 1 and the cellwise rate bounds) and the
 * distance-sensitive Bloom filter that reaches them (K, L, t; Theorem 1 with
 * the threshold taken as t/m, the choices of t, B and L in the proof of the
 * test-cost theorem) for N points, a query whose K-th and (K+1)-th nearest
 * neighbours have per-hash collision probabilities s_k > s_k1, and failure
 * probability delta.  L is computed for the integer K (the paper's closed
 * form, which takes K real-valued, is returned as m_paper).
 * FLINNG_EINVAL: N < 2, N <= 118 (the bound on R needs more points),
 * similarities outside 0 < s_k1 < s_k < 1, delta outside (0, 1), or values
 * out of range.
 */
int flinng_theory_params(uint64_t N, double s_k, double s_k1, double delta,
                         flinng_theory *out);

/* ---- serving: continuous batching over resident indexes ----------------- */
typedef struct flinng_server flinng_server;

typedef struct flinng_serve_config {
    uint64_t mem_budget;      /* device bytes the batch workspaces of all
                                 streams may hold together (staged inputs,
                                 codes, results, hash scratch); a workspace
                                 is kept between batches and given back when
                                 another stream needs the room                */
    uint32_t max_inflight;    /* batches on the GPU at once (streams), 1..16  */
    uint32_t max_batch;       /* queries per launched batch, >= 1             */
    uint32_t max_queue;       /* queued requests before submit refuses        */
    uint32_t persistent;      /* launch batches with the persistent grid      */
    uint64_t linger_ns;       /* hold a batch that is not full until its
                                 oldest request has waited this long (0: launch
                                 as soon as a stream is free)                 */
} flinng_serve_config;

typedef struct flinng_serve_stats {
    uint64_t submitted, completed, rejected, batches, queries;
    double wall_s;            /* since create                                 */
    double qps;               /* completed queries / wall_s                   */
    double p50_ms, p99_ms, max_ms; /* completion - submit latency per request */
    double mean_batch;        /* queries per launched batch                   */
    uint64_t peak_mem_bytes;  /* peak device bytes held by the workspaces     */
} flinng_serve_stats;

/* Create a server over n_idx resident indexes (borrowed; they must outlive
 * the server).  One scheduler thread, cfg->max_inflight HIP streams. */
int flinng_serve_create(flinng_index *const *indexes, uint32_t n_idx,
                        const flinng_serve_config *cfg, flinng_server **out);

/* Submit one request (a batch of queries for index slot idx_slot); *ticket
 * identifies it.  Host input (q->on_device = 0) is copied before return.
 * Device input (q->on_device = 1) is borrowed: it must hold its final
 * values at the call (the caller has synchronized the work producing it)
 * and stay valid until the request completes (poll returns 1 or wait
 * returns); the batch stages it from device memory.  For device sets the
 * call reads the count+1 offsets back once (a small synchronous copy);
 * q->on_device = 2 (device items, host offsets) avoids that read.
 * FLINNG_EBUSY when the queue is full or the request alone exceeds the
 * memory budget; FLINNG_EINVAL for bad arguments (k outside 1..4096, empty
 * request, decreasing offsets, bad slot). */
int flinng_serve_submit(flinng_server *srv, uint32_t idx_slot,
                        const flinng_input *q, uint32_t k, uint64_t *ticket);

/* As flinng_serve_submit, but the batch writes the request's results into
 * device buffers: ids (device, count*k uint32, required) and scores (device,
 * count*k uint32, may be NULL), borrowed until the request completes; they
 * hold the results once poll returns 1 or wait returns.  A serving loop
 * whose queries and answers stay in HBM (e.g. embeddings produced on the
 * GPU) moves nothing over PCIe. */
int flinng_serve_submit_to(flinng_server *srv, uint32_t idx_slot,
                           const flinng_input *q, uint32_t k, uint32_t *ids,
                           uint32_t *scores, uint64_t *ticket);

/* Submit a request of symbol sequences (flinng_text, for a MinHash index
 * slot): the batch extracts their n-gram items on the device, so no host
 * preprocessing stands in the served path.  Host text is copied before
 * return; device text is borrowed until the request completes.  ids and
 * scores: device buffers (count*k each; scores may be NULL) as in
 * flinng_serve_submit_to, or both NULL to take the results with
 * flinng_serve_wait.  Requests are batched with others of the same slot, k
 * and text parameters. */
int flinng_serve_submit_text(flinng_server *srv, uint32_t idx_slot,
                             const flinng_text *q, uint32_t k, uint32_t *ids,
                             uint32_t *scores, uint64_t *ticket);

/* Wait for a request and release the ticket.  Requests submitted with
 * flinng_serve_submit: copies the results (count*k each) into the host
 * buffers ids (required) and scores (may be NULL).  Requests submitted with
 * flinng_serve_submit_to: ids and scores are ignored (may be NULL).
 * timeout_ns < 0 waits forever.  FLINNG_ETIMEDOUT leaves the ticket valid;
 * FLINNG_ESTATE for an unknown ticket. */
int flinng_serve_wait(flinng_server *srv, uint64_t ticket, uint32_t *ids,
                      uint32_t *scores, int64_t timeout_ns);

/* 1 if done, 0 if not yet, negative on error. */
int flinng_serve_poll(flinng_server *srv, uint64_t ticket);

int flinng_serve_stats_get(flinng_server *srv, flinng_serve_stats *st);

/* Start the statistics afresh (counters, latencies, wall clock; the peak
 * memory restarts at what the workspaces hold now), e.g. after a warm-up.
 * Requests in flight at the call are counted when they complete. */
int flinng_serve_stats_reset(flinng_server *srv);

/* Drain in-flight work, then stop the scheduler and free the server.
 * Requests not yet waited on are discarded. */
void flinng_serve_destroy(flinng_server *srv);

#ifdef __cplusplus
}
#endif
#endif /* FLINNG_H */
