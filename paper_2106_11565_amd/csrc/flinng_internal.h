// Internal declarations of the gfx950 FLINNG library (not part of the ABI).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <mutex>
#include <shared_mutex>
#include <string>
#include <vector>

#include "../../include/flinng.h"

namespace flinng {

// ---------------------------------------------------------------------------
// Errors: every ABI function catches flinng::Error and maps it to a code and
// the thread-local message.
struct Error {
    int code;
    std::string msg;
};
[[noreturn]] void fail(int code, const std::string &msg);
void set_last_error(const std::string &msg);

#define FL_HIP(call)                                                          \
    do {                                                                      \
        hipError_t e_ = (call);                                               \
        if (e_ != hipSuccess)                                                 \
            ::flinng::fail(e_ == hipErrorOutOfMemory ? FLINNG_ENOMEM          \
                                                     : FLINNG_EDEVICE,        \
                           std::string(#call) + ": " + hipGetErrorString(e_)); \
    } while (0)

#define FL_CHECK_LAUNCH() FL_HIP(hipGetLastError())

// ---------------------------------------------------------------------------
// Counter-based generator shared by every random object of the method:
// SplitMix64's output function (Steele, Lea and Flood, OOPSLA 2014) applied to
// state s + (i+1) * 0x9E3779B97F4A7C15, i.e. the i-th output of a SplitMix64
// stream started at s.  Stream keys: sm64(seed, tag).
enum : uint64_t { TAG_HYP = 1, TAG_MINHASH = 2, TAG_GROUP = 3, TAG_STREAM = 4 };

__host__ __device__ inline uint64_t splitmix_finalize(uint64_t z) {
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}
__host__ __device__ inline uint64_t sm64(uint64_t s, uint64_t i) {
    return splitmix_finalize(s + (i + 1ull) * 0x9E3779B97F4A7C15ull);
}

// ---------------------------------------------------------------------------
// A built index.  Device layout (all arrays owned by the index):
//   offsets   [L][nbuckets+1] uint32  absolute positions into `cells`
//   cells     [list_entries]  uint16 (R*B <= 65536) or uint32 cell ids,
//             each bucket's list ascending (a Bloom filter bit set once)
//   grp       [N][Rp]         uint16 group of point x in repetition r
//             (Rp = R rounded up to a power of two; point-major so one
//             vector load gathers all R groups of a candidate)
//   mem       [R][B][mstride] uint32 members of cell (r,b), ascending id,
//             padded with 0xFFFFFFFF to mstride = ceil(N/B) rounded up to 4,
//             so every cell starts 16-byte aligned (4 ids per lane per load)
//   cmg       [R][B][mstride][Rp] uint16 cell-major copy of the groups: the
//             row of the member in each slot of mem, so a decode pass reads
//             every candidate's R groups sequentially beside its id
//   cfl       [R][B][mstride] uint32 the member's groups in repetitions
//             r+1 and r+2 (mod R), low and high 16 bits: a decode pass of
//             repetition r reads these 4 bytes per member and gathers the
//             id and the full row only for the few members whose counts in
//             those repetitions reach the level
//   gsize     [R][B]          uint32 members of each cell
//   hyp       [L*K][dpad]     bf16 hyperplanes (dense families)
//   hypnorm   [L*K]           fp32 Euclidean norms of the hyperplanes
//   hypt      [ceil(L*K/16)][dpad/32][16][32]  bf16 family: the hyperplanes
//             again, in 16 x 32 tiles (one MFMA operand fragment each, 1 KB
//             contiguous; rows past L*K zero)
// Points inserted after the build (ids N0, N0+1, ...) are added by building
// new offsets/cells/mem/cmg/cfl/gsize arrays beside the old ones and swapping
// them in under `rw` (exclusive), so a query enqueued under `rw` (shared)
// sees one version; the old arrays are freed once the device is idle.
struct Index {
    flinng_params p{};
    uint64_t N = 0;
    uint64_t N0 = 0;             // points of the one-pass build
    uint64_t grp_cap = 0;        // point rows allocated in grp
    uint32_t nbits = 0;          // bucket width (K for SRP)
    uint32_t dpad = 0;           // dense: dim rounded up to 32
    uint32_t Rp = 1;
    uint32_t mstride = 4;        // member slots per cell
    uint32_t cell_bytes = 2;
    uint64_t list_entries = 0;
    uint64_t device_bytes = 0;
    uint64_t srp_rechecked = 0, srp_exact = 0;
    int device = 0;
    uint32_t *offsets = nullptr;
    void *cells = nullptr;
    uint16_t *grp = nullptr;
    uint32_t *mem = nullptr;
    uint16_t *cmg = nullptr;
    uint32_t *cfl = nullptr;
    uint16_t *hyp = nullptr;
    float *hypnorm = nullptr;
    uint16_t *hypt = nullptr;
    uint32_t *gsize = nullptr;
    uint32_t gmax = 0;                    // the largest cell
    std::vector<uint32_t> gsize_host;     // host copy of gsize
    std::vector<uint64_t> tstart;         // [L+1] first list entry of each table
    mutable std::shared_mutex rw;         // query enqueue (shared) / insert swap
    std::mutex insert_mu;                 // one insert at a time
    // Device scratch for the codes of one query batch, one region per
    // stream the index is queried on: work on one stream runs in order, so
    // a region is reused without waiting.  Grown (and evicted) with a
    // synchronous free; released with the index.
    struct StreamScratch {
        hipStream_t stream;
        void *ptr;
        size_t cap;
    };
    mutable std::mutex scratch_mu;
    mutable std::vector<StreamScratch> scratch;
};

inline uint64_t nbuckets(const Index &ix) { return 1ull << ix.nbits; }
// Bytes allocated for n list entries of csz bytes: rounded up to 16 bytes
// plus 16 more (zeroed), so aligned 16-byte reads covering any entry are in
// bounds.
inline size_t cells_alloc_bytes(uint64_t n, size_t csz) {
    return ((n * csz + 15) & ~(size_t)15) + 16;
}
inline bool is_dense(uint32_t fam) { return fam == FLINNG_SRP_F32 || fam == FLINNG_SRP_BF16; }
// Device bytes an index holds (all its arrays).
inline uint64_t index_device_bytes(const Index &ix) {
    const uint64_t ncells = (uint64_t)ix.p.R * ix.p.B;
    uint64_t b = (uint64_t)ix.p.L * (nbuckets(ix) + 1) * 4 +
                 cells_alloc_bytes(ix.list_entries, ix.cell_bytes) + ix.grp_cap * ix.Rp * 2 +
                 ncells * ix.mstride * (8 + 2ull * ix.Rp) + ncells * 4;
    if (is_dense(ix.p.family)) b += (uint64_t)ix.p.L * ix.p.K * (ix.dpad * 2 + 4);
    if (ix.p.family == FLINNG_SRP_BF16) b += ((uint64_t)ix.p.L * ix.p.K + 15) / 16 * 16 * ix.dpad * 2;
    return b;
}

// Device scratch allocated on a stream (stream-ordered allocator).
struct DevBuf {
    void *ptr = nullptr;
    hipStream_t stream = nullptr;
    DevBuf() = default;
    DevBuf(size_t bytes, hipStream_t s);
    ~DevBuf();
    DevBuf(const DevBuf &) = delete;
    DevBuf &operator=(const DevBuf &) = delete;
    DevBuf(DevBuf &&o) noexcept : ptr(o.ptr), stream(o.stream) { o.ptr = nullptr; }
    DevBuf &operator=(DevBuf &&o) noexcept {
        if (this != &o) {
            release();
            ptr = o.ptr;
            stream = o.stream;
            o.ptr = nullptr;
        }
        return *this;
    }
    void release();
    template <class T> T *as() const { return static_cast<T *>(ptr); }
};

// A device region owned by the caller, handed out by a bump pointer in
// 256-byte aligned pieces.  Running past its end is an internal sizing error.
struct Arena {
    char *base = nullptr;
    size_t cap = 0, used = 0;
    static size_t round(size_t b) { return (b + 255) & ~(size_t)255; }
    void *take(size_t bytes) {
        if (bytes == 0) return nullptr;
        const size_t b = round(bytes);
        if (used + b > cap) fail(FLINNG_EDEVICE, "internal: batch workspace undersized");
        void *p = base + used;
        used += b;
        return p;
    }
};

// Scratch of one call: carved from an arena when one is given, otherwise
// allocated on the stream and freed on it when the Scratch goes away.
struct Scratch {
    Arena *arena;
    hipStream_t stream;
    std::vector<DevBuf> owned;
    Scratch(Arena *a, hipStream_t s) : arena(a), stream(s) {}
    template <class T = void> T *get(size_t bytes) {
        if (bytes == 0) return nullptr;
        if (arena) return static_cast<T *>(arena->take(bytes));
        owned.emplace_back(bytes, stream);
        return static_cast<T *>(owned.back().ptr);
    }
};

// ---------------------------------------------------------------------------
// Hashing (hash_srp.hip, hash_minhash.hip).  All write codes[n][L] uint32.
void srp_make_hyperplanes(Index &ix, hipStream_t s);
// Returns (rechecked, exact) counts when counters != nullptr (synchronizes).
// Scratch comes from ws when given (srp_scratch_bytes bounds what it takes).
// proj_dev (optional, device, n*L*K fp32): receives the MFMA projections
// before any recheck.
void srp_hash(const Index &ix, const flinng_input &in, uint32_t *codes_dev,
              hipStream_t s, uint64_t *counters_host, Arena *ws = nullptr,
              float *proj_dev = nullptr);
// The error bound the MFMA stage uses for a trusted sign: |v32 - v| <=
// gamma * |x|_2 * |w|_2 + tau_abs (rounding of the norms included).
void srp_bound(const Index &ix, double *gamma, double *tau_abs);
// Upper bound of the scratch srp_hash takes for n rows already on the device
// (exact when the rows' device address xdev is given).
size_t srp_scratch_bytes(const Index &ix, uint64_t n, const void *xdev = nullptr);
void minhash_hash(const Index &ix, const flinng_input &in, uint32_t *codes_dev,
                  hipStream_t s, double mean_hint = -1.0);
// mean_hint: mean items per set of a device-resident set batch (<= 0: unknown).
// Device-resident inputs take no scratch beyond ws (MinHash takes none).
void hash_batch(const Index &ix, const flinng_input &in, uint32_t *codes_dev,
                hipStream_t s, uint64_t *counters_host, double mean_hint = -1.0,
                Arena *ws = nullptr);
// Device bytes one served batch of nq queries (nitems set items) occupies:
// staged input, codes, results and hash scratch, as the server carves them.
uint64_t batch_device_bytes(const Index &ix, uint64_t nq, uint64_t nitems, uint32_t k,
                            bool text);

// N-gram text (text.hip).  validate_text: argument checks (FLINNG_EINVAL);
// text_symbols: symbols the sequences span (reads two offsets back for a
// device input); text_to_items: the item sets on the device (buffers from
// sc), described by a device flinng_input of the family's item type.
void validate_text(const flinng_text *t, uint32_t family);
uint64_t text_symbols(const flinng_text &t);
void text_to_items(const flinng_text &t, uint32_t family, uint64_t nsym, hipStream_t s,
                   Scratch &sc, flinng_input *out);
// Device bytes text_to_items takes from an arena for n sequences of nsym symbols.
inline size_t text_scratch_bytes(uint32_t family, uint64_t n, uint64_t nsym) {
    const size_t isz = family == FLINNG_MINHASH_U64 ? 8 : 4;
    return Arena::round((n + 1) * 8) + Arena::round((nsym ? nsym : 1) * isz);
}

// Segment copies by kernel (stage.hip): each segment copies `bytes` from
// src to dst, both device-visible addresses (device memory, or mapped pinned
// host memory).  Segments must not overlap their destinations.
struct CopySeg {
    uint64_t src, dst, bytes;
};
constexpr int MAX_COPY_SEGS = 128;  // per launch (kernel-argument space)
void copy_segments(const CopySeg *segs, size_t nseg, hipStream_t s);

// Sorting and scans (radix.hip).
void device_exclusive_scan_u32(const uint32_t *in, uint32_t *out, uint64_t n,
                               hipStream_t s);
// Stable LSD radix sort of 64-bit keys (bits [0, end_bit)) with optional
// uint32 values; result in keys/vals (tmp buffers of the same size needed).
// Keys alone (vals == nullptr) with `sorted` given: the result stays in
// whichever of keys / keys_tmp the last pass wrote, returned in *sorted.
void radix_sort_u64(uint64_t *keys, uint64_t *keys_tmp, uint32_t *vals,
                    uint32_t *vals_tmp, uint64_t n, int end_bit, hipStream_t s,
                    uint64_t **sorted = nullptr);

// Build pieces (build.hip).
void build_groups(Index &ix, hipStream_t s);
void build_lists(Index &ix, const uint32_t *codes_dev, hipStream_t s);
// The filter plane cfl of member arrays `mem` (stride mstride) from the
// point rows `grp`.
void build_filter(const Index &ix, const uint32_t *mem, const uint16_t *grp, uint32_t mstride,
                  uint32_t *cfl, hipStream_t s);
// Add n points (ids ix.N ..) whose codes [n][L] are on the device: groups by
// the arrival rule, members, reverse index; swaps the new arrays in.  The
// caller holds ix.insert_mu.  Synchronizes the device.
void insert_points(Index &ix, const uint32_t *codes_dev, uint64_t n, hipStream_t s);

// Query (query.hip).
void query_launch(const Index &ix, const uint32_t *codes_dev, uint64_t nq,
                  uint32_t k, uint32_t *ids_dev, uint32_t *scores_dev,
                  bool persistent, hipStream_t s, uint32_t *work_counter,
                  unsigned long long *stats = nullptr);
void counts_launch(const Index &ix, const uint32_t *codes_dev, uint64_t nq,
                   uint8_t *counts_dev, hipStream_t s);
size_t query_lds_bytes(const Index &ix, uint32_t k);
uint32_t query_max_k();

// Scratch bytes flinng_query_noalloc carves for nq queries (noalloc.hip).
size_t noalloc_scratch_bytes(const Index &ix, uint64_t nq, const void *xdev);

// Fixed-threshold query (threshold.hip): ids [nq][max_out] of the points with
// m(x) >= t, counts [nq] the size of each answer.
void threshold_launch(const Index &ix, const uint32_t *codes_dev, uint64_t nq, uint32_t t,
                      uint32_t max_out, uint32_t *ids_dev, uint32_t *counts_dev, hipStream_t s);

}  // namespace flinng
