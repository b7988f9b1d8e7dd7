// Batched FLINNG query on gfx950: count, threshold, decode.
//
// One workgroup owns one query at a time (a persistent grid pulls queries
// from a device counter).  All per-query state lives in LDS:
//   * the B*R cell counters as bytes, 4 per dword, holding 255 - count
//     (count <= L <= 255), decremented with 32-bit LDS atomics while the
//     workgroup walks the L reverse-index lists selected by the query's codes
//     (Section 6: count how often each cell collides with the query);
//   * per-repetition histograms of the nonzero counts (as counts-at-least);
//   * the list of cells the query touched (sparse queries), a list of
//     positive cells and a top-k key buffer.
// Decode (Algorithm 3, threshold relaxation).  Walking cells by descending
// count and reporting a point when all R of its cells have been walked means
// a point x completes at its last-ranked cell, so the output is the k
// smallest keys (255 - m(x), c*(x), x) with m(x) = min_r C[r, g_r(x)] and
// c*(x) the largest cell id among x's cells of count m(x).  {x : m(x) >= t}
// is Algorithm 2's answer at threshold t, and it lies inside the cells of
// count >= t of any single repetition.  So a pass streams the members of one
// repetition's cells with count >= t (t chosen from the histograms) together
// with each member's R group ids (stored cell-major beside the member ids, so
// the whole pass is sequential reads), computes every key and keeps the
// smallest; the pass is final once at least k candidates have m >= t.  When
// fewer than k points have m >= 1, the answer is completed from repetition
// R-1: its positive cells hold every point whose last zero-count cell lies in
// an earlier repetition, and the rest follow in (cell, id) order from its
// zero-count cells.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "flinng_internal.h"

namespace flinng {

// Threads per query workgroup: 256, or 1024 when the per-query LDS state
// leaves room for only one workgroup per CU (more wavefronts to hide
// latency).  Dense queries build the count histograms in HC copies (thread t
// adds to copy t mod HC) so that the many increments of the few low count
// values do not serialise on one LDS address; HC is a power of two sized to
// the LDS left over.
constexpr uint32_t HC_MAX = 32;
// Target members for the first pass.  The pass schedule does not change the
// answer, only how many members are read: dense indexes (many candidates at
// every level) do best with a tight first pass, sparse ones (few candidates,
// near-duplicate clusters) with one large enough to be final more often.
// (Measured on the 1M x 4096 ReLU index for dense, 2048-16384 tried, and on
// the 5M URL and configured genome indexes for sparse, 8192-65536 tried.)
constexpr uint32_t BUDGET_DENSE = 4096, BUDGET_SPARSE = 32768;
// positive-cell list capacity (at least one round of T cells)
__host__ __device__ constexpr uint32_t cl_for(int T) { return T <= 256 ? 256u : 1024u; }
// capacity of the list of cells a sparse query touched (fast path)
__host__ __device__ constexpr uint32_t tl_for(int T) { return (uint32_t)T; }

struct QArgs {
    const uint32_t *codes;
    uint64_t nq;
    const uint32_t *offsets;
    const void *cells;
    const uint32_t *mem;   // [R][B][mstride] member ids
    const uint16_t *cmg;   // [R][B][mstride][Rp] member group rows
    const uint32_t *cfl;   // [R][B][mstride] groups in repetitions r+1, r+2
    uint64_t N;
    const uint32_t *gsize; // [R][B] members of each cell
    uint32_t gmax;         // the largest cell
    uint32_t L, R, Rp, B, Bp, nbits, k, cap;
    uint32_t mstride;      // member slots per cell (multiple of 4)
    uint32_t threads;      // workgroup size the kernel is launched with
    uint32_t hc;           // histogram copies (a power of two)
    float inv_bp;          // 1 / Bp, for cell id -> repetition
    uint32_t *ids;
    uint32_t *scores;
    uint8_t *counts_out;   // debug: write counters and skip decode
    uint32_t *work;        // persistent: next query counter (nullptr: 1 WG/query)
    uint32_t budget;
    unsigned long long *stats;  // optional per-launch totals: list entries read,
                                // members read (all passes), members read in
                                // final passes, passes, group rows read in
                                // final passes
};

struct QLayout {
    uint32_t cnt_words, hist_words, cap;
    size_t off_cnt, off_hist, off_pre, off_pree, off_start, off_end, off_buf, off_lb, off_lp, off_tl,
        off_fp, off_fs, off_misc, total;
};

// gk: the general-k decode, which also needs the per-thread prefix slots.
__host__ __device__ inline QLayout q_layout(uint32_t L, uint32_t R, uint32_t Bp, uint32_t cap,
                                            int T, uint32_t hc, bool gk) {
    QLayout l;
    l.cnt_words = ((R * Bp) / 4 + 3) & ~3u;  // whole 16-byte units
    l.hist_words = hc * R * (L + 1);
    l.cap = cap;
    size_t o = 0;
    l.off_cnt = o;   o += (size_t)l.cnt_words * 4;  // first: a counter's LDS address is its cell id
    l.off_buf = o;   o += (size_t)cap * 8;          // 8-byte aligned (16-byte counter units)
    l.off_pre = o;   o += (size_t)(L + 1) * 4;
    l.off_pree = o;  o += (size_t)(L + 1) * 4;
    l.off_start = o; o += (size_t)L * 4;
    l.off_end = o;   o += (size_t)L * 4;
    l.off_lb = o;    o += cl_for(T) * 4;
    l.off_lp = o;    o += gk ? (size_t)T * 4 : 0;
    l.off_tl = o;    o += gk ? 0 : (size_t)tl_for(T) * 4;
    // the flattened walk of the 1024-thread fast path: 4-rounded prefix
    // sums and sizes of the listed cells
    const bool flat = !gk && T == 1024;
    l.off_fp = o;    o += flat ? (size_t)(cl_for(T) + 1) * 4 : 0;
    l.off_fs = o;    o += flat ? (size_t)cl_for(T) * 4 : 0;
    l.off_misc = o;  o += 64 * 4;
    l.off_hist = o;  o += (size_t)l.hist_words * 4;  // last: only its size varies with hc
    l.total = (o + 15) & ~(size_t)15;
    return l;
}

// misc slots
enum { M_Q = 0, M_BUFN, M_NGE, M_NALL, M_LEVEL, M_REP, M_KEEPALL, M_NEXT, M_THRLO,
       M_THRHI, M_LCNT, M_MEMB, M_THI, M_ST_ALL, M_ST_FINAL, M_ST_PASSES, M_NT, M_GATH,
       M_ST_GATH, M_SCAN0 };

// c / d for c < 2^24 and d >= 1, from the float quotient (within one of the
// true quotient: c is exact in float and the two roundings of c * (1/d)
// perturb it by less than one for d >= 2; d = 1 is exact) and one correction.
// A copy of a lane-dependent value that the compiler cannot merge with the
// original: an LDS address derived from it is then recomputed where it is
// used instead of being kept live (and spilled) across the whole query.
__device__ inline uint32_t fresh_copy(uint32_t x) {
    uint32_t y;
    asm volatile("v_mov_b32 %0, %1" : "=v"(y) : "v"(x));
    return y;
}

__device__ inline uint32_t div_small(uint32_t c, uint32_t d, float inv) {
    uint32_t q = (uint32_t)((float)c * inv);
    const int32_t rr = (int32_t)(c - q * d);
    return rr < 0 ? q - 1 : (rr >= (int32_t)d ? q + 1 : q);
}

template <int T>
__device__ inline uint32_t wg_excl_scan(uint32_t v, uint32_t *scr, uint32_t *total) {
    constexpr int TW = T / 64;
    const int lane = threadIdx.x % 64, wave = threadIdx.x / 64;
    uint32_t inc = v;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        uint32_t y = __shfl_up(inc, o, 64);
        if (lane >= o) inc += y;
    }
    if (lane == 63) scr[wave] = inc;
    __syncthreads();
    uint32_t pre = 0, tot = 0;
#pragma unroll
    for (int w = 0; w < TW; ++w) {
        uint32_t c = scr[w];
        pre += (w < wave) ? c : 0u;
        tot += c;
    }
    __syncthreads();
    *total = tot;
    return pre + inc - v;
}

// Bitonic sort of buf[0, cap) ascending (cap a power of two).
template <int T>
__device__ inline void wg_bitonic(uint64_t *buf, uint32_t cap) {
    for (uint32_t size = 2; size <= cap; size <<= 1) {
        for (uint32_t stride = size >> 1; stride > 0; stride >>= 1) {
            for (uint32_t i = threadIdx.x; i < cap / 2; i += T) {
                uint32_t lo = 2 * i - (i & (stride - 1));
                uint32_t hi = lo + stride;
                bool up = ((lo & size) == 0);
                uint64_t a = buf[lo], b = buf[hi];
                if ((a > b) == up) {
                    buf[lo] = b;
                    buf[hi] = a;
                }
            }
            __syncthreads();
        }
    }
}

__device__ inline uint64_t shfl64(uint64_t v, int src) {
    const uint32_t lo = (uint32_t)__shfl((int)(uint32_t)v, src, 64);
    const uint32_t hi = (uint32_t)__shfl((int)(uint32_t)(v >> 32), src, 64);
    return ((uint64_t)hi << 32) | lo;
}
__device__ inline uint64_t shfl64_up1(uint64_t v) {
    const uint32_t lo = (uint32_t)__shfl_up((int)(uint32_t)v, 1, 64);
    const uint32_t hi = (uint32_t)__shfl_up((int)(uint32_t)(v >> 32), 1, 64);
    return ((uint64_t)hi << 32) | lo;
}

// Per-wavefront decode state: its top-k list (lane i holds the i-th smallest
// key), the k-th key, and tallies (uniform across the wavefront).
struct WaveState {
    uint64_t wl, kth;
    uint32_t n_ge, n_all, members, gathered;
};

// Broadcast a 64-bit value from one lane (src uniform across the wavefront).
__device__ inline uint64_t bcast64(uint64_t v, int src) {
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)v, src);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(v >> 32), src);
    return ((uint64_t)hi << 32) | lo;
}

// The value of lane (lane ^ J) (every lane active): quad permutations and a
// row rotation by 8 move data within the VALU (DPP); the other distances go
// through the LDS crossbar (swizzle within 32 lanes, permute across halves).
template <int J>
__device__ inline uint32_t lane_xor(uint32_t v, int lane) {
    if constexpr (J == 1) {
        return (uint32_t)__builtin_amdgcn_mov_dpp((int)v, 0xB1, 0xF, 0xF, false);  // quad [1,0,3,2]
    } else if constexpr (J == 2) {
        return (uint32_t)__builtin_amdgcn_mov_dpp((int)v, 0x4E, 0xF, 0xF, false);  // quad [2,3,0,1]
    } else if constexpr (J == 8) {
        return (uint32_t)__builtin_amdgcn_mov_dpp((int)v, 0x128, 0xF, 0xF, false);  // row rotate 8
    } else if constexpr (J < 32) {
        return (uint32_t)__builtin_amdgcn_ds_swizzle((int)v, (J << 10) | 0x1F);  // xor J, 32-lane groups
    } else {
        return (uint32_t)__builtin_amdgcn_ds_bpermute((lane ^ J) << 2, (int)v);
    }
}

// One compare-exchange step of a bitonic sort across the wavefront: lanes
// l and l ^ J exchange so that the lower lane keeps the smaller key in
// ascending blocks (bit S of l clear) and the larger one in descending
// blocks.
// Lanes l of a wavefront with bit S of l equal to bit J of l, as a mask
// (a compile-time constant, rematerialised where it is used).
constexpr unsigned long long keep_min_mask(int S, int J) {
    unsigned long long m = 0;
    for (int l = 0; l < 64; ++l)
        if (((l & S) == 0) == ((l & J) == 0)) m |= 1ull << l;
    return m;
}

template <int S, int J>
__device__ inline uint64_t bitonic_step(uint64_t v, int lane) {
    const uint32_t plo = lane_xor<J>((uint32_t)v, lane);
    const uint32_t phi = lane_xor<J>((uint32_t)(v >> 32), lane);
    const uint64_t p = ((uint64_t)phi << 32) | plo;
    // take the partner's key where it is smaller in a keep-min lane, or
    // larger in a keep-max lane
    constexpr unsigned long long km = keep_min_mask(S, J);
    const unsigned long long take = ~(__ballot(p < v) ^ km);
    return __builtin_amdgcn_inverse_ballot_w64(take) ? p : v;
}

// Sort one key per lane ascending across the 64 lanes (every lane active).
__device__ inline uint64_t wave_sort64(uint64_t v, int lane) {
    v = bitonic_step<2, 1>(v, lane);
    v = bitonic_step<4, 2>(v, lane);
    v = bitonic_step<4, 1>(v, lane);
    v = bitonic_step<8, 4>(v, lane);
    v = bitonic_step<8, 2>(v, lane);
    v = bitonic_step<8, 1>(v, lane);
    v = bitonic_step<16, 8>(v, lane);
    v = bitonic_step<16, 4>(v, lane);
    v = bitonic_step<16, 2>(v, lane);
    v = bitonic_step<16, 1>(v, lane);
    v = bitonic_step<32, 16>(v, lane);
    v = bitonic_step<32, 8>(v, lane);
    v = bitonic_step<32, 4>(v, lane);
    v = bitonic_step<32, 2>(v, lane);
    v = bitonic_step<32, 1>(v, lane);
    v = bitonic_step<64, 32>(v, lane);
    v = bitonic_step<64, 16>(v, lane);
    v = bitonic_step<64, 8>(v, lane);
    v = bitonic_step<64, 4>(v, lane);
    v = bitonic_step<64, 2>(v, lane);
    v = bitonic_step<64, 1>(v, lane);
    return v;
}

// Insert the keys of the lanes in `tk` into the wavefront's sorted top-k
// list, all at once (called with every lane of the wavefront active; keys
// are distinct).  Into an empty list many candidates are sorted across the
// wavefront and the first k kept, a few are ranked among themselves and
// permuted to their ranks.  Otherwise each candidate below the k-th key is
// broadcast in turn (readlane) and its place in the merged order found by
// ballot (its rank among the list plus its rank among the candidates); the
// places taken form a lane mask and each place notes its candidate.  Then
// each lane pulls its new entry: the candidate's key, or the list entry
// shifted up by the candidates placed before it.
__device__ inline bool wave_insert(WaveState &ws, uint64_t key, unsigned long long tk, uint32_t k,
                                   int lane) {
    const unsigned long long cm = __ballot(key < ws.kth) & tk;
    if (!cm) return false;
    const bool in = __builtin_amdgcn_inverse_ballot_w64(cm);
    if (bcast64(ws.wl, 0) == ~0ull) {
        // empty list (keys never equal ~0: their cell field is below 2^24 - 1)
        const uint32_t c = (uint32_t)__popcll(cm);
        if (c > 16) {
            const uint64_t v = wave_sort64(in ? key : ~0ull, lane);
            ws.wl = ((uint32_t)lane < k) ? v : ~0ull;
        } else {
            uint32_t rank = 0;
            for (unsigned long long m = cm; m; m &= m - 1) {
                const uint64_t kk = bcast64(key, __ffsll((long long)m) - 1);
                rank += (kk < key) ? 1u : 0u;
            }
            // the other lanes take the places after the candidates, in order
            const uint32_t dest = in ? rank : c + __builtin_amdgcn_mbcnt_hi(
                                                     (uint32_t)(~cm >> 32),
                                                     __builtin_amdgcn_mbcnt_lo((uint32_t)~cm, 0u));
            const uint32_t lo = (uint32_t)__builtin_amdgcn_ds_permute((int)(dest * 4), (int)(uint32_t)key);
            const uint32_t hi =
                (uint32_t)__builtin_amdgcn_ds_permute((int)(dest * 4), (int)(uint32_t)(key >> 32));
            ws.wl = ((uint32_t)lane < (c < k ? c : k)) ? (((uint64_t)hi << 32) | lo) : ~0ull;
        }
        ws.kth = bcast64(ws.wl, (int)k - 1);
        return true;
    }
    unsigned long long placed = 0;  // list places taken by candidates
    int from = 0;                   // the candidate lane placed at this place
    for (unsigned long long m = cm; m; m &= m - 1) {
        const int src = __ffsll((long long)m) - 1;
        const uint64_t kk = bcast64(key, src);
        const uint32_t pos = (uint32_t)__popcll(__ballot(ws.wl < kk)) +
                             (uint32_t)__popcll(__ballot(key < kk) & cm);
        if (pos < k) {
            placed |= 1ull << pos;
            from = (lane == (int)pos) ? src : from;
        }
    }
    // candidates placed before this lane; the list entry that moves here
    const uint32_t before =
        __builtin_amdgcn_mbcnt_hi((uint32_t)(placed >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)placed, 0u));
    const int li = lane - (int)before;
    const bool fromc = __builtin_amdgcn_inverse_ballot_w64(placed);
    const uint32_t clo = (uint32_t)__shfl((int)(uint32_t)key, from, 64);
    const uint32_t chi = (uint32_t)__shfl((int)(uint32_t)(key >> 32), from, 64);
    const uint32_t llo = (uint32_t)__shfl((int)(uint32_t)ws.wl, li, 64);
    const uint32_t lhi = (uint32_t)__shfl((int)(uint32_t)(ws.wl >> 32), li, 64);
    const uint64_t v = fromc ? (((uint64_t)chi << 32) | clo) : (((uint64_t)lhi << 32) | llo);
    ws.wl = ((uint32_t)lane < k) ? v : ~0ull;
    ws.kth = bcast64(ws.wl, (int)k - 1);
    return true;
}

// Compare-exchange of two keys held by the same lane (ascending).
__device__ inline void ce64(uint64_t &a, uint64_t &b) {
    const bool sw = b < a;
    const uint64_t lo = sw ? b : a, hi = sw ? a : b;
    a = lo;
    b = hi;
}

// Load the group rows of 4 consecutive member slots (4*RP uint16, 16-byte
// aligned for RP >= 2, 8-byte for RP = 1) as 2*RP dwords.
template <int RP>
__device__ inline void load_rows(const uint16_t *p, uint32_t (&w)[2 * RP]) {
    if constexpr (RP == 1) {
        const uint2 v = *reinterpret_cast<const uint2 *>(p);
        w[0] = v.x;
        w[1] = v.y;
    } else {
#pragma unroll
        for (int i = 0; i < RP / 2; ++i) {
            const uint4 v = reinterpret_cast<const uint4 *>(p)[i];
            w[4 * i + 0] = v.x;
            w[4 * i + 1] = v.y;
            w[4 * i + 2] = v.z;
            w[4 * i + 3] = v.w;
        }
    }
}

template <int RP>
__device__ inline uint32_t row_group(const uint32_t (&w)[2 * RP], int e, int r) {
    const int q = e * RP + r;
    return (w[q >> 1] >> (16 * (q & 1))) & 0xFFFFu;
}

// A byte of LDS by its address.  The query kernel uses no static LDS, so its
// dynamic LDS (where the counters come first) starts at address 0 and the
// counter of cell c sits at address c (the launcher checks that the kernel
// has no static LDS).
typedef __attribute__((address_space(3))) const uint8_t lds_byte;
__device__ inline uint32_t lds_u8_at(uint32_t addr) {
    return *reinterpret_cast<lds_byte *>((size_t)addr);
}

// Stream the members of the cells lbs[0, nl) of one repetition: for each
// member, its id and its group row give m and c* from the LDS counters; keys
// with m >= level (all keys when `keep`) go into the wavefront's top-k.
// Work items are (cell, 256-member chunk); each lane takes 4 consecutive
// members (one 16-byte id load plus RP/2 16-byte row loads) and keeps U items
// in flight.  The loads are unconditional (slots past an item's end, or of an
// item past the last, read the cell's first slots and are marked invalid), so
// that all U items' loads are issued before any of them is waited on.
template <int RP, int U, int T>
__device__ inline void walk_cells(const uint32_t *lbs, uint32_t nl, const uint32_t *__restrict__ memr,
                                  const uint16_t *__restrict__ cmgr, const uint8_t *cnt8, uint32_t R,
                                  uint32_t Bp, uint32_t mstride, uint32_t level, bool keep,
                                  const uint32_t *__restrict__ gsz, uint32_t cpc, uint32_t k, int lane,
                                  int wave, WaveState &ws) {
    constexpr int TW = T / 64;
    const uint32_t nitems = nl * cpc;
    const uint32_t wv = __builtin_amdgcn_readfirstlane(wave);
    for (uint32_t i0 = wv; i0 < nitems; i0 += TW * U) {
        uint4 idv[U];
        uint32_t rows[U][2 * RP];
        uint32_t nv[U];
#pragma unroll
        for (int g = 0; g < U; ++g) {
            // wavefront-uniform item; the last item stands in past the end
            const uint32_t i = i0 + (uint32_t)g * TW;
            const uint32_t ic = i < nitems ? i : nitems - 1;
            const uint32_t ci = cpc == 1 ? ic : ic / cpc;
            const uint32_t bb = __builtin_amdgcn_readfirstlane(lbs[ci]);
            const uint32_t j0 = (ic - ci * cpc) * 256;
            const uint32_t j = j0 + 4 * lane;
            // slots clamped into the cell's stride, so that the loads need
            // not wait for the size; slots past it are masked by nv
            const uint64_t slot = (uint64_t)bb * mstride + (j < mstride ? j : 0u);
            idv[g] = *reinterpret_cast<const uint4 *>(memr + slot);
            load_rows<RP>(cmgr + slot * RP, rows[g]);
            const uint32_t sz = __builtin_amdgcn_readfirstlane(gsz[bb]);
            nv[g] = (i < nitems && j < sz) ? ((sz - j < 4) ? sz - j : 4u) : 0u;
            if (i < nitems && j0 < sz) {
                ws.members += (sz - j0 < 256) ? sz - j0 : 256u;
                ws.gathered += (sz - j0 < 256) ? sz - j0 : 256u;
            }
        }
        // repetition r's counters start at rb[r]; the padding repetitions
        // r >= R repeat repetition R-1 (its group is repeated in the rows)
        uint32_t rb[RP];
#pragma unroll
        for (int r = 0; r < RP; ++r) rb[r] = ((uint32_t)r < R ? (uint32_t)r : R - 1) * Bp;
#pragma unroll
        for (int g = 0; g < U; ++g) {
            const uint32_t xs[4] = {idv[g].x, idv[g].y, idv[g].z, idv[g].w};
            // key of member e of this lane and the lane mask of the kept
            // members.  The counters hold 255 - count at LDS byte address =
            // cell id, so t = max over the member's cells of
            // ((255 - count) << 24 | cell) is the key's high word
            // ((255 - m) << 24) | c*: the smallest count and, among equal
            // counts, the largest cell id (cell ids stay below 2^24: the
            // counters of all cells fit in LDS).  m >= level iff
            // t < (256 - level) << 24 (level >= 1).
            auto member_key = [&](int e, unsigned long long &tm) -> uint64_t {
                uint32_t t = 0;
#pragma unroll
                for (int r = 0; r < RP; ++r) {
                    const uint32_t c = rb[r] + row_group<RP>(rows[g], e, r);
                    const uint32_t tv = (lds_u8_at(c) << 24) | c;
                    t = tv > t ? tv : t;
                }
                // lane masks of the valid members, of those with m >= level,
                // and of those kept
                const unsigned long long vm = __ballot((uint32_t)e < nv[g]);
                const unsigned long long gm = __ballot(t < ((256u - level) << 24)) & vm;
                tm = keep ? vm : gm;
                ws.n_ge += (uint32_t)__popcll(gm);
                ws.n_all += (uint32_t)__popcll(tm);
                return ((uint64_t)t << 32) | xs[e];
            };
            if (keep) {
                // every valid member is kept: each lane's keys in ascending
                // order (~0, which no key equals, for the invalid ones), so
                // that the e-th batch holds every lane's e-th smallest key and
                // once a batch has no candidate the later ones have none
                uint64_t kv[4];
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    unsigned long long tm;
                    const uint64_t key = member_key(e, tm);
                    kv[e] = __builtin_amdgcn_inverse_ballot_w64(tm) ? key : ~0ull;
                }
                ce64(kv[0], kv[1]);
                ce64(kv[2], kv[3]);
                ce64(kv[0], kv[2]);
                ce64(kv[1], kv[3]);
                ce64(kv[1], kv[2]);
#pragma unroll
                for (int e = 0; e < 4; ++e)
                    if (!wave_insert(ws, kv[e], __ballot(kv[e] != ~0ull), k, lane)) break;
            } else {
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    unsigned long long tm;
                    const uint64_t key = member_key(e, tm);
                    wave_insert(ws, key, tm, k, lane);
                }
            }
        }
    }
}

// The group row of one member slot (RP uint16) as (RP + 1) / 2 dwords.
template <int RP>
__device__ inline void load_row1(const uint16_t *p, uint32_t (&w)[(RP + 1) / 2]) {
    if constexpr (RP == 1) {
        w[0] = *p;
    } else if constexpr (RP == 2) {
        w[0] = *reinterpret_cast<const uint32_t *>(p);
    } else if constexpr (RP == 4) {
        const uint2 v = *reinterpret_cast<const uint2 *>(p);
        w[0] = v.x;
        w[1] = v.y;
    } else {
#pragma unroll
        for (int i = 0; i < RP / 8; ++i) {
            const uint4 v = reinterpret_cast<const uint4 *>(p)[i];
            w[4 * i + 0] = v.x;
            w[4 * i + 1] = v.y;
            w[4 * i + 2] = v.z;
            w[4 * i + 3] = v.w;
        }
    }
}

// walk_cells for a pass that keeps only keys with m >= level (R >= 2): a
// member's m is at most its counts in repetitions r+1 and r+2 (mod R), read
// from the 4-byte filter word of its slot, so each lane first reads the
// filter words of its 4 members of each of U items (one 16-byte load per
// item, all in flight together) and gathers the id and the full group row
// only of the members whose counts there reach the level (about 1% of them
// on the ReLU and URL workloads).  The survivors are then taken one per lane
// per round (a lane with several takes them in later rounds), so a batch of
// U items costs two rounds of memory latency in the common case.  Every
// member with m >= level survives the filter, so the keys offered to the
// top-k, and the tallies, are those of walk_cells.
template <int RP, int U, int T>
__device__ inline void walk_cells_filtered(const uint32_t *lbs, uint32_t nl,
                                           const uint32_t *__restrict__ memr,
                                           const uint16_t *__restrict__ cmgr,
                                           const uint32_t *__restrict__ cflr, uint32_t R, uint32_t Bp,
                                           uint32_t mstride, uint32_t level, uint32_t f1b, uint32_t f2b,
                                           const uint32_t *__restrict__ gsz, uint32_t cpc, uint32_t k,
                                           int lane, int wave, WaveState &ws) {
    constexpr int TW = T / 64;
    constexpr int RW = (RP + 1) / 2;
    const uint32_t nitems = nl * cpc;
    const uint32_t wv = __builtin_amdgcn_readfirstlane(wave);
    // counter bytes hold 255 - count: count >= level iff byte < 256 - level
    const uint32_t lim = 256u - level;
    uint32_t rb[RP];
#pragma unroll
    for (int r = 0; r < RP; ++r) rb[r] = ((uint32_t)r < R ? (uint32_t)r : R - 1) * Bp;
    for (uint32_t i0 = wv; i0 < nitems; i0 += TW * U) {
        uint4 fv[U];
        uint32_t slot[U];  // within the repetition: B * mstride < 2^32
        uint32_t nv[U], szv[U];
#pragma unroll
        for (int g = 0; g < U; ++g) {
            // the filter words (clamped into the cell's stride) and the
            // cell's size are loaded together; slots past the size are
            // padding, masked out below
            const uint32_t i = i0 + (uint32_t)g * TW;
            const uint32_t ic = i < nitems ? i : nitems - 1;
            const uint32_t ci = cpc == 1 ? ic : ic / cpc;
            const uint32_t bb = __builtin_amdgcn_readfirstlane(lbs[ci]);
            const uint32_t j = (ic - ci * cpc) * 256 + 4 * lane;
            slot[g] = bb * mstride + (j < mstride ? j : 0u);
            fv[g] = *reinterpret_cast<const uint4 *>(cflr + slot[g]);
            szv[g] = __builtin_amdgcn_readfirstlane(gsz[bb]);
        }
#pragma unroll
        for (int g = 0; g < U; ++g) {
            const uint32_t i = i0 + (uint32_t)g * TW;
            const uint32_t ic = i < nitems ? i : nitems - 1;
            const uint32_t ci = cpc == 1 ? ic : ic / cpc;
            const uint32_t j0 = (ic - ci * cpc) * 256, j = j0 + 4 * lane, sz = szv[g];
            nv[g] = (i < nitems && j < sz) ? ((sz - j < 4) ? sz - j : 4u) : 0u;
            if (i < nitems && j0 < sz) ws.members += (sz - j0 < 256) ? sz - j0 : 256u;
        }
        // survivors: bit 4g + e for member e of item g
        uint32_t pend = 0;
#pragma unroll
        for (int g = 0; g < U; ++g) {
            const uint32_t fw[4] = {fv[g].x, fv[g].y, fv[g].z, fv[g].w};
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const uint32_t b1 = lds_u8_at(f1b + (fw[e] & 0xFFFFu));
                const uint32_t b2 = lds_u8_at(f2b + (fw[e] >> 16));
                if ((uint32_t)e < nv[g] && b1 < lim && b2 < lim) pend |= 1u << (4 * g + e);
            }
        }
        while (__ballot(pend != 0)) {
            const bool act = pend != 0;
            const uint32_t m = act ? (uint32_t)__builtin_ctz(pend) : 0u;
            pend &= pend - 1;
            uint32_t sl = slot[0];
#pragma unroll
            for (int g = 1; g < U; ++g) sl = (m >> 2) == (uint32_t)g ? slot[g] : sl;
            sl += m & 3u;
            uint32_t xid = 0, rw[RW];
#pragma unroll
            for (int i = 0; i < RW; ++i) rw[i] = 0;
            if (act) {
                xid = memr[sl];
                load_row1<RP>(cmgr + (uint64_t)sl * RP, rw);
            }
            ws.gathered += (uint32_t)__popcll(__ballot(act));
            uint32_t t = 0;
#pragma unroll
            for (int r = 0; r < RP; ++r) {
                const uint32_t c = rb[r] + ((rw[r >> 1] >> (16 * (r & 1))) & 0xFFFFu);
                const uint32_t tv = (lds_u8_at(c) << 24) | c;
                t = tv > t ? tv : t;
            }
            const unsigned long long gm = __ballot(act && t < (lim << 24));
            ws.n_ge += (uint32_t)__popcll(gm);
            ws.n_all += (uint32_t)__popcll(gm);
            wave_insert(ws, ((uint64_t)t << 32) | xid, gm, k, lane);
        }
    }
}

// walk_cells_filtered over the listed cells' members as one flattened
// sequence (each cell's run padded to a multiple of 4 inside its stride):
// items of 256 consecutive positions, so that a wavefront's lanes stay busy
// however the cell sizes fall (cells of 122 members would leave half the
// lanes of a per-cell item idle, cells of 305 a second item nearly empty).
// A lane finds the cell of its 4 positions by a binary search over the
// prefix sums fp (LDS), then reads their filter words; survivors as in
// walk_cells_filtered.
template <int RP, int U, int T>
__device__ inline void walk_flat_filtered(const uint32_t *lbs, const uint32_t *fp, const uint32_t *fs,
                                          uint32_t nl, uint32_t total,
                                          const uint32_t *__restrict__ memr,
                                          const uint16_t *__restrict__ cmgr,
                                          const uint32_t *__restrict__ cflr, uint32_t R, uint32_t Bp,
                                          uint32_t mstride, uint32_t level, uint32_t f1b, uint32_t f2b,
                                          uint32_t k, int lane, int wave, WaveState &ws) {
    constexpr int TW = T / 64;
    constexpr int RW = (RP + 1) / 2;
    const uint32_t nitems = (total + 255) / 256;
    const uint32_t wv = __builtin_amdgcn_readfirstlane(wave);
    const uint32_t lim = 256u - level;
    uint32_t rb[RP];
#pragma unroll
    for (int r = 0; r < RP; ++r) rb[r] = ((uint32_t)r < R ? (uint32_t)r : R - 1) * Bp;
    for (uint32_t i0 = wv; i0 < nitems; i0 += TW * U) {
        uint4 fv[U];
        uint32_t slot[U];  // within the repetition: B * mstride < 2^32
        uint32_t nv[U];
#pragma unroll
        for (int g = 0; g < U; ++g) {
            const uint32_t i = i0 + (uint32_t)g * TW;
            const uint32_t pos = i * 256 + 4 * lane;
            const bool valid = i < nitems && pos < total;
            const uint32_t pp = valid ? pos : 0u;
            uint32_t lo = 0, hi = nl;  // the last cell whose run starts at or before pp
            while (hi - lo > 1) {
                const uint32_t mid = (lo + hi) >> 1;
                if (fp[mid] <= pp) lo = mid; else hi = mid;
            }
            const uint32_t o = pp - fp[lo], sz = fs[lo];
            nv[g] = (valid && o < sz) ? ((sz - o < 4) ? sz - o : 4u) : 0u;
            slot[g] = lbs[lo] * mstride + o;
            fv[g] = *reinterpret_cast<const uint4 *>(cflr + slot[g]);
        }
        uint32_t pend = 0;
#pragma unroll
        for (int g = 0; g < U; ++g) {
            const uint32_t fw[4] = {fv[g].x, fv[g].y, fv[g].z, fv[g].w};
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                ws.members += (uint32_t)__popcll(__ballot((uint32_t)e < nv[g]));
                const uint32_t b1 = lds_u8_at(f1b + (fw[e] & 0xFFFFu));
                const uint32_t b2 = lds_u8_at(f2b + (fw[e] >> 16));
                if ((uint32_t)e < nv[g] && b1 < lim && b2 < lim) pend |= 1u << (4 * g + e);
            }
        }
        while (__ballot(pend != 0)) {
            const bool act = pend != 0;
            const uint32_t m = act ? (uint32_t)__builtin_ctz(pend) : 0u;
            pend &= pend - 1;
            uint32_t sl = slot[0];
#pragma unroll
            for (int g = 1; g < U; ++g) sl = (m >> 2) == (uint32_t)g ? slot[g] : sl;
            sl += m & 3u;
            uint32_t xid = 0, rw[RW];
#pragma unroll
            for (int i = 0; i < RW; ++i) rw[i] = 0;
            if (act) {
                xid = memr[sl];
                load_row1<RP>(cmgr + (uint64_t)sl * RP, rw);
            }
            ws.gathered += (uint32_t)__popcll(__ballot(act));
            uint32_t t = 0;
#pragma unroll
            for (int r = 0; r < RP; ++r) {
                const uint32_t c = rb[r] + ((rw[r >> 1] >> (16 * (r & 1))) & 0xFFFFu);
                const uint32_t tv = (lds_u8_at(c) << 24) | c;
                t = tv > t ? tv : t;
            }
            const unsigned long long gm = __ballot(act && t < (lim << 24));
            ws.n_ge += (uint32_t)__popcll(gm);
            ws.n_all += (uint32_t)__popcll(gm);
            wave_insert(ws, ((uint64_t)t << 32) | xid, gm, k, lane);
        }
    }
}

// m and c* of one member from its group row (general-k path).
__device__ inline void slot_min_cell(const uint16_t *row, uint32_t R, uint32_t Bp, const uint8_t *cnt8,
                                     uint32_t &m, uint32_t &cs) {
    m = 0xFFFFFFFFu;
    cs = 0;
    for (uint32_t r = 0; r < R; ++r) {
        const uint32_t c = r * Bp + row[r];
        const uint32_t v = 255u - cnt8[c];
        if (v <= m) {
            m = v;
            cs = c;
        }
    }
}

// GK: the general-k decode (k > 64) instead of the per-wavefront register
// top-k.  PERS: the persistent grid, whose workgroups pull queries from a
// device counter; otherwise one workgroup per query.  Each combination is
// compiled separately so that the common path carries only its own code and
// registers (the persistent loop keeps more values live).  WAVES: the
// wavefronts per SIMD the register allocation must allow.
template <typename CellT, int RP, int QT, bool GK, bool PERS, int WAVES>
__global__ __launch_bounds__(QT, WAVES) void query_kernel(QArgs A) {
    constexpr int QW = QT / 64;
    extern __shared__ __align__(16) unsigned char lds[];
    const uint32_t HC = A.hc;
    const QLayout lay = q_layout(A.L, A.R, A.Bp, A.cap, QT, HC, GK);
    constexpr uint32_t CL = cl_for(QT);
    uint64_t *buf = reinterpret_cast<uint64_t *>(lds + lay.off_buf);
    uint32_t *cnt32 = reinterpret_cast<uint32_t *>(lds + lay.off_cnt);
    const uint8_t *cnt8 = lds + lay.off_cnt;
    uint32_t *hist = reinterpret_cast<uint32_t *>(lds + lay.off_hist);
    uint32_t *pre = reinterpret_cast<uint32_t *>(lds + lay.off_pre);
    uint32_t *pree = reinterpret_cast<uint32_t *>(lds + lay.off_pree);
    uint32_t *lstart = reinterpret_cast<uint32_t *>(lds + lay.off_start);
    uint32_t *lend = reinterpret_cast<uint32_t *>(lds + lay.off_end);
    uint32_t *lb = reinterpret_cast<uint32_t *>(lds + lay.off_lb);
    uint32_t *lp = reinterpret_cast<uint32_t *>(lds + lay.off_lp);
    uint32_t *tl = reinterpret_cast<uint32_t *>(lds + lay.off_tl);
    constexpr uint32_t TLC = tl_for(QT);
    uint32_t *misc = reinterpret_cast<uint32_t *>(lds + lay.off_misc);
    uint32_t *scr = misc + M_SCAN0;

    const int tid = threadIdx.x, lane = tid % 64, wave = tid / 64;
    const uint32_t L = A.L, R = A.R, B = A.B, Bp = A.Bp, k = A.k, cap = A.cap;
    const uint64_t nbk1 = (1ull << A.nbits) + 1;
    const uint32_t gmax = A.gmax;
    const uint32_t cpc = (gmax + 255) / 256;  // 256-member chunks per cell
    const uint64_t rstride = (uint64_t)B * A.mstride;
    const CellT *cells = static_cast<const CellT *>(A.cells);

    uint64_t q = blockIdx.x;
    for (;;) {
        if constexpr (PERS) {
            if (tid == 0) misc[M_Q] = atomicAdd(A.work, 1u);
            __syncthreads();
            q = misc[M_Q];
            __syncthreads();
        }
        if (q >= A.nq) break;

        // ---- 1. the query's L list ranges (loads issued first, so that they
        // are in flight while the counters are cleared), as 16-byte chunks
        constexpr uint32_t CE = 16 / sizeof(CellT);  // list entries per chunk
        uint32_t nch = 0, st = 0, en = 0;
        if ((uint32_t)tid < L) {
            // a code outside the table (caller-supplied codes) matches no
            // bucket: its table adds nothing
            const uint32_t h = A.codes[q * L + tid];
            if ((uint64_t)h + 1 < nbk1) {
                const uint32_t *o = A.offsets + (uint64_t)tid * nbk1 + h;
                st = o[0];
                en = o[1];
            }
        }
        {
            uint4 *c16 = reinterpret_cast<uint4 *>(cnt32);
            for (uint32_t w = tid; w < lay.cnt_words / 4; w += QT)
                c16[w] = make_uint4(~0u, ~0u, ~0u, ~0u);  // count 0
        }
        for (uint32_t w = tid; w < lay.hist_words; w += QT) hist[w] = 0u;
        if (tid == 0) {
            misc[M_NT] = 0;
            misc[M_THI] = 0;
            misc[M_NEXT] = 0;
        }
        if (en > st) nch = (en + CE - 1) / CE - st / CE;
        const uint32_t ne = en - st;  // entries
        uint32_t total, nent;  // chunks and entries over all tables
        if (L <= 64) {
            // the tables fit in wavefront 0: the scans stay in it
            if (wave == 0) {
                uint32_t inc = nch, ince = ne;
#pragma unroll
                for (int o = 1; o < 64; o <<= 1) {
                    const uint32_t y = (uint32_t)__shfl_up((int)inc, o, 64);
                    const uint32_t ye = (uint32_t)__shfl_up((int)ince, o, 64);
                    if (lane >= o) {
                        inc += y;
                        ince += ye;
                    }
                }
                if ((uint32_t)lane < L) {
                    pre[lane] = inc - nch;
                    pree[lane] = ince - ne;
                    lstart[lane] = st;
                    lend[lane] = en;
                }
                if (lane == 63) {  // lanes past L add nothing
                    pre[L] = inc;
                    pree[L] = ince;
                }
            }
            __syncthreads();
            total = pre[L];
            nent = pree[L];
        } else {
            const uint32_t ex = wg_excl_scan<QT>(nch, scr, &total);
            const uint32_t exe = wg_excl_scan<QT>(ne, scr, &nent);
            if ((uint32_t)tid < L) {
                pre[tid] = ex;
                pree[tid] = exe;
                lstart[tid] = st;
                lend[tid] = en;
            }
            if (tid == 0) {
                pre[L] = total;
                pree[L] = nent;
            }
            __syncthreads();
        }

        // ---- 2. count: one increment per listed cell per table.
        // Dense (many entries for the number of cells): chunk ci belongs to
        // the last table t with pre[t] <= ci; a thread's chunks only grow, so
        // after one binary search its table index only moves forward.  Four
        // aligned 16-byte chunks per thread are loaded before their
        // increments; entries outside the table's list are skipped.
        // Sparse: one entry per thread (entry j in the last table t with
        // pre_e[t] <= j), and each increment also adds one to the
        // count-at-least histogram of the cell's repetition at the new count
        // (the old count comes back from the atomic), which replaces the
        // scan of all counters below; a cell's first increment notes it.
        const bool sparse = nent <= lay.cnt_words;
        // (the sparse increments are few: one copy takes them all)
        uint32_t *hwc = hist + (sparse ? 0u : ((uint32_t)tid & (HC - 1)) * R * (L + 1));
        if (sparse) {
            for (uint32_t j = tid; j < nent; j += QT) {
                uint32_t lo = 0, hi = L;
                while (hi - lo > 1) {
                    const uint32_t mid = (lo + hi) >> 1;
                    if (pree[mid] <= j) lo = mid; else hi = mid;
                }
                const uint32_t c = cells[lstart[lo] + (j - pree[lo])];
                const uint32_t sh = 8 * (c & 3);
                const uint32_t old = atomicSub(&cnt32[c >> 2], 1u << sh);
                const uint32_t ob = 255u - ((old >> sh) & 255u);  // count before
                const uint32_t r = div_small(c, Bp, A.inv_bp);
                atomicAdd(&hwc[r * (L + 1) + ob + 1], 1u);
                if constexpr (!GK) {
                    if (ob == 0) {
                        const uint32_t slot = atomicAdd(&misc[M_NT], 1u);
                        if (slot < TLC) tl[slot] = c;
                    }
                }
            }
        } else {
            const uint4 *cells16 = static_cast<const uint4 *>(A.cells);
            uint32_t t = 0;
            if ((uint32_t)tid < total) {
                uint32_t lo = 0, hi = L;
                const uint32_t idx = tid;
                while (hi - lo > 1) {
                    const uint32_t mid = (lo + hi) >> 1;
                    if (pre[mid] <= idx) lo = mid; else hi = mid;
                }
                t = lo;
            }
            for (uint32_t base = tid; base < total; base += 4 * QT) {
                uint4 v[4];
                uint32_t chunk[4], tt[4];
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    const uint32_t ci = base + (uint32_t)u * QT;
                    tt[u] = 0xFFFFFFFFu;
                    chunk[u] = 0;
                    v[u] = make_uint4(0, 0, 0, 0);
                    if (ci < total) {
                        while (t + 1 < L && pre[t + 1] <= ci) ++t;
                        tt[u] = t;
                        chunk[u] = lstart[t] / CE + (ci - pre[t]);
                        v[u] = cells16[chunk[u]];
                    }
                }
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    if (tt[u] == 0xFFFFFFFFu) continue;
                    const uint32_t lo = lstart[tt[u]], hi = lend[tt[u]];
                    const uint32_t w4[4] = {v[u].x, v[u].y, v[u].z, v[u].w};
#pragma unroll
                    for (uint32_t e = 0; e < CE; ++e) {
                        const uint32_t j = chunk[u] * CE + e;
                        const uint32_t c = (CE == 8) ? ((w4[e / 2] >> (16 * (e & 1))) & 0xFFFFu)
                                                     : w4[e % 4];
                        if (j >= lo && j < hi) atomicSub(&cnt32[c >> 2], 1u << (8 * (c & 3)));
                    }
                }
            }
        }
        __syncthreads();

        if (A.counts_out) {
            // debug: export counters as [R][B] bytes
            uint8_t *out = A.counts_out + q * (uint64_t)R * B;
            for (uint32_t c = tid; c < R * B; c += QT) out[c] = 255u - cnt8[(c / B) * Bp + c % B];
            __syncthreads();
            if constexpr (!PERS) break;
            continue;
        }

        // ---- 3. per-repetition histograms, as counts-at-least: hist[r][v] =
        // cells of repetition r with count >= v for v >= 1 (sparse: built
        // while counting; dense: a scan of the counters into HC copies, the
        // copies merged, then suffix sums)
        if (!sparse) {
            for (uint32_t w = tid; w < lay.cnt_words; w += QT) {
                const uint32_t v = ~cnt32[w];  // four counts
                if (!v) continue;
                const uint32_t r = div_small(4 * w, Bp, A.inv_bp);
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    const uint32_t cv = (v >> (8 * j)) & 255u;
                    if (cv) atomicAdd(&hwc[r * (L + 1) + cv], 1u);
                }
            }
            __syncthreads();
            for (uint32_t i = tid; i < R * (L + 1); i += QT) {
                uint32_t sacc = 0;
                // constant trip counts: a loop bounded by HC alone costs registers
                if (HC <= 4) {
#pragma unroll
                    for (uint32_t w = 0; w < 4; ++w)
                        if (w < HC) sacc += hist[w * R * (L + 1) + i];
                } else {
                    for (uint32_t w = 0; w < HC_MAX; ++w)
                        if (w < HC) sacc += hist[w * R * (L + 1) + i];
                }
                hist[i] = sacc;
            }
            __syncthreads();
            // suffix sums (one wavefront per repetition, 4 levels per lane)
            for (uint32_t r = wave; r < R; r += QW) {
                uint32_t *h = hist + r * (L + 1);
                uint32_t v[4], loc = 0;
#pragma unroll
                for (int j = 3; j >= 0; --j) {
                    const uint32_t idx = 4 * lane + j;
                    v[j] = (idx <= L && idx >= 1) ? h[idx] : 0u;
                    loc += v[j];
                    v[j] = loc;  // suffix within the lane's 4 levels
                }
                uint32_t above = loc;  // inclusive suffix over lanes >= lane
#pragma unroll
                for (int o = 1; o < 64; o <<= 1) {
                    const uint32_t y = (uint32_t)__shfl_down((int)above, o, 64);
                    if (lane + o < 64) above += y;
                }
                const uint32_t after = above - loc;  // lanes > lane
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    const uint32_t idx = 4 * lane + j;
                    if (idx <= L && idx >= 1) h[idx] = v[j] + after;
                }
                if (lane == 0) h[0] = B;
            }
            __syncthreads();
        }
        // ms[t] = min over repetitions of cells with count >= t (the list
        // offsets are no longer needed, so `pre` holds it).  Enumerating the
        // level-t cells of the cheapest repetition reads about ms[t]*ceil(N/B)
        // members; ms is non-increasing in t.  Level t belongs to thread
        // t - 1 (L < QT), here and when the level is lowered.
        // t_hi = #{t in 1..L : ms[t]*gmax >= k} (a prefix of levels);
        // t_lo = #{t in 1..L : ms[t]*gmax <= budget} (a suffix of levels).
        uint32_t *ms = pre;
        {
            const uint32_t t = 1 + tid;
            uint64_t sz = 0;
            if (t <= L) {
                uint32_t mn = 0xFFFFFFFFu;
                for (uint32_t r = 0; r < R; ++r) {
                    const uint32_t c = hist[r * (L + 1) + t];
                    mn = c < mn ? c : mn;
                }
                ms[t] = mn;
                sz = (uint64_t)mn * gmax;
            }
            const unsigned long long mh = __ballot(t <= L && sz >= k);
            const unsigned long long ml = __ballot(t <= L && sz <= A.budget);
            uint32_t thi = 0, tlo = 0;
            if (L <= 64) {
                // every level is in wavefront 0
                thi = (uint32_t)__popcll(mh);
                tlo = L + 1 - (uint32_t)__popcll(ml);
            } else {
                if (lane == 0 && (uint32_t)wave * 64 < L) {
                    atomicAdd(&misc[M_THI], (uint32_t)__popcll(mh));
                    atomicAdd(&misc[M_NEXT], (uint32_t)__popcll(ml));
                }
                __syncthreads();
                thi = misc[M_THI];
                tlo = L + 1 - misc[M_NEXT];
            }
            // the lowest level within the budget, but at most t_hi
            if (tid == 0) misc[M_LEVEL] = (thi == 0) ? 0u : (tlo <= thi ? tlo : thi);
        }

        // ---- 4. decode passes
        // per-query work tallies (members read, in the final pass, passes) in
        // LDS rather than registers: they live across the whole decode
        if (tid == 0) {
            misc[M_ST_ALL] = 0;
            misc[M_ST_FINAL] = 0;
            misc[M_ST_GATH] = 0;
            misc[M_ST_PASSES] = 0;
        }
        for (;;) {
            if (tid == 0) {
                uint32_t level = misc[M_LEVEL];
                uint32_t rep, keep = 0;
                if (level == 0) {
                    level = 1;
                    rep = R - 1;
                    keep = 1;
                } else {
                    uint32_t best = 0xFFFFFFFFu;
                    rep = 0;
                    for (uint32_t r = 0; r < R; ++r) {
                        const uint32_t sc = hist[r * (L + 1) + level];
                        if (sc < best) { best = sc; rep = r; }
                    }
                    // level 1: one pass over repetition R-1 keeping every key
                    // serves both outcomes (m >= 1 for k points, or the
                    // zero-count completion) when it is not much larger.  Not
                    // where the fast decode filters (R >= 2): its filtered
                    // pass at level 1 reads a fraction of the bytes and most
                    // often finds the k keys alone
                    if (level == 1 && (GK || R < 2) &&
                        (uint64_t)hist[(R - 1) * (L + 1) + 1] * gmax <= 2ull * A.budget) {
                        rep = R - 1;
                        keep = 1;
                    }
                }
                misc[M_LEVEL] = level;
                misc[M_REP] = rep;
                misc[M_KEEPALL] = keep;
                misc[M_BUFN] = 0;
                misc[M_NGE] = 0;
                misc[M_NALL] = 0;
                misc[M_THRLO] = 0xFFFFFFFFu;
                misc[M_THRHI] = 0xFFFFFFFFu;
                misc[M_LCNT] = 0;
                misc[M_MEMB] = 0;
                misc[M_GATH] = 0;
            }
            __syncthreads();
            // uniform across the workgroup: kept in scalar registers
            const uint32_t level = __builtin_amdgcn_readfirstlane(misc[M_LEVEL]);
            const uint32_t rep = __builtin_amdgcn_readfirstlane(misc[M_REP]);
            const bool keep = misc[M_KEEPALL] != 0;
            const uint32_t *memr = A.mem + rep * rstride;
            const uint16_t *cmgr = A.cmg + rep * rstride * RP;

          if constexpr (!GK) {
            // Fast decode (k <= 64): the positive cells of `rep` go into an
            // LDS list (one word-wide scan, or 256 cells at a time when they
            // do not fit); each wavefront streams (cell, 256-member chunk)
            // items with several in flight per lane and keeps its own top-k
            // in registers; the lists are merged by rank at the end.
            WaveState ws{~0ull, ~0ull, 0u, 0u, 0u, 0u};
            // walk items in flight per lane: one where the rows are wide or
            // many wavefronts share a SIMD
            constexpr int WU = (RP >= 4 || (QT == 256 && !PERS)) ? 1 : 2;
            // the filtered walk: a pass keeping only m >= level, R >= 2
            constexpr int WF = (QT == 256 || PERS) ? (WAVES >= 8 ? 1 : 2) : 4;
            const bool filt = !keep && R >= 2 && rstride < (1ull << 32);  // 32-bit slots
            const uint32_t *cflr = A.cfl + rep * rstride;
            const uint32_t f1b = ((rep + 1) % R) * Bp, f2b = ((rep + 2) % R) * Bp;
            const uint32_t nrep = hist[rep * (L + 1) + level];
            if (nrep <= CL) {
                const uint32_t nt = misc[M_NT];
                if (sparse && nt <= TLC) {
                    // from the cells the query touched
                    const uint32_t c0 = rep * Bp;
                    for (uint32_t i = tid; i < nt; i += QT) {
                        const uint32_t c = tl[i];
                        if (c - c0 < B && 255u - cnt8[c] >= level) lb[atomicAdd(&misc[M_LCNT], 1u)] = c - c0;
                    }
                } else {
                    for (uint32_t w = tid; w < Bp / 4; w += QT) {
                        const uint32_t v = ~cnt32[rep * (Bp / 4) + w];  // four counts
                        if (!v) continue;
#pragma unroll
                        for (int j = 0; j < 4; ++j) {
                            const uint32_t b = 4 * w + j;
                            if (b < B && ((v >> (8 * j)) & 255u) >= level)
                                lb[atomicAdd(&misc[M_LCNT], 1u)] = b;
                        }
                    }
                }
                __syncthreads();
                if (QT == 1024 && filt) {
                    // sizes and 4-rounded prefix sums of the listed cells
                    // (nrep <= CL = QT: one cell per thread)
                    uint32_t *fp = reinterpret_cast<uint32_t *>(lds + lay.off_fp);
                    uint32_t *fs = reinterpret_cast<uint32_t *>(lds + lay.off_fs);
                    const uint32_t csz = (uint32_t)tid < nrep ? A.gsize[rep * B + lb[tid]] : 0u;
                    uint32_t ftot;
                    const uint32_t fex = wg_excl_scan<QT>((csz + 3) & ~3u, scr, &ftot);
                    if ((uint32_t)tid < nrep) {
                        fp[tid] = fex;
                        fs[tid] = csz;
                    }
                    __syncthreads();
                    walk_flat_filtered<RP, WF, QT>(lb, fp, fs, nrep, ftot, memr, cmgr, cflr, R, Bp,
                                                   A.mstride, level, f1b, f2b, k, lane, wave, ws);
                } else if (filt)
                    walk_cells_filtered<RP, WF, QT>(lb, nrep, memr, cmgr, cflr, R, Bp, A.mstride,
                                                    level, f1b, f2b, A.gsize + rep * B, cpc, k, lane,
                                                    wave, ws);
                else
                    walk_cells<RP, WU, QT>(lb, nrep, memr, cmgr, cnt8, R, Bp, A.mstride, level, keep,
                                           A.gsize + rep * B, cpc, k, lane, wave, ws);
            } else {
                const unsigned long long ltmask = (lane == 0) ? 0ull : ((~0ull) >> (64 - lane));
                for (uint32_t cb0 = 0; cb0 < B; cb0 += QT) {
                    const uint32_t b = cb0 + tid;
                    const bool pos = (b < B) && (255u - cnt8[rep * Bp + b] >= level);
                    const unsigned long long pm = __ballot(pos);
                    uint32_t wbase = 0;
                    if (lane == 0 && pm) wbase = atomicAdd(&misc[M_LCNT], (uint32_t)__popcll(pm));
                    wbase = (uint32_t)__shfl((int)wbase, 0, 64);
                    if (pos) lb[wbase + (uint32_t)__popcll(pm & ltmask)] = b;
                    __syncthreads();
                    const uint32_t nl = misc[M_LCNT];
                    if (nl > CL - QT || cb0 + QT >= B) {
                        if (filt)
                            walk_cells_filtered<RP, WF, QT>(lb, nl, memr, cmgr, cflr, R, Bp,
                                                            A.mstride, level, f1b, f2b,
                                                            A.gsize + rep * B, cpc, k, lane, wave, ws);
                        else
                            walk_cells<RP, WU, QT>(lb, nl, memr, cmgr, cnt8, R, Bp, A.mstride, level,
                                                   keep, A.gsize + rep * B, cpc, k, lane, wave, ws);
                        __syncthreads();
                        if (tid == 0) misc[M_LCNT] = 0;
                        __syncthreads();
                    }
                }
            }
            // merge the per-wave lists: when they fit in one wavefront, one
            // sort across it; else the rank of each key among all keys
            uint64_t *wlist = buf + k;  // one k-key list per wavefront
            if ((uint32_t)lane < k) wlist[wave * k + lane] = ws.wl;
            if (lane == 0) {
                atomicAdd(&misc[M_NGE], ws.n_ge);
                atomicAdd(&misc[M_NALL], ws.n_all);
                atomicAdd(&misc[M_MEMB], ws.members);
                atomicAdd(&misc[M_GATH], ws.gathered);
            }
            __syncthreads();
            if (QW * k <= 64) {
                // only a final pass needs the result, and then wavefront 0
                // alone emits it (lane i writes and reads entry i): the other
                // wavefronts are done
                const bool fin = misc[M_NGE] >= k || keep;
                if (fin && wave == 0) {
                    const uint64_t v = wave_sort64((uint32_t)lane < QW * k ? wlist[lane] : ~0ull, lane);
                    if ((uint32_t)lane < k) buf[fresh_copy((uint32_t)lane)] = v;
                }
                if (fin && wave != 0) break;
            } else if ((uint32_t)tid < QW * k) {
                // rank = the keys of all lists below this one (keys are
                // distinct; empty entries, ~0, are below none): independent
                // broadcast reads of the whole set rather than dependent
                // binary searches
                const uint64_t key = wlist[tid];
                if (key != ~0ull) {
                    // (1024 threads: sixteen reads issued before any
                    // compare, so the LDS latency is paid once per sixteen
                    // keys; the 256-thread kernels lack the registers)
                    constexpr uint32_t RB16 = QT == 1024 ? 16u : 1u;
                    const uint32_t nkeys = QW * k;
                    uint32_t rank = 0, j = 0;
                    if constexpr (RB16 > 1)
                    for (; j + 16 <= nkeys; j += 16) {
                        uint64_t v[16];
#pragma unroll
                        for (int u = 0; u < 16; ++u) v[u] = wlist[j + u];
#pragma unroll
                        for (int u = 0; u < 16; ++u) rank += (v[u] < key) ? 1u : 0u;
                    }
                    for (; j < nkeys; ++j) rank += (wlist[j] < key) ? 1u : 0u;
                    if (rank < k) buf[rank] = key;
                }
            }
            if (QW * k > 64) __syncthreads();
          } else {
            // General k: cells 256 at a time, candidates appended to a
            // capacity-cap LDS buffer under a tightening threshold; the
            // buffer is sorted and cut to k when nearly full.
            uint32_t n_ge = 0, n_all = 0;  // per-wave tallies (lane 0 of each wave)
            unsigned long long pass_members = 0;
            for (uint32_t cb0 = 0; cb0 < B; cb0 += QT) {
                const uint32_t b = cb0 + tid;
                uint32_t cval = 0;
                if (b < B) cval = 255u - cnt8[rep * Bp + b];
                const bool pos = (b < B) && (cval >= level);
                const uint32_t sz = pos ? A.gsize[rep * B + b] : 0u;
                uint32_t npos, tsz;
                const uint32_t ci = wg_excl_scan<QT>(pos ? 1u : 0u, scr, &npos);
                const uint32_t ps = wg_excl_scan<QT>(sz, scr, &tsz);
                if (pos) {
                    lb[ci] = b;
                    lp[ci] = ps;
                }
                pass_members += tsz;
                __syncthreads();
                for (uint32_t off = 0; off < tsz; off += QT) {
                    const uint32_t idx = off + tid;
                    bool take = false;
                    uint64_t key = 0;
                    bool ge = false;
                    if (idx < tsz) {
                        uint32_t lo = 0, hi = npos;
                        while (hi - lo > 1) {
                            uint32_t mid = (lo + hi) >> 1;
                            if (lp[mid] <= idx) lo = mid; else hi = mid;
                        }
                        const uint64_t slot = (uint64_t)lb[lo] * A.mstride + (idx - lp[lo]);
                        const uint32_t x = memr[slot];
                        uint32_t m, cs;
                        slot_min_cell(cmgr + slot * RP, R, Bp, cnt8, m, cs);
                        ge = m >= level;
                        take = keep || ge;
                        key = ((uint64_t)(255u - m) << 56) | ((uint64_t)cs << 32) | x;
                        if (take) {
                            const uint64_t thr = ((uint64_t)misc[M_THRHI] << 32) | misc[M_THRLO];
                            if (key < thr) {
                                const uint32_t slotb = atomicAdd(&misc[M_BUFN], 1u);
                                buf[slotb] = key;
                            }
                        }
                    }
                    const unsigned long long mg = __ballot(take && ge);
                    const unsigned long long ma = __ballot(take);
                    if (lane == 0) {
                        n_ge += __popcll(mg);
                        n_all += __popcll(ma);
                    }
                    __syncthreads();
                    if (misc[M_BUFN] > cap - QT) {
                        // merge: sort, keep the k smallest, tighten the threshold
                        const uint32_t nb = misc[M_BUFN];
                        for (uint32_t i = nb + tid; i < cap; i += QT) buf[i] = ~0ull;
                        __syncthreads();
                        wg_bitonic<QT>(buf, cap);
                        if (tid == 0) {
                            const uint32_t keepn = nb < k ? nb : k;
                            misc[M_BUFN] = keepn;
                            if (keepn == k) {
                                misc[M_THRLO] = (uint32_t)buf[k - 1];
                                misc[M_THRHI] = (uint32_t)(buf[k - 1] >> 32);
                            }
                        }
                        __syncthreads();
                    }
                }
                __syncthreads();
            }
            if (lane == 0) {
                atomicAdd(&misc[M_NGE], n_ge);
                atomicAdd(&misc[M_NALL], n_all);
            }
            if (tid == 0) {
                atomicAdd(&misc[M_MEMB], (uint32_t)pass_members);
                atomicAdd(&misc[M_GATH], (uint32_t)pass_members);
            }
            __syncthreads();
            {
                const uint32_t nb = misc[M_BUFN];
                for (uint32_t i = nb + tid; i < cap; i += QT) buf[i] = ~0ull;
            }
            __syncthreads();
            wg_bitonic<QT>(buf, cap);
          }
            const uint32_t nge = misc[M_NGE], nall = misc[M_NALL];
            const bool ok = nge >= k;
            if (tid == 0) {
                misc[M_ST_ALL] += misc[M_MEMB];
                misc[M_ST_PASSES] += 1;
                if (ok || keep) {
                    misc[M_ST_FINAL] = misc[M_MEMB];
                    misc[M_ST_GATH] = misc[M_GATH];
                }
            }
            if (ok || keep) {
                // emit the buffered keys (and, for the fill path, zero cells)
                const uint32_t nres = (nall < k ? nall : k);
                uint32_t *oid = A.ids + q * (uint64_t)k;
                uint32_t *osc = A.scores ? A.scores + q * (uint64_t)k : nullptr;
                for (uint32_t i = tid; i < nres; i += QT) {
                    const uint64_t key = buf[i];
                    oid[i] = (uint32_t)key;
                    if (osc) osc[i] = 255u - (uint32_t)(key >> 56);
                }
                if (!ok && nres < k && wave == 0) {
                    // zero fill from repetition R-1, cells ascending, ids ascending
                    uint32_t need = k - nres, outp = nres;
                    const uint32_t *memz = A.mem + (R - 1) * rstride;
                    for (uint32_t b0 = 0; b0 < B && need; b0 += 64) {
                        const uint32_t b = b0 + lane;
                        const bool z = (b < B) && (cnt8[(R - 1) * Bp + b] == 255u);  // count 0
                        unsigned long long zm = __ballot(z);
                        while (zm && need) {
                            const uint32_t bb = b0 + (uint32_t)(__ffsll((long long)zm) - 1);
                            zm &= zm - 1;
                            const uint32_t sz = A.gsize[(R - 1) * B + bb];
                            const uint32_t takeN = sz < need ? sz : need;
                            const uint64_t mo = (uint64_t)bb * A.mstride;
                            for (uint32_t j = lane; j < takeN; j += 64) {
                                oid[outp + j] = memz[mo + j];
                                if (osc) osc[outp + j] = 0u;
                            }
                            outp += takeN;
                            need -= takeN;
                        }
                    }
                    for (uint32_t j = outp + lane; j < k; j += 64) {
                        oid[j] = 0xFFFFFFFFu;
                        if (osc) osc[j] = 0u;
                    }
                }
                break;  // the decision is the same in every thread
            } else {
                // lower the level: the lowest level whose cheapest enumeration
                // stays within 8x the larger of the budget and this pass
                const uint32_t lv = misc[M_LEVEL];
                const uint64_t lim = 8ull * (A.budget > nall ? A.budget : nall);
                __syncthreads();
                if (tid == 0) misc[M_NEXT] = 0;
                __syncthreads();
                {
                    const uint32_t t = 1 + fresh_copy((uint32_t)tid);
                    const unsigned long long ml = __ballot(t <= L && (uint64_t)ms[t] * gmax <= lim);
                    if (lane == 0 && (uint32_t)wave * 64 < L) atomicAdd(&misc[M_NEXT], (uint32_t)__popcll(ml));
                }
                __syncthreads();
                if (tid == 0) {
                    const uint32_t t1 = L + 1 - misc[M_NEXT];
                    misc[M_LEVEL] = (t1 < lv) ? t1 : lv - 1;  // 0 selects the fill path
                }
            }
            __syncthreads();
        }
        if (A.stats && tid == 0) {
            unsigned long long entries = 0;
            for (uint32_t t = 0; t < L; ++t) entries += lend[t] - lstart[t];
            atomicAdd(&A.stats[0], entries);
            atomicAdd(&A.stats[1], (unsigned long long)misc[M_ST_ALL]);
            atomicAdd(&A.stats[2], (unsigned long long)misc[M_ST_FINAL]);
            atomicAdd(&A.stats[3], (unsigned long long)misc[M_ST_PASSES]);
            atomicAdd(&A.stats[4], (unsigned long long)misc[M_ST_GATH]);
        }
        if constexpr (!PERS) break;
        __syncthreads();  // before the next query reuses the LDS state
    }
}

// ---------------------------------------------------------------------------
uint32_t query_max_k() { return 4096; }

// Top-k buffer capacity.  Fast path (k <= 64): the k results, then one
// k-key list per wavefront (an even count, so that the counters after it
// stay 16-byte aligned).  General path: room for k kept keys plus one round
// of T appends, a power of two for the bitonic sort.
static uint32_t cap_for(uint32_t k, int T) {
    if (k <= 64) return (k * (1u + (uint32_t)T / 64) + 1) & ~1u;
    uint32_t need = std::max<uint32_t>(512u, k + (uint32_t)T);
    uint32_t c = 1;
    while (c < need) c <<= 1;
    return c;
}

static int max_lds();

// Launch shape of the query kernel for one index and k.
struct QShape {
    int T;
    uint32_t cap, hc;
    size_t lds;
};

// 256 threads when four such workgroups fit in a CU's LDS (the register
// budget admits four per CU: 16 wavefronts), else 1024 threads with one
// workgroup per CU (also 16).  The histogram copies take what the LDS share
// of one workgroup has left, up to HC_MAX.
// sparse: the index's lists are short enough that its queries are expected
// to count sparsely, with the histogram built while counting (no copies).
static QShape q_shape(uint32_t L, uint32_t R, uint32_t Bp, uint32_t k, bool sparse) {
    const size_t lim = (size_t)max_lds();
    const size_t bins = (size_t)R * (L + 1) * 4;
    QShape sh;
    const bool gk = k > 64;
    const size_t small = q_layout(L, R, Bp, cap_for(k, 256), 256, 1, gk).total;
    if (small * 4 <= lim) {
        // a state this small holds few cells, so few counts collide: four
        // copies (more only add clearing and merging), none for sparse
        // queries, whose smaller state may then let one more workgroup in
        sh.T = 256;
        sh.hc = sparse ? 1u : (uint32_t)std::min<size_t>(4, 1 + (lim / 4 - small) / bins);
    } else {
        const size_t big = q_layout(L, R, Bp, cap_for(k, 1024), 1024, 1, gk).total;
        sh.T = big <= lim ? 1024 : 256;
        sh.hc = big <= lim ? (uint32_t)std::min<size_t>(HC_MAX, 1 + (lim - big) / bins) : 1u;
    }
    while (sh.hc & (sh.hc - 1)) sh.hc &= sh.hc - 1;  // round down to a power of two
    sh.cap = cap_for(k, sh.T);
    sh.lds = q_layout(L, R, Bp, sh.cap, sh.T, sh.hc, gk).total;
    return sh;
}

// Whether an index's queries are expected to count sparsely: the mean list
// entries a query meets (all lists over all buckets) at most a quarter of the
// counter words (the per-query test is entries <= counter words).
static bool sparse_index(const Index &ix) {
    const uint32_t Bp = (ix.p.B + 3) & ~3u;
    const uint64_t words = ((uint64_t)ix.p.R * Bp) / 4;
    return (ix.list_entries >> ix.nbits) * 4 <= words;
}

size_t query_lds_bytes(const Index &ix, uint32_t k) {
    const uint32_t Bp = (ix.p.B + 3) & ~3u;
    return q_shape(ix.p.L, ix.p.R, Bp, k, sparse_index(ix)).lds;
}

// Device attributes read once per process (function-local statics are
// initialised exactly once even when several threads launch at the same time;
// every device this library runs on is an MI355X, so one reading serves all).
static int device_attr(hipDeviceAttribute_t attr, int fallback) {
    int dev = 0;
    (void)hipGetDevice(&dev);
    int x = 0;
    if (hipDeviceGetAttribute(&x, attr, dev) != hipSuccess || x <= 0) {
        (void)hipGetLastError();
        x = fallback;
    }
    return x;
}

static int max_lds() {
    static const int v = device_attr(hipDeviceAttributeMaxSharedMemoryPerBlock, 65536);
    return v;
}

static int num_cus() {
    static const int v = device_attr(hipDeviceAttributeMultiprocessorCount, 256);
    return v;
}

template <typename CellT, int RP, int QT, bool GK, bool PERS, int WAVES>
static void launch_kernel(const QArgs &a, size_t lds, unsigned grid, hipStream_t s) {
    // once per kernel variant and process (a throwing initialiser is retried)
    static const bool attrs_ok = [] {
        const void *fn = reinterpret_cast<const void *>(&query_kernel<CellT, RP, QT, GK, PERS, WAVES>);
        (void)hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, max_lds());
        // the counters are addressed from LDS address 0 (dynamic LDS first)
        hipFuncAttributes fa{};
        if (hipFuncGetAttributes(&fa, fn) != hipSuccess || fa.sharedSizeBytes != 0)
            fail(FLINNG_EDEVICE, "query kernel: static LDS in use or attributes unavailable");
        return true;
    }();
    (void)attrs_ok;
    hipLaunchKernelGGL((query_kernel<CellT, RP, QT, GK, PERS, WAVES>), dim3(grid), dim3(QT), lds, s, a);
}

template <typename CellT, int RP, int QT, bool GK>
static void launch_rp(const QArgs &a, size_t lds, bool persistent, hipStream_t s) {
    uint64_t grid = a.nq;
    if (persistent) {
        const uint64_t per_cu = std::max<uint64_t>(
            1, std::min<uint64_t>(8, (uint64_t)(160 * 1024) / std::max<size_t>(lds, 1)));
        grid = std::min<uint64_t>(a.nq, per_cu * (uint64_t)num_cus());
    }
    if (grid == 0) return;
    if (grid > 0x7FFFFFFFull) fail(FLINNG_EINVAL, "query batch too large for one launch");
    // Register budgets: the one-query fast kernel at 256 threads asks for as
    // many wavefronts per SIMD as the LDS lets share a CU (six to eight
    // four-wavefront workgroups); the others take what they need.
    if constexpr (QT == 256 && !GK) {
        if (persistent)
            launch_kernel<CellT, RP, QT, GK, true, 4>(a, lds, (unsigned)grid, s);
        else if (lds * 8 <= (size_t)max_lds())
            launch_kernel<CellT, RP, QT, GK, false, 8>(a, lds, (unsigned)grid, s);
        else if (lds * 7 <= (size_t)max_lds())
            launch_kernel<CellT, RP, QT, GK, false, 7>(a, lds, (unsigned)grid, s);
        else
            launch_kernel<CellT, RP, QT, GK, false, 6>(a, lds, (unsigned)grid, s);
    } else {
        constexpr int W = QT == 256 ? 4 : 1;
        if (persistent)
            launch_kernel<CellT, RP, QT, GK, true, W>(a, lds, (unsigned)grid, s);
        else
            launch_kernel<CellT, RP, QT, GK, false, W>(a, lds, (unsigned)grid, s);
    }
    FL_CHECK_LAUNCH();
}

template <typename CellT, int QT, bool GK>
static void launch_t(const QArgs &a, size_t lds, bool persistent, hipStream_t s) {
    switch (a.Rp) {
        case 1: launch_rp<CellT, 1, QT, GK>(a, lds, persistent, s); break;
        case 2: launch_rp<CellT, 2, QT, GK>(a, lds, persistent, s); break;
        case 4: launch_rp<CellT, 4, QT, GK>(a, lds, persistent, s); break;
        case 8: launch_rp<CellT, 8, QT, GK>(a, lds, persistent, s); break;
        default: launch_rp<CellT, 16, QT, GK>(a, lds, persistent, s); break;
    }
}

template <typename CellT>
static void launch_q(const QArgs &a, size_t lds, bool persistent, hipStream_t s) {
    const bool gk = a.k > 64;
    if (a.threads == 1024) {
        if (gk) launch_t<CellT, 1024, true>(a, lds, persistent, s);
        else launch_t<CellT, 1024, false>(a, lds, persistent, s);
    } else {
        if (gk) launch_t<CellT, 256, true>(a, lds, persistent, s);
        else launch_t<CellT, 256, false>(a, lds, persistent, s);
    }
}

__global__ void zero_u32_kernel(uint32_t *p) {
    if (threadIdx.x == 0) *p = 0u;
}

static QArgs make_args(const Index &ix, const uint32_t *codes, uint64_t nq, uint32_t k) {
    QArgs a{};
    a.codes = codes;
    a.nq = nq;
    a.offsets = ix.offsets;
    a.cells = ix.cells;
    a.mem = ix.mem;
    a.cmg = ix.cmg;
    a.cfl = ix.cfl;
    a.N = ix.N;
    a.gsize = ix.gsize;
    a.gmax = ix.gmax;
    a.L = ix.p.L;
    a.R = ix.p.R;
    a.Rp = ix.Rp;
    a.B = ix.p.B;
    a.Bp = (ix.p.B + 3) & ~3u;
    a.nbits = ix.nbits;
    a.k = k;
    const QShape sh = q_shape(a.L, a.R, a.Bp, k, sparse_index(ix));
    a.threads = (uint32_t)sh.T;
    a.cap = sh.cap;
    a.hc = sh.hc;
    a.mstride = ix.mstride;
    a.inv_bp = 1.0f / (float)a.Bp;
    a.budget = sparse_index(ix) ? BUDGET_SPARSE : BUDGET_DENSE;
    return a;
}

void query_launch(const Index &ix, const uint32_t *codes_dev, uint64_t nq, uint32_t k,
                  uint32_t *ids_dev, uint32_t *scores_dev, bool persistent, hipStream_t s,
                  uint32_t *work_counter, unsigned long long *stats) {
    if (nq == 0) return;
    QArgs a = make_args(ix, codes_dev, nq, k);
    a.ids = ids_dev;
    a.scores = scores_dev;
    a.work = persistent ? work_counter : nullptr;
    a.stats = stats;
    const size_t lds = q_layout(a.L, a.R, a.Bp, a.cap, (int)a.threads, a.hc, a.k > 64).total;
    if ((int)lds > max_lds())
        fail(FLINNG_EINVAL, "per-query state (" + std::to_string(lds) +
                                " bytes) exceeds the workgroup LDS limit; reduce B*R or k");
    // the persistent grid's query counter starts at 0 (cleared by a kernel,
    // so that the launch can be captured into a graph)
    if (persistent) {
        hipLaunchKernelGGL(zero_u32_kernel, dim3(1), dim3(64), 0, s, work_counter);
        FL_CHECK_LAUNCH();
    }
    if (ix.cell_bytes == 2)
        launch_q<uint16_t>(a, lds, persistent, s);
    else
        launch_q<uint32_t>(a, lds, persistent, s);
}

void counts_launch(const Index &ix, const uint32_t *codes_dev, uint64_t nq, uint8_t *counts_dev,
                   hipStream_t s) {
    if (nq == 0) return;
    QArgs a = make_args(ix, codes_dev, nq, 1);
    a.counts_out = counts_dev;
    const size_t lds = q_layout(a.L, a.R, a.Bp, a.cap, (int)a.threads, a.hc, a.k > 64).total;
    if ((int)lds > max_lds()) fail(FLINNG_EINVAL, "per-query state exceeds the LDS limit");
    if (ix.cell_bytes == 2)
        launch_q<uint16_t>(a, lds, false, s);
    else
        launch_q<uint32_t>(a, lds, false, s);
}

}  // namespace flinng
