// Fixed-threshold query (Algorithm 2) on gfx950.
//
// Algorithm 2 marks a cell positive when its group test fires -- its count
// of colliding tables reaches the threshold t (positive means count >= t) --
// takes in each repetition the union of the positive cells' points and
// reports the intersection of those unions over the R repetitions.  A point
// x is therefore reported iff m(x) = min_r C[r, g_r(x)] >= t, and every
// reported point lies in a positive cell of any single repetition.
//
// One workgroup per query:
//   1. counts: the B*R cell counters as bytes in LDS (4 per dword), one
//      32-bit LDS atomic add per reverse-index list entry of the query's L
//      buckets (Section 6, Implementation);
//   2. the number of positive cells of each repetition; the repetition with
//      the fewest is enumerated (ties: the lowest);
//   3. its positive cells, taken in ascending order up to T at a time, and
//      their members (cell-major member ids beside their R group ids): a
//      member is reported iff all R of its cells are positive, written in
//      enumeration order (cells ascending, members by ascending id) by an
//      ordered compaction across the workgroup.
// Up to max_out ids are written per query; counts[q] receives the size of the
// answer even when it is larger.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "flinng_internal.h"

namespace flinng {

namespace {

struct TArgs {
    const uint32_t *codes;
    uint64_t nq;
    const uint32_t *offsets;
    const void *cells;
    const uint32_t *mem;
    const uint16_t *cmg;
    uint32_t L, R, Rp, B, Bp, nbits, t, max_out;
    const uint32_t *gsize;  // [R][B] members of each cell
    uint32_t gmax, mstride, cnt_words;
    uint32_t *ids;
    uint32_t *counts;
};

// misc slots after the counters
enum { T_TOTAL = 0, T_REP, T_NL, T_SCAN, T_NPOS = T_SCAN + 16 };  // T_NPOS: R words

template <int T>
__device__ inline uint32_t block_scan_excl(uint32_t v, uint32_t *scr, uint32_t *total) {
    constexpr int TW = T / 64;
    const int lane = threadIdx.x % 64, wave = threadIdx.x / 64;
    uint32_t inc = v;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const uint32_t y = (uint32_t)__shfl_up((int)inc, o, 64);
        if (lane >= o) inc += y;
    }
    if (lane == 63) scr[wave] = inc;
    __syncthreads();
    uint32_t pre = 0, tot = 0;
#pragma unroll
    for (int w = 0; w < TW; ++w) {
        const uint32_t c = scr[w];
        pre += (w < wave) ? c : 0u;
        tot += c;
    }
    __syncthreads();
    *total = tot;
    return pre + inc - v;
}

__device__ inline uint32_t count_of(const uint32_t *cnt32, uint32_t c) {
    return (cnt32[c >> 2] >> (8 * (c & 3))) & 255u;
}

template <typename CellT, int T>
__global__ __launch_bounds__(T) void threshold_kernel(TArgs A) {
    extern __shared__ __align__(16) uint32_t tl[];
    uint32_t *cnt32 = tl;
    uint32_t *misc = tl + A.cnt_words;
    uint32_t *npos = misc + T_NPOS;
    uint32_t *lb = npos + 16;  // up to T positive cells of one round
    const int tid = threadIdx.x;
    const uint64_t q = blockIdx.x;
    if (q >= A.nq) return;
    const uint32_t L = A.L, R = A.R, B = A.B, Bp = A.Bp, t = A.t;
    const uint64_t nbk1 = (1ull << A.nbits) + 1;
    const CellT *cells = static_cast<const CellT *>(A.cells);

    for (uint32_t w = tid; w < A.cnt_words; w += T) cnt32[w] = 0u;
    if (tid < 16) npos[tid] = 0u;
    if (tid == 0) misc[T_TOTAL] = 0u;
    __syncthreads();

    // 1. counts (a code outside the table matches no bucket)
    for (uint32_t tb = 0; tb < L; ++tb) {
        const uint32_t h = A.codes[q * L + tb];
        if ((uint64_t)h + 1 >= nbk1) continue;
        const uint32_t *o = A.offsets + (uint64_t)tb * nbk1 + h;
        const uint32_t st = o[0], en = o[1];
        for (uint32_t j = st + tid; j < en; j += T) {
            const uint32_t c = cells[j];
            atomicAdd(&cnt32[c >> 2], 1u << (8 * (c & 3)));
        }
    }
    __syncthreads();

    // 2. positive cells per repetition (a counter word holds four cells of
    // one repetition: Bp is a multiple of 4)
    for (uint32_t w = tid; w < A.cnt_words; w += T) {
        const uint32_t v = cnt32[w];
        const uint32_t r = (4 * w) / Bp;
        if (r >= R) continue;
        uint32_t n = 0;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const uint32_t b = 4 * w + j - r * Bp;
            n += (b < B && ((v >> (8 * j)) & 255u) >= t) ? 1u : 0u;
        }
        if (n) atomicAdd(&npos[r], n);
    }
    __syncthreads();
    if (tid == 0) {
        uint32_t best = 0;
        for (uint32_t r = 1; r < R; ++r)
            if (npos[r] < npos[best]) best = r;
        misc[T_REP] = best;
    }
    __syncthreads();
    const uint32_t rep = misc[T_REP];
    const uint64_t rstride = (uint64_t)B * A.mstride;
    const uint32_t *memr = A.mem + rep * rstride;
    const uint16_t *cmgr = A.cmg + rep * rstride * A.Rp;
    uint32_t *out = A.ids + q * (uint64_t)A.max_out;

    // 3. positive cells of `rep`, T at a time, and their members
    if (npos[rep] != 0) {
        for (uint32_t b0 = 0; b0 < B; b0 += T) {
            const uint32_t b = b0 + tid;
            const bool pos = b < B && count_of(cnt32, rep * Bp + b) >= t;
            uint32_t nl;
            const uint32_t at = block_scan_excl<T>(pos ? 1u : 0u, misc + T_SCAN, &nl);
            if (pos) lb[at] = b;
            __syncthreads();
            const uint64_t items = (uint64_t)nl * A.gmax;
            for (uint64_t i0 = 0; i0 < items; i0 += T) {
                const uint64_t i = i0 + tid;
                bool rep_ok = false;
                uint32_t x = 0;
                if (i < items) {
                    const uint32_t ci = (uint32_t)(i / A.gmax);
                    const uint32_t cb = lb[ci], j = (uint32_t)(i - (uint64_t)ci * A.gmax);
                    const uint32_t sz = A.gsize[rep * B + cb];
                    if (j < sz) {
                        const uint64_t slot = (uint64_t)cb * A.mstride + j;
                        x = memr[slot];
                        const uint16_t *row = cmgr + slot * A.Rp;
                        rep_ok = true;
                        for (uint32_t r = 0; r < R; ++r)
                            rep_ok &= count_of(cnt32, r * Bp + row[r]) >= t;
                    }
                }
                uint32_t nnew;
                const uint32_t p = block_scan_excl<T>(rep_ok ? 1u : 0u, misc + T_SCAN, &nnew);
                const uint32_t base = misc[T_TOTAL];
                if (rep_ok && base + p < A.max_out) out[base + p] = x;
                __syncthreads();
                if (tid == 0) misc[T_TOTAL] = base + nnew;
                __syncthreads();
            }
        }
    }
    const uint32_t total = misc[T_TOTAL];
    for (uint32_t j = total + tid; j < A.max_out; j += T) out[j] = 0xFFFFFFFFu;
    if (tid == 0) A.counts[q] = total;
}

}  // namespace

size_t threshold_lds_bytes(const Index &ix, int T) {
    const uint32_t Bp = (ix.p.B + 3) & ~3u;
    const size_t cnt_words = ((size_t)ix.p.R * Bp / 4 + 3) & ~(size_t)3;
    return (cnt_words + T_NPOS + 16 + T) * 4;
}

void threshold_launch(const Index &ix, const uint32_t *codes_dev, uint64_t nq, uint32_t t,
                      uint32_t max_out, uint32_t *ids_dev, uint32_t *counts_dev, hipStream_t s) {
    if (nq == 0) return;
    if (nq > 0x7FFFFFFFull) fail(FLINNG_EINVAL, "query batch too large for one launch");
    TArgs a{};
    a.codes = codes_dev;
    a.nq = nq;
    a.offsets = ix.offsets;
    a.cells = ix.cells;
    a.mem = ix.mem;
    a.cmg = ix.cmg;
    a.L = ix.p.L;
    a.R = ix.p.R;
    a.Rp = ix.Rp;
    a.B = ix.p.B;
    a.Bp = (ix.p.B + 3) & ~3u;
    a.nbits = ix.nbits;
    a.t = t;
    a.max_out = max_out;
    a.gsize = ix.gsize;
    a.gmax = ix.gmax;
    a.mstride = ix.mstride;
    a.cnt_words = (uint32_t)((((size_t)a.R * a.Bp) / 4 + 3) & ~(size_t)3);
    a.ids = ids_dev;
    a.counts = counts_dev;
    int dev = 0;
    FL_HIP(hipGetDevice(&dev));
    int max_lds = 0;
    FL_HIP(hipDeviceGetAttribute(&max_lds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev));
    const bool big = threshold_lds_bytes(ix, 256) > 32 * 1024;
    const size_t lds = threshold_lds_bytes(ix, big ? 1024 : 256);
    if (lds > (size_t)max_lds)
        fail(FLINNG_EINVAL, "per-query counters (" + std::to_string(lds) +
                                " bytes) exceed the workgroup LDS limit; reduce B*R");
    auto go = [&](auto kern, int T) {
        FL_HIP(hipFuncSetAttribute(reinterpret_cast<const void *>(kern),
                                   hipFuncAttributeMaxDynamicSharedMemorySize, max_lds));
        hipLaunchKernelGGL(kern, dim3((unsigned)nq), dim3(T), lds, s, a);
        FL_CHECK_LAUNCH();
    };
    if (ix.cell_bytes == 2) {
        if (big) go(threshold_kernel<uint16_t, 1024>, 1024);
        else go(threshold_kernel<uint16_t, 256>, 256);
    } else {
        if (big) go(threshold_kernel<uint32_t, 1024>, 1024);
        else go(threshold_kernel<uint32_t, 256>, 256);
    }
}

}  // namespace flinng
