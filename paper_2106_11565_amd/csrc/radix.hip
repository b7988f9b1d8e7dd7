// Device-wide exclusive scan and stable LSD radix sort (8-bit digits) used by
// the one-pass index build: grouping points by cell and bucketing
// (bucket, cell) pairs into the reverse index.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "flinng_internal.h"

namespace flinng {

constexpr int SCAN_THREADS = 256;
constexpr int SCAN_ITEMS = 8;
constexpr int SCAN_TILE = SCAN_THREADS * SCAN_ITEMS;

// Exclusive scan of a workgroup's per-thread totals; returns this thread's
// exclusive prefix, and the workgroup total in *total.
__device__ inline uint32_t block_exclusive_scan(uint32_t v, uint32_t *lds, uint32_t *total) {
    const int lane = threadIdx.x % 64, wave = threadIdx.x / 64;
    uint32_t inc = v;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        uint32_t y = __shfl_up(inc, o, 64);
        if (lane >= o) inc += y;
    }
    if (lane == 63) lds[wave] = inc;
    __syncthreads();
    uint32_t wpre = 0, tot = 0;
    for (int w = 0; w < (int)(blockDim.x / 64); ++w) {
        uint32_t c = lds[w];
        if (w < wave) wpre += c;
        tot += c;
    }
    __syncthreads();
    *total = tot;
    return wpre + inc - v;
}

__global__ __launch_bounds__(SCAN_THREADS) void scan_reduce_kernel(const uint32_t *__restrict__ in,
                                                                   uint64_t n,
                                                                   uint32_t *__restrict__ sums) {
    __shared__ uint32_t lds[SCAN_THREADS / 64];
    const uint64_t base = (uint64_t)blockIdx.x * SCAN_TILE + threadIdx.x * SCAN_ITEMS;
    uint32_t s = 0;
#pragma unroll
    for (int i = 0; i < SCAN_ITEMS; ++i)
        if (base + i < n) s += in[base + i];
    uint32_t tot;
    block_exclusive_scan(s, lds, &tot);
    if (threadIdx.x == 0) sums[blockIdx.x] = tot;
}

__global__ __launch_bounds__(SCAN_THREADS) void scan_apply_kernel(const uint32_t *__restrict__ in,
                                                                  uint64_t n,
                                                                  const uint32_t *__restrict__ offs,
                                                                  uint32_t *__restrict__ out) {
    __shared__ uint32_t lds[SCAN_THREADS / 64];
    const uint64_t base = (uint64_t)blockIdx.x * SCAN_TILE + threadIdx.x * SCAN_ITEMS;
    uint32_t v[SCAN_ITEMS];
    uint32_t s = 0;
#pragma unroll
    for (int i = 0; i < SCAN_ITEMS; ++i) {
        v[i] = (base + i < n) ? in[base + i] : 0u;
        s += v[i];
    }
    uint32_t tot;
    uint32_t pre = block_exclusive_scan(s, lds, &tot) + (offs ? offs[blockIdx.x] : 0u);
#pragma unroll
    for (int i = 0; i < SCAN_ITEMS; ++i) {
        if (base + i < n) out[base + i] = pre;
        pre += v[i];
    }
}

void device_exclusive_scan_u32(const uint32_t *in, uint32_t *out, uint64_t n, hipStream_t s) {
    if (n == 0) return;
    const uint64_t nb = (n + SCAN_TILE - 1) / SCAN_TILE;
    if (nb == 1) {
        hipLaunchKernelGGL(scan_apply_kernel, dim3(1), dim3(SCAN_THREADS), 0, s, in, n,
                           (const uint32_t *)nullptr, out);
        FL_CHECK_LAUNCH();
        return;
    }
    DevBuf sums(nb * 4, s), soffs(nb * 4, s);
    hipLaunchKernelGGL(scan_reduce_kernel, dim3((unsigned)nb), dim3(SCAN_THREADS), 0, s, in, n,
                       sums.as<uint32_t>());
    FL_CHECK_LAUNCH();
    device_exclusive_scan_u32(sums.as<uint32_t>(), soffs.as<uint32_t>(), nb, s);
    hipLaunchKernelGGL(scan_apply_kernel, dim3((unsigned)nb), dim3(SCAN_THREADS), 0, s, in, n,
                       soffs.as<uint32_t>(), out);
    FL_CHECK_LAUNCH();
}

// ---------------------------------------------------------------------------
constexpr int RS_THREADS = 256;
constexpr int RS_ITEMS = 16;
constexpr int RS_TILE = RS_THREADS * RS_ITEMS;

// Digit histogram of one tile; hist is digit-major: hist[digit * nb + block].
__global__ __launch_bounds__(RS_THREADS) void rs_hist_kernel(const uint64_t *__restrict__ keys,
                                                             uint64_t n, int shift, uint64_t nb,
                                                             uint32_t *__restrict__ hist) {
    __shared__ uint32_t h[256];
    h[threadIdx.x] = 0;
    __syncthreads();
    const uint64_t base = (uint64_t)blockIdx.x * RS_TILE;
#pragma unroll 4
    for (int i = 0; i < RS_ITEMS; ++i) {
        uint64_t p = base + (uint64_t)i * RS_THREADS + threadIdx.x;
        if (p < n) atomicAdd(&h[(keys[p] >> shift) & 255u], 1u);
    }
    __syncthreads();
    hist[(uint64_t)threadIdx.x * nb + blockIdx.x] = h[threadIdx.x];
}

// Stable scatter: rounds of 256 keys in input order; within a round each
// key's rank among equal digits comes from the wavefront's digit-match mask
// (8 ballots) and per-wave digit counts combined in LDS.  The ranks place the
// tile's keys in LDS ordered by digit (the tile's digit counts from hist give
// each digit's start there); the tile is then written out in that order, so
// consecutive threads store consecutive addresses of a digit's run.
template <bool VALS>
__global__ __launch_bounds__(RS_THREADS) void rs_scatter_kernel(
    const uint64_t *__restrict__ keys, const uint32_t *__restrict__ vals, uint64_t n, int shift,
    uint64_t nb, const uint32_t *__restrict__ hist, const uint32_t *__restrict__ goff,
    uint64_t *__restrict__ okeys, uint32_t *__restrict__ ovals) {
    __shared__ uint32_t wcnt[RS_THREADS / 64][256];
    __shared__ uint32_t woff[RS_THREADS / 64][256];
    __shared__ uint32_t run[256];    // next local position per digit
    __shared__ uint32_t gdel[256];   // global start minus local start, per digit
    __shared__ uint32_t sl[RS_THREADS / 64];
    __shared__ uint64_t tk[RS_TILE];
    __shared__ uint32_t tv[VALS ? RS_TILE : 1];
    const int t = threadIdx.x, lane = t % 64, wave = t / 64;
    uint32_t tot;
    const uint32_t ls = block_exclusive_scan(hist[(uint64_t)t * nb + blockIdx.x], sl, &tot);
    run[t] = ls;
    gdel[t] = goff[(uint64_t)t * nb + blockIdx.x] - ls;
#pragma unroll
    for (int w = 0; w < RS_THREADS / 64; ++w) wcnt[w][t] = 0;
    __syncthreads();
    const uint64_t base = (uint64_t)blockIdx.x * RS_TILE;
    const unsigned long long lt = (lane == 0) ? 0ull : ((~0ull) >> (64 - lane));
    for (int i = 0; i < RS_ITEMS; ++i) {
        const uint64_t p = base + (uint64_t)i * RS_THREADS + t;
        const bool valid = p < n;
        uint64_t key = valid ? keys[p] : 0ull;
        uint32_t val = (VALS && valid) ? vals[p] : 0u;
        const uint32_t dgt = (uint32_t)((key >> shift) & 255u);
        unsigned long long peers = __ballot(valid);
#pragma unroll
        for (int b = 0; b < 8; ++b) {
            const bool bit = (dgt >> b) & 1u;
            const unsigned long long m = __ballot(bit);
            peers &= bit ? m : ~m;
        }
        const uint32_t rank = (uint32_t)__popcll(peers & lt);
        if (valid && rank == 0) wcnt[wave][dgt] = (uint32_t)__popcll(peers);
        __syncthreads();
        {
            uint32_t r = run[t];
#pragma unroll
            for (int w = 0; w < RS_THREADS / 64; ++w) {
                woff[w][t] = r;
                r += wcnt[w][t];
                wcnt[w][t] = 0;
            }
            run[t] = r;
        }
        __syncthreads();
        if (valid) {
            const uint32_t lp = woff[wave][dgt] + rank;  // < the tile's key count
            tk[lp] = key;
            if (VALS) tv[lp] = val;
        }
    }
    __syncthreads();
    const uint64_t m = n - base < (uint64_t)RS_TILE ? n - base : (uint64_t)RS_TILE;
    for (uint32_t j = t; j < m; j += RS_THREADS) {
        const uint64_t key = tk[j];
        const uint32_t gp = gdel[(uint32_t)((key >> shift) & 255u)] + j;
        okeys[gp] = key;
        if (VALS) ovals[gp] = tv[j];
    }
}

void radix_sort_u64(uint64_t *keys, uint64_t *keys_tmp, uint32_t *vals, uint32_t *vals_tmp,
                    uint64_t n, int end_bit, hipStream_t s, uint64_t **sorted) {
    if (sorted && vals) fail(FLINNG_EDEVICE, "internal: radix sort result left in place with values");
    if (sorted) *sorted = keys;
    if (n <= 1 || end_bit <= 0) return;
    const uint64_t nb = (n + RS_TILE - 1) / RS_TILE;
    DevBuf hist(256 * nb * 4, s), goff(256 * nb * 4, s);
    uint64_t *kin = keys, *kout = keys_tmp;
    uint32_t *vin = vals, *vout = vals_tmp;
    int passes = 0;
    for (int shift = 0; shift < end_bit; shift += 8, ++passes) {
        hipLaunchKernelGGL(rs_hist_kernel, dim3((unsigned)nb), dim3(RS_THREADS), 0, s, kin, n,
                           shift, nb, hist.as<uint32_t>());
        FL_CHECK_LAUNCH();
        device_exclusive_scan_u32(hist.as<uint32_t>(), goff.as<uint32_t>(), 256 * nb, s);
        if (vals)
            hipLaunchKernelGGL(rs_scatter_kernel<true>, dim3((unsigned)nb), dim3(RS_THREADS), 0, s,
                               kin, vin, n, shift, nb, hist.as<uint32_t>(), goff.as<uint32_t>(),
                               kout, vout);
        else
            hipLaunchKernelGGL(rs_scatter_kernel<false>, dim3((unsigned)nb), dim3(RS_THREADS), 0,
                               s, kin, (const uint32_t *)nullptr, n, shift, nb,
                               hist.as<uint32_t>(), goff.as<uint32_t>(), kout, (uint32_t *)nullptr);
        FL_CHECK_LAUNCH();
        std::swap(kin, kout);
        std::swap(vin, vout);
    }
    if (sorted) {
        *sorted = kin;  // no copy back
        return;
    }
    if (passes % 2 == 1) {
        FL_HIP(hipMemcpyAsync(keys, kin, n * 8, hipMemcpyDeviceToDevice, s));
        if (vals) FL_HIP(hipMemcpyAsync(vals, vin, n * 4, hipMemcpyDeviceToDevice, s));
    }
}

}  // namespace flinng
