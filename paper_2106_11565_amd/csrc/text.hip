// N-gram item sets of symbol sequences, extracted on the device: the step
// before MinHash (the paper hashes genome reads and URLs as sets of n-grams,
// Section 7, Experiments, "Datasets").
//
// Sequence s (symbols s_0 .. s_{len-1}, each below the radix) is the set of
// its windows p = 0 .. len - n: the window's value is the base-radix number
// v = sum_i s_{p+i} radix^(n-1-i), and its item is MurmurHash3's 64-bit
// finaliser of v XOR key (64-bit items) or its 32-bit finaliser of the low
// 32 bits of v XOR key (32-bit items) (Appleby, MurmurHash3, public domain).
// A sequence shorter than n has no items (its MinHash is that of the empty
// set).  Duplicate windows give duplicate items, which MinHash ignores.
//
// Layout: item offsets are the exclusive sum of the window counts (one
// workgroup walks the sequences in 1024-sequence rounds with a carry, so no
// scratch or host round trip is needed), then one wavefront per sequence
// writes its items, lanes over windows.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <vector>

#include "flinng_internal.h"

namespace flinng {

__host__ __device__ inline uint64_t murmur_fmix64(uint64_t k) {
    k ^= k >> 33;
    k *= 0xFF51AFD7ED558CCDull;
    k ^= k >> 33;
    k *= 0xC4CEB9FE1A85EC53ull;
    k ^= k >> 33;
    return k;
}

__host__ __device__ inline uint32_t murmur_fmix32(uint32_t h) {
    h ^= h >> 16;
    h *= 0x85EBCA6Bu;
    h ^= h >> 13;
    h *= 0xC2B2AE35u;
    h ^= h >> 16;
    return h;
}

namespace {

constexpr int TO_T = 1024;

__global__ __launch_bounds__(TO_T) void text_offsets_kernel(const uint64_t *__restrict__ soff,
                                                            uint64_t count, uint32_t gram,
                                                            uint64_t *__restrict__ ioff) {
    __shared__ uint64_t wsum[TO_T / 64];
    __shared__ uint64_t carry;
    const int tid = threadIdx.x, lane = tid % 64, wave = tid / 64;
    if (tid == 0) carry = 0;
    __syncthreads();
    for (uint64_t b0 = 0; b0 < count; b0 += TO_T) {
        const uint64_t i = b0 + tid;
        uint64_t w = 0;
        if (i < count) {
            const uint64_t len = soff[i + 1] - soff[i];
            w = len >= gram ? len - gram + 1 : 0;
        }
        uint64_t inc = w;
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
            const uint64_t y = __shfl_up(inc, o, 64);
            if (lane >= o) inc += y;
        }
        if (lane == 63) wsum[wave] = inc;
        __syncthreads();
        uint64_t pre = carry;
        for (int v = 0; v < wave; ++v) pre += wsum[v];
        if (i < count) ioff[i] = pre + inc - w;
        __syncthreads();
        if (tid == TO_T - 1) carry = pre + inc;
        __syncthreads();
    }
    if (tid == 0) ioff[count] = carry;
}

template <typename ItemT>
__global__ __launch_bounds__(256) void text_items_kernel(const uint8_t *__restrict__ sym,
                                                         const uint64_t *__restrict__ soff,
                                                         const uint64_t *__restrict__ ioff,
                                                         uint64_t count, uint32_t gram,
                                                         uint32_t radix, uint64_t key,
                                                         ItemT *__restrict__ items) {
    const int lane = threadIdx.x % 64;
    const uint64_t s = (uint64_t)blockIdx.x * (blockDim.x / 64) + threadIdx.x / 64;
    if (s >= count) return;
    const uint64_t beg = soff[s];
    const uint64_t nw = ioff[s + 1] - ioff[s];
    ItemT *out = items + ioff[s];
    for (uint64_t p = lane; p < nw; p += 64) {
        uint64_t v = 0;
        for (uint32_t i = 0; i < gram; ++i) v = v * radix + sym[beg + p + i];
        if constexpr (sizeof(ItemT) == 8)
            out[p] = murmur_fmix64(v ^ key);
        else
            out[p] = murmur_fmix32((uint32_t)v ^ (uint32_t)key);
    }
}

}  // namespace

void validate_text(const flinng_text *t, uint32_t family) {
    if (!t) fail(FLINNG_EINVAL, "text input is NULL");
    if (t->reserved != 0) fail(FLINNG_EINVAL, "text.reserved must be 0");
    if (t->on_device > 1) fail(FLINNG_EINVAL, "text.on_device must be 0 or 1");
    if (family != FLINNG_MINHASH_U32 && family != FLINNG_MINHASH_U64)
        fail(FLINNG_EINVAL, "n-gram text feeds a MinHash index");
    if (t->radix < 2 || t->radix > 256) fail(FLINNG_EINVAL, "text.radix must be in 2..256");
    if (t->gram < 1) fail(FLINNG_EINVAL, "text.gram must be >= 1");
    // radix^gram <= 2^64: the window value fits 64 bits
    long double cap = 1.0L;
    for (uint32_t i = 0; i < t->gram; ++i) {
        cap *= t->radix;
        if (cap > 18446744073709551616.0L) fail(FLINNG_EINVAL, "text.radix^gram exceeds 2^64");
    }
    if (t->count && !t->offsets) fail(FLINNG_EINVAL, "text.offsets is NULL");
}

uint64_t text_symbols(const flinng_text &t) {
    if (t.count == 0) return 0;
    uint64_t first = 0, last = 0;
    if (t.on_device) {
        FL_HIP(hipMemcpy(&first, t.offsets, 8, hipMemcpyDeviceToHost));
        FL_HIP(hipMemcpy(&last, t.offsets + t.count, 8, hipMemcpyDeviceToHost));
    } else {
        first = t.offsets[0];
        last = t.offsets[t.count];
    }
    if (last < first) fail(FLINNG_EINVAL, "text offsets must be nondecreasing");
    return last - first;
}

void text_to_items(const flinng_text &t, uint32_t family, uint64_t nsym, hipStream_t s,
                   Scratch &sc, flinng_input *out) {
    const uint64_t n = t.count;
    const size_t isz = family == FLINNG_MINHASH_U64 ? 8 : 4;
    const uint8_t *sym = t.symbols;
    const uint64_t *soff = t.offsets;
    if (!t.on_device) {
        // symbols of the sequences and their offsets rebased to them
        std::vector<uint64_t> ro(n + 1);
        for (uint64_t i = 0; i <= n; ++i) {
            if (i && t.offsets[i] < t.offsets[i - 1])
                fail(FLINNG_EINVAL, "text offsets must be nondecreasing");
            ro[i] = t.offsets[i] - t.offsets[0];
        }
        uint8_t *dsym = sc.get<uint8_t>(std::max<uint64_t>(nsym, 1));
        uint64_t *doff = sc.get<uint64_t>((n + 1) * 8);
        if (nsym) FL_HIP(hipMemcpyAsync(dsym, t.symbols + t.offsets[0], nsym, hipMemcpyHostToDevice, s));
        FL_HIP(hipMemcpyAsync(doff, ro.data(), (n + 1) * 8, hipMemcpyHostToDevice, s));
        FL_HIP(hipStreamSynchronize(s));  // ro is the copy's source
        sym = dsym;
        soff = doff;
    }
    // at most one item per symbol
    uint64_t *ioff = sc.get<uint64_t>((n + 1) * 8);
    void *items = sc.get<void>(std::max<uint64_t>(nsym, 1) * isz);
    hipLaunchKernelGGL(text_offsets_kernel, dim3(1), dim3(TO_T), 0, s, soff, n, t.gram, ioff);
    FL_CHECK_LAUNCH();
    if (n) {
        const dim3 grid((unsigned)((n + 3) / 4));
        if (isz == 8)
            hipLaunchKernelGGL(text_items_kernel<uint64_t>, grid, dim3(256), 0, s, sym, soff, ioff, n,
                               t.gram, t.radix, t.key, static_cast<uint64_t *>(items));
        else
            hipLaunchKernelGGL(text_items_kernel<uint32_t>, grid, dim3(256), 0, s, sym, soff, ioff, n,
                               t.gram, t.radix, t.key, static_cast<uint32_t *>(items));
        FL_CHECK_LAUNCH();
    }
    *out = flinng_input{};
    out->values = items;
    out->offsets = ioff;
    out->count = n;
    out->on_device = 1;
}

}  // namespace flinng
