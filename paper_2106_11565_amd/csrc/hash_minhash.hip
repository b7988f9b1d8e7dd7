// MinHash hashing of item sets on gfx950.
//
// The set-similarity LSH instance (the paper hashes genome n-gram sets with
// MinHash, Section 7, Experiments, "Datasets"; the concatenation trick of Section 3 joins K
// minima per table):
//   a[t][j]  = sm64(key_MH, t*K + j)
//   pi_tj(e) = top 32 bits of splitmix_finalize(e XOR a[t][j])
//   mh_tj(S) = min over e in S of pi_tj(e)        (empty set: 0xFFFFFFFF)
//   h = sm64(key_MH, L*K + t); for j < K: h = splitmix_finalize(h XOR mh_tj)
//   bucket_t = h >> (64 - bucket_bits)
//
// Mapping: one wavefront per set.  The 64 lanes are F = floor(64/S) hash
// functions times S item slices; lane (f, s) takes the minimum over items s,
// s+S, ... of its function, then the S partial minima of each function are
// combined by LDS atomic minima.  S (any count up to 16) is chosen per batch
// from the mean set size so that the lanes stay busy.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <vector>

#include "flinng_internal.h"

namespace flinng {

template <typename ItemT>
__global__ __launch_bounds__(256) void minhash_kernel(
    const ItemT *__restrict__ items, const uint64_t *__restrict__ offsets, uint64_t nsets,
    uint32_t K, uint32_t L, uint32_t bbits, uint64_t key, uint32_t S, uint32_t *__restrict__ codes) {
    extern __shared__ uint32_t mins_all[];
    const int lane = threadIdx.x % 64;
    const int wave = threadIdx.x / 64;
    const uint64_t set = (uint64_t)blockIdx.x * (blockDim.x / 64) + wave;
    if (set >= nsets) return;
    const uint32_t LK = L * K;
    uint32_t *mins = mins_all + wave * LK;
    for (uint32_t f = lane; f < LK; f += 64) mins[f] = 0xFFFFFFFFu;
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    const uint64_t beg = offsets[set], end = offsets[set + 1];
    const uint32_t F = 64 / S;
    const uint32_t fl = (uint32_t)lane / S, sl = (uint32_t)lane % S;
    for (uint32_t f0 = 0; f0 < LK; f0 += F) {
        const uint32_t fi = f0 + fl;
        if (fl < F && fi < LK) {
            const uint64_t a = sm64(key, fi);
            uint32_t mn = 0xFFFFFFFFu;
            for (uint64_t p = beg + sl; p < end; p += S) {
                const uint64_t e = (uint64_t)items[p];
                const uint32_t v = (uint32_t)(splitmix_finalize(e ^ a) >> 32);
                mn = v < mn ? v : mn;
            }
            atomicMin(&mins[fi], mn);
        }
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    for (uint32_t t = lane; t < L; t += 64) {
        uint64_t h = sm64(key, (uint64_t)LK + t);
        for (uint32_t j = 0; j < K; ++j) h = splitmix_finalize(h ^ (uint64_t)mins[t * K + j]);
        codes[set * L + t] = (uint32_t)(h >> (64 - bbits));
    }
}

// Slices per function minimising (passes over functions) x (items per lane)
// for the batch's mean set size, plus one atomic minimum per lane and pass.
static int choose_slices(uint32_t LK, double mean_items) {
    int best = 1;
    double best_cost = 1e300;
    for (int S = 1; S <= 16; ++S) {
        const double F = (double)(64 / S);
        const double passes = std::ceil((double)LK / F);
        const double cost = passes * (std::ceil(mean_items / S) + 1.0);
        if (cost < best_cost - 1e-9) {
            best_cost = cost;
            best = S;
        }
    }
    return best;
}

template <typename ItemT>
static void launch_minhash(int S, const ItemT *items, const uint64_t *offs, uint64_t n,
                           uint32_t K, uint32_t L, uint32_t b, uint64_t key, uint32_t *codes,
                           hipStream_t s) {
    // one wavefront per set, up to four per workgroup: as many as keep the
    // per-wavefront minima (L*K words each) within 64 KiB of LDS, so every
    // valid (K, L) launches (L*K <= 255*32 needs 32 KiB for one wavefront)
    const size_t per_wave = (size_t)L * K * sizeof(uint32_t);
    unsigned waves = 4;
    while (waves > 1 && waves * per_wave > 65536) waves >>= 1;
    dim3 grid((unsigned)((n + waves - 1) / waves)), block(64 * waves);
    size_t lds = waves * per_wave;
    hipLaunchKernelGGL((minhash_kernel<ItemT>), grid, block, lds, s, items, offs, n, K, L, b, key,
                       (uint32_t)S, codes);
    FL_CHECK_LAUNCH();
}

void minhash_hash(const Index &ix, const flinng_input &in, uint32_t *codes_dev, hipStream_t s,
                  double mean_hint) {
    const uint64_t n = in.count;
    if (n == 0) return;
    const bool u64 = ix.p.family == FLINNG_MINHASH_U64;
    const size_t isz = u64 ? 8 : 4;
    const void *items = in.values;
    const uint64_t *offs = in.offsets;
    DevBuf ibuf, obuf;
    uint64_t first = 0, last = 0;
    if (!in.on_device) {
        first = in.offsets[0];
        last = in.offsets[n];
        if (last < first) fail(FLINNG_EINVAL, "offsets must be nondecreasing");
        // copy offsets rebased to 0 and the item range they cover
        std::vector<uint64_t> ro(n + 1);
        for (uint64_t i = 0; i <= n; ++i) {
            if (i && in.offsets[i] < in.offsets[i - 1])
                fail(FLINNG_EINVAL, "offsets must be nondecreasing");
            ro[i] = in.offsets[i] - first;
        }
        obuf = DevBuf((n + 1) * 8, s);
        FL_HIP(hipMemcpyAsync(obuf.ptr, ro.data(), (n + 1) * 8, hipMemcpyHostToDevice, s));
        const uint64_t nit = last - first;
        ibuf = DevBuf(std::max<uint64_t>(nit, 1) * isz, s);
        if (nit)
            FL_HIP(hipMemcpyAsync(ibuf.ptr, static_cast<const char *>(in.values) + first * isz,
                                  nit * isz, hipMemcpyHostToDevice, s));
        // the host copy must finish before the vector goes out of scope
        FL_HIP(hipStreamSynchronize(s));
        items = ibuf.ptr;
        offs = obuf.as<uint64_t>();
    }
    // device inputs are not read back (no host synchronisation): the slice
    // count then comes from the caller's hint, else a 64-item default
    const double mean = !in.on_device ? (double)(last - first) / (double)n
                                      : (mean_hint > 0 ? mean_hint : 64.0);
    const int S = choose_slices(ix.p.L * ix.p.K, mean);
    const uint64_t key = sm64(ix.p.seed, TAG_MINHASH);
    if (u64)
        launch_minhash<uint64_t>(S, static_cast<const uint64_t *>(items), offs, n, ix.p.K,
                                 ix.p.L, ix.nbits, key, codes_dev, s);
    else
        launch_minhash<uint32_t>(S, static_cast<const uint32_t *>(items), offs, n, ix.p.K,
                                 ix.p.L, ix.nbits, key, codes_dev, s);
}

void hash_batch(const Index &ix, const flinng_input &in, uint32_t *codes_dev, hipStream_t s,
                uint64_t *counters_host, double mean_hint, Arena *ws) {
    if (is_dense(ix.p.family))
        srp_hash(ix, in, codes_dev, s, counters_host, ws);
    else
        minhash_hash(ix, in, codes_dev, s, mean_hint);
}

}  // namespace flinng
