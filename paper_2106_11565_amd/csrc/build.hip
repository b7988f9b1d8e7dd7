// One-pass index build on gfx950 (Algorithm 1 and the reverse index of
// Section 6, Implementation).
//
// Groups: repetition r permutes the points with a keyed bijection P_r of
// [0, N) and point x joins group P_r(x) mod B (Algorithm 1: a random
// permutation, then blocks by modulo), so group b holds exactly
// floor(N/B) + [b < N mod B] points.  P_r is a 4-round balanced Feistel
// network on [0, 2^nb) (nb the smallest even width >= 2 covering N) with
// round function F_i(v) = splitmix_finalize(v XOR k_{r,i}) mod 2^(nb/2) and
// keys k_{r,i} = sm64(sm64(seed, GROUP), 4r + i), restricted to [0, N) by
// cycle walking (Black and Rogaway 2002).
//
// Reverse index: for each table t the pairs (bucket_t(x), cell of x in rep
// r) over all points and repetitions are radix-sorted, duplicates dropped (a
// filter bit is set once), and bucket offsets built by a count + scan.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "flinng_internal.h"

namespace flinng {

__device__ inline uint64_t feistel(uint64_t v, uint32_t half, const uint64_t *keys) {
    const uint64_t mask = (1ull << half) - 1ull;
    uint64_t hi = v >> half, lo = v & mask;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const uint64_t f = splitmix_finalize(lo ^ keys[i]) & mask;
        const uint64_t nlo = hi ^ f;
        hi = lo;
        lo = nlo;
    }
    return (hi << half) | lo;
}

struct GroupKeys {
    uint64_t k[16][4];
};

// grp[x*Rp + r] = P_r(x) mod B; the padding repetitions R..Rp-1 repeat
// repetition R-1's group, so a reader may take the minimum over all Rp
// entries (a repeated cell changes neither the minimum nor its cell).
__global__ void groups_kernel(uint64_t N, uint32_t R, uint32_t Rp, uint32_t B, uint32_t half,
                              GroupKeys gk, uint16_t *__restrict__ grp) {
    const uint64_t x = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (x >= N) return;
    for (uint32_t r = 0; r < R; ++r) {
        uint64_t y = feistel(x, half, gk.k[r]);
        while (y >= N) y = feistel(y, half, gk.k[r]);
        grp[x * Rp + r] = (uint16_t)(y % B);
    }
    for (uint32_t r = R; r < Rp; ++r) grp[x * Rp + r] = grp[x * Rp + R - 1];
}

__global__ void member_keys_kernel(const uint16_t *__restrict__ grp, uint64_t N, uint32_t Rp,
                                   uint32_t r, uint64_t *__restrict__ keys,
                                   uint32_t *__restrict__ vals) {
    const uint64_t x = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (x >= N) return;
    keys[x] = grp[x * Rp + r];
    vals[x] = (uint32_t)x;
}

// sorted position p of group b = keys[p] sits at run offset
// p - (b*floor(N/B) + min(b, N mod B)); copy it to slot b*mstride + that.
__global__ void member_slots_kernel(const uint64_t *__restrict__ keys, const uint32_t *__restrict__ ids,
                                    uint64_t N, uint32_t B, uint32_t mstride,
                                    uint32_t *__restrict__ mem) {
    const uint64_t p = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= N) return;
    const uint64_t b = keys[p];
    const uint64_t q0 = N / B, rem = N % B;
    const uint64_t run = b * q0 + (b < rem ? b : rem);
    mem[b * mstride + (p - run)] = ids[p];
}

// cmg[slot][r] = group in repetition r of the member stored in mem[slot]
// (zeros for the padding slots).
__global__ void cell_groups_kernel(const uint32_t *__restrict__ mem, const uint16_t *__restrict__ grp,
                                   uint64_t nslots, uint32_t Rp, uint16_t *__restrict__ cmg) {
    const uint64_t sl = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (sl >= nslots) return;
    const uint32_t x = mem[sl];
    for (uint32_t r = 0; r < Rp; ++r)
        cmg[sl * Rp + r] = (x == 0xFFFFFFFFu) ? (uint16_t)0 : grp[(uint64_t)x * Rp + r];
}

void build_groups(Index &ix, hipStream_t s) {
    const uint64_t N = ix.N;
    const uint32_t R = ix.p.R, B = ix.p.B;
    uint32_t nb = 2;
    while (nb < 64 && (1ull << nb) < N) nb += 2;
    GroupKeys gk{};
    const uint64_t key = sm64(ix.p.seed, TAG_GROUP);
    for (uint32_t r = 0; r < R; ++r)
        for (int i = 0; i < 4; ++i) gk.k[r][i] = sm64(key, (uint64_t)r * 4 + i);
    const unsigned grid = (unsigned)((N + 255) / 256);
    hipLaunchKernelGGL(groups_kernel, dim3(grid), dim3(256), 0, s, N, R, ix.Rp, B, nb / 2, gk,
                       ix.grp);
    FL_CHECK_LAUNCH();
    // members of each cell, ascending id: stable sort of ids by group, then
    // each group's run (at b*floor(N/B) + min(b, N mod B)) moves to its
    // 16-byte aligned slot b*mstride; unused slot tails hold 0xFFFFFFFF
    DevBuf k1(N * 8, s), k2(N * 8, s), v1(N * 4, s), v2(N * 4, s);
    int gbits = 1;
    while ((1u << gbits) < B) ++gbits;
    FL_HIP(hipMemsetAsync(ix.mem, 0xFF, (size_t)R * B * ix.mstride * 4, s));
    for (uint32_t r = 0; r < R; ++r) {
        hipLaunchKernelGGL(member_keys_kernel, dim3(grid), dim3(256), 0, s, ix.grp, N, ix.Rp, r,
                           k1.as<uint64_t>(), v1.as<uint32_t>());
        FL_CHECK_LAUNCH();
        radix_sort_u64(k1.as<uint64_t>(), k2.as<uint64_t>(), v1.as<uint32_t>(), v2.as<uint32_t>(),
                       N, gbits, s);
        hipLaunchKernelGGL(member_slots_kernel, dim3(grid), dim3(256), 0, s, k1.as<uint64_t>(),
                           v1.as<uint32_t>(), N, B, ix.mstride, ix.mem + (uint64_t)r * B * ix.mstride);
        FL_CHECK_LAUNCH();
    }
    const uint64_t nslots = (uint64_t)R * B * ix.mstride;
    hipLaunchKernelGGL(cell_groups_kernel, dim3((unsigned)((nslots + 255) / 256)), dim3(256), 0, s,
                       ix.mem, ix.grp, nslots, ix.Rp, ix.cmg);
    FL_CHECK_LAUNCH();
}

// ---------------------------------------------------------------------------
// keys[x*R + r] = bucket_t(x) << cb | (r*Bp + g_r(x))
__global__ void emit_pairs_kernel(const uint32_t *__restrict__ codes, const uint16_t *__restrict__ grp,
                                  uint64_t N, uint32_t L, uint32_t t, uint32_t R, uint32_t Rp,
                                  uint32_t Bp, int cb, uint64_t *__restrict__ keys) {
    const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N * R) return;
    const uint64_t x = i / R;
    const uint32_t r = (uint32_t)(i % R);
    const uint64_t h = codes[x * L + t];
    keys[i] = (h << cb) | (uint64_t)(r * Bp + grp[x * Rp + r]);
}

__global__ void unique_kernel(const uint64_t *__restrict__ keys, uint64_t n, int cb,
                              uint32_t *__restrict__ flag, uint32_t *__restrict__ bcnt) {
    const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const uint64_t k = keys[i];
    const uint32_t u = (i == 0 || keys[i - 1] != k) ? 1u : 0u;
    flag[i] = u;
    if (u) atomicAdd(&bcnt[k >> cb], 1u);
}

template <typename CellT>
__global__ void compact_kernel(const uint64_t *__restrict__ keys, const uint32_t *__restrict__ flag,
                               const uint32_t *__restrict__ pos, uint64_t n, uint64_t cmask,
                               CellT *__restrict__ out) {
    const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n || !flag[i]) return;
    out[pos[i]] = (CellT)(keys[i] & cmask);
}

__global__ void add_const_kernel(const uint32_t *__restrict__ in, uint64_t n, uint32_t c,
                                 uint32_t *__restrict__ out) {
    const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) out[i] = in[i] + c;
}

void build_lists(Index &ix, const uint32_t *codes, hipStream_t s) {
    const uint64_t N = ix.N;
    const uint32_t L = ix.p.L, R = ix.p.R;
    const uint32_t Bp = (ix.p.B + 3) & ~3u;
    int cb = 1;
    while ((1ull << cb) < (uint64_t)R * Bp) ++cb;
    const uint64_t NR = N * R;
    const uint64_t nbk = nbuckets(ix);
    const int end_bit = (int)ix.nbits + cb;
    const uint64_t cap = NR * L;  // upper bound on list entries
    const size_t csz = ix.cell_bytes;

    DevBuf keys(NR * 8, s), tmp(NR * 8, s), flag(NR * 4, s), pos(NR * 4, s);
    DevBuf bcnt((nbk + 1) * 4, s), boff((nbk + 1) * 4, s);
    void *big = nullptr;
    FL_HIP(hipMalloc(&big, std::max<uint64_t>(cap, 1) * csz));
    uint64_t base = 0;
    const unsigned g1 = (unsigned)((NR + 255) / 256);
    const unsigned gb = (unsigned)((nbk + 1 + 255) / 256);
    try {
        for (uint32_t t = 0; t < L; ++t) {
            hipLaunchKernelGGL(emit_pairs_kernel, dim3(g1), dim3(256), 0, s, codes, ix.grp, N, L, t,
                               R, ix.Rp, Bp, cb, keys.as<uint64_t>());
            FL_CHECK_LAUNCH();
            radix_sort_u64(keys.as<uint64_t>(), tmp.as<uint64_t>(), nullptr, nullptr, NR, end_bit, s);
            FL_HIP(hipMemsetAsync(bcnt.ptr, 0, (nbk + 1) * 4, s));
            hipLaunchKernelGGL(unique_kernel, dim3(g1), dim3(256), 0, s, keys.as<uint64_t>(), NR, cb,
                               flag.as<uint32_t>(), bcnt.as<uint32_t>());
            FL_CHECK_LAUNCH();
            device_exclusive_scan_u32(flag.as<uint32_t>(), pos.as<uint32_t>(), NR, s);
            uint32_t last[2];
            FL_HIP(hipMemcpyAsync(&last[0], pos.as<uint32_t>() + NR - 1, 4, hipMemcpyDeviceToHost, s));
            FL_HIP(hipMemcpyAsync(&last[1], flag.as<uint32_t>() + NR - 1, 4, hipMemcpyDeviceToHost, s));
            FL_HIP(hipStreamSynchronize(s));
            const uint64_t nt = (uint64_t)last[0] + last[1];
            const uint64_t cmask = (1ull << cb) - 1;
            if (csz == 2)
                hipLaunchKernelGGL(compact_kernel<uint16_t>, dim3(g1), dim3(256), 0, s,
                                   keys.as<uint64_t>(), flag.as<uint32_t>(), pos.as<uint32_t>(), NR,
                                   cmask, static_cast<uint16_t *>(big) + base);
            else
                hipLaunchKernelGGL(compact_kernel<uint32_t>, dim3(g1), dim3(256), 0, s,
                                   keys.as<uint64_t>(), flag.as<uint32_t>(), pos.as<uint32_t>(), NR,
                                   cmask, static_cast<uint32_t *>(big) + base);
            FL_CHECK_LAUNCH();
            // bucket offsets: exclusive scan of per-bucket counts (+ trailing 0)
            device_exclusive_scan_u32(bcnt.as<uint32_t>(), boff.as<uint32_t>(), nbk + 1, s);
            if (base + nt > 0xFFFFFFFFull) fail(FLINNG_EINVAL, "reverse index exceeds 2^32 entries");
            hipLaunchKernelGGL(add_const_kernel, dim3(gb), dim3(256), 0, s, boff.as<uint32_t>(),
                               nbk + 1, (uint32_t)base, ix.offsets + (uint64_t)t * (nbk + 1));
            FL_CHECK_LAUNCH();
            base += nt;
        }
        // shrink the list buffer to its size plus a zeroed tail, so that the
        // query kernel's 16-byte chunk reads past a list's end stay inside it
        void *exact = nullptr;
        const size_t used = (size_t)base * csz;
        FL_HIP(hipMalloc(&exact, cells_alloc_bytes(base, csz)));
        if (base) FL_HIP(hipMemcpyAsync(exact, big, used, hipMemcpyDeviceToDevice, s));
        FL_HIP(hipMemsetAsync(static_cast<char *>(exact) + used, 0,
                              cells_alloc_bytes(base, csz) - used, s));
        FL_HIP(hipStreamSynchronize(s));
        FL_HIP(hipFree(big));
        big = nullptr;
        ix.cells = exact;
        ix.list_entries = base;
    } catch (...) {
        if (big) (void)hipFree(big);
        throw;
    }
}

}  // namespace flinng
