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
// filter bit is set once), and each bucket's offset is written by the one
// sorted position where the bucket starts (no atomics, no count array).
//
// Points arriving after the build (ids N0, N0+1, ...): the arrivals are cut
// into blocks of B; within block j the point at position u joins group
// pi_{r,j}(u) of repetition r, pi_{r,j} a 4-round balanced Feistel network
// on [0, 2^nb) (nb the smallest even width >= 2 covering B) restricted to
// [0, B) by cycle walking, round keys sm64(sm64(seed, STREAM), 4(16j + r) + i).
// Every complete block adds one point to each group, so group sizes stay
// within two of each other.  An insert rebuilds each table's list from its
// old entries plus the new pairs, and appends the new members (ascending id
// is preserved: new ids exceed every old one) into copies of the member
// arrays, growing their per-cell stride when a cell outgrows it.
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

// keys[i] = group of point x0 + i in repetition r (rows from x0 on), vals[i] = its id
__global__ void member_keys_kernel(const uint16_t *__restrict__ grp, uint64_t x0, uint64_t N,
                                   uint32_t Rp, uint32_t r, uint64_t *__restrict__ keys,
                                   uint32_t *__restrict__ vals) {
    const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N) return;
    keys[i] = grp[(x0 + i) * Rp + r];
    vals[i] = (uint32_t)(x0 + i);
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

// cfl[r][b][j] = the groups, in repetitions r+1 and r+2 (mod R), of the
// member in slot j of cell (r, b): low and high 16 bits (zero for padding
// slots).  One launch per repetition r.
__global__ void filter_groups_kernel(const uint32_t *__restrict__ mem_r,
                                     const uint16_t *__restrict__ grp, uint64_t nslots, uint32_t Rp,
                                     uint32_t r1, uint32_t r2, uint32_t *__restrict__ cfl_r) {
    const uint64_t sl = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (sl >= nslots) return;
    const uint32_t x = mem_r[sl];
    cfl_r[sl] = (x == 0xFFFFFFFFu)
                    ? 0u
                    : (uint32_t)grp[(uint64_t)x * Rp + r1] | ((uint32_t)grp[(uint64_t)x * Rp + r2] << 16);
}

void build_filter(const Index &ix, const uint32_t *mem, const uint16_t *grp, uint32_t mstride,
                  uint32_t *cfl, hipStream_t s) {
    const uint32_t R = ix.p.R, B = ix.p.B;
    const uint64_t per = (uint64_t)B * mstride;
    for (uint32_t r = 0; r < R; ++r) {
        hipLaunchKernelGGL(filter_groups_kernel, dim3((unsigned)((per + 255) / 256)), dim3(256), 0, s,
                           mem + r * per, grp, per, ix.Rp, (r + 1) % R, (r + 2) % R, cfl + r * per);
        FL_CHECK_LAUNCH();
    }
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
        hipLaunchKernelGGL(member_keys_kernel, dim3(grid), dim3(256), 0, s, ix.grp, (uint64_t)0, N,
                           ix.Rp, r, k1.as<uint64_t>(), v1.as<uint32_t>());
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
    build_filter(ix, ix.mem, ix.grp, ix.mstride, ix.cfl, s);
    // cell sizes (Algorithm 1's balanced design), on the device and the host
    ix.gsize_host.assign((size_t)R * B, 0);
    for (uint32_t r = 0; r < R; ++r)
        for (uint32_t b = 0; b < B; ++b)
            ix.gsize_host[(size_t)r * B + b] = (uint32_t)(N / B + (b < N % B ? 1 : 0));
    ix.gmax = (uint32_t)((N + B - 1) / B);
    FL_HIP(hipMemcpyAsync(ix.gsize, ix.gsize_host.data(), (size_t)R * B * 4, hipMemcpyHostToDevice, s));
    FL_HIP(hipStreamSynchronize(s));  // the host vector is the copy's source
}

// ---------------------------------------------------------------------------
// keys[x*R + r] = bucket_t(x) << cb | (r*Bp + g_r(x)) for the n points whose
// codes and group rows are given
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

// The n entries of one table's existing list (positions e0 .. e0+n-1 of the
// cells array) as sorted keys again: the bucket of an entry is the last one
// whose offset does not exceed its position.
template <typename CellT>
__global__ void expand_list_kernel(const uint32_t *__restrict__ off, uint64_t nbk,
                                   const CellT *__restrict__ cells, uint64_t e0, uint64_t n, int cb,
                                   uint64_t *__restrict__ keys) {
    const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const uint64_t pos = e0 + i;
    uint64_t lo = 0, hi = nbk;  // off[lo] <= pos < off[hi]
    while (hi - lo > 1) {
        const uint64_t mid = (lo + hi) >> 1;
        if (off[mid] <= pos) lo = mid; else hi = mid;
    }
    keys[i] = (lo << cb) | (uint64_t)cells[pos];
}

// flag[i] = 1 for the first of each run of equal sorted keys
__global__ void unique_kernel(const uint64_t *__restrict__ keys, uint64_t n,
                              uint32_t *__restrict__ flag) {
    const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    flag[i] = (i == 0 || keys[i - 1] != keys[i]) ? 1u : 0u;
}

template <typename CellT>
__global__ void compact_kernel(const uint64_t *__restrict__ keys, const uint32_t *__restrict__ flag,
                               const uint32_t *__restrict__ pos, uint64_t n, uint64_t cmask,
                               const uint64_t *__restrict__ tbase, CellT *__restrict__ out) {
    const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n || !flag[i]) return;
    out[*tbase + pos[i]] = (CellT)(keys[i] & cmask);
}

// The running start of the tables' lists on the device: tb[t + 1] = tb[t] +
// the unique entries of table t (pos and flag of its last key), so that the
// tables' kernels queue without a host round trip per table.
__global__ void list_total_kernel(const uint32_t *__restrict__ pos,
                                  const uint32_t *__restrict__ flag, uint64_t n,
                                  uint64_t *__restrict__ tb, uint32_t t) {
    if (threadIdx.x == 0 && blockIdx.x == 0)
        tb[t + 1] = tb[t] + (n ? (uint64_t)pos[n - 1] + flag[n - 1] : 0ull);
}

// Bucket offsets without atomics, as a merge of two sorted sequences: the
// bucket numbers 0 .. nbk and the buckets of the n sorted keys, where bucket b
// goes before the keys of buckets >= b.  The offset of bucket b is base plus
// the unique entries among the keys before it.  Each thread takes OB_ITEMS
// consecutive items of the merged order: a binary search on its diagonal finds
// how many keys precede its first item, then it walks its items, consuming a
// key or writing one offset per step.  The work per thread is bounded however
// the keys crowd into few buckets (SRP codes of clustered data leave gaps of
// millions of empty buckets); each offset is written exactly once.  32 items
// per thread: a few thousand workgroups for a table of millions of keys.  A
// workgroup's offsets form one contiguous run of at most OB_BLOCK buckets, so
// they are gathered in LDS and written out with whole-line stores.
constexpr uint32_t OB_ITEMS = 32;
constexpr uint64_t OB_BLOCK = 256ull * OB_ITEMS;  // merged items per workgroup
constexpr uint32_t OB_LDS = OB_BLOCK + OB_BLOCK / 32;  // one pad word per 32
__device__ inline uint32_t ob_pad(uint64_t j) { return (uint32_t)(j + (j >> 5)); }

// Where the merge path crosses diagonal d: the first key index i in [lo, hi)
// that does not go before bucket d-1-i.
__device__ inline uint64_t ob_cross(const uint64_t *__restrict__ keys, int cb, uint64_t d,
                                    uint64_t lo, uint64_t hi) {
    while (lo < hi) {
        const uint64_t m = (lo + hi) / 2;
        if ((keys[m] >> cb) + 1 + m < d) lo = m + 1;  // bucket(keys[m]) < d-1-m
        else hi = m;
    }
    return lo;
}

// The crossings of the workgroups' first diagonals (one thread each): the
// crossing only grows along the path, so a thread of bucket_offsets_kernel
// then searches its workgroup's stretch of at most OB_BLOCK keys, mostly in
// cache, instead of the whole table.
__global__ void bucket_blocks_kernel(const uint64_t *__restrict__ keys, uint64_t n, int cb,
                                     uint64_t nbk, uint64_t nblk, uint64_t *__restrict__ blo) {
    const uint64_t b = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (b > nblk) return;
    const uint64_t total = nbk + 1 + n;
    const uint64_t d = b * OB_BLOCK < total ? b * OB_BLOCK : total;
    blo[b] = ob_cross(keys, cb, d, d > nbk + 1 ? d - (nbk + 1) : 0, d < n ? d : n);
}

__global__ __launch_bounds__(256) void bucket_offsets_kernel(const uint64_t *__restrict__ keys,
                                                             const uint32_t *__restrict__ pos,
                                                             const uint32_t *__restrict__ flag,
                                                             uint64_t n, int cb, uint64_t nbk,
                                                             const uint64_t *__restrict__ blo,
                                                             const uint64_t *__restrict__ tbase,
                                                             uint32_t *__restrict__ off) {
    __shared__ uint32_t run[OB_LDS];
    const uint64_t total = nbk + 1 + n;
    const uint32_t base = (uint32_t)*tbase;  // an overflow past 2^32 fails the build
    // the workgroup's diagonals [d0, d1) emit the buckets [b0, b1)
    const uint64_t d0 = (uint64_t)blockIdx.x * OB_BLOCK;
    const uint64_t d1 = d0 + OB_BLOCK < total ? d0 + OB_BLOCK : total;
    const uint64_t c0 = blo[blockIdx.x], c1 = blo[blockIdx.x + 1];
    const uint64_t b0 = d0 - c0, b1 = d1 - c1;
    const uint64_t d = d0 + (uint64_t)threadIdx.x * OB_ITEMS;
    if (d < total) {
        // the crossing of d lies between those of the workgroup's diagonals
        uint64_t lo = d > nbk + 1 ? d - (nbk + 1) : 0, hi = d < n ? d : n;
        lo = lo > c0 ? lo : c0;
        hi = hi < c1 ? hi : c1;
        uint64_t i = ob_cross(keys, cb, d, lo, hi), b = d - i;
        const uint32_t last = n ? pos[n - 1] + flag[n - 1] : 0u;
        const uint64_t end = d + OB_ITEMS < total ? d + OB_ITEMS : total;
        uint64_t kb = i < n ? keys[i] >> cb : 0;  // bucket of key i
        uint32_t pv = 0;                          // pos of key i, once read
        bool have = false;
        for (uint64_t e = d; e < end; ++e) {
            if (i < n && (b > nbk || kb < b)) {
                ++i;
                if (i < n) kb = keys[i] >> cb;
                have = false;
            } else {
                if (!have) {
                    pv = i < n ? pos[i] : last;
                    have = true;
                }
                run[ob_pad(b - b0)] = base + pv;
                ++b;
            }
        }
    }
    __syncthreads();
    uint32_t *o = off + b0;
    for (uint64_t j = threadIdx.x; j < b1 - b0; j += blockDim.x) o[j] = run[ob_pad(j)];
}

namespace {

// The reverse index of all tables into fresh arrays: for table t the keys of
// its old list (when `old_cells` is given: entries tstart_old[t] ..
// tstart_old[t+1] of old_cells, offsets old_off) and the pairs of the n
// points whose codes and group rows are given, sorted, deduplicated and
// compacted.  Returns the new offsets [L][nbk+1] and cells (with the zeroed
// 16-byte tail the query kernel's chunk reads need) and fills tstart.
struct Lists {
    uint32_t *offsets = nullptr;
    void *cells = nullptr;
    uint64_t entries = 0;
    std::vector<uint64_t> tstart;
};

Lists assemble_lists(const Index &ix, const uint32_t *old_off, const void *old_cells,
                     const std::vector<uint64_t> &tstart_old, const uint32_t *codes,
                     const uint16_t *grp_rows, uint64_t n, hipStream_t s) {
    const uint32_t L = ix.p.L, R = ix.p.R;
    const uint32_t Bp = (ix.p.B + 3) & ~3u;
    int cb = 1;
    while ((1ull << cb) < (uint64_t)R * Bp) ++cb;
    const uint64_t nbk = nbuckets(ix);
    const int end_bit = (int)ix.nbits + cb;
    const size_t csz = ix.cell_bytes;
    const uint64_t nr = n * R;
    uint64_t most_old = 0, old_total = 0;
    if (old_cells)
        for (uint32_t t = 0; t < L; ++t) {
            most_old = std::max<uint64_t>(most_old, tstart_old[t + 1] - tstart_old[t]);
            old_total += tstart_old[t + 1] - tstart_old[t];
        }
    const uint64_t most = most_old + nr;           // keys of the largest table
    const uint64_t cap = old_total + nr * L;       // upper bound on the entries

    Lists out;
    out.tstart.assign(L + 1, 0);
    DevBuf keys(most * 8, s), tmp(most * 8, s), flag(most * 4, s), pos(most * 4, s);
    DevBuf tbd((L + 1) * 8, s);  // the tables' list starts
    uint64_t *tb = tbd.as<uint64_t>();
    const uint64_t nblk_most = (nbk + 1 + most + OB_BLOCK - 1) / OB_BLOCK;
    DevBuf blod((nblk_most + 1) * 8, s);  // merge-path crossings per workgroup
    void *big = nullptr;
    try {
        FL_HIP(hipMalloc(&out.offsets, (size_t)L * (nbk + 1) * 4));
        FL_HIP(hipMalloc(&big, std::max<uint64_t>(cap, 1) * csz));
        FL_HIP(hipMemsetAsync(tb, 0, 8, s));
        for (uint32_t t = 0; t < L; ++t) {
            const uint64_t nold = old_cells ? tstart_old[t + 1] - tstart_old[t] : 0;
            const uint64_t nk = nold + nr;
            uint64_t *k = keys.as<uint64_t>();
            if (nold) {
                const uint32_t *ot = old_off + (uint64_t)t * (nbk + 1);
                const unsigned g = (unsigned)((nold + 255) / 256);
                if (csz == 2)
                    hipLaunchKernelGGL(expand_list_kernel<uint16_t>, dim3(g), dim3(256), 0, s, ot,
                                       nbk, static_cast<const uint16_t *>(old_cells),
                                       tstart_old[t], nold, cb, k);
                else
                    hipLaunchKernelGGL(expand_list_kernel<uint32_t>, dim3(g), dim3(256), 0, s, ot,
                                       nbk, static_cast<const uint32_t *>(old_cells),
                                       tstart_old[t], nold, cb, k);
                FL_CHECK_LAUNCH();
            }
            if (nr) {
                hipLaunchKernelGGL(emit_pairs_kernel, dim3((unsigned)((nr + 255) / 256)), dim3(256),
                                   0, s, codes, grp_rows, n, L, t, R, ix.Rp, Bp, cb, k + nold);
                FL_CHECK_LAUNCH();
            }
            // the sorted keys stay in whichever buffer the last pass wrote
            uint64_t *ks = k;
            radix_sort_u64(k, tmp.as<uint64_t>(), nullptr, nullptr, nk, end_bit, s, &ks);
            if (nk) {
                const unsigned g1 = (unsigned)((nk + 255) / 256);
                hipLaunchKernelGGL(unique_kernel, dim3(g1), dim3(256), 0, s, ks, nk,
                                   flag.as<uint32_t>());
                FL_CHECK_LAUNCH();
                device_exclusive_scan_u32(flag.as<uint32_t>(), pos.as<uint32_t>(), nk, s);
                const uint64_t cmask = (1ull << cb) - 1;
                // the list starts at tb[t]; big holds every key, so the
                // writes stay inside it whatever the total comes to
                if (csz == 2)
                    hipLaunchKernelGGL(compact_kernel<uint16_t>, dim3(g1), dim3(256), 0, s, ks,
                                       flag.as<uint32_t>(), pos.as<uint32_t>(), nk, cmask, tb + t,
                                       static_cast<uint16_t *>(big));
                else
                    hipLaunchKernelGGL(compact_kernel<uint32_t>, dim3(g1), dim3(256), 0, s, ks,
                                       flag.as<uint32_t>(), pos.as<uint32_t>(), nk, cmask, tb + t,
                                       static_cast<uint32_t *>(big));
                FL_CHECK_LAUNCH();
            }
            hipLaunchKernelGGL(list_total_kernel, dim3(1), dim3(64), 0, s, pos.as<uint32_t>(),
                               flag.as<uint32_t>(), nk, tb, t);
            FL_CHECK_LAUNCH();
            const uint64_t nblk = (nbk + 1 + nk + OB_BLOCK - 1) / OB_BLOCK;
            hipLaunchKernelGGL(bucket_blocks_kernel, dim3((unsigned)((nblk + 1 + 255) / 256)),
                               dim3(256), 0, s, ks, nk, cb, nbk, nblk, blod.as<uint64_t>());
            FL_CHECK_LAUNCH();
            hipLaunchKernelGGL(bucket_offsets_kernel, dim3((unsigned)nblk), dim3(256), 0, s, ks,
                               pos.as<uint32_t>(), flag.as<uint32_t>(), nk, cb, nbk,
                               blod.as<uint64_t>(), tb + t, out.offsets + (uint64_t)t * (nbk + 1));
            FL_CHECK_LAUNCH();
        }
        // one read-back of the tables' list starts
        FL_HIP(hipMemcpyAsync(out.tstart.data(), tb, (L + 1) * 8, hipMemcpyDeviceToHost, s));
        FL_HIP(hipStreamSynchronize(s));
        const uint64_t base = out.tstart[L];
        if (base > 0xFFFFFFFFull) fail(FLINNG_EINVAL, "reverse index exceeds 2^32 entries");
        // shrink the list buffer to its size plus a zeroed tail, so that the
        // query kernel's 16-byte chunk reads past a list's end stay inside it
        const size_t used = (size_t)base * csz;
        FL_HIP(hipMalloc(&out.cells, cells_alloc_bytes(base, csz)));
        if (base) FL_HIP(hipMemcpyAsync(out.cells, big, used, hipMemcpyDeviceToDevice, s));
        FL_HIP(hipMemsetAsync(static_cast<char *>(out.cells) + used, 0,
                              cells_alloc_bytes(base, csz) - used, s));
        FL_HIP(hipStreamSynchronize(s));
        FL_HIP(hipFree(big));
        big = nullptr;
        out.entries = base;
    } catch (...) {
        if (big) (void)hipFree(big);
        if (out.offsets) (void)hipFree(out.offsets);
        if (out.cells) (void)hipFree(out.cells);
        throw;
    }
    return out;
}

}  // namespace

void build_lists(Index &ix, const uint32_t *codes, hipStream_t s) {
    Lists l = assemble_lists(ix, nullptr, nullptr, {}, codes, ix.grp, ix.N, s);
    if (ix.offsets) (void)hipFree(ix.offsets);
    ix.offsets = l.offsets;
    ix.cells = l.cells;
    ix.list_entries = l.entries;
    ix.tstart = std::move(l.tstart);
}

// ---------------------------------------------------------------------------
// inserts

// Groups of the arrivals x0 .. x0+n-1 (the build had N0 points).
__global__ void stream_groups_kernel(uint64_t x0, uint64_t n, uint64_t N0, uint32_t R, uint32_t Rp,
                                     uint32_t B, uint32_t half, uint64_t skey,
                                     uint16_t *__restrict__ grp) {
    const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const uint64_t x = x0 + i, a = x - N0;
    const uint64_t j = a / B, u = a % B;
    for (uint32_t r = 0; r < R; ++r) {
        uint64_t keys[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) keys[k] = sm64(skey, 4 * (16 * j + r) + (uint64_t)k);
        uint64_t y = feistel(u, half, keys);
        while (y >= B) y = feistel(y, half, keys);
        grp[x * Rp + r] = (uint16_t)y;
    }
    for (uint32_t r = R; r < Rp; ++r) grp[x * Rp + r] = grp[x * Rp + R - 1];
}

// Where each group's run starts and ends in the arrivals sorted by group.
__global__ void run_bounds_kernel(const uint64_t *__restrict__ keys, uint64_t n,
                                  uint32_t *__restrict__ start, uint32_t *__restrict__ end) {
    const uint64_t p = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= n) return;
    const uint64_t b = keys[p];
    if (p == 0 || keys[p - 1] != b) start[b] = (uint32_t)p;
    if (p == n - 1 || keys[p + 1] != b) end[b] = (uint32_t)(p + 1);
}

__global__ void run_counts_kernel(const uint32_t *__restrict__ start, const uint32_t *__restrict__ end,
                                  uint32_t B, uint32_t *__restrict__ cnt) {
    const uint32_t b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b < B) cnt[b] = end[b] - start[b];
}

// Copy each cell's member ids and group rows into arrays of a larger stride.
__global__ void restride_kernel(const uint32_t *__restrict__ mem, const uint16_t *__restrict__ cmg,
                                uint64_t ncells, uint32_t s0, uint32_t s1, uint32_t Rp,
                                uint32_t *__restrict__ mem1, uint16_t *__restrict__ cmg1) {
    const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= ncells * s0) return;
    const uint64_t c = i / s0, j = i % s0;
    mem1[c * s1 + j] = mem[i];
    for (uint32_t r = 0; r < Rp; ++r) cmg1[(c * s1 + j) * Rp + r] = cmg[i * Rp + r];
}

// The sorted arrivals of one repetition join their cells after the members
// already there: member id and its group row.
__global__ void place_members_kernel(const uint64_t *__restrict__ keys, const uint32_t *__restrict__ ids,
                                     uint64_t n, const uint32_t *__restrict__ start,
                                     const uint32_t *__restrict__ gsize_r, uint32_t mstride,
                                     const uint16_t *__restrict__ grp, uint32_t Rp,
                                     uint32_t *__restrict__ mem_r, uint16_t *__restrict__ cmg_r) {
    const uint64_t p = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= n) return;
    const uint64_t b = keys[p];
    const uint64_t slot = b * mstride + gsize_r[b] + (p - start[b]);
    const uint32_t x = ids[p];
    mem_r[slot] = x;
    for (uint32_t r = 0; r < Rp; ++r) cmg_r[slot * Rp + r] = grp[(uint64_t)x * Rp + r];
}

__global__ void add_u32_kernel(const uint32_t *__restrict__ a, const uint32_t *__restrict__ b,
                               uint64_t n, uint32_t *__restrict__ out) {
    const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) out[i] = a[i] + b[i];
}

void insert_points(Index &ix, const uint32_t *codes, uint64_t n, hipStream_t s) {
    if (n == 0) return;
    const uint64_t x0 = ix.N;
    if (x0 + n > 0xFFFFFFFEull) fail(FLINNG_EINVAL, "at most 2^32-2 points");
    const uint32_t R = ix.p.R, B = ix.p.B, Rp = ix.Rp;
    const uint64_t ncells = (uint64_t)R * B;
    auto dfree = [](void *p) { if (p) (void)hipFree(p); };
    // arrays of the new version (freed on failure)
    uint16_t *grp1 = nullptr, *cmg1 = nullptr;
    uint32_t *mem1 = nullptr, *gsize1 = nullptr, *cfl1 = nullptr;
    Lists lists;
    try {
        // 1. group rows of the arrivals (grp is not read by queries; a larger
        //    copy replaces it under the lock below)
        uint16_t *grp = ix.grp;
        if (x0 + n > ix.grp_cap) {
            const uint64_t cap = std::max<uint64_t>(x0 + n, ix.grp_cap + ix.grp_cap / 2);
            FL_HIP(hipMalloc(&grp1, cap * Rp * 2));
            FL_HIP(hipMemcpyAsync(grp1, ix.grp, x0 * Rp * 2, hipMemcpyDeviceToDevice, s));
            grp = grp1;
        }
        uint32_t nb = 2;
        while (nb < 64 && (1ull << nb) < B) nb += 2;
        const unsigned gn = (unsigned)((n + 255) / 256);
        hipLaunchKernelGGL(stream_groups_kernel, dim3(gn), dim3(256), 0, s, x0, n, ix.N0, R, Rp, B,
                           nb / 2, sm64(ix.p.seed, TAG_STREAM), grp);
        FL_CHECK_LAUNCH();
        // 2. arrivals sorted by group, per repetition; new cell sizes
        int gbits = 1;
        while ((1u << gbits) < B) ++gbits;
        std::vector<DevBuf> skeys, sids;
        DevBuf tk(n * 8, s), tv(n * 4, s), starts(ncells * 4, s), ends(ncells * 4, s),
            cnt(ncells * 4, s);
        FL_HIP(hipMemsetAsync(starts.ptr, 0, ncells * 4, s));
        FL_HIP(hipMemsetAsync(ends.ptr, 0, ncells * 4, s));
        for (uint32_t r = 0; r < R; ++r) {
            skeys.emplace_back(n * 8, s);
            sids.emplace_back(n * 4, s);
            hipLaunchKernelGGL(member_keys_kernel, dim3(gn), dim3(256), 0, s, grp, x0, n, Rp, r,
                               skeys.back().as<uint64_t>(), sids.back().as<uint32_t>());
            FL_CHECK_LAUNCH();
            radix_sort_u64(skeys.back().as<uint64_t>(), tk.as<uint64_t>(), sids.back().as<uint32_t>(),
                           tv.as<uint32_t>(), n, gbits, s);
            hipLaunchKernelGGL(run_bounds_kernel, dim3(gn), dim3(256), 0, s,
                               skeys.back().as<uint64_t>(), n, starts.as<uint32_t>() + (uint64_t)r * B,
                               ends.as<uint32_t>() + (uint64_t)r * B);
            FL_CHECK_LAUNCH();
        }
        hipLaunchKernelGGL(run_counts_kernel, dim3((unsigned)((ncells + 255) / 256)), dim3(256), 0, s,
                           starts.as<uint32_t>(), ends.as<uint32_t>(), (uint32_t)ncells,
                           cnt.as<uint32_t>());
        FL_CHECK_LAUNCH();
        std::vector<uint32_t> add(ncells);
        FL_HIP(hipMemcpyAsync(add.data(), cnt.ptr, ncells * 4, hipMemcpyDeviceToHost, s));
        FL_HIP(hipStreamSynchronize(s));
        std::vector<uint32_t> gs1(ix.gsize_host);
        uint32_t gmax1 = 0;
        for (uint64_t c = 0; c < ncells; ++c) {
            gs1[c] += add[c];
            gmax1 = std::max(gmax1, gs1[c]);
        }
        // 3. member arrays of the new version: a copy, at a larger stride when
        //    a cell outgrows the old one, then the arrivals appended
        uint32_t ms1 = ix.mstride;
        if (gmax1 > ms1) ms1 = (uint32_t)((std::max<uint64_t>(gmax1, ms1 + ms1 / 2) + 3) & ~3ull);
        FL_HIP(hipMalloc(&mem1, ncells * ms1 * 4));
        FL_HIP(hipMalloc(&cmg1, ncells * ms1 * Rp * 2));
        if (ms1 == ix.mstride) {
            FL_HIP(hipMemcpyAsync(mem1, ix.mem, ncells * ms1 * 4, hipMemcpyDeviceToDevice, s));
            FL_HIP(hipMemcpyAsync(cmg1, ix.cmg, ncells * ms1 * Rp * 2, hipMemcpyDeviceToDevice, s));
        } else {
            FL_HIP(hipMemsetAsync(mem1, 0xFF, ncells * ms1 * 4, s));
            FL_HIP(hipMemsetAsync(cmg1, 0, ncells * ms1 * Rp * 2, s));
            const uint64_t tot = ncells * ix.mstride;
            hipLaunchKernelGGL(restride_kernel, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s,
                               ix.mem, ix.cmg, ncells, ix.mstride, ms1, Rp, mem1, cmg1);
            FL_CHECK_LAUNCH();
        }
        for (uint32_t r = 0; r < R; ++r) {
            hipLaunchKernelGGL(place_members_kernel, dim3(gn), dim3(256), 0, s,
                               skeys[r].as<uint64_t>(), sids[r].as<uint32_t>(), n,
                               starts.as<uint32_t>() + (uint64_t)r * B, ix.gsize + (uint64_t)r * B,
                               ms1, grp, Rp, mem1 + (uint64_t)r * B * ms1,
                               cmg1 + (uint64_t)r * B * ms1 * Rp);
            FL_CHECK_LAUNCH();
        }
        FL_HIP(hipMalloc(&cfl1, ncells * ms1 * 4));
        build_filter(ix, mem1, grp, ms1, cfl1, s);
        FL_HIP(hipMalloc(&gsize1, ncells * 4));
        hipLaunchKernelGGL(add_u32_kernel, dim3((unsigned)((ncells + 255) / 256)), dim3(256), 0, s,
                           ix.gsize, cnt.as<uint32_t>(), ncells, gsize1);
        FL_CHECK_LAUNCH();
        // 4. reverse index: old entries plus the arrivals' pairs
        lists = assemble_lists(ix, ix.offsets, ix.cells, ix.tstart, codes, grp + x0 * Rp, n, s);
        FL_HIP(hipStreamSynchronize(s));
        // 5. swap the new version in while no query is being enqueued, and
        //    free the old one once the device has finished all work using it
        std::unique_lock<std::shared_mutex> lk(ix.rw);
        void *old[7] = {ix.offsets, ix.cells, ix.mem, ix.cmg, ix.cfl, ix.gsize,
                        grp1 ? ix.grp : nullptr};
        ix.offsets = lists.offsets;
        ix.cells = lists.cells;
        ix.list_entries = lists.entries;
        ix.tstart = std::move(lists.tstart);
        ix.mem = mem1;
        ix.cmg = cmg1;
        ix.cfl = cfl1;
        ix.gsize = gsize1;
        if (grp1) {
            ix.grp = grp1;
            ix.grp_cap = std::max<uint64_t>(x0 + n, ix.grp_cap + ix.grp_cap / 2);
        }
        ix.mstride = ms1;
        ix.gsize_host = std::move(gs1);
        ix.gmax = gmax1;
        ix.N = x0 + n;
        ix.device_bytes = index_device_bytes(ix);
        lists = Lists();
        mem1 = nullptr;
        cmg1 = nullptr;
        cfl1 = nullptr;
        gsize1 = nullptr;
        grp1 = nullptr;
        FL_HIP(hipDeviceSynchronize());
        for (void *p : old) dfree(p);
    } catch (...) {
        dfree(grp1);
        dfree(mem1);
        dfree(cmg1);
        dfree(cfl1);
        dfree(gsize1);
        dfree(lists.offsets);
        dfree(lists.cells);
        throw;
    }
}

}  // namespace flinng
