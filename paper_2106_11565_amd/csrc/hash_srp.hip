// Signed random projection hashing on gfx950.
//
// The dense LSH of the method (Section 3, Locality-Sensitive Hashing, and the
// concatenation trick): bit j of table t is 1 iff the exact dot product of
// the row with hyperplane h = t*K + j is positive (an exact zero gives 0);
// the table's bucket is sum_j bit_j 2^j.  Hashing is shared by every filter
// and done once per point or query (Section 6, Implementation).
//
// bf16 rows take one fused kernel (srp_fused_kernel) for all of the steps
// below; fp32 rows take them as three kernels.
//
// Pipeline (one batch of n rows, H = L*K hyperplanes):
//   1. prep: bf16 operand planes (fp32 rows split exactly into 3 bf16 terms)
//      and fp32 row norms.
//   2. MFMA: P = X * W^T on v_mfma_f32_16x16x32_bf16 with fp32 accumulation.
//      A projection is trusted when |P| > tau = gamma * |x| * |w| (plus a
//      denormal allowance), gamma = n*u/(1-n*u) with u = 2^-23 and n the
//      number of accumulated products: a bound on the accumulation error for
//      any summation order with round-to-nearest or truncating adds, applied
//      through sum|x_i w_i| <= |x|_2 |w|_2.  Trusted signs become bits by
//      wavefront ballot; the rest are flagged.
//   3. recheck: each flagged projection is recomputed in FP64 across a
//      wavefront; its sign is certified when |v| > 2*d*2^-53 * sum|x_i w_i|,
//      else an exact fixed-point sum decides.  Then bits are packed into the
//      per-table codes.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>

#include "flinng_internal.h"

namespace flinng {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

// ---------------------------------------------------------------------------
// Hyperplanes: entry (h, i) = (popcount(sm64(key_HYP, h*d + i)) - 32) / 4, a
// centred Binomial(64,1/2)/4 value, exact in bf16.  Stored [H][dpad], zero
// padded.
__global__ void hyp_kernel(uint16_t *__restrict__ w, uint32_t H, uint32_t d,
                           uint32_t dpad, uint64_t key) {
    uint64_t id = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    uint64_t total = (uint64_t)H * dpad;
    if (id >= total) return;
    uint32_t h = (uint32_t)(id / dpad), i = (uint32_t)(id % dpad);
    uint16_t bits = 0;
    if (i < d) {
        int pc = __popcll(sm64(key, (uint64_t)h * d + i));
        float f = (float)(pc - 32) * 0.25f;
        bits = (uint16_t)(__float_as_uint(f) >> 16);
    }
    w[id] = bits;
}

__device__ inline float bf16_to_f32(uint16_t b) { return __uint_as_float((uint32_t)b << 16); }

__device__ inline float wave_sum_f32(float v) {
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}
__device__ inline double wave_sum_f64(double v) {
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// Norms of the hyperplanes (sums of squares of quarter-integers are exact in
// fp32 for the supported dimensions).  One wavefront per hyperplane.
__global__ void hypnorm_kernel(const uint16_t *__restrict__ w, float *__restrict__ nw,
                               uint32_t H, uint32_t dpad) {
    uint32_t h = blockIdx.x * (blockDim.x / 64) + threadIdx.x / 64;
    uint32_t lane = threadIdx.x % 64;
    if (h >= H) return;
    float s = 0.f;
    for (uint32_t i = lane; i < dpad; i += 64) {
        float v = bf16_to_f32(w[(uint64_t)h * dpad + i]);
        s += v * v;
    }
    s = wave_sum_f32(s);
    if (lane == 0) nw[h] = sqrtf(s);
}

// The tiled copy: element (h, i) at ((h / 16) * (dpad / 32) + i / 32) * 512
// + (h % 16) * 32 + i % 32, zero for h >= H.
__global__ void hyp_tile_kernel(const uint16_t *__restrict__ w, uint16_t *__restrict__ wt,
                                uint32_t H, uint32_t dpad) {
    const uint64_t id = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const uint64_t hp = (H + 15) / 16 * 16;
    if (id >= hp * dpad) return;
    const uint32_t h = (uint32_t)(id / dpad), i = (uint32_t)(id % dpad);
    const uint64_t o = ((uint64_t)(h / 16) * (dpad / 32) + i / 32) * 512 + (h % 16) * 32 + i % 32;
    wt[o] = h < H ? w[(uint64_t)h * dpad + i] : (uint16_t)0;
}

void srp_make_hyperplanes(Index &ix, hipStream_t s) {
    const uint32_t H = ix.p.L * ix.p.K;
    uint64_t total = (uint64_t)H * ix.dpad;
    hipLaunchKernelGGL(hyp_kernel, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s,
                       ix.hyp, H, ix.p.dim, ix.dpad, sm64(ix.p.seed, TAG_HYP));
    FL_CHECK_LAUNCH();
    hipLaunchKernelGGL(hypnorm_kernel, dim3((H + 3) / 4), dim3(256), 0, s, ix.hyp,
                       ix.hypnorm, H, ix.dpad);
    FL_CHECK_LAUNCH();
    if (ix.hypt) {
        const uint64_t tot = (uint64_t)(H + 15) / 16 * 16 * ix.dpad;
        hipLaunchKernelGGL(hyp_tile_kernel, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s,
                           ix.hyp, ix.hypt, H, ix.dpad);
        FL_CHECK_LAUNCH();
    }
}

// ---------------------------------------------------------------------------
// Prep: one wavefront per row.  Writes nsplit bf16 planes [n][dpad] (unless
// planes == nullptr) and the row norm, rounded to fp32 (unless nx ==
// nullptr), and clears the sign and flag words and the counters (those given).  fp32 values are
// split by truncation: x = x1 + x2 + x3, each a bf16 (exact except below
// 2^-133, which the denormal allowance of tau covers).
// The sum of squares is accumulated in FP64: the square of any fp32 or bf16
// value (at least 2^-298) is a normal double, so the norm cannot underflow
// for rows whose entries all lie below 2^-63, where fp32 squares would
// vanish and leave the sign certificate with the absolute term alone.
template <bool F32>
__global__ void prep_kernel(const void *__restrict__ xin, uint64_t n, uint32_t d,
                            uint32_t dpad, uint16_t *__restrict__ planes,
                            float *__restrict__ nx, uint32_t *__restrict__ bits,
                            uint32_t *__restrict__ flags, uint32_t Hw,
                            unsigned long long *__restrict__ ctr) {
    uint64_t row = (uint64_t)blockIdx.x * (blockDim.x / 64) + threadIdx.x / 64;
    uint32_t lane = threadIdx.x % 64;
    if (row >= n) return;
    // clear this row's sign and flag words (the projection kernel leaves the
    // words past the last hyperplane untouched) and the flag counters
    for (uint32_t w = lane; w < Hw; w += 64) {
        bits[row * Hw + w] = 0u;
        flags[row * Hw + w] = 0u;
    }
    if (ctr && row == 0 && lane < 2) ctr[lane] = 0ull;
    const uint64_t plane_stride = n * dpad;
    double s = 0.0;
    if (!F32 && planes == nullptr && d == dpad) {
        // bf16 rows used in place (16-byte aligned, d a multiple of 32):
        // only the norm, from 16-byte loads (eight values per lane)
        const uint4 *xr = reinterpret_cast<const uint4 *>(static_cast<const uint16_t *>(xin) + row * d);
        for (uint32_t i = lane; i < d / 8; i += 64) {
            const uint4 v = xr[i];
            const uint32_t w[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const double lo = (double)__uint_as_float(w[j] << 16);
                const double hi = (double)__uint_as_float(w[j] & 0xFFFF0000u);
                s += lo * lo + hi * hi;
            }
        }
        s = wave_sum_f64(s);
        if (lane == 0 && nx) nx[row] = (float)sqrt(s);
        return;
    }
    for (uint32_t i = lane; i < dpad; i += 64) {
        float x = 0.f;
        if (i < d) {
            if (F32)
                x = static_cast<const float *>(xin)[row * d + i];
            else
                x = bf16_to_f32(static_cast<const uint16_t *>(xin)[row * d + i]);
        }
        s += (double)x * (double)x;
        if (planes) {
            uint64_t o = row * dpad + i;
            if (F32) {
                uint32_t b1 = __float_as_uint(x) & 0xFFFF0000u;
                float r1 = x - __uint_as_float(b1);
                uint32_t b2 = __float_as_uint(r1) & 0xFFFF0000u;
                float r2 = r1 - __uint_as_float(b2);
                uint32_t b3 = __float_as_uint(r2) & 0xFFFF0000u;
                planes[o] = (uint16_t)(b1 >> 16);
                planes[plane_stride + o] = (uint16_t)(b2 >> 16);
                planes[2 * plane_stride + o] = (uint16_t)(b3 >> 16);
            } else {
                planes[o] = static_cast<const uint16_t *>(xin)[row * d + i];
            }
        } else {
            (void)plane_stride;
        }
    }
    s = wave_sum_f64(s);
    if (lane == 0 && nx) nx[row] = (float)sqrt(s);
}

// ---------------------------------------------------------------------------
// MFMA projection + trusted-sign bits.
// Wave tile: (16*MR) rows x (16*NR) hyperplanes; workgroup: WM x WN waves.
// Operand fragments are loaded straight from global memory (16 bytes per
// lane per fragment); lane l supplies row/column (l % 16) and the 8
// consecutive k values at 8*(l/16) of each 32-wide k step, identically for
// X and W, so every product pairs x[row][k] with w[col][k].
// Output of a 16x16 tile: lane l holds rows 4*(l/16)+i, column l%16.
template <int MR, int NR, int WM, int WN, int NSPLIT>
__global__ __launch_bounds__(64 * WM * WN) void srp_mfma_kernel(
    const uint16_t *__restrict__ planes, uint64_t plane_stride, uint32_t ld,
    const uint16_t *__restrict__ w, uint32_t dpad, const float *__restrict__ nx,
    const float *__restrict__ nw, uint64_t n, uint32_t H, uint32_t Hw,
    float gamma, float tau_abs, uint16_t *__restrict__ bits16,
    uint16_t *__restrict__ flags16, unsigned long long *__restrict__ nflag,
    float *__restrict__ proj) {
    const int lane = threadIdx.x % 64;
    const int wave = threadIdx.x / 64;
    const int wm = wave / WN, wn = wave % WN;
    const uint64_t row0 = (uint64_t)blockIdx.y * (16 * MR * WM) + (uint64_t)wm * 16 * MR;
    const uint32_t col0 = blockIdx.x * (16 * NR * WN) + wn * 16 * NR;
    if (row0 >= n || col0 >= H) return;

    f32x4 acc[MR][NR];
#pragma unroll
    for (int a = 0; a < MR; ++a)
#pragma unroll
        for (int b = 0; b < NR; ++b) acc[a][b] = f32x4{0.f, 0.f, 0.f, 0.f};

    const int lr = lane % 16, lk = (lane / 16) * 8;
    const uint16_t *pa[MR];
    const uint16_t *pb[NR];
#pragma unroll
    for (int a = 0; a < MR; ++a) {
        uint64_t r = row0 + 16 * a + lr;
        if (r >= n) r = n - 1;
        pa[a] = planes + r * ld + lk;
    }
#pragma unroll
    for (int b = 0; b < NR; ++b) {
        uint32_t c = col0 + 16 * b + lr;
        if (c >= H) c = H - 1;
        pb[b] = w + (uint64_t)c * dpad + lk;
    }

    for (uint32_t k0 = 0; k0 < dpad; k0 += 32) {
        bf16x8 fb[NR];
#pragma unroll
        for (int b = 0; b < NR; ++b)
            fb[b] = __builtin_bit_cast(bf16x8, *reinterpret_cast<const uint4 *>(pb[b] + k0));
#pragma unroll
        for (int sp = 0; sp < NSPLIT; ++sp) {
            bf16x8 fa[MR];
#pragma unroll
            for (int a = 0; a < MR; ++a)
                fa[a] = __builtin_bit_cast(
                    bf16x8, *reinterpret_cast<const uint4 *>(pa[a] + sp * plane_stride + k0));
#pragma unroll
            for (int a = 0; a < MR; ++a)
#pragma unroll
                for (int b = 0; b < NR; ++b)
                    acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(fa[a], fb[b], acc[a][b],
                                                                        0, 0, 0);
        }
    }

    // Epilogue: trusted sign bits and flags, 16 columns per ballot group.
    unsigned long long flagged = 0;
#pragma unroll
    for (int b = 0; b < NR; ++b) {
        const uint32_t cbase = col0 + 16 * b;
        if (cbase >= H) continue;
        const uint32_t col = cbase + lr;
        const float wn_ = (col < H) ? nw[col] : 0.f;
#pragma unroll
        for (int a = 0; a < MR; ++a) {
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const uint64_t row = row0 + 16 * a + 4 * (lane / 16) + i;
                const float xn = (row < n) ? nx[row] : 0.f;
                const float v = acc[a][b][i];
                if (proj && row < n && col < H) proj[row * H + col] = v;
                const float tau = gamma * xn * wn_ + tau_abs;
                const bool ok = (col < H) && (fabsf(v) > tau);
                const bool bit = ok && (v > 0.f);
                const bool flg = (col < H) && !ok;
                const unsigned long long mb = __ballot(bit);
                const unsigned long long mf = __ballot(flg);
                if ((lane % 16) == 0 && row < n) {
                    const int g = lane / 16;
                    const uint64_t o = row * (2 * (uint64_t)Hw) + cbase / 16;
                    bits16[o] = (uint16_t)(mb >> (16 * g));
                    flags16[o] = (uint16_t)(mf >> (16 * g));
                    flagged += __popcll((mf >> (16 * g)) & 0xFFFFull);
                }
            }
        }
    }
    if ((lane % 16) == 0 && flagged) atomicAdd(nflag, flagged);
}

// ---------------------------------------------------------------------------
// Exact sign of sum_i x_i * w_i when FP64 cannot certify it.  Every product
// is an exact double m * 2^e with |m| < 2^31 and e >= -151 (x: fp32/bf16,
// w: quarter-integer); products are added into 32-bit digits of a signed
// fixed-point number spanning 2^-160 .. 2^224, then carries are propagated
// and the sign read from the top.  The whole wavefront calls it: lane l adds
// the products i = l, l + 64, ... into its own int64 digits, which are then
// summed across the wavefront (no overflow for up to 2^30 terms in all), so
// every lane returns the same sign.
__device__ int exact_sign_wave(const void *xin, bool f32, uint64_t row, uint32_t d, uint32_t ld,
                               const uint16_t *__restrict__ wh) {
    constexpr int NLIMB = 12;
    constexpr int BASE = -160;
    long long limb[NLIMB];
#pragma unroll
    for (int j = 0; j < NLIMB; ++j) limb[j] = 0;
    for (uint32_t i = threadIdx.x % 64; i < d; i += 64) {
        const double xv = f32 ? (double)static_cast<const float *>(xin)[row * ld + i]
                              : (double)bf16_to_f32(static_cast<const uint16_t *>(xin)[row * ld + i]);
        const double p = xv * (double)bf16_to_f32(wh[i]);
        if (p == 0.0) continue;
        const unsigned long long bits = (unsigned long long)__double_as_longlong(p);
        const bool neg = bits >> 63;
        const int ex = (int)((bits >> 52) & 0x7FF);
        unsigned long long m = bits & ((1ull << 52) - 1);
        int pos;
        if (ex == 0) {
            pos = -1074;
        } else {
            m |= (1ull << 52);
            pos = ex - 1075;
        }
        const int tz = __builtin_ctzll(m);  // m != 0: p is not zero
        m >>= tz;
        pos += tz;
        const int sh = pos - BASE;  // >= 9 for the supported inputs
        const int j = sh / 32, o = sh % 32;
        // m < 2^31 after stripping: (m << o) < 2^63
        const unsigned long long v = m << o;
        long long lo = (long long)(v & 0xFFFFFFFFull), hi = (long long)(v >> 32);
        if (neg) {
            lo = -lo;
            hi = -hi;
        }
        // registers, not a dynamically indexed array
#pragma unroll
        for (int q = 0; q < NLIMB; ++q) {
            limb[q] += (q == j) ? lo : 0ll;
            limb[q] += (q == j + 1) ? hi : 0ll;
        }
    }
#pragma unroll
    for (int q = 0; q < NLIMB; ++q)
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) limb[q] += __shfl_xor(limb[q], o, 64);
#pragma unroll
    for (int j = 0; j < NLIMB - 1; ++j) {
        const long long c = limb[j] >> 32;  // arithmetic shift: floor division
        limb[j] -= c * (1ll << 32);
        limb[j + 1] += c;
    }
    if (limb[NLIMB - 1] != 0) return limb[NLIMB - 1] > 0 ? 1 : -1;
    int any = 0;
#pragma unroll
    for (int j = NLIMB - 2; j >= 0; --j) any |= limb[j] != 0;
    return any;
}

// Recheck + pack: one wavefront per row.  Bits of the row are staged in LDS
// (Hw words), flagged projections are recomputed in FP64 across the wave,
// then lanes t < L extract the K-bit code of table t.
__global__ __launch_bounds__(256) void srp_recheck_pack_kernel(
    const void *__restrict__ xin, int f32, uint64_t n, uint32_t d,
    const uint16_t *__restrict__ w, uint32_t dpad, const uint32_t *__restrict__ bits,
    const uint32_t *__restrict__ flags, uint32_t Hw, uint32_t H, uint32_t K, uint32_t L,
    uint32_t *__restrict__ codes, unsigned long long *__restrict__ nexact) {
    extern __shared__ uint32_t sm[];
    const int lane = threadIdx.x % 64;
    const int wave = threadIdx.x / 64;
    const uint64_t row = (uint64_t)blockIdx.x * (blockDim.x / 64) + wave;
    if (row >= n) return;
    uint32_t *rb = sm + wave * Hw;
    for (uint32_t j = lane; j < Hw; j += 64) rb[j] = bits[row * Hw + j];
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    for (uint32_t j0 = 0; j0 < Hw; j0 += 64) {
        uint32_t fw = (j0 + lane < Hw) ? flags[row * Hw + j0 + lane] : 0u;
        unsigned long long any = __ballot(fw != 0);
        while (any) {
            int src = __ffsll((long long)any) - 1;
            any &= any - 1;
            uint32_t word = __shfl(fw, src, 64);
            while (word) {
                int bit = __ffs(word) - 1;
                word &= word - 1;
                uint32_t h = (j0 + src) * 32 + bit;
                if (h >= H) continue;
                const uint16_t *wh = w + (uint64_t)h * dpad;
                double v = 0.0, a = 0.0;
                for (uint32_t i = lane; i < d; i += 64) {
                    double xv = f32 ? (double)static_cast<const float *>(xin)[row * d + i]
                                    : (double)bf16_to_f32(static_cast<const uint16_t *>(xin)[row * d + i]);
                    double p = xv * (double)bf16_to_f32(wh[i]);
                    v += p;
                    a += fabs(p);
                }
                v = wave_sum_f64(v);
                a = wave_sum_f64(a);
                int sgn;
                // the butterfly sums are bit-identical in every lane; take
                // lane 0's verdict so the branch is uniform by construction
                if (__builtin_amdgcn_readfirstlane(fabs(v) > 2.0 * (double)d * 0x1p-53 * a ? 1 : 0)) {
                    sgn = v > 0.0 ? 1 : -1;
                } else {
                    sgn = exact_sign_wave(xin, f32 != 0, row, d, d, wh);
                    if (lane == 0) atomicAdd(nexact, 1ull);
                }
                if (lane == 0) {
                    uint32_t m = 1u << bit;
                    if (sgn > 0)
                        rb[j0 + src] |= m;
                    else
                        rb[j0 + src] &= ~m;
                }
                __builtin_amdgcn_wave_barrier();
            }
        }
    }
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    for (uint32_t t = lane; t < L; t += 64) {
        uint32_t b0 = t * K;
        uint32_t wi = b0 / 32, sh = b0 % 32;
        uint64_t v = rb[wi];
        if (sh + K > 32 && wi + 1 < Hw) v |= (uint64_t)rb[wi + 1] << 32;
        uint32_t code = (uint32_t)((v >> sh) & ((K >= 32) ? 0xFFFFFFFFull : ((1ull << K) - 1)));
        codes[row * L + t] = code;
    }
}

// The bf16 stage in one kernel: projection, sign certificate, FP64 recheck
// of the flagged projections and packing of the codes.
//
// A workgroup takes a tile of TM = 16*MR rows against one group of whole
// tables (gt consecutive tables, at most 48*NW hyperplanes), with NW*KS
// wavefronts: column wavefront c owns the group's hyperplanes 48c .. 48c+47
// (MR x 3 MFMA tiles of 16 x 16, v_mfma_f32_16x16x32_bf16), and each of the
// KS k groups of NW wavefronts takes one contiguous run of whole 128-wide k
// chunks.  A group walks its run in 64-wide steps: its rows are staged once
// in LDS (double-buffered, rows padded by 16 bytes against bank conflicts)
// and multiplied by its NW wavefronts, while each wavefront reads its own
// hyperplanes' fragments straight from global memory (no other wavefront of
// the group uses them; the hyperplanes of an index stay in L2); both are
// prefetched one step ahead.  Each step waits on one round of memory
// latency, so the KS groups (KS times the loads in flight, a chain of steps
// KS times shorter) are what keeps a small grid busy.
//
// Accumulation is chunked: every 128 consecutive k accumulate into a fresh
// partial (MFMA accumulate), the partials are added in fp32 within the
// group, and the KS group sums are added in group order.  A product then
// passes through at most 128 roundings inside its chunk (whatever order an
// instruction sums its 32 products and its accumulator in), one per chunk of
// its group and KS - 1 group additions.  With nch = ceil(d / 128) chunks,
// cpg = ceil(nch / KS) per group and nch >= 2 KS, cpg + KS - 1 <= nch, so
// |v32 - v| <= gamma_m * sum|x_i w_i| with m = min(128, d) + nch
// (srp_lds_terms), far below the gamma_d of one long chain.
//
// The norms |x| are summed in FP64 from the staged pieces (squares of bf16
// values are exact doubles, so they cannot underflow), per group and then
// in group order.  Epilogue: trusted signs and flags become 16-bit words in
// LDS by ballot; all wavefronts take the tile's rows in turn and recompute
// each flagged projection in FP64 (8 bf16 values per lane per 16-byte load,
// partials reduced by butterfly), certified when |v| > 2*d*2^-53*sum|x_i
// w_i|, else by exact_sign_wave; then the codes of the group's tables are
// written.
//
// Workgroup order: the hardware hands consecutive workgroup ids to the eight
// XCDs in turn; ids are renumbered so that the groups of one row tile (which
// read the same rows) run on one XCD, close in time, and share its L2.
constexpr int LK = 64;        // k per pipeline step (two 32-wide MFMA slices)
constexpr int LROW = LK + 8;  // bf16 per LDS row (16 bytes of padding)
constexpr int LCHK = 128;     // k per accumulation chunk
constexpr int FW = 48;        // hyperplanes per wavefront
constexpr int FMAXW = 6;      // column wavefronts per workgroup at most
constexpr int FMAXH = FW * FMAXW;  // hyperplanes per group at most
constexpr int FWRD = FMAXH / 32;   // sign / flag words per row in LDS

// Roundings a product passes through in srp_fused_kernel (see above).
inline uint32_t srp_lds_terms(uint32_t dpad) {
    return (dpad < (uint32_t)LCHK ? dpad : (uint32_t)LCHK) + (dpad + LCHK - 1) / LCHK;
}

// Sizes of one srp_fused_kernel variant.
template <int MR, int NW, int KS>
struct FusedShape {
    static constexpr int TM = 16 * MR;
    static constexpr int GT = 64 * NW;              // threads of one k group
    static constexpr int XP = TM * LK / 8;          // 16-byte pieces of one step's rows
    static constexpr int PPT = (XP + GT - 1) / GT;  // pieces per thread
    static constexpr int XB = TM * LROW;            // bf16 per row buffer
    static constexpr size_t XBYTES = (size_t)KS * 2 * XB * 2;
    static constexpr size_t PBYTES = (size_t)(KS - 1) * TM * FW * NW * 4;  // group sums
    static constexpr size_t LDS = XBYTES > PBYTES ? XBYTES : PBYTES;      // dynamic LDS
};

template <int MR, int NW, int KS>
__global__ __launch_bounds__(64 * NW * KS) void srp_fused_kernel(
    const uint16_t *__restrict__ x, uint32_t ld, uint32_t d, const uint16_t *__restrict__ w,
    const uint16_t *__restrict__ wt, uint32_t dpad, const float *__restrict__ nw, uint64_t n,
    uint32_t K, uint32_t L, uint32_t gt, float gamma, float tau_abs, uint32_t *__restrict__ codes,
    unsigned long long *__restrict__ ctr, float *__restrict__ proj) {
    using SH = FusedShape<MR, NW, KS>;
    constexpr int TM = SH::TM, GT = SH::GT, XP = SH::XP, PPT = SH::PPT, XB = SH::XB;
    constexpr int NWV = NW * KS;
    // row buffers during the k loop, then the group sums (fp32)
    extern __shared__ __align__(16) unsigned char dyn[];
    uint16_t *sxa = reinterpret_cast<uint16_t *>(dyn);
    float *part = reinterpret_cast<float *>(dyn);
    __shared__ uint32_t sbits[TM * FWRD];
    __shared__ uint32_t sflag[TM * FWRD];
    __shared__ float snx[TM];
    __shared__ double snx2[KS * TM];
    uint16_t *sb16 = reinterpret_cast<uint16_t *>(sbits);
    uint16_t *sf16 = reinterpret_cast<uint16_t *>(sflag);

    const int tid = threadIdx.x, lane = tid % 64;
    const int wave = __builtin_amdgcn_readfirstlane(tid / 64);
    const int cw = wave % NW, kg = wave / NW;  // column wavefront, k group
    const int gtid = tid - kg * GT;            // thread within the k group
    const uint32_t ng = (L + gt - 1) / gt;
    uint32_t lid = blockIdx.x;
    {
        const uint32_t per = gridDim.x / 8;
        if (lid < per * 8) lid = (lid % 8) * per + lid / 8;
    }
    const uint32_t rt = lid / ng, g = lid - rt * ng;
    const uint64_t r0 = (uint64_t)rt * TM;
    const uint32_t t0 = g * gt;
    const uint32_t ntab = (L - t0 < gt) ? L - t0 : gt;
    const uint32_t h0 = t0 * K, gcols = ntab * K, H = K * L;

    // this group's k range (whole chunks) and step count; group 0 has the most
    const uint32_t nch = (d + LCHK - 1) / LCHK, cpg = (nch + KS - 1) / KS;
    const uint32_t c0 = (uint32_t)kg * cpg < nch ? (uint32_t)kg * cpg : nch;
    const uint32_t kb = c0 * LCHK;
    const uint32_t ke = (c0 + cpg) * LCHK < d ? (c0 + cpg) * LCHK : d;
    const uint32_t nst = ke > kb ? (ke - kb + LK - 1) / LK : 0u;
    const uint32_t kmax = cpg * LCHK < d ? cpg * LCHK : d;
    const uint32_t nmax = (kmax + LK - 1) / LK;

    // this thread's pieces of the rows: piece p covers tile row p / 8, k
    // offset 8 * (p % 8) of the step (rows past n clamped, never output)
    const uint16_t *xp[PPT];
#pragma unroll
    for (int j = 0; j < PPT; ++j) {
        const uint32_t p = gtid + GT * j;
        const uint64_t r = (p < XP && r0 + p / 8 < n) ? r0 + p / 8 : n - 1;
        xp[j] = x + r * ld + 8 * (p % 8);
    }
    // this lane's hyperplanes: column 16b + lane % 16 of the wavefront's 48
    // (clamped into the group; the clamped columns' outputs are unused), read
    // from the tiled copy, where a fragment (16 hyperplanes x 32 k) is 1 KB
    // contiguous: the next 32 k lie 512 values further
    const int lr = lane % 16, lk = (lane / 16) * 8;
    const uint16_t *wp[3];
#pragma unroll
    for (int b = 0; b < 3; ++b) {
        const uint32_t hr = FW * cw + 16 * b + lr;
        const uint32_t c = h0 + (hr < gcols ? hr : gcols - 1);
        wp[b] = wt + (uint64_t)(c / 16) * (dpad / 32) * 512 + (c % 16) * 32 + lk;
    }
    uint16_t *sx = sxa + kg * 2 * XB;  // this group's two row buffers

    uint4 xr[PPT];
    uint4 wf[2][3], wn[2][3];
    double ss[PPT];
#pragma unroll
    for (int j = 0; j < PPT; ++j) ss[j] = 0.0;
    auto fetch_x = [&](uint32_t k0) {
#pragma unroll
        for (int j = 0; j < PPT; ++j) {
            const uint32_t p = gtid + GT * j;
            const bool in = p < XP && k0 + 8 * (p % 8) < ke;
            xr[j] = in ? *reinterpret_cast<const uint4 *>(xp[j] + k0) : uint4{0u, 0u, 0u, 0u};
        }
    };
    auto fetch_w = [&](uint32_t k0, uint4(&f)[2][3]) {
#pragma unroll
        for (int hs = 0; hs < 2; ++hs) {
            const bool in = k0 + 32 * hs < ke;
#pragma unroll
            for (int b = 0; b < 3; ++b)
                f[hs][b] = in ? *reinterpret_cast<const uint4 *>(wp[b] + (k0 / 32 + hs) * 512)
                              : uint4{0u, 0u, 0u, 0u};
        }
    };
    auto stage = [&](int buf) {
#pragma unroll
        for (int j = 0; j < PPT; ++j) {
            const uint32_t p = gtid + GT * j;
            if (p < XP) {
                *reinterpret_cast<uint4 *>(&sx[buf * XB + (p / 8) * LROW + 8 * (p % 8)]) = xr[j];
                const uint32_t v[4] = {xr[j].x, xr[j].y, xr[j].z, xr[j].w};
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    const double lo = (double)__uint_as_float(v[e] << 16);
                    const double hi = (double)__uint_as_float(v[e] & 0xFFFF0000u);
                    ss[j] += lo * lo + hi * hi;
                }
            }
        }
    };

    if (nst > 0) {
        fetch_x(kb);
        fetch_w(kb, wf);
        stage(0);
    }
    __syncthreads();

    f32x4 acc[MR][3], prt[MR][3];
#pragma unroll
    for (int a = 0; a < MR; ++a)
#pragma unroll
        for (int b = 0; b < 3; ++b) {
            acc[a][b] = f32x4{0.f, 0.f, 0.f, 0.f};
            prt[a][b] = f32x4{0.f, 0.f, 0.f, 0.f};
        }
    for (uint32_t st = 0; st < nmax; ++st) {
        // every group passes every barrier; a group past its last step idles
        const bool act = st < nst;
        const bool more = st + 1 < nst;
        const uint32_t k0 = kb + st * LK;
        if (more) {
            fetch_x(k0 + LK);
            fetch_w(k0 + LK, wn);
        }
        if (act) {
            const uint16_t *cx = sx + (st & 1) * XB;
#pragma unroll
            for (int hs = 0; hs < 2; ++hs) {
                if (k0 + 32 * hs < ke) {  // uniform: ke is a multiple of 32
                    bf16x8 fa[MR];
#pragma unroll
                    for (int a = 0; a < MR; ++a)
                        fa[a] = __builtin_bit_cast(
                            bf16x8,
                            *reinterpret_cast<const uint4 *>(&cx[(16 * a + lr) * LROW + 32 * hs + lk]));
#pragma unroll
                    for (int a = 0; a < MR; ++a)
#pragma unroll
                        for (int b = 0; b < 3; ++b)
                            prt[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(
                                fa[a], __builtin_bit_cast(bf16x8, wf[hs][b]), prt[a][b], 0, 0, 0);
                }
            }
            if ((k0 + LK - kb) % LCHK == 0 || !more) {
                // close the chunk: one fp32 addition per output
#pragma unroll
                for (int a = 0; a < MR; ++a)
#pragma unroll
                    for (int b = 0; b < 3; ++b) {
#pragma unroll
                        for (int i = 0; i < 4; ++i) acc[a][b][i] += prt[a][b][i];
                        prt[a][b] = f32x4{0.f, 0.f, 0.f, 0.f};
                    }
            }
        }
        if (more) {
            stage((st + 1) & 1);
#pragma unroll
            for (int hs = 0; hs < 2; ++hs)
#pragma unroll
                for (int b = 0; b < 3; ++b) wf[hs][b] = wn[hs][b];
        }
        __syncthreads();
    }

    // row norms: the 8 lanes holding one row's pieces are adjacent; the
    // groups' sums are added in group order
#pragma unroll
    for (int j = 0; j < PPT; ++j) {
        double v = ss[j];
        v += __shfl_xor(v, 1, 64);
        v += __shfl_xor(v, 2, 64);
        v += __shfl_xor(v, 4, 64);
        const uint32_t p = gtid + GT * j;
        if (p < XP && p % 8 == 0) snx2[kg * TM + p / 8] = v;
    }
    // the group sums (the row buffers are free: every group left the loop)
    if (KS > 1 && kg > 0) {
        float *pp = part + (size_t)(kg - 1) * TM * FW * NW + (size_t)cw * MR * 3 * 4 * 64;
#pragma unroll
        for (int a = 0; a < MR; ++a)
#pragma unroll
            for (int b = 0; b < 3; ++b)
#pragma unroll
                for (int i = 0; i < 4; ++i) pp[((a * 3 + b) * 4 + i) * 64 + lane] = acc[a][b][i];
    }
    __syncthreads();
    if (tid < TM) {
        double v = 0.0;
#pragma unroll
        for (int q = 0; q < KS; ++q) v += snx2[q * TM + tid];
        snx[tid] = (float)sqrt(v);
    }
    if (KS > 1 && kg == 0) {
#pragma unroll
        for (int q = 1; q < KS; ++q) {
            const float *pp = part + (size_t)(q - 1) * TM * FW * NW + (size_t)cw * MR * 3 * 4 * 64;
#pragma unroll
            for (int a = 0; a < MR; ++a)
#pragma unroll
                for (int b = 0; b < 3; ++b)
#pragma unroll
                    for (int i = 0; i < 4; ++i) acc[a][b][i] += pp[((a * 3 + b) * 4 + i) * 64 + lane];
        }
    }
    __syncthreads();

    // trusted signs and flags (group 0), 16 hyperplanes per ballot group
    if (kg == 0) {
#pragma unroll
        for (int b = 0; b < 3; ++b) {
            const uint32_t hr = FW * cw + 16 * b + lr;
            const bool cv = hr < gcols;
            const float wn_ = nw[h0 + (cv ? hr : 0u)];
#pragma unroll
            for (int a = 0; a < MR; ++a) {
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    const uint32_t rl = 16 * a + 4 * (lane / 16) + i;
                    const float v = acc[a][b][i];
                    if (proj && cv && r0 + rl < n) proj[(r0 + rl) * H + h0 + hr] = v;
                    const float tau = gamma * snx[rl] * wn_ + tau_abs;
                    const bool ok = cv && fabsf(v) > tau;
                    const unsigned long long mb = __ballot(ok && v > 0.f);
                    const unsigned long long mf = __ballot(cv && !ok);
                    if (lr == 0) {
                        const int q = lane / 16;
                        sb16[rl * 2 * FWRD + 3 * cw + b] = (uint16_t)(mb >> (16 * q));
                        sf16[rl * 2 * FWRD + 3 * cw + b] = (uint16_t)(mf >> (16 * q));
                    }
                }
            }
        }
    }
    __syncthreads();

    // recheck: wavefront w takes rows w, w + NW*KS, ...; a row's sign words
    // are changed by its wavefront's lane 0 only
    const uint32_t nrow = (n - r0 < (uint64_t)TM) ? (uint32_t)(n - r0) : (uint32_t)TM;
    const uint32_t gw = (gcols + 31) / 32;
    unsigned long long nflag = 0, nexact = 0;
    for (uint32_t rl = wave; rl < nrow; rl += NWV) {
        // only the group's gcols bits: the ballots leave the upper half of
        // the last word unwritten when gcols / 16 is odd
        uint32_t fw = 0u;
        if ((uint32_t)lane < gw) {
            fw = sflag[rl * FWRD + lane];
            const uint32_t nb = gcols - 32u * (uint32_t)lane;
            if (nb < 32u) fw &= (1u << nb) - 1u;
        }
        unsigned long long any = __ballot(fw != 0);
        const uint16_t *xrow = x + (r0 + rl) * ld;
        while (any) {
            const int src = __ffsll((long long)any) - 1;
            any &= any - 1;
            uint32_t word = (uint32_t)__shfl((int)fw, src, 64);
            while (word) {
                const int bit = __ffs(word) - 1;
                word &= word - 1;
                const uint32_t hr = (uint32_t)src * 32 + bit;
                const uint16_t *wh = w + (uint64_t)(h0 + hr) * dpad;
                double v = 0.0, a = 0.0;
#pragma unroll 8
                for (uint32_t i = 8 * lane; i < d; i += 512) {
                    const uint4 xv = *reinterpret_cast<const uint4 *>(xrow + i);
                    const uint4 wv = *reinterpret_cast<const uint4 *>(wh + i);
                    const uint32_t xs4[4] = {xv.x, xv.y, xv.z, xv.w};
                    const uint32_t ws4[4] = {wv.x, wv.y, wv.z, wv.w};
#pragma unroll
                    for (int e = 0; e < 4; ++e) {
                        const double x0 = (double)__uint_as_float(xs4[e] << 16);
                        const double x1 = (double)__uint_as_float(xs4[e] & 0xFFFF0000u);
                        const double w0 = (double)__uint_as_float(ws4[e] << 16);
                        const double w1 = (double)__uint_as_float(ws4[e] & 0xFFFF0000u);
                        const double p0 = x0 * w0, p1 = x1 * w1;
                        v += p0;
                        v += p1;
                        a += fabs(p0);
                        a += fabs(p1);
                    }
                }
                v = wave_sum_f64(v);
                a = wave_sum_f64(a);
                int sgn;
                // the butterfly sums are bit-identical in every lane; lane
                // 0's verdict keeps the branch uniform by construction
                if (__builtin_amdgcn_readfirstlane(fabs(v) > 2.0 * (double)d * 0x1p-53 * a ? 1 : 0)) {
                    sgn = v > 0.0 ? 1 : -1;
                } else {
                    sgn = exact_sign_wave(x, false, r0 + rl, d, ld, wh);
                    ++nexact;
                }
                if (lane == 0) {
                    const uint32_t m = 1u << bit;
                    if (sgn > 0)
                        sbits[rl * FWRD + src] |= m;
                    else
                        sbits[rl * FWRD + src] &= ~m;
                }
                ++nflag;
            }
        }
    }
    if (ctr && lane == 0) {
        if (nflag) atomicAdd(&ctr[0], nflag);
        if (nexact) atomicAdd(&ctr[1], nexact);
    }
    __syncthreads();

    // codes of the group's tables (K <= 24 bits, within two words)
    for (uint32_t idx = tid; idx < nrow * ntab; idx += 64 * NWV) {
        const uint32_t rl = idx / ntab, t = idx - rl * ntab;
        const uint32_t b0 = t * K, wi = b0 / 32, sh = b0 % 32;
        uint64_t v = sbits[rl * FWRD + wi];
        if (sh + K > 32) v |= (uint64_t)sbits[rl * FWRD + wi + 1] << 32;
        codes[(r0 + rl) * L + t0 + t] = (uint32_t)((v >> sh) & ((1ull << K) - 1));
    }
}

// ---------------------------------------------------------------------------
// Roundings a product can pass through: one long chain of 3 * dpad terms for
// the fp32 kernel (three bf16 planes); chunked for the fused kernel (bf16).
// gamma_m = m u / (1 - m u) with u = 2^-23, widened by 2^-6 for the fp32
// rounding of the two norms and of gamma itself; the absolute term covers
// products and partial sums that the matrix cores flush below 2^-126.
void srp_bound(const Index &ix, double *gamma, double *tau_abs) {
    const int nsplit = ix.p.family == FLINNG_SRP_F32 ? 3 : 1;
    const double nterms =
        nsplit == 1 ? (double)srp_lds_terms(ix.dpad) : (double)nsplit * ix.dpad;
    const double u = 0x1p-23;
    *gamma = nterms * u / (1.0 - nterms * u) * (1.0 + 0x1p-6);
    *tau_abs = (double)nsplit * ix.dpad * 0x1p-100;
}

// bf16 rows are projected in place (no operand planes) when d is a multiple
// of 32 and the rows start 16-byte aligned.
static bool srp_inplace(const Index &ix, const void *xdev) {
    return ix.p.family == FLINNG_SRP_BF16 && ix.p.dim == ix.dpad &&
           (reinterpret_cast<uintptr_t>(xdev) & 15) == 0;
}

// How srp_fused_kernel covers n rows: MR (tile rows / 16), NW (column
// wavefronts), KS (k groups) and gt (tables per group), from a model fitted
// to kernel traces on MI355X (ReLU embeddings, d = 4096, K*L = 288 and 1024,
// batches of 128 to 65,536 rows: at every size measured its plan is within
// 16% of the best one, and the best one from 8,192 rows up).  A workgroup
// takes steps = 2 ceil(nch / KS) 64-wide steps, each about 0.2 us + 0.1 us
// per KB that one wavefront loads in it (its share of the rows and its 48
// hyperplanes: TM / (8 NW) + 6 KB), longer by 4% per further wavefront of
// the workgroup (they step together) in proportion to how full the chip is.
// Workgroups run in rounds of 256 times the number a compute unit holds (8,
// 12 or 16 wavefronts for MR = 4, 2, 1).  The grid's loads take at least
// their bytes at 10 TB/s, counting each row once per row tile (the table
// groups of a tile run on one XCD and share its L2) and the hyperplanes once
// per workgroup; plus a fixed 4 us.  Within 2% the plan with more workgroups
// wins.  KS needs nch >= 2 KS (the rounding bound).
struct SrpPlan {
    int mr, nw, ks;
    uint32_t gt;
    uint64_t wgs;
};

// The compiled variants: KS = 8 only with one column wavefront and tiles of
// at most 32 rows (the row buffers of 8 groups).
static bool srp_variant(int mr, int nw, int ks) {
    return ks == 1 || (ks == 2 && nw <= 4) || (ks == 4 && nw <= 2) || (ks == 8 && nw == 1 && mr <= 2);
}

static SrpPlan srp_plan(uint32_t K, uint32_t L, uint64_t n, uint32_t d) {
    static const int NWS[] = {1, 2, 3, 4, 6};
    static const int MRS[] = {1, 2, 4};
    static const int KSS[] = {1, 2, 4, 8};
    const double A = 0.2e-6, B = 0.1e-6, C = 0.04, BWG = 10e12, FIX = 4e-6;
    const uint32_t nch = (d + LCHK - 1) / LCHK;
    SrpPlan best{4, FMAXW, 1, 1, 0};
    double best_t = -1.0;
    for (int mr : MRS) {
        const uint64_t tm = 16 * (uint64_t)mr, nrt = (n + tm - 1) / tm;
        const int wcu = mr == 4 ? 8 : (mr == 2 ? 12 : 16);
        for (uint32_t ng = 1; ng <= L; ++ng) {
            const uint32_t gt = (L + ng - 1) / ng;
            if ((L + gt - 1) / gt != ng || gt * K > (uint32_t)FMAXH) continue;
            const uint32_t need = (gt * K + FW - 1) / FW;
            int nw = FMAXW;
            for (int c : NWS)
                if ((uint32_t)c >= need) {
                    nw = c;
                    break;
                }
            for (int ks : KSS) {
                if (!srp_variant(mr, nw, ks) || (ks > 1 && nch < 2u * ks)) continue;
                const uint64_t wgs = nrt * ng;
                const double steps = 2.0 * ((nch + ks - 1) / ks);
                const double kbw = (double)tm / (8.0 * nw) + 6.0;
                const uint64_t occ = (uint64_t)std::max(1, wcu / (nw * ks));
                const double rounds = (double)((wgs + 256 * occ - 1) / (256 * occ));
                const double bytes = 2.0 * d * (double)(nrt * tm + wgs * (uint64_t)(FW * nw));
                const double load = std::min(1.0, (double)wgs / (256.0 * (double)occ));
                const double step = (A + B * kbw) * (1.0 + C * (nw * ks - 1) * load);
                const double t = std::max(rounds * steps * step, bytes / BWG) + FIX;
                // within 2% of the best so far, the plan with more workgroups
                // (the bandwidth bound ties plans the traces tell apart)
                if (best_t < 0.0 || t < 0.98 * best_t || (t <= 1.02 * best_t && wgs > best.wgs)) {
                    best = SrpPlan{mr, nw, ks, gt, wgs};
                    best_t = t;
                }
            }
        }
    }
    return best;
}

struct SrpFusedArgs {
    const uint16_t *x;
    uint32_t ld, d;
    const Index *ix;
    uint64_t n;
    float gamma, tau_abs;
    uint32_t *codes;
    unsigned long long *ctr;
    float *proj;
};

template <int MR, int NW, int KS>
static void srp_launch(const SrpPlan &pl, const SrpFusedArgs &a, hipStream_t s) {
    constexpr size_t lds = FusedShape<MR, NW, KS>::LDS;
    // once per variant and process (a throwing initialiser is retried)
    static const bool attrs_ok = [] {
        const void *fn = reinterpret_cast<const void *>(&srp_fused_kernel<MR, NW, KS>);
        if (hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds) !=
            hipSuccess)
            fail(FLINNG_EDEVICE, "SRP kernel: its LDS does not fit");
        return true;
    }();
    (void)attrs_ok;
    hipLaunchKernelGGL((srp_fused_kernel<MR, NW, KS>), dim3((unsigned)pl.wgs), dim3(64 * NW * KS),
                       lds, s, a.x, a.ld, a.d, a.ix->hyp, a.ix->hypt, a.ix->dpad, a.ix->hypnorm, a.n,
                       a.ix->p.K, a.ix->p.L, pl.gt, a.gamma, a.tau_abs, a.codes, a.ctr, a.proj);
}

template <int MR, int KS>
static void srp_launch_nw(const SrpPlan &pl, const SrpFusedArgs &a, hipStream_t s) {
    if constexpr (KS == 1) {
        switch (pl.nw) {
            case 1: srp_launch<MR, 1, 1>(pl, a, s); break;
            case 2: srp_launch<MR, 2, 1>(pl, a, s); break;
            case 3: srp_launch<MR, 3, 1>(pl, a, s); break;
            case 4: srp_launch<MR, 4, 1>(pl, a, s); break;
            default: srp_launch<MR, 6, 1>(pl, a, s); break;
        }
    } else if constexpr (KS == 2) {
        switch (pl.nw) {
            case 1: srp_launch<MR, 1, 2>(pl, a, s); break;
            case 2: srp_launch<MR, 2, 2>(pl, a, s); break;
            case 3: srp_launch<MR, 3, 2>(pl, a, s); break;
            default: srp_launch<MR, 4, 2>(pl, a, s); break;
        }
    } else if constexpr (KS == 4) {
        if (pl.nw == 1)
            srp_launch<MR, 1, 4>(pl, a, s);
        else
            srp_launch<MR, 2, 4>(pl, a, s);
    } else if constexpr (MR <= 2) {
        srp_launch<MR, 1, 8>(pl, a, s);
    } else {
        fail(FLINNG_EDEVICE, "internal: no SRP kernel variant for the plan");
    }
}

template <int MR>
static void srp_launch_ks(const SrpPlan &pl, const SrpFusedArgs &a, hipStream_t s) {
    switch (pl.ks) {
        case 1: srp_launch_nw<MR, 1>(pl, a, s); break;
        case 2: srp_launch_nw<MR, 2>(pl, a, s); break;
        case 4: srp_launch_nw<MR, 4>(pl, a, s); break;
        default: srp_launch_nw<MR, 8>(pl, a, s); break;
    }
}

__global__ void srp_zero_ctr_kernel(unsigned long long *ctr) {
    if (threadIdx.x < 2) ctr[threadIdx.x] = 0ull;
}

size_t srp_scratch_bytes(const Index &ix, uint64_t n, const void *xdev) {
    const bool planes = !(xdev && srp_inplace(ix, xdev));
    if (ix.p.family != FLINNG_SRP_F32)
        return (planes ? Arena::round((size_t)n * ix.dpad * 2) : 0) + Arena::round(16);
    const uint64_t Hw = ((uint64_t)ix.p.K * ix.p.L + 31) / 32;
    return Arena::round((size_t)3 * n * ix.dpad * 2) + Arena::round(n * 4) +
           2 * Arena::round(n * Hw * 4) + Arena::round(16);
}

void srp_hash(const Index &ix, const flinng_input &in, uint32_t *codes_dev, hipStream_t s,
              uint64_t *counters_host, Arena *ws, float *proj_dev) {
    const uint64_t n = in.count;
    if (n == 0) return;
    const uint32_t d = ix.p.dim, dpad = ix.dpad;
    const uint32_t K = ix.p.K, L = ix.p.L, H = K * L;
    const uint32_t Hw = (H + 31) / 32;
    const bool f32 = ix.p.family == FLINNG_SRP_F32;
    Scratch sc(ws, s);

    // stage values on the device (host inputs never come with an arena)
    const size_t esz = f32 ? 4 : 2;
    const void *xdev = in.values;
    DevBuf xcopy;
    if (!in.on_device) {
        xcopy = DevBuf(n * d * esz, s);
        FL_HIP(hipMemcpyAsync(xcopy.ptr, in.values, n * d * esz, hipMemcpyHostToDevice, s));
        xdev = xcopy.ptr;
    }
    double gam = 0.0, tabs = 0.0;
    srp_bound(ix, &gam, &tabs);
    const float gamma = (float)gam;
    const float tau_abs = (float)tabs;

    if (!f32) {
        // bf16 rows: one fused kernel, on the rows in place or on a padded
        // copy (zeros past d, which add nothing to any sum)
        const bool inplace = srp_inplace(ix, xdev);
        uint16_t *planes = sc.get<uint16_t>(inplace ? 0 : (size_t)n * dpad * 2);
        // counters only when asked for (the kernel skips them otherwise)
        unsigned long long *ctr = counters_host ? sc.get<unsigned long long>(16) : nullptr;
        if (ctr) {
            hipLaunchKernelGGL(srp_zero_ctr_kernel, dim3(1), dim3(64), 0, s, ctr);
            FL_CHECK_LAUNCH();
        }
        if (!inplace) {
            hipLaunchKernelGGL(prep_kernel<false>, dim3((unsigned)((n + 3) / 4)), dim3(256), 0, s,
                               xdev, n, d, dpad, planes, nullptr, nullptr, nullptr, 0u, nullptr);
            FL_CHECK_LAUNCH();
        }
        const SrpPlan pl = srp_plan(K, L, n, dpad);
        if (pl.wgs > 0x7FFFFFFFull) fail(FLINNG_EINVAL, "SRP batch too large for one launch");
        const SrpFusedArgs a{inplace ? static_cast<const uint16_t *>(xdev) : planes,
                             dpad, dpad, &ix, n, gamma, tau_abs, codes_dev,
                             ctr, proj_dev};
        switch (pl.mr) {
            case 1: srp_launch_ks<1>(pl, a, s); break;
            case 2: srp_launch_ks<2>(pl, a, s); break;
            default: srp_launch_ks<4>(pl, a, s); break;
        }
        FL_CHECK_LAUNCH();
        if (counters_host) {
            unsigned long long c[2];
            FL_HIP(hipMemcpyAsync(c, ctr, 16, hipMemcpyDeviceToHost, s));
            FL_HIP(hipStreamSynchronize(s));
            counters_host[0] = c[0];
            counters_host[1] = c[1];
        }
        return;
    }

    // fp32 rows: three bf16 planes, srp_mfma_kernel, then recheck + pack
    uint16_t *planes = sc.get<uint16_t>((size_t)3 * n * dpad * 2);
    float *nx = sc.get<float>(n * 4);
    uint32_t *bits = sc.get<uint32_t>(n * Hw * 4);
    uint32_t *flags = sc.get<uint32_t>(n * Hw * 4);
    unsigned long long *ctr = sc.get<unsigned long long>(16);
    hipLaunchKernelGGL(prep_kernel<true>, dim3((unsigned)((n + 3) / 4)), dim3(256), 0, s, xdev, n,
                       d, dpad, planes, nx, bits, flags, Hw, ctr);
    FL_CHECK_LAUNCH();
    constexpr int MR = 4, NR = 4, WM = 2, WN = 2;
    dim3 grid((H + 16 * NR * WN - 1) / (16 * NR * WN),
              (unsigned)((n + 16 * MR * WM - 1) / (16 * MR * WM)));
    hipLaunchKernelGGL((srp_mfma_kernel<MR, NR, WM, WN, 3>), grid, dim3(64 * WM * WN), 0, s,
                       planes, (uint64_t)n * dpad, dpad, ix.hyp, dpad, nx, ix.hypnorm, n, H, Hw,
                       gamma, tau_abs, reinterpret_cast<uint16_t *>(bits),
                       reinterpret_cast<uint16_t *>(flags), ctr, proj_dev);
    FL_CHECK_LAUNCH();
    hipLaunchKernelGGL(srp_recheck_pack_kernel, dim3((unsigned)((n + 3) / 4)), dim3(256),
                       4 * Hw * sizeof(uint32_t), s, xdev, 1, n, d, ix.hyp, dpad, bits, flags, Hw,
                       H, K, L, codes_dev, ctr + 1);
    FL_CHECK_LAUNCH();
    if (counters_host) {
        unsigned long long c[2];
        FL_HIP(hipMemcpyAsync(c, ctr, 16, hipMemcpyDeviceToHost, s));
        FL_HIP(hipStreamSynchronize(s));
        counters_host[0] = c[0];
        counters_host[1] = c[1];
    }
}

}  // namespace flinng
