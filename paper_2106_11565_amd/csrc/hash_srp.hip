// Signed random projection hashing on gfx950.
//
// The dense LSH of the method (Section 3, Locality-Sensitive Hashing, and the
// concatenation trick): bit j of table t is 1 iff the exact dot product of
// the row with hyperplane h = t*K + j is positive (an exact zero gives 0);
// the table's bucket is sum_j bit_j 2^j.  Hashing is shared by every filter
// and done once per point or query (Section 6, Implementation).
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

void srp_make_hyperplanes(Index &ix, hipStream_t s) {
    const uint32_t H = ix.p.L * ix.p.K;
    uint64_t total = (uint64_t)H * ix.dpad;
    hipLaunchKernelGGL(hyp_kernel, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s,
                       ix.hyp, H, ix.p.dim, ix.dpad, sm64(ix.p.seed, TAG_HYP));
    FL_CHECK_LAUNCH();
    hipLaunchKernelGGL(hypnorm_kernel, dim3((H + 3) / 4), dim3(256), 0, s, ix.hyp,
                       ix.hypnorm, H, ix.dpad);
    FL_CHECK_LAUNCH();
}

// ---------------------------------------------------------------------------
// Prep: one wavefront per row.  Writes nsplit bf16 planes [n][dpad] (unless
// planes == nullptr) and the row norm, rounded to fp32.  fp32 values are
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
    if (row == 0 && lane < 2) ctr[lane] = 0ull;
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
        if (lane == 0) nx[row] = (float)sqrt(s);
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
    if (lane == 0) nx[row] = (float)sqrt(s);
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

// The same products for one bf16 operand plane with both operands staged in
// LDS: a 256-thread workgroup computes a 128 x 128 tile (four wavefronts of
// 64 x 64); each 32-wide k slice of the 128 rows and the 128 hyperplanes is
// loaded once per workgroup (two 16-byte loads per thread and operand),
// prefetched into registers while the previous slice is multiplied, and
// double-buffered in LDS with rows padded against bank conflicts.
// Accumulation is chunked: every LCH consecutive slices accumulate into a
// fresh partial (MFMA accumulate), and the partials are added in fp32 by the
// wavefront.  A product then passes through at most LCH*32 roundings inside
// its chunk (whatever order an instruction sums its 32 products and its
// accumulator in) plus one per chunk, so |v32 - v| <= gamma_m * sum|x_i w_i|
// with m = min(LCH*32, d) + ceil(d / (LCH*32)) (srp_lds_terms), far below
// the gamma_d of one long accumulation chain.
constexpr int LT = 128;          // tile rows and hyperplanes
constexpr int LK = 32;           // k slice
constexpr int LROW = LK + 8;     // bf16 per LDS row (16 bytes of padding)
constexpr int LCH = 4;           // slices per accumulation chunk

// Roundings a product passes through in srp_mfma_lds_kernel (see above).
inline uint32_t srp_lds_terms(uint32_t dpad) {
    const uint32_t chunk = LCH * LK;
    return (dpad < chunk ? dpad : chunk) + (dpad + chunk - 1) / chunk;
}

__global__ __launch_bounds__(256, 2) void srp_mfma_lds_kernel(
    const uint16_t *__restrict__ planes, uint32_t ld, const uint16_t *__restrict__ w,
    uint32_t dpad, const float *__restrict__ nx, const float *__restrict__ nw, uint64_t n,
    uint32_t H, uint32_t Hw, float gamma, float tau_abs, uint16_t *__restrict__ bits16,
    uint16_t *__restrict__ flags16, unsigned long long *__restrict__ nflag,
    float *__restrict__ proj) {
    __shared__ __align__(16) uint16_t sa[2][LT * LROW];
    __shared__ __align__(16) uint16_t sb[2][LT * LROW];
    const int tid = threadIdx.x, lane = tid % 64, wave = tid / 64;
    const int wm = wave / 2, wn = wave % 2;
    const uint64_t tr0 = (uint64_t)blockIdx.y * LT;
    const uint32_t tc0 = blockIdx.x * LT;

    // this thread's two 16-byte pieces of each operand slice: piece u covers
    // tile row u / 4, k offset 8 * (u % 4), for u = tid and tid + 256 (named
    // registers and no branches, so the prefetch stays in registers)
    const int u0 = tid, u1 = tid + 256;
    const int rr0 = u0 / 4, rr1 = u1 / 4, kk0 = 8 * (u0 % 4), kk1 = 8 * (u1 % 4);
    const uint64_t r0 = (tr0 + rr0 < n) ? tr0 + rr0 : n - 1;
    const uint64_t r1 = (tr0 + rr1 < n) ? tr0 + rr1 : n - 1;
    const uint32_t c0 = (tc0 + rr0 < H) ? tc0 + rr0 : H - 1;
    const uint32_t c1 = (tc0 + rr1 < H) ? tc0 + rr1 : H - 1;
    const uint16_t *ga0 = planes + r0 * ld + kk0;
    const uint16_t *ga1 = planes + r1 * ld + kk1;
    const uint16_t *gb0 = w + (uint64_t)c0 * dpad + kk0;
    const uint16_t *gb1 = w + (uint64_t)c1 * dpad + kk1;
    const int so0 = rr0 * LROW + kk0, so1 = rr1 * LROW + kk1;

    uint4 ra0 = *reinterpret_cast<const uint4 *>(ga0);
    uint4 ra1 = *reinterpret_cast<const uint4 *>(ga1);
    uint4 rb0 = *reinterpret_cast<const uint4 *>(gb0);
    uint4 rb1 = *reinterpret_cast<const uint4 *>(gb1);
    *reinterpret_cast<uint4 *>(&sa[0][so0]) = ra0;
    *reinterpret_cast<uint4 *>(&sa[0][so1]) = ra1;
    *reinterpret_cast<uint4 *>(&sb[0][so0]) = rb0;
    *reinterpret_cast<uint4 *>(&sb[0][so1]) = rb1;
    __syncthreads();

    f32x4 acc[4][4], part[4][4];
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) {
            acc[a][b] = f32x4{0.f, 0.f, 0.f, 0.f};
            part[a][b] = f32x4{0.f, 0.f, 0.f, 0.f};
        }
    const int lr = lane % 16, lk = (lane / 16) * 8;

    for (uint32_t k0 = 0; k0 < dpad; k0 += LK) {
        const uint32_t step = k0 / LK;
        const int cur = step & 1;
        // next slice (the last iteration reloads its own slice into the
        // buffer nobody reads any more)
        const uint32_t kn = (k0 + LK < dpad) ? k0 + LK : k0;
        ra0 = *reinterpret_cast<const uint4 *>(ga0 + kn);
        ra1 = *reinterpret_cast<const uint4 *>(ga1 + kn);
        rb0 = *reinterpret_cast<const uint4 *>(gb0 + kn);
        rb1 = *reinterpret_cast<const uint4 *>(gb1 + kn);
        const uint16_t *ca = sa[cur];
        const uint16_t *cb = sb[cur];
        bf16x8 fa[4], fb[4];
#pragma unroll
        for (int a = 0; a < 4; ++a)
            fa[a] = __builtin_bit_cast(
                bf16x8, *reinterpret_cast<const uint4 *>(&ca[(wm * 64 + 16 * a + lr) * LROW + lk]));
#pragma unroll
        for (int b = 0; b < 4; ++b)
            fb[b] = __builtin_bit_cast(
                bf16x8, *reinterpret_cast<const uint4 *>(&cb[(wn * 64 + 16 * b + lr) * LROW + lk]));
#pragma unroll
        for (int a = 0; a < 4; ++a)
#pragma unroll
            for (int b = 0; b < 4; ++b)
                part[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(fa[a], fb[b], part[a][b], 0, 0, 0);
        if ((step + 1) % LCH == 0 || k0 + LK >= dpad) {
            // close the chunk: one fp32 addition per output
#pragma unroll
            for (int a = 0; a < 4; ++a)
#pragma unroll
                for (int b = 0; b < 4; ++b) {
#pragma unroll
                    for (int i = 0; i < 4; ++i) acc[a][b][i] += part[a][b][i];
                    part[a][b] = f32x4{0.f, 0.f, 0.f, 0.f};
                }
        }
        uint16_t *na = sa[cur ^ 1];
        uint16_t *nb = sb[cur ^ 1];
        *reinterpret_cast<uint4 *>(&na[so0]) = ra0;
        *reinterpret_cast<uint4 *>(&na[so1]) = ra1;
        *reinterpret_cast<uint4 *>(&nb[so0]) = rb0;
        *reinterpret_cast<uint4 *>(&nb[so1]) = rb1;
        __syncthreads();
    }

    // Epilogue: trusted sign bits and flags, 16 columns per ballot group.
    const uint64_t row0 = tr0 + (uint64_t)wm * 64;
    const uint32_t col0 = tc0 + wn * 64;
    unsigned long long flagged = 0;
#pragma unroll
    for (int b = 0; b < 4; ++b) {
        const uint32_t cbase = col0 + 16 * b;
        if (cbase >= H) continue;
        const uint32_t col = cbase + lr;
        const float wn_ = (col < H) ? nw[col] : 0.f;
#pragma unroll
        for (int a = 0; a < 4; ++a) {
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
// fixed-point number spanning 2^-160 .. 2^224 (int64 digits absorb carries
// for up to 2^30 terms), then carries are propagated and the sign read from
// the top.  Runs on one lane; reached only for near-exact cancellations.
__device__ int exact_sign_fixed(const void *xin, bool f32, uint64_t row, uint32_t d,
                                const uint16_t *__restrict__ wh) {
    constexpr int NLIMB = 12;
    constexpr int BASE = -160;
    long long limb[NLIMB];
    for (int j = 0; j < NLIMB; ++j) limb[j] = 0;
    for (uint32_t i = 0; i < d; ++i) {
        double xv = f32 ? (double)static_cast<const float *>(xin)[row * d + i]
                        : (double)bf16_to_f32(static_cast<const uint16_t *>(xin)[row * d + i]);
        double p = xv * (double)bf16_to_f32(wh[i]);
        if (p == 0.0) continue;
        unsigned long long bits = (unsigned long long)__double_as_longlong(p);
        bool neg = bits >> 63;
        int ex = (int)((bits >> 52) & 0x7FF);
        unsigned long long m = bits & ((1ull << 52) - 1);
        int pos;
        if (ex == 0) {
            pos = -1074;
        } else {
            m |= (1ull << 52);
            pos = ex - 1075;
        }
        while ((m & 1ull) == 0) {
            m >>= 1;
            ++pos;
        }
        int sh = pos - BASE;  // >= 9 for the supported inputs
        int j = sh / 32, o = sh % 32;
        // m < 2^31 after stripping: (m << o) < 2^63
        unsigned long long v = m << o;
        long long lo = (long long)(v & 0xFFFFFFFFull), hi = (long long)(v >> 32);
        if (neg) {
            lo = -lo;
            hi = -hi;
        }
        limb[j] += lo;
        if (j + 1 < NLIMB) limb[j + 1] += hi;
    }
    for (int j = 0; j < NLIMB - 1; ++j) {
        long long c = limb[j] >> 32;  // arithmetic shift: floor division
        limb[j] -= c * (1ll << 32);
        limb[j + 1] += c;
    }
    if (limb[NLIMB - 1] != 0) return limb[NLIMB - 1] > 0 ? 1 : -1;
    for (int j = NLIMB - 2; j >= 0; --j)
        if (limb[j] != 0) return 1;
    return 0;
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
                if (fabs(v) > 2.0 * (double)d * 0x1p-53 * a) {
                    sgn = v > 0.0 ? 1 : -1;
                } else {
                    sgn = 0;
                    if (lane == 0) {
                        sgn = exact_sign_fixed(xin, f32 != 0, row, d, wh);
                        atomicAdd(nexact, 1ull);
                    }
                    sgn = __shfl(sgn, 0, 64);
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

// Recheck + pack for bf16 rows read in place (d a multiple of 32, rows
// 16-byte aligned).  One wavefront per row: its flagged hyperplanes are
// listed in LDS, then recomputed four at a time, 16 lanes each, with 16-byte
// loads of 8 bf16 values of the row and of the hyperplane and FP64 partial
// sums reduced within the 16 lanes.  Same certificate and exact fallback as
// srp_recheck_pack_kernel.
__global__ __launch_bounds__(256) void srp_recheck_pack_vec_kernel(
    const uint16_t *__restrict__ x, uint64_t n, uint32_t d, const uint16_t *__restrict__ w,
    const uint32_t *__restrict__ bits, const uint32_t *__restrict__ flags, uint32_t Hw,
    uint32_t H, uint32_t K, uint32_t L, uint32_t *__restrict__ codes,
    unsigned long long *__restrict__ nexact) {
    extern __shared__ uint32_t sm[];
    const int lane = threadIdx.x % 64;
    const int wave = threadIdx.x / 64;
    const uint64_t row = (uint64_t)blockIdx.x * (blockDim.x / 64) + wave;
    if (row >= n) return;
    const uint32_t per_wave = Hw + (Hw * 32) / 2;  // bit words + uint16 flagged list
    uint32_t *rb = sm + wave * per_wave;
    uint16_t *fl = reinterpret_cast<uint16_t *>(rb + Hw);
    for (uint32_t j = lane; j < Hw; j += 64) rb[j] = bits[row * Hw + j];
    // list the flagged hyperplanes (wave prefix sums over flag words)
    uint32_t nf = 0;
    for (uint32_t j0 = 0; j0 < Hw; j0 += 64) {
        const uint32_t j = j0 + lane;
        uint32_t fw = (j < Hw) ? flags[row * Hw + j] : 0u;
        const uint32_t c = (uint32_t)__popc(fw);
        uint32_t inc = c;
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
            const uint32_t y = (uint32_t)__shfl_up((int)inc, o, 64);
            if (lane >= o) inc += y;
        }
        uint32_t pos = nf + inc - c;
        while (fw) {
            const uint32_t b = (uint32_t)(__ffs(fw) - 1);
            fw &= fw - 1;
            const uint32_t h = j * 32 + b;
            if (h < H) fl[pos] = (uint16_t)h;
            ++pos;
        }
        nf += (uint32_t)__shfl((int)inc, 63, 64);
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    const int g = lane >> 4, sl = lane & 15;
    const uint16_t *xr = x + row * d;
    for (uint32_t p0 = 0; p0 < nf; p0 += 4) {
        const uint32_t p = p0 + g;
        const bool act = p < nf;
        const uint32_t h = fl[act ? p : nf - 1];
        if (h >= H) continue;  // never: flags past H are zero
        const uint16_t *wh = w + (uint64_t)h * d;
        double v = 0.0, a = 0.0;
#pragma unroll 4
        for (uint32_t i = 8 * sl; i < d; i += 128) {
            const uint4 xv = *reinterpret_cast<const uint4 *>(xr + i);
            const uint4 wv = *reinterpret_cast<const uint4 *>(wh + i);
            const uint32_t xs[4] = {xv.x, xv.y, xv.z, xv.w};
            const uint32_t ws[4] = {wv.x, wv.y, wv.z, wv.w};
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const double x0 = (double)__uint_as_float(xs[e] << 16);
                const double x1 = (double)__uint_as_float(xs[e] & 0xFFFF0000u);
                const double w0 = (double)__uint_as_float(ws[e] << 16);
                const double w1 = (double)__uint_as_float(ws[e] & 0xFFFF0000u);
                const double p0_ = x0 * w0, p1_ = x1 * w1;
                v += p0_;
                v += p1_;
                a += fabs(p0_);
                a += fabs(p1_);
            }
        }
#pragma unroll
        for (int o = 8; o > 0; o >>= 1) {
            v += __shfl_xor(v, o, 64);
            a += __shfl_xor(a, o, 64);
        }
        int sgn = 0;
        if (act && sl == 0) {
            if (fabs(v) > 2.0 * (double)d * 0x1p-53 * a) {
                sgn = v > 0.0 ? 1 : -1;
            } else {
                sgn = exact_sign_fixed(x, false, row, d, wh);
                atomicAdd(nexact, 1ull);
            }
            const uint32_t m = 1u << (h & 31);
            if (sgn > 0)
                atomicOr(&rb[h >> 5], m);
            else
                atomicAnd(&rb[h >> 5], ~m);
        }
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    for (uint32_t t = lane; t < L; t += 64) {
        const uint32_t b0 = t * K;
        const uint32_t wi = b0 / 32, sh = b0 % 32;
        uint64_t vv = rb[wi];
        if (sh + K > 32 && wi + 1 < Hw) vv |= (uint64_t)rb[wi + 1] << 32;
        codes[row * L + t] = (uint32_t)((vv >> sh) & ((K >= 32) ? 0xFFFFFFFFull : ((1ull << K) - 1)));
    }
}

// ---------------------------------------------------------------------------
// Roundings a product can pass through: one long chain of 3 * dpad terms for
// the fp32 kernel (three bf16 planes); chunked for the LDS kernel (bf16).
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

size_t srp_scratch_bytes(const Index &ix, uint64_t n, const void *xdev) {
    const uint64_t Hw = ((uint64_t)ix.p.K * ix.p.L + 31) / 32;
    const int nsplit = ix.p.family == FLINNG_SRP_F32 ? 3 : 1;
    const bool planes = !(xdev && srp_inplace(ix, xdev));
    return (planes ? Arena::round((size_t)nsplit * n * ix.dpad * 2) : 0) + Arena::round(n * 4) +
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
    const int nsplit = f32 ? 3 : 1;
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
    const bool inplace = srp_inplace(ix, xdev);
    uint16_t *planes = sc.get<uint16_t>(inplace ? 0 : (size_t)nsplit * n * dpad * 2);
    float *nx = sc.get<float>(n * 4);
    uint32_t *bits = sc.get<uint32_t>(n * Hw * 4);
    uint32_t *flags = sc.get<uint32_t>(n * Hw * 4);
    unsigned long long *ctr = sc.get<unsigned long long>(16);
    {
        dim3 grid((unsigned)((n + 3) / 4));
        if (f32)
            hipLaunchKernelGGL(prep_kernel<true>, grid, dim3(256), 0, s, xdev, n, d, dpad, planes,
                               nx, bits, flags, Hw, ctr);
        else
            hipLaunchKernelGGL(prep_kernel<false>, grid, dim3(256), 0, s, xdev, n, d, dpad,
                               inplace ? nullptr : planes, nx, bits, flags, Hw, ctr);
        FL_CHECK_LAUNCH();
    }
    const uint16_t *pl = inplace ? static_cast<const uint16_t *>(xdev) : planes;
    const uint32_t ld = inplace ? d : dpad;
    const uint64_t pstride = (uint64_t)n * dpad;

    double gam = 0.0, tabs = 0.0;
    srp_bound(ix, &gam, &tabs);
    const float gamma = (float)gam;
    const float tau_abs = (float)tabs;

    constexpr int MR = 4, NR = 4, WM = 2, WN = 2;
    dim3 grid((H + 16 * NR * WN - 1) / (16 * NR * WN),
              (unsigned)((n + 16 * MR * WM - 1) / (16 * MR * WM)));
    unsigned long long *nflag = ctr;
    if (nsplit == 3)
        hipLaunchKernelGGL((srp_mfma_kernel<MR, NR, WM, WN, 3>), grid, dim3(64 * WM * WN), 0, s,
                           pl, pstride, ld, ix.hyp, dpad, nx, ix.hypnorm, n, H, Hw, gamma, tau_abs,
                           reinterpret_cast<uint16_t *>(bits), reinterpret_cast<uint16_t *>(flags),
                           nflag, proj_dev);
    else
        hipLaunchKernelGGL(srp_mfma_lds_kernel,
                           dim3((H + LT - 1) / LT, (unsigned)((n + LT - 1) / LT)), dim3(256), 0, s,
                           pl, ld, ix.hyp, dpad, nx, ix.hypnorm, n, H, Hw, gamma, tau_abs,
                           reinterpret_cast<uint16_t *>(bits), reinterpret_cast<uint16_t *>(flags),
                           nflag, proj_dev);
    FL_CHECK_LAUNCH();
    if (inplace)
        hipLaunchKernelGGL(srp_recheck_pack_vec_kernel, dim3((unsigned)((n + 3) / 4)), dim3(256),
                           4 * (Hw + Hw * 16) * sizeof(uint32_t), s,
                           static_cast<const uint16_t *>(xdev), n, d, ix.hyp, bits, flags, Hw, H,
                           K, L, codes_dev, nflag + 1);
    else
        hipLaunchKernelGGL(srp_recheck_pack_kernel, dim3((unsigned)((n + 3) / 4)), dim3(256),
                           4 * Hw * sizeof(uint32_t), s, xdev, (int)f32, n, d, ix.hyp, dpad, bits,
                           flags, Hw, H, K, L, codes_dev, nflag + 1);
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
