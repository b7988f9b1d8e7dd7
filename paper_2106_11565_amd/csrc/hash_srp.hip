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
// 64 x 64) over one range of k.  Each 64-wide k step of the 128 rows and the
// 128 hyperplanes is loaded once per workgroup (four 16-byte loads per thread
// and operand), prefetched into registers while the previous step is
// multiplied, and double-buffered in LDS with rows padded against bank
// conflicts.  Accumulation is chunked: every 128 consecutive k accumulate into
// a fresh partial (MFMA accumulate), and the partials are added in fp32 by the
// wavefront.  A product then passes through at most 128 roundings inside its
// chunk (whatever order an instruction sums its 32 products and its
// accumulator in) plus one per chunk, so |v32 - v| <= gamma_m * sum|x_i w_i|
// with m = min(128, d) + ceil(d / 128) (srp_lds_terms), far below the gamma_d
// of one long accumulation chain.
//
// Split k: small batches give fewer tiles than the chip has compute units,
// and a long k loop is a chain of dependent steps, so the k range is cut into
// ns pieces of whole chunks, each its own workgroup, writing fp32 partial
// projections that srp_finish_kernel adds in piece order.  A product then
// passes through ceil(kpiece / 128) chunk additions and ns - 1 piece
// additions, which for kpiece a multiple of 128 is at most ceil(d / 128): the
// bound above holds unchanged.
//
// Workgroup order: the hardware hands consecutive workgroup ids to the eight
// XCDs in turn; ids are renumbered so that the column tiles of one row tile
// (which read the same rows) run on one XCD, close in time, and share its L2.
constexpr int LT = 128;          // tile rows and hyperplanes
constexpr int LK = 64;           // k per pipeline step (two 32-wide MFMA slices)
constexpr int LROW = LK + 8;     // bf16 per LDS row (16 bytes of padding)
constexpr int LCHK = 128;        // k per accumulation chunk
constexpr int LPC = LT * LK / 8 / 256;  // 16-byte pieces per thread and operand

// Roundings a product passes through in srp_mfma_lds_kernel (see above).
inline uint32_t srp_lds_terms(uint32_t dpad) {
    return (dpad < (uint32_t)LCHK ? dpad : (uint32_t)LCHK) + (dpad + LCHK - 1) / LCHK;
}

// How the LDS kernel covers n rows: tiles of 128 x 128 and k pieces.
struct SrpSplit {
    uint32_t nct, nrt, ns, kpiece;
};

static SrpSplit srp_split(uint32_t H, uint64_t n, uint32_t dpad) {
    SrpSplit sp;
    sp.nct = (H + LT - 1) / LT;
    sp.nrt = (uint32_t)((n + LT - 1) / LT);
    const uint64_t tiles = (uint64_t)sp.nct * sp.nrt;
    const uint32_t nch = (dpad + LCHK - 1) / LCHK;
    // Two workgroups fit on each of the 256 compute units.  Estimated time:
    // (rounds of resident workgroups) x (chunks per piece) x the time of one
    // chunk at full load (about 2.8 us measured), plus writing and reading
    // the fp32 partials of more than one piece (at about 5000 bytes per ns).
    constexpr uint64_t SLOTS = 512;
    constexpr double CHUNK_NS = 2800.0, NS_PER_BYTE = 1.0 / 5000.0;
    uint32_t best = 1;
    double best_cost = 0.0;
    for (uint32_t ns = 1; ns <= nch; ++ns) {
        const uint32_t cps = (nch + ns - 1) / ns;
        if (ns > 1 && (nch + cps - 1) / cps < ns) continue;  // same split as fewer pieces
        const uint64_t rounds = (tiles * ns + SLOTS - 1) / SLOTS;
        double cost = (double)rounds * cps * CHUNK_NS;
        if (ns > 1) cost += NS_PER_BYTE * 8.0 * ns * (double)n * H;
        if (ns == 1 || cost < best_cost) {
            best_cost = cost;
            best = ns;
        }
    }
    const uint32_t cps = (nch + best - 1) / best;
    sp.kpiece = cps * LCHK;
    sp.ns = (nch + cps - 1) / cps;
    return sp;
}

__global__ __launch_bounds__(256, 2) void srp_mfma_lds_kernel(
    const uint16_t *__restrict__ planes, uint32_t ld, const uint16_t *__restrict__ w,
    uint32_t dpad, const float *__restrict__ nx, const float *__restrict__ nw, uint64_t n,
    uint32_t H, uint32_t Hw, float gamma, float tau_abs, uint32_t nct, uint32_t nrt,
    uint32_t kpiece, float *__restrict__ part, uint16_t *__restrict__ bits16,
    uint16_t *__restrict__ flags16, unsigned long long *__restrict__ nflag,
    float *__restrict__ proj) {
    __shared__ __align__(16) uint16_t sa[2][LT * LROW];
    __shared__ __align__(16) uint16_t sb[2][LT * LROW];
    const int tid = threadIdx.x, lane = tid % 64, wave = tid / 64;
    const int wm = wave / 2, wn = wave % 2;
    uint32_t lid = blockIdx.x;
    {
        const uint32_t per = gridDim.x / 8;
        if (lid < per * 8) lid = (lid % 8) * per + lid / 8;
    }
    const uint32_t ct = lid % nct, rt = (lid / nct) % nrt, ks = lid / (nct * nrt);
    const uint64_t tr0 = (uint64_t)rt * LT;
    const uint32_t tc0 = ct * LT;
    const uint32_t kbeg = ks * kpiece;
    const uint32_t kend = (kbeg + kpiece < dpad) ? kbeg + kpiece : dpad;

    // this thread's pieces of each operand step: piece u = tid + 256 j covers
    // tile row u / 8 (= tid / 8 + 32 j), k offset 8 * (tid % 8); pieces at or
    // past kend (the last step of an odd number of 32-wide slices) are zero
    const int kk = 8 * (tid % 8), rr = tid / 8;
    const uint16_t *ga[LPC];
    const uint16_t *gb[LPC];
#pragma unroll
    for (int j = 0; j < LPC; ++j) {
        const uint64_t r = (tr0 + rr + 32 * j < n) ? tr0 + rr + 32 * j : n - 1;
        const uint32_t c = (tc0 + rr + 32 * j < H) ? tc0 + rr + 32 * j : H - 1;
        ga[j] = planes + r * ld + kk;
        gb[j] = w + (uint64_t)c * dpad + kk;
    }
    const int so = rr * LROW + kk;
    uint4 ra[LPC], rb[LPC];
    auto fetch = [&](uint32_t k) {
        const bool in = k + kk < kend;
#pragma unroll
        for (int j = 0; j < LPC; ++j) {
            ra[j] = in ? *reinterpret_cast<const uint4 *>(ga[j] + k) : uint4{0u, 0u, 0u, 0u};
            rb[j] = in ? *reinterpret_cast<const uint4 *>(gb[j] + k) : uint4{0u, 0u, 0u, 0u};
        }
    };
    auto stage = [&](int buf) {
#pragma unroll
        for (int j = 0; j < LPC; ++j) {
            *reinterpret_cast<uint4 *>(&sa[buf][so + 32 * j * LROW]) = ra[j];
            *reinterpret_cast<uint4 *>(&sb[buf][so + 32 * j * LROW]) = rb[j];
        }
    };
    fetch(kbeg);
    stage(0);
    __syncthreads();

    f32x4 acc[4][4], prt[4][4];
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) {
            acc[a][b] = f32x4{0.f, 0.f, 0.f, 0.f};
            prt[a][b] = f32x4{0.f, 0.f, 0.f, 0.f};
        }
    const int lr = lane % 16, lk = (lane / 16) * 8;

    for (uint32_t k0 = kbeg; k0 < kend; k0 += LK) {
        const int cur = ((k0 - kbeg) / LK) & 1;
        const bool more = k0 + LK < kend;
        if (more) fetch(k0 + LK);
        const uint16_t *ca = sa[cur];
        const uint16_t *cb = sb[cur];
#pragma unroll
        for (int hs = 0; hs < LK / 32; ++hs) {
            bf16x8 fa[4], fb[4];
#pragma unroll
            for (int a = 0; a < 4; ++a)
                fa[a] = __builtin_bit_cast(
                    bf16x8, *reinterpret_cast<const uint4 *>(
                                &ca[(wm * 64 + 16 * a + lr) * LROW + 32 * hs + lk]));
#pragma unroll
            for (int b = 0; b < 4; ++b)
                fb[b] = __builtin_bit_cast(
                    bf16x8, *reinterpret_cast<const uint4 *>(
                                &cb[(wn * 64 + 16 * b + lr) * LROW + 32 * hs + lk]));
#pragma unroll
            for (int a = 0; a < 4; ++a)
#pragma unroll
                for (int b = 0; b < 4; ++b)
                    prt[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(fa[a], fb[b], prt[a][b], 0, 0, 0);
        }
        if ((k0 + LK - kbeg) % LCHK == 0 || !more) {
            // close the chunk: one fp32 addition per output
#pragma unroll
            for (int a = 0; a < 4; ++a)
#pragma unroll
                for (int b = 0; b < 4; ++b) {
#pragma unroll
                    for (int i = 0; i < 4; ++i) acc[a][b][i] += prt[a][b][i];
                    prt[a][b] = f32x4{0.f, 0.f, 0.f, 0.f};
                }
        }
        if (more) stage(cur ^ 1);
        __syncthreads();
    }

    const uint64_t row0 = tr0 + (uint64_t)wm * 64;
    const uint32_t col0 = tc0 + wn * 64;
    if (part) {
        // one k piece of several: its partial projections
        float *pp = part + (uint64_t)ks * n * H;
#pragma unroll
        for (int b = 0; b < 4; ++b) {
            const uint32_t col = col0 + 16 * b + lr;
#pragma unroll
            for (int a = 0; a < 4; ++a)
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    const uint64_t row = row0 + 16 * a + 4 * (lane / 16) + i;
                    if (row < n && col < H) pp[row * H + col] = acc[a][b][i];
                }
        }
        return;
    }

    // Epilogue: trusted sign bits and flags, 16 columns per ballot group.
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

// Sum of the k pieces' partial projections, in piece order, then the same
// certificate as the single-piece epilogue.  A thread takes one hyperplane of
// RB consecutive rows; the 16 lanes 16j .. 16j+15 of a wavefront hold one
// group of 16 hyperplanes (reads of consecutive hyperplanes are coalesced),
// and each row's sign and flag words of the group come from two ballots.
// Loads carry no branches (rows and hyperplanes are clamped into range, the
// clamped values unused), so that they are in flight together.
template <int RB>
__global__ __launch_bounds__(256) void srp_finish_kernel(
    const float *__restrict__ part, uint32_t ns, uint64_t n, uint64_t r0, uint32_t nr,
    uint32_t H, uint32_t Hw, const float *__restrict__ nx, const float *__restrict__ nw,
    float gamma, float tau_abs, uint16_t *__restrict__ bits16, uint16_t *__restrict__ flags16,
    unsigned long long *__restrict__ nflag, float *__restrict__ proj) {
    // rows r0 .. r0 + nr - 1; the thread count is below 2^31, so the
    // indexing is 32-bit
    const uint32_t G = (H + 15) / 16;
    const int lane = threadIdx.x % 64;
    const uint32_t t = blockIdx.x * blockDim.x + threadIdx.x;
    const uint32_t grp = t / 16;
    const uint32_t rbk = grp / G;
    const uint32_t g = grp - rbk * G, col = 16 * g + t % 16;
    const uint32_t rl0 = rbk * RB;
    const uint64_t pstride = n * H;
    const uint32_t cc = col < H ? col : H - 1;
    uint64_t ro[RB];
#pragma unroll
    for (int r = 0; r < RB; ++r) ro[r] = (r0 + (rl0 + r < nr ? rl0 + r : nr - 1)) * H + cc;
    float v[RB];
#pragma unroll
    for (int r = 0; r < RB; ++r) v[r] = 0.f;
    if (rl0 < nr) {
        if constexpr (RB == 1) {
#pragma unroll 8
            for (uint32_t s = 0; s < ns; ++s) v[0] += part[(uint64_t)s * pstride + ro[0]];
        } else {
            for (uint32_t s = 0; s < ns; ++s) {
                const float *ps = part + (uint64_t)s * pstride;
#pragma unroll
                for (int r = 0; r < RB; ++r) v[r] += ps[ro[r]];
            }
        }
    }
    unsigned long long nf = 0;
    const float wn_ = nw[cc];
    float xn[RB];
#pragma unroll
    for (int r = 0; r < RB; ++r) xn[r] = nx[r0 + (rl0 + r < nr ? rl0 + r : nr - 1)];
#pragma unroll
    for (int r = 0; r < RB; ++r) {
        const uint32_t rl = rl0 + r;
        const uint64_t row = r0 + rl;
        bool bit = false, flg = false;
        if (rl < nr && col < H) {
            if (proj) proj[row * H + col] = v[r];
            const float tau = gamma * xn[r] * wn_ + tau_abs;
            const bool ok = fabsf(v[r]) > tau;
            bit = ok && (v[r] > 0.f);
            flg = !ok;
        }
        const unsigned long long mb = __ballot(bit);
        const unsigned long long mf = __ballot(flg);
        if (lane % 16 == 0 && rl < nr) {
            const uint64_t o = row * (2 * (uint64_t)Hw) + g;
            bits16[o] = (uint16_t)(mb >> lane);
            flags16[o] = (uint16_t)(mf >> lane);
        }
        nf += (unsigned long long)__popcll(mf);
    }
    if (lane == 0 && nf) atomicAdd(nflag, nf);
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
__device__ int exact_sign_wave(const void *xin, bool f32, uint64_t row, uint32_t d,
                               const uint16_t *__restrict__ wh) {
    constexpr int NLIMB = 12;
    constexpr int BASE = -160;
    long long limb[NLIMB];
#pragma unroll
    for (int j = 0; j < NLIMB; ++j) limb[j] = 0;
    for (uint32_t i = threadIdx.x % 64; i < d; i += 64) {
        const double xv = f32 ? (double)static_cast<const float *>(xin)[row * d + i]
                              : (double)bf16_to_f32(static_cast<const uint16_t *>(xin)[row * d + i]);
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
                    sgn = exact_sign_wave(xin, f32 != 0, row, d, wh);
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

// Recheck + pack for bf16 rows read in place (d a multiple of 32, rows
// 16-byte aligned).  One wavefront per row: its flagged hyperplanes are
// listed in LDS, then recomputed one at a time across the wavefront, with
// 16-byte loads of 8 bf16 values of the row and of the hyperplane and FP64
// partial sums reduced across the lanes (one round of memory latency per
// flagged projection).  Same certificate and exact fallback as
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
            fl[pos++] = (uint16_t)(j * 32 + b);
        }
        nf += (uint32_t)__shfl((int)inc, 63, 64);
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    // each flagged projection is recomputed by the whole wavefront: lane l
    // takes the 8-value pieces l, l + 64, ... of the row and the hyperplane,
    // all loads in flight at once
    const uint16_t *xr = x + row * d;
    for (uint32_t p = 0; p < nf; ++p) {
        const uint32_t h = fl[p];
        if (h >= H) continue;  // never: flags past H are zero
        const uint16_t *wh = w + (uint64_t)h * d;
        double v = 0.0, a = 0.0;
#pragma unroll 8
        for (uint32_t i = 8 * lane; i < d; i += 512) {
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
        v = wave_sum_f64(v);
        a = wave_sum_f64(a);
        int sgn;
        // the butterfly sums are bit-identical in every lane; lane 0's
        // verdict keeps the branch uniform by construction
        if (__builtin_amdgcn_readfirstlane(fabs(v) > 2.0 * (double)d * 0x1p-53 * a ? 1 : 0)) {
            sgn = v > 0.0 ? 1 : -1;
        } else {
            sgn = exact_sign_wave(x, false, row, d, wh);
            if (lane == 0) atomicAdd(nexact, 1ull);
        }
        if (lane == 0) {
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
    size_t partial = 0;
    if (nsplit == 1) {
        const SrpSplit sp = srp_split(ix.p.K * ix.p.L, n, ix.dpad);
        if (sp.ns > 1) partial = Arena::round((size_t)sp.ns * n * ix.p.K * ix.p.L * 4);
    }
    return (planes ? Arena::round((size_t)nsplit * n * ix.dpad * 2) : 0) + Arena::round(n * 4) +
           2 * Arena::round(n * Hw * 4) + Arena::round(16) + partial;
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
    // bf16 rows: the LDS kernel, with k split into pieces for small batches
    SrpSplit sp{};
    float *part = nullptr;
    if (nsplit == 1) {
        sp = srp_split(H, n, dpad);
        if ((uint64_t)sp.nct * sp.nrt * sp.ns > 0x7FFFFFFFull)
            fail(FLINNG_EINVAL, "SRP batch too large for one launch");
        if (sp.ns > 1) part = sc.get<float>((size_t)sp.ns * n * H * 4);
    }
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
    else {
        hipLaunchKernelGGL(srp_mfma_lds_kernel, dim3(sp.nct * sp.nrt * sp.ns), dim3(256), 0, s, pl,
                           ld, ix.hyp, dpad, nx, ix.hypnorm, n, H, Hw, gamma, tau_abs, sp.nct,
                           sp.nrt, sp.kpiece, part, reinterpret_cast<uint16_t *>(bits),
                           reinterpret_cast<uint16_t *>(flags), nflag, part ? nullptr : proj_dev);
        if (part) {
            FL_CHECK_LAUNCH();
            // rows per thread: RB * ns loads in flight
            const int rb = sp.ns >= 8 ? 1 : 4;
            const uint64_t per_rb = (uint64_t)((H + 15) / 16) * 16;
            const uint64_t rows_max = ((1ull << 30) / per_rb) * rb;
            uint16_t *b16 = reinterpret_cast<uint16_t *>(bits);
            uint16_t *f16 = reinterpret_cast<uint16_t *>(flags);
            for (uint64_t r0 = 0; r0 < n; r0 += rows_max) {
                const uint32_t nr = (uint32_t)std::min<uint64_t>(rows_max, n - r0);
                const uint64_t nt = (nr + rb - 1) / rb * per_rb;
                const dim3 g((unsigned)((nt + 255) / 256));
                if (rb == 1)
                    hipLaunchKernelGGL(srp_finish_kernel<1>, g, dim3(256), 0, s, part, sp.ns, n, r0,
                                       nr, H, Hw, nx, ix.hypnorm, gamma, tau_abs, b16, f16, nflag,
                                       proj_dev);
                else
                    hipLaunchKernelGGL(srp_finish_kernel<4>, g, dim3(256), 0, s, part, sp.ns, n, r0,
                                       nr, H, Hw, nx, ix.hypnorm, gamma, tau_abs, b16, f16, nflag,
                                       proj_dev);
                FL_CHECK_LAUNCH();
            }
        }
    }
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
