// Segment copies between device memory and host memory the device can map
// (pinned, mapped, coherent host allocations), done by a kernel rather than
// by the runtime's copy calls: the server moves each batch in with one launch
// (every request's payload is one segment, read straight from the pinned
// block the request was copied into at submit) and its results out with
// another.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "flinng_internal.h"

namespace flinng {

namespace {

constexpr int COPY_THREADS = 256;
constexpr uint64_t CHUNK = 16384;  // bytes per workgroup

struct CopyArgs {
    uint32_t nseg;
    CopySeg seg[MAX_COPY_SEGS];
};

template <typename T>
__device__ inline void copy_words(const char *__restrict__ s, char *__restrict__ d, uint64_t n) {
    const T *src = reinterpret_cast<const T *>(s);
    T *dst = reinterpret_cast<T *>(d);
    const uint64_t w = n / sizeof(T);
    for (uint64_t i = threadIdx.x; i < w; i += COPY_THREADS) dst[i] = src[i];
    for (uint64_t i = w * sizeof(T) + threadIdx.x; i < n; i += COPY_THREADS) d[i] = s[i];
}

// blockIdx.y: segment; blockIdx.x: CHUNK-sized piece of it.  Each piece
// starts at a multiple of CHUNK, so it keeps the segment's alignment.
__global__ void __launch_bounds__(COPY_THREADS) copy_segments_kernel(const CopyArgs a) {
    const CopySeg g = a.seg[blockIdx.y];
    const uint64_t off = (uint64_t)blockIdx.x * CHUNK;
    if (off >= g.bytes) return;
    const uint64_t n = std::min<uint64_t>(CHUNK, g.bytes - off);
    const char *s = reinterpret_cast<const char *>(g.src) + off;
    char *d = reinterpret_cast<char *>(g.dst) + off;
    const uint64_t al = (g.src | g.dst) & 15;
    if (al == 0)
        copy_words<uint4>(s, d, n);
    else if ((al & 3) == 0)
        copy_words<uint32_t>(s, d, n);
    else
        copy_words<unsigned char>(s, d, n);
}

}  // namespace

void copy_segments(const CopySeg *segs, size_t nseg, hipStream_t s) {
    for (size_t i = 0; i < nseg; i += MAX_COPY_SEGS) {
        CopyArgs a{};
        a.nseg = (uint32_t)std::min<size_t>(MAX_COPY_SEGS, nseg - i);
        uint64_t most = 0;
        for (uint32_t j = 0; j < a.nseg; ++j) {
            a.seg[j] = segs[i + j];
            most = std::max<uint64_t>(most, a.seg[j].bytes);
        }
        if (most == 0) continue;
        const uint64_t chunks = (most + CHUNK - 1) / CHUNK;
        if (chunks > 0x7FFFFFFFull) fail(FLINNG_EINVAL, "copy segment too large");
        hipLaunchKernelGGL(copy_segments_kernel, dim3((unsigned)chunks, a.nseg), dim3(COPY_THREADS),
                           0, s, a);
        FL_CHECK_LAUNCH();
    }
}

}  // namespace flinng
