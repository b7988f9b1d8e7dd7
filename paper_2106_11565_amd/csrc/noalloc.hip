// flinng_query_noalloc: the batched query (hash, count, threshold
// relaxation, top-k) with every piece of scratch -- the batch's bucket codes,
// the SRP stage's norms, sign and flag words and counters, the persistent
// grid's query counter -- carved from one file-scope device array instead of
// allocated, for callers that cannot allocate (code under graph capture,
// tight serving loops, harnesses that forbid allocation).
//
// Each GPU holds its own copy of the array, at its own address, until the
// process ends.  In host code the array's name is only a stand-in, so its
// device address is looked up once per device (with that device current)
// and that address is what the kernels receive.  Every call on a GPU shares
// that GPU's array: calls that overlap on one GPU (on any streams) race, and
// each call clears what must start at zero with kernels (no memset call).
#include <hip/hip_runtime.h>

#include <mutex>

#include "flinng_internal.h"

namespace flinng {

constexpr size_t NOALLOC_SCRATCH_BYTES = (size_t)64 << 20;

static __device__ __align__(256) unsigned char scratch[NOALLOC_SCRATCH_BYTES];

namespace {

constexpr int MAX_DEVICES = 64;

struct ScratchAddr {
    std::once_flag once[MAX_DEVICES];
    void *ptr[MAX_DEVICES] = {};
    hipError_t err[MAX_DEVICES] = {};
};

ScratchAddr &scratch_addr() {
    static ScratchAddr a;
    return a;
}

// The device address of this GPU's scratch array (the current device).
char *device_scratch() {
    int dev = 0;
    FL_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= MAX_DEVICES) fail(FLINNG_EDEVICE, "device ordinal out of range");
    ScratchAddr &a = scratch_addr();
    std::call_once(a.once[dev], [&] {
        void *p = nullptr;
        a.err[dev] = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (a.err[dev] == hipSuccess) a.ptr[dev] = p;
        else (void)hipGetLastError();
    });
    if (a.err[dev] != hipSuccess || !a.ptr[dev])
        fail(FLINNG_EDEVICE, std::string("scratch symbol lookup failed: ") +
                                 hipGetErrorString(a.err[dev]));
    return static_cast<char *>(a.ptr[dev]);
}

}  // namespace

size_t noalloc_scratch_bytes(const Index &ix, uint64_t nq, const void *xdev) {
    size_t b = Arena::round(nq * (size_t)ix.p.L * 4) + Arena::round(4);
    if (is_dense(ix.p.family)) b += srp_scratch_bytes(ix, nq, xdev);
    return b;
}

}  // namespace flinng

using namespace flinng;

extern "C" int flinng_query_noalloc(const flinng_index *idx, const flinng_input *q, uint32_t k,
                                    uint32_t *ids, uint32_t *scores, uint32_t persistent,
                                    void *stream) {
    try {
        if (!idx || !q || !ids) fail(FLINNG_EINVAL, "NULL argument");
        const Index &ix = *reinterpret_cast<const Index *>(idx);
        if (q->reserved != 0) fail(FLINNG_EINVAL, "queries.reserved must be 0");
        if (q->on_device != 1) fail(FLINNG_EINVAL, "flinng_query_noalloc takes device inputs");
        if (k < 1 || k > query_max_k()) fail(FLINNG_EINVAL, "k must be in 1..4096");
        const uint64_t nq = q->count;
        if (nq == 0) {
            set_last_error("");
            return FLINNG_OK;
        }
        if (!q->values) fail(FLINNG_EINVAL, "queries.values is NULL");
        if (!is_dense(ix.p.family) && !q->offsets) fail(FLINNG_EINVAL, "queries.offsets is NULL");
        const size_t need = noalloc_scratch_bytes(ix, nq, q->values);
        if (need > NOALLOC_SCRATCH_BYTES)
            fail(FLINNG_EINVAL, "batch needs " + std::to_string(need) +
                                    " bytes of scratch, more than the " +
                                    std::to_string(NOALLOC_SCRATCH_BYTES) +
                                    " the allocation-free query holds; split the batch");
        FL_HIP(hipSetDevice(ix.device));
        hipStream_t s = static_cast<hipStream_t>(stream);
        std::shared_lock<std::shared_mutex> rl(ix.rw);  // one index version per call
        Arena ws{device_scratch(), NOALLOC_SCRATCH_BYTES, 0};
        uint32_t *codes = static_cast<uint32_t *>(ws.take(nq * (size_t)ix.p.L * 4));
        uint32_t *work = static_cast<uint32_t *>(ws.take(4));
        // device sets: no slice-count hint is read back, so the launch uses
        // the default (the result does not depend on it)
        hash_batch(ix, *q, codes, s, nullptr, -1.0, &ws);
        query_launch(ix, codes, nq, k, ids, scores, persistent != 0, s, work);
        set_last_error("");
        return FLINNG_OK;
    } catch (const Error &e) {
        set_last_error(e.msg);
        return e.code;
    } catch (...) {
        set_last_error("internal error");
        return FLINNG_EDEVICE;
    }
}
