// Exported C ABI: argument validation, orchestration of the build and query
// pipelines, and error mapping (no C++ exception crosses the boundary).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "flinng_internal.h"

namespace flinng {

static thread_local std::string g_err;

void set_last_error(const std::string &msg) { g_err = msg; }

[[noreturn]] void fail(int code, const std::string &msg) { throw Error{code, msg}; }

DevBuf::DevBuf(size_t bytes, hipStream_t s) : stream(s) {
    if (bytes == 0) return;
    hipError_t e = hipMallocAsync(&ptr, bytes, s);
    if (e != hipSuccess) {
        ptr = nullptr;
        (void)hipGetLastError();
        fail(e == hipErrorOutOfMemory ? FLINNG_ENOMEM : FLINNG_EDEVICE,
             "device allocation of " + std::to_string(bytes) + " bytes failed: " +
                 hipGetErrorString(e));
    }
}

void DevBuf::release() {
    if (ptr) (void)hipFreeAsync(ptr, stream);
    ptr = nullptr;
}

DevBuf::~DevBuf() { release(); }

template <class F>
static int guard(F &&f) {
    try {
        f();
        set_last_error("");
        return FLINNG_OK;
    } catch (const Error &e) {
        set_last_error(e.msg);
        return e.code;
    } catch (const std::bad_alloc &) {
        set_last_error("host allocation failed");
        return FLINNG_ENOMEM;
    } catch (const std::exception &e) {
        set_last_error(std::string("internal error: ") + e.what());
        return FLINNG_EDEVICE;
    } catch (...) {
        set_last_error("internal error");
        return FLINNG_EDEVICE;
    }
}

static void require(bool ok, const std::string &msg) {
    if (!ok) fail(FLINNG_EINVAL, msg);
}

static void validate_params(const flinng_params &p, uint64_t N) {
    require(p.family <= FLINNG_MINHASH_U64, "unknown family");
    require(p.reserved == 0, "reserved must be 0");
    require(p.L >= 1 && p.L <= 255, "L (tables) must be in 1..255");
    require(p.R >= 1 && p.R <= 16, "R (repetitions) must be in 1..16");
    require(p.B >= 1 && p.B <= 65536, "B (groups) must be in 1..65536");
    require(N >= 1, "empty dataset");
    require(N <= 0xFFFFFFFEull, "at most 2^32-2 points");
    require(p.B <= N, "B must not exceed N");
    if (is_dense(p.family)) {
        require(p.dim >= 1 && p.dim <= (1u << 20), "dim must be in 1..2^20");
        require(p.K >= 1 && p.K <= 24, "SRP K (bits per table) must be in 1..24");
        require(p.bucket_bits == 0 || p.bucket_bits == p.K, "SRP bucket_bits must be 0 or K");
    } else {
        require(p.K >= 1 && p.K <= 32, "MinHash K must be in 1..32");
        require(p.bucket_bits >= 1 && p.bucket_bits <= 24, "MinHash bucket_bits must be in 1..24");
    }
}

static void validate_input(const flinng_input *in, uint32_t family, const char *what) {
    require(in != nullptr, std::string(what) + " is NULL");
    require(in->reserved == 0, std::string(what) + ".reserved must be 0");
    require(in->on_device <= 1, std::string(what) + ".on_device must be 0 or 1");
    if (in->count == 0) return;
    require(in->values != nullptr || !is_dense(family), std::string(what) + ".values is NULL");
    if (!is_dense(family)) require(in->offsets != nullptr, std::string(what) + ".offsets is NULL");
}

static flinng_input slice(const flinng_input &in, const Index &ix, uint64_t begin, uint64_t n) {
    flinng_input s = in;
    s.count = n;
    if (is_dense(ix.p.family)) {
        const size_t esz = ix.p.family == FLINNG_SRP_F32 ? 4 : 2;
        s.values = static_cast<const char *>(in.values) + begin * ix.p.dim * esz;
    } else {
        s.offsets = in.offsets + begin;
    }
    return s;
}

static void free_index(Index *ix) {
    if (!ix) return;
    (void)hipSetDevice(ix->device);
    for (auto &e : ix->scratch)
        if (e.ptr) (void)hipFree(e.ptr);
    if (ix->offsets) (void)hipFree(ix->offsets);
    if (ix->cells) (void)hipFree(ix->cells);
    if (ix->grp) (void)hipFree(ix->grp);
    if (ix->mem) (void)hipFree(ix->mem);
    if (ix->cmg) (void)hipFree(ix->cmg);
    if (ix->cfl) (void)hipFree(ix->cfl);
    if (ix->hyp) (void)hipFree(ix->hyp);
    if (ix->hypnorm) (void)hipFree(ix->hypnorm);
    if (ix->hypt) (void)hipFree(ix->hypt);
    if (ix->gsize) (void)hipFree(ix->gsize);
    delete ix;
}

template <class T>
static T *dmalloc(uint64_t n, uint64_t &acc) {
    void *p = nullptr;
    const size_t bytes = std::max<uint64_t>(n, 1) * sizeof(T);
    hipError_t e = hipMalloc(&p, bytes);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        fail(e == hipErrorOutOfMemory ? FLINNG_ENOMEM : FLINNG_EDEVICE,
             "device allocation of " + std::to_string(bytes) + " bytes failed");
    }
    acc += bytes;
    return static_cast<T *>(p);
}

}  // namespace flinng

using namespace flinng;

extern "C" {

const char *flinng_last_error(void) { return g_err.c_str(); }

}  // extern "C"

static void build_impl(const flinng_params *p, const flinng_input *data, hipStream_t s,
                       flinng_index **out) {
    require(p && data && out, "NULL argument");
    *out = nullptr;
    validate_input(data, p->family, "data");
    validate_params(*p, data->count);
    Index *ix = new Index();
    try {
        ix->p = *p;
        ix->N = data->count;
        FL_HIP(hipGetDevice(&ix->device));
        const bool dense = is_dense(p->family);
        ix->nbits = dense ? p->K : p->bucket_bits;
        if (dense) ix->p.bucket_bits = p->K;
        ix->dpad = dense ? ((p->dim + 31) / 32) * 32 : 0;
        ix->Rp = 1;
        while (ix->Rp < p->R) ix->Rp <<= 1;
        const uint32_t Bp = (p->B + 3) & ~3u;
        ix->cell_bytes = ((uint64_t)p->R * Bp <= 65536) ? 2 : 4;
        const uint64_t N = ix->N;
        uint64_t bytes = 0;
        ix->N0 = N;
        ix->grp_cap = N;
        ix->grp = dmalloc<uint16_t>(N * ix->Rp, bytes);
        ix->gsize = dmalloc<uint32_t>((uint64_t)p->R * p->B, bytes);
        const uint64_t gmax = (N + p->B - 1) / p->B;
        ix->mstride = (uint32_t)((gmax + 3) & ~3ull);
        ix->mem = dmalloc<uint32_t>((uint64_t)p->R * p->B * ix->mstride, bytes);
        ix->cmg = dmalloc<uint16_t>((uint64_t)p->R * p->B * ix->mstride * ix->Rp, bytes);
        ix->cfl = dmalloc<uint32_t>((uint64_t)p->R * p->B * ix->mstride, bytes);
        if (dense) {
            ix->hyp = dmalloc<uint16_t>((uint64_t)p->L * p->K * ix->dpad, bytes);
            ix->hypnorm = dmalloc<float>((uint64_t)p->L * p->K, bytes);
            if (p->family == FLINNG_SRP_BF16)
                ix->hypt = dmalloc<uint16_t>(((uint64_t)p->L * p->K + 15) / 16 * 16 * ix->dpad, bytes);
            srp_make_hyperplanes(*ix, s);
        }
        // hash all points (in chunks to bound scratch memory)
        DevBuf codes(N * p->L * 4, s);
        // dense chunks bound the SRP scratch (a device copy of host rows,
        // operand planes): 512 MB of bf16 rows (the fused kernel takes them
        // in place, and larger batches fill more rounds of workgroups), or
        // 512 MB of fp32 rows with their three bf16 planes
        const uint64_t per_row =
            (uint64_t)ix->dpad * (p->family == FLINNG_SRP_BF16 ? 2 : 16);
        const uint64_t chunk = dense ? std::max<uint64_t>(1, (1ull << 29) / per_row) : (1ull << 20);
        for (uint64_t b0 = 0; b0 < N; b0 += chunk) {
            const uint64_t n = std::min(chunk, N - b0);
            flinng_input part = slice(*data, *ix, b0, n);
            uint64_t ctr[2] = {0, 0};
            hash_batch(*ix, part, codes.as<uint32_t>() + b0 * p->L, s, dense ? ctr : nullptr);
            ix->srp_rechecked += ctr[0];
            ix->srp_exact += ctr[1];
        }
        build_groups(*ix, s);
        build_lists(*ix, codes.as<uint32_t>(), s);
        FL_HIP(hipStreamSynchronize(s));
        ix->device_bytes = index_device_bytes(*ix);
    } catch (...) {
        free_index(ix);
        throw;
    }
    *out = reinterpret_cast<flinng_index *>(ix);
}

extern "C" {

int flinng_build(const flinng_params *p, const flinng_input *data, void *stream,
                 flinng_index **out) {
    return guard([&] { build_impl(p, data, static_cast<hipStream_t>(stream), out); });
}

int flinng_build_text(const flinng_params *p, const flinng_text *data, void *stream,
                      flinng_index **out) {
    return guard([&] {
        require(p && data && out, "NULL argument");
        *out = nullptr;
        validate_text(data, p->family);
        hipStream_t s = static_cast<hipStream_t>(stream);
        const uint64_t nsym = text_symbols(*data);
        Scratch sc(nullptr, s);
        flinng_input items{};
        text_to_items(*data, p->family, nsym, s, sc, &items);
        build_impl(p, &items, s, out);
    });
}

void flinng_index_free(flinng_index *idx) { free_index(reinterpret_cast<Index *>(idx)); }

int flinng_index_insert(flinng_index *idx, const flinng_input *data, void *stream) {
    return guard([&] {
        require(idx != nullptr, "index is NULL");
        Index &ix = *reinterpret_cast<Index *>(idx);
        validate_input(data, ix.p.family, "data");
        const uint64_t n = data->count;
        if (n == 0) return;
        FL_HIP(hipSetDevice(ix.device));
        hipStream_t s = static_cast<hipStream_t>(stream);
        std::lock_guard<std::mutex> one(ix.insert_mu);
        require(ix.N + n <= 0xFFFFFFFEull, "at most 2^32-2 points");
        const bool dense = is_dense(ix.p.family);
        DevBuf codes(n * ix.p.L * 4, s);
        const uint64_t per_row =
            (uint64_t)ix.dpad * (ix.p.family == FLINNG_SRP_BF16 ? 2 : 16);  // as in the build
        const uint64_t chunk = dense ? std::max<uint64_t>(1, (1ull << 29) / per_row)
                                     : (1ull << 20);
        uint64_t rechecked = 0, exact = 0;
        for (uint64_t b0 = 0; b0 < n; b0 += chunk) {
            const uint64_t m = std::min(chunk, n - b0);
            flinng_input part = slice(*data, ix, b0, m);
            uint64_t ctr[2] = {0, 0};
            hash_batch(ix, part, codes.as<uint32_t>() + b0 * ix.p.L, s, dense ? ctr : nullptr);
            rechecked += ctr[0];
            exact += ctr[1];
        }
        insert_points(ix, codes.as<uint32_t>(), n, s);
        std::unique_lock<std::shared_mutex> lk(ix.rw);
        ix.srp_rechecked += rechecked;
        ix.srp_exact += exact;
    });
}

int flinng_index_get_info(const flinng_index *idx, flinng_index_info *info) {
    return guard([&] {
        require(idx && info, "NULL argument");
        const Index &ix = *reinterpret_cast<const Index *>(idx);
        std::shared_lock<std::shared_mutex> rl(ix.rw);
        std::memset(info, 0, sizeof(*info));
        info->N = ix.N;
        info->list_entries = ix.list_entries;
        info->device_bytes = ix.device_bytes;
        info->family = ix.p.family;
        info->dim = ix.p.dim;
        info->K = ix.p.K;
        info->L = ix.p.L;
        info->R = ix.p.R;
        info->B = ix.p.B;
        info->bucket_bits = ix.nbits;
        info->cell_id_bytes = ix.cell_bytes;
        info->srp_rechecked = ix.srp_rechecked;
        info->srp_exact = ix.srp_exact;
    });
}

// The index's codes region for stream s, at least `bytes` long (see
// Index::scratch), with ix.scratch_mu held by the caller until the work that
// uses it is queued (two threads queueing on one stream must not interleave
// their hash and query launches).  At most 8 streams are remembered; the
// oldest is evicted.
static uint32_t *codes_scratch(const Index &ix, hipStream_t s, size_t bytes) {
    Index::StreamScratch *slot = nullptr;
    for (auto &e : ix.scratch)
        if (e.stream == s) slot = &e;
    if (slot && slot->cap >= bytes) return static_cast<uint32_t *>(slot->ptr);
    if (!slot) {
        if (ix.scratch.size() >= 8) {
            if (ix.scratch.front().ptr) (void)hipFree(ix.scratch.front().ptr);
            ix.scratch.erase(ix.scratch.begin());
        }
        ix.scratch.push_back({s, nullptr, 0});
        slot = &ix.scratch.back();
    }
    if (slot->ptr) (void)hipFree(slot->ptr);  // waits for the work using it
    slot->ptr = nullptr;
    slot->cap = 0;
    const size_t cap = std::max<size_t>(bytes, 64 * 1024);
    void *p = nullptr;
    const hipError_t e = hipMalloc(&p, cap);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        fail(e == hipErrorOutOfMemory ? FLINNG_ENOMEM : FLINNG_EDEVICE,
             "device allocation of " + std::to_string(cap) + " bytes failed");
    }
    slot->ptr = p;
    slot->cap = cap;
    return static_cast<uint32_t *>(p);
}

}  // extern "C"

static void query_impl(const flinng_index *idx, const flinng_input *q, uint32_t k, uint32_t *ids,
                       uint32_t *scores, uint32_t out_on_device, uint32_t persistent,
                       void *stream) {
    require(idx != nullptr, "index is NULL");
    const Index &ix = *reinterpret_cast<const Index *>(idx);
    validate_input(q, ix.p.family, "queries");
    require(ids != nullptr, "ids is NULL");
    require(k >= 1 && k <= query_max_k(), "k must be in 1..4096");
    const uint64_t nq = q->count;
    if (nq == 0) return;
    FL_HIP(hipSetDevice(ix.device));
    hipStream_t s = static_cast<hipStream_t>(stream);
    std::shared_lock<std::shared_mutex> rl(ix.rw);  // one index version per call
    std::unique_lock<std::mutex> lock(ix.scratch_mu);
    uint32_t *codes = codes_scratch(ix, s, (size_t)nq * ix.p.L * 4);
    hash_batch(ix, *q, codes, s, nullptr);
    DevBuf work(persistent ? 4 : 0, s);
    if (out_on_device) {
        query_launch(ix, codes, nq, k, ids, scores, persistent != 0, s, work.as<uint32_t>());
        lock.unlock();
        rl.unlock();
    } else {
        DevBuf dids(nq * k * 4, s), dsc(scores ? nq * k * 4 : 0, s);
        query_launch(ix, codes, nq, k, dids.as<uint32_t>(), scores ? dsc.as<uint32_t>() : nullptr,
                     persistent != 0, s, work.as<uint32_t>());
        lock.unlock();
        rl.unlock();
        FL_HIP(hipMemcpyAsync(ids, dids.ptr, nq * k * 4, hipMemcpyDeviceToHost, s));
        if (scores) FL_HIP(hipMemcpyAsync(scores, dsc.ptr, nq * k * 4, hipMemcpyDeviceToHost, s));
        FL_HIP(hipStreamSynchronize(s));
    }
}

extern "C" {

int flinng_query(const flinng_index *idx, const flinng_input *q, uint32_t k, uint32_t *ids,
                 uint32_t *scores, uint32_t out_on_device, uint32_t persistent, void *stream) {
    return guard([&] { query_impl(idx, q, k, ids, scores, out_on_device, persistent, stream); });
}

int flinng_query_text(const flinng_index *idx, const flinng_text *q, uint32_t k, uint32_t *ids,
                      uint32_t *scores, uint32_t out_on_device, uint32_t persistent, void *stream) {
    return guard([&] {
        require(idx != nullptr, "index is NULL");
        const Index &ix = *reinterpret_cast<const Index *>(idx);
        validate_text(q, ix.p.family);
        if (q->count == 0) return;
        FL_HIP(hipSetDevice(ix.device));
        hipStream_t s = static_cast<hipStream_t>(stream);
        const uint64_t nsym = text_symbols(*q);
        Scratch sc(nullptr, s);
        flinng_input items{};
        text_to_items(*q, ix.p.family, nsym, s, sc, &items);
        query_impl(idx, &items, k, ids, scores, out_on_device, persistent, stream);
    });
}

int flinng_query_threshold(const flinng_index *idx, const flinng_input *q, uint32_t t,
                           uint32_t max_per_query, uint32_t *ids, uint32_t *counts,
                           uint32_t out_on_device, void *stream) {
    return guard([&] {
        require(idx != nullptr, "index is NULL");
        const Index &ix = *reinterpret_cast<const Index *>(idx);
        validate_input(q, ix.p.family, "queries");
        require(counts != nullptr, "counts is NULL");
        require(ids != nullptr || max_per_query == 0, "ids is NULL");
        const uint64_t nq = q->count;
        if (nq == 0) return;
        require(nq * (uint64_t)max_per_query <= (1ull << 40), "nq * max_per_query too large");
        FL_HIP(hipSetDevice(ix.device));
        hipStream_t s = static_cast<hipStream_t>(stream);
        DevBuf codes(nq * ix.p.L * 4, s);
        hash_batch(ix, *q, codes.as<uint32_t>(), s, nullptr);
        std::shared_lock<std::shared_mutex> rl(ix.rw);
        if (out_on_device) {
            threshold_launch(ix, codes.as<uint32_t>(), nq, t, max_per_query, ids, counts, s);
        } else {
            DevBuf dids(nq * max_per_query * 4, s), dcnt(nq * 4, s);
            threshold_launch(ix, codes.as<uint32_t>(), nq, t, max_per_query, dids.as<uint32_t>(),
                             dcnt.as<uint32_t>(), s);
            if (max_per_query)
                FL_HIP(hipMemcpyAsync(ids, dids.ptr, nq * max_per_query * 4, hipMemcpyDeviceToHost, s));
            FL_HIP(hipMemcpyAsync(counts, dcnt.ptr, nq * 4, hipMemcpyDeviceToHost, s));
            FL_HIP(hipStreamSynchronize(s));
        }
    });
}

int flinng_query_codes(const flinng_index *idx, const uint32_t *codes, uint64_t nq, uint32_t k,
                       uint32_t *ids, uint32_t *scores, uint32_t persistent, uint64_t *stats,
                       void *stream) {
    return guard([&] {
        require(idx && codes && ids, "NULL argument");
        require(k >= 1 && k <= query_max_k(), "k must be in 1..4096");
        if (nq == 0) return;
        const Index &ix = *reinterpret_cast<const Index *>(idx);
        FL_HIP(hipSetDevice(ix.device));
        hipStream_t s = static_cast<hipStream_t>(stream);
        DevBuf work(persistent ? 4 : 0, s);
        std::shared_lock<std::shared_mutex> rl(ix.rw);
        query_launch(ix, codes, nq, k, ids, scores, persistent != 0, s, work.as<uint32_t>(),
                     reinterpret_cast<unsigned long long *>(stats));
    });
}

int flinng_debug_hash(const flinng_index *idx, const flinng_input *q, uint32_t *codes,
                      uint32_t out_on_device, void *stream) {
    return guard([&] {
        require(idx && codes, "NULL argument");
        const Index &ix = *reinterpret_cast<const Index *>(idx);
        validate_input(q, ix.p.family, "queries");
        const uint64_t nq = q->count;
        if (nq == 0) return;
        FL_HIP(hipSetDevice(ix.device));
        hipStream_t s = static_cast<hipStream_t>(stream);
        if (out_on_device) {
            hash_batch(ix, *q, codes, s, nullptr);
        } else {
            DevBuf d(nq * ix.p.L * 4, s);
            hash_batch(ix, *q, d.as<uint32_t>(), s, nullptr);
            FL_HIP(hipMemcpyAsync(codes, d.ptr, nq * ix.p.L * 4, hipMemcpyDeviceToHost, s));
            FL_HIP(hipStreamSynchronize(s));
        }
    });
}

int flinng_debug_projections(const flinng_index *idx, const flinng_input *q, float *proj,
                             double *bound, uint32_t out_on_device, void *stream) {
    return guard([&] {
        require(idx != nullptr, "index is NULL");
        const Index &ix = *reinterpret_cast<const Index *>(idx);
        require(is_dense(ix.p.family), "projections exist for dense (SRP) indexes only");
        if (bound) srp_bound(ix, &bound[0], &bound[1]);
        if (!proj) return;
        validate_input(q, ix.p.family, "queries");
        const uint64_t nq = q->count;
        if (nq == 0) return;
        FL_HIP(hipSetDevice(ix.device));
        hipStream_t s = static_cast<hipStream_t>(stream);
        const uint64_t H = (uint64_t)ix.p.L * ix.p.K;
        DevBuf codes(nq * ix.p.L * 4, s);
        if (out_on_device) {
            srp_hash(ix, *q, codes.as<uint32_t>(), s, nullptr, nullptr, proj);
        } else {
            DevBuf d(nq * H * 4, s);
            srp_hash(ix, *q, codes.as<uint32_t>(), s, nullptr, nullptr, d.as<float>());
            FL_HIP(hipMemcpyAsync(proj, d.ptr, nq * H * 4, hipMemcpyDeviceToHost, s));
            FL_HIP(hipStreamSynchronize(s));
        }
    });
}

int flinng_debug_counts(const flinng_index *idx, const flinng_input *q, uint8_t *counts,
                        uint32_t out_on_device, void *stream) {
    return guard([&] {
        require(idx && counts, "NULL argument");
        const Index &ix = *reinterpret_cast<const Index *>(idx);
        validate_input(q, ix.p.family, "queries");
        const uint64_t nq = q->count;
        if (nq == 0) return;
        FL_HIP(hipSetDevice(ix.device));
        hipStream_t s = static_cast<hipStream_t>(stream);
        const uint64_t nc = (uint64_t)ix.p.R * ix.p.B;
        DevBuf codes(nq * ix.p.L * 4, s);
        hash_batch(ix, *q, codes.as<uint32_t>(), s, nullptr);
        std::shared_lock<std::shared_mutex> rl(ix.rw);
        if (out_on_device) {
            counts_launch(ix, codes.as<uint32_t>(), nq, counts, s);
        } else {
            DevBuf d(nq * nc, s);
            counts_launch(ix, codes.as<uint32_t>(), nq, d.as<uint8_t>(), s);
            FL_HIP(hipMemcpyAsync(counts, d.ptr, nq * nc, hipMemcpyDeviceToHost, s));
            FL_HIP(hipStreamSynchronize(s));
        }
    });
}

int flinng_index_export(const flinng_index *idx, uint64_t *offsets, uint32_t *cells,
                        uint32_t *groups, void *stream) {
    return guard([&] {
        require(idx != nullptr, "index is NULL");
        const Index &ix = *reinterpret_cast<const Index *>(idx);
        FL_HIP(hipSetDevice(ix.device));
        hipStream_t s = static_cast<hipStream_t>(stream);
        std::shared_lock<std::shared_mutex> rl(ix.rw);
        const uint64_t nbk = nbuckets(ix);
        const uint32_t B = ix.p.B, Bp = (B + 3) & ~3u;
        if (offsets) {
            std::vector<uint32_t> o((size_t)ix.p.L * (nbk + 1));
            FL_HIP(hipMemcpyAsync(o.data(), ix.offsets, o.size() * 4, hipMemcpyDeviceToHost, s));
            FL_HIP(hipStreamSynchronize(s));
            for (size_t i = 0; i < o.size(); ++i) offsets[i] = o[i];
        }
        if (cells) {
            const uint64_t n = ix.list_entries;
            if (ix.cell_bytes == 2) {
                std::vector<uint16_t> c(n);
                if (n) FL_HIP(hipMemcpyAsync(c.data(), ix.cells, n * 2, hipMemcpyDeviceToHost, s));
                FL_HIP(hipStreamSynchronize(s));
                for (uint64_t i = 0; i < n; ++i) cells[i] = (c[i] / Bp) * B + c[i] % Bp;
            } else {
                std::vector<uint32_t> c(n);
                if (n) FL_HIP(hipMemcpyAsync(c.data(), ix.cells, n * 4, hipMemcpyDeviceToHost, s));
                FL_HIP(hipStreamSynchronize(s));
                for (uint64_t i = 0; i < n; ++i) cells[i] = (c[i] / Bp) * B + c[i] % Bp;
            }
        }
        if (groups) {
            std::vector<uint16_t> g(ix.N * ix.Rp);
            FL_HIP(hipMemcpyAsync(g.data(), ix.grp, g.size() * 2, hipMemcpyDeviceToHost, s));
            FL_HIP(hipStreamSynchronize(s));
            for (uint32_t r = 0; r < ix.p.R; ++r)
                for (uint64_t x = 0; x < ix.N; ++x) groups[(uint64_t)r * ix.N + x] = g[x * ix.Rp + r];
        }
    });
}

}  // extern "C"
