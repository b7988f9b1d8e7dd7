// Continuous-batching query server over resident FLINNG indexes.
//
// Requests (a batch of queries for one index slot) are copied at submit and
// queued; device-resident requests are borrowed instead (their values are
// staged from device memory by the batch, and their results can be written
// straight into device buffers).  One scheduler thread keeps up to
// max_inflight batches on the GPU,
// one per HIP stream (all at the default priority): whenever a stream is free
// and the memory budget admits it, it coalesces queued requests of the same
// (index, k) into one batch and enqueues a copy kernel that pulls every
// request's payload from pinned host memory, hash + count + decode, a copy
// kernel that writes the results into pinned host memory, and an event.  Each
// stream keeps its device workspace (staged input, codes, results, hash
// scratch) and pinned buffers between batches, so a steady stream of batches
// allocates nothing; the workspaces of all streams together stay within the
// memory budget, idle streams giving theirs back when another needs room.  Batches of
// different indexes (hash families) run concurrently on different streams.
// Completed batches are detected by event query; each request's results are
// sliced out and its latency (completion - submit, host steady clock) is
// recorded.  Every query is decoded by its own workgroup from its own codes,
// so a request's results do not depend on what it was batched with.
#include <hip/hip_runtime.h>
#include <sys/prctl.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <memory>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <vector>

#include "flinng_internal.h"

namespace flinng {

using Clock = std::chrono::steady_clock;

// Layout of one served batch inside its lane's device workspace (byte
// offsets, each piece 256-byte aligned).  The staged input holds the values,
// then (sets) the rebased offsets at an 8-byte aligned position, so one copy
// moves both; ids and scores are adjacent so one copy brings both back.
struct BatchPlan {
    size_t in = 0, in_bytes = 0, offs = 0;
    size_t codes = 0, out = 0, work = 0, hash = 0, total = 0;
};

// nitems: set items, or symbols of text requests (one byte each; their
// n-gram items are extracted into the hash scratch).
static BatchPlan plan_batch(const Index &ix, uint64_t nq, uint64_t nitems, uint32_t k,
                            bool text = false) {
    BatchPlan b;
    const bool dense = is_dense(ix.p.family);
    const size_t vbytes = dense ? nq * (size_t)ix.p.dim * (ix.p.family == FLINNG_SRP_F32 ? 4 : 2)
                          : text ? nitems
                                 : nitems * (ix.p.family == FLINNG_MINHASH_U64 ? 8 : 4);
    b.offs = (vbytes + 7) & ~(size_t)7;
    b.in_bytes = dense ? vbytes : b.offs + (nq + 1) * 8;
    size_t o = 0;
    b.in = o;
    o += Arena::round(b.in_bytes);
    b.codes = o;
    o += Arena::round(nq * (size_t)ix.p.L * 4);
    b.out = o;
    o += Arena::round(2 * nq * (size_t)k * 4);
    b.work = o;
    o += Arena::round(4);
    b.hash = o;
    o += dense ? srp_scratch_bytes(ix, nq) : 0;
    o += text ? text_scratch_bytes(ix.p.family, nq, nitems) : 0;
    b.total = o;
    return b;
}

uint64_t batch_device_bytes(const Index &ix, uint64_t nq, uint64_t nitems, uint32_t k, bool text) {
    return plan_batch(ix, nq, nitems, k, text).total;
}

// Pinned host memory mapped into the device's address space, coherent, so
// kernels read request payloads from it and write results into it directly.
struct Pinned {
    unsigned char *host = nullptr;
    uint64_t dev = 0;  // the same memory as a device address
};

static bool pinned_alloc(size_t bytes, Pinned *out) {
    void *h = nullptr;
    if (hipHostMalloc(&h, bytes, hipHostMallocMapped | hipHostMallocCoherent) != hipSuccess) {
        (void)hipGetLastError();
        return false;
    }
    void *d = nullptr;
    if (hipHostGetDevicePointer(&d, h, 0) != hipSuccess || !d) {
        (void)hipGetLastError();
        (void)hipHostFree(h);
        return false;
    }
    out->host = static_cast<unsigned char *>(h);
    out->dev = reinterpret_cast<uint64_t>(d);
    return true;
}

// Pinned blocks for large request payloads, reused from request to request
// (size classes of 64 KiB * 2^c): a payload is copied once, at submit, into
// memory the device reads directly, with no page faults once the pool is
// warm.  At most `cap` bytes are pinned; beyond that payloads stay in the
// heap and are packed like small ones.
struct PinnedPool {
    static constexpr size_t MIN = (size_t)64 << 10;
    std::mutex mu;
    std::vector<std::vector<Pinned>> free_;
    size_t held = 0, cap = (size_t)1 << 30;
    static int cls_of(size_t b) {
        int c = 0;
        while ((MIN << c) < b) ++c;
        return c;
    }
    bool get(size_t bytes, Pinned *out, int *cls) {
        const int c = cls_of(bytes);
        {
            std::lock_guard<std::mutex> lk(mu);
            if ((int)free_.size() > c && !free_[c].empty()) {
                *out = free_[c].back();
                free_[c].pop_back();
                *cls = c;
                return true;
            }
            if (held + (MIN << c) > cap) return false;
            held += MIN << c;
        }
        if (!pinned_alloc(MIN << c, out)) {
            std::lock_guard<std::mutex> lk(mu);
            held -= MIN << c;
            return false;
        }
        *cls = c;
        return true;
    }
    void put(const Pinned &p, int c) {
        std::lock_guard<std::mutex> lk(mu);
        if ((int)free_.size() <= c) free_.resize(c + 1);
        free_[c].push_back(p);
    }
    ~PinnedPool() {
        for (auto &v : free_)
            for (const Pinned &p : v) (void)hipHostFree(p.host);
    }
};

struct Request {
    uint64_t ticket = 0;
    uint32_t slot = 0, k = 0;
    uint64_t nq = 0, nitems = 0;
    size_t vbytes = 0;
    std::vector<unsigned char> values;  // small payloads (or the pool is full)
    Pinned pinned;                       // large payloads: a block of the pool
    uint64_t dev_values = 0;             // device-resident payload (borrowed)
    bool text = false;                   // symbol sequences (payload: symbols)
    uint32_t gram = 0, radix = 0;
    uint64_t tkey = 0, nwin = 0;         // item key; n-gram windows
    uint32_t *out_ids = nullptr;         // device outputs (borrowed), or null:
    uint32_t *out_scores = nullptr;      // results are kept for wait()
    int pcls = -1;
    PinnedPool *pool = nullptr;
    std::vector<uint64_t> offsets;  // rebased to 0 (sets)
    Clock::time_point t_submit, t_done;
    std::vector<uint32_t> ids, scores;
    int status = 0;
    bool done = false;
    uint64_t mem = 0;
    void set_payload(const unsigned char *src, size_t n) {
        vbytes = n;
        if (n >= PinnedPool::MIN && pool && pool->get(n, &pinned, &pcls))
            std::memcpy(pinned.host, src, n);
        else
            values.assign(src, src + n);
    }
    // the payload is not needed once the batch's input copy has completed
    void release_payload() {
        if (pinned.host) pool->put(pinned, pcls);
        pinned = Pinned();
        std::vector<unsigned char>().swap(values);
        std::vector<uint64_t>().swap(offsets);
    }
    ~Request() { release_payload(); }
};

struct Lane {  // one stream, its in-flight batch and its reusable buffers
    hipStream_t stream = nullptr;
    hipEvent_t done = nullptr;
    bool busy = false;
    std::vector<Request *> reqs;
    uint64_t nq = 0, nitems = 0;
    uint32_t k = 0;
    BatchPlan plan;
    Pinned hin;                     // packed small payloads and offsets
    size_t hin_cap = 0;
    Pinned hout;                    // ids then scores of the batch
    size_t hout_cap = 0;
    std::vector<CopySeg> segs;
    char *arena = nullptr;          // device workspace, kept between batches
    size_t arena_cap = 0;
    int status = 0;
};

struct Server {
    PinnedPool pool;
    std::vector<Index *> idx;
    flinng_serve_config cfg{};
    int device = 0;
    std::mutex mu;
    std::condition_variable cv_sched, cv_done;
    std::deque<Request *> queue;
    std::unordered_map<uint64_t, Request *> tickets;
    std::vector<Lane> lanes;
    std::thread sched;
    bool stop = false;
    uint64_t next_ticket = 1;
    // stats
    Clock::time_point t0;
    uint64_t submitted = 0, completed = 0, rejected = 0, batches = 0, queries = 0;
    uint64_t peak_mem = 0;
    std::vector<double> lat_ms;
};

// Device bytes held by all lane workspaces.
static uint64_t held_bytes(const Server &S) {
    uint64_t h = 0;
    for (const Lane &ln : S.lanes) h += ln.arena_cap;
    return h;
}

static void ensure_pinned(Pinned *p, size_t *cap, size_t need) {
    if (*cap >= need) return;
    const size_t c = std::max<size_t>({need, 2 * *cap, (size_t)1 << 20});
    if (p->host) (void)hipHostFree(p->host);
    *p = Pinned();
    *cap = 0;
    if (!pinned_alloc(c, p)) fail(FLINNG_ENOMEM, "pinned host allocation failed");
    *cap = c;
}

// Give lane ln a workspace of at least `need` bytes without letting the
// workspaces of all lanes exceed the budget: the other busy lanes' holdings
// are fixed, idle lanes give theirs back when room is needed.  The caller has
// checked need <= budget - (other busy lanes' holdings).  Lock held.
static void grow_arena(Server &S, Lane &ln, uint64_t need) {
    if (ln.arena_cap >= need) return;
    const uint64_t budget = S.cfg.mem_budget;
    uint64_t busy_other = 0;
    for (const Lane &o : S.lanes)
        if (&o != &ln && o.busy) busy_other += o.arena_cap;
    const uint64_t allowed = budget - busy_other;
    uint64_t want = std::min<uint64_t>(std::max<uint64_t>(need, 2 * (uint64_t)ln.arena_cap), allowed);
    if (held_bytes(S) - ln.arena_cap + want > budget) {
        for (Lane &o : S.lanes)
            if (&o != &ln && !o.busy && o.arena) {
                (void)hipFreeAsync(o.arena, o.stream);
                o.arena = nullptr;
                o.arena_cap = 0;
            }
    }
    if (ln.arena) (void)hipFreeAsync(ln.arena, ln.stream);
    ln.arena = nullptr;
    ln.arena_cap = 0;
    void *p = nullptr;
    hipError_t e = hipMallocAsync(&p, want, ln.stream);
    if (e != hipSuccess && want > need) {
        (void)hipGetLastError();
        want = need;
        e = hipMallocAsync(&p, want, ln.stream);
    }
    if (e != hipSuccess) {
        (void)hipGetLastError();
        fail(FLINNG_ENOMEM, "serving workspace allocation failed");
    }
    ln.arena = static_cast<char *>(p);
    ln.arena_cap = want;
    S.peak_mem = std::max<uint64_t>(S.peak_mem, held_bytes(S));
}

// Launch one batch on a lane (scheduler thread, without the lock): pack the
// requests into pinned memory, one copy in, hash + count + decode, one copy
// out, then the completion event.
static void launch(Server &S, Lane &ln) {
    const Index &ix = *S.idx[ln.reqs[0]->slot];
    const bool dense = is_dense(ix.p.family);
    const uint32_t k = ln.k;
    const uint64_t nq = ln.nq;
    const BatchPlan &pl = ln.plan;
    ensure_pinned(&ln.hin, &ln.hin_cap, pl.in_bytes + 16 * (ln.reqs.size() + 2));
    hipStream_t s = ln.stream;
    char *base = ln.arena;
    const uint64_t dev_in = reinterpret_cast<uint64_t>(base + pl.in);
    // one segment per pooled payload (read from its pinned block), one per
    // run of small payloads packed into the lane's pinned buffer, and (sets)
    // one for the offsets rebased to the batch; values stay in query order
    ln.segs.clear();
    size_t dst = 0, hpos = 0, run_dst = 0, run_src = 0, run_len = 0;
    auto flush = [&] {
        if (run_len) ln.segs.push_back({ln.hin.dev + run_src, dev_in + run_dst, run_len});
        run_len = 0;
    };
    for (Request *r : ln.reqs) {
        if (r->dev_values) {
            flush();
            if (r->vbytes) ln.segs.push_back({r->dev_values, dev_in + dst, r->vbytes});
        } else if (r->pinned.host) {
            flush();
            ln.segs.push_back({r->pinned.dev, dev_in + dst, r->vbytes});
        } else if (r->vbytes) {
            if (!run_len) {
                hpos = (hpos + 15) & ~(size_t)15;
                run_dst = dst;
                run_src = hpos;
            }
            std::memcpy(ln.hin.host + hpos, r->values.data(), r->vbytes);
            hpos += r->vbytes;
            run_len += r->vbytes;
        }
        dst += r->vbytes;
    }
    flush();
    if (!dense) {
        hpos = (hpos + 15) & ~(size_t)15;
        uint64_t *ho = reinterpret_cast<uint64_t *>(ln.hin.host + hpos);
        uint64_t qi = 0, ibase = 0;
        for (Request *r : ln.reqs) {
            for (uint64_t i = 0; i < r->nq; ++i) ho[qi + i] = ibase + r->offsets[i];
            qi += r->nq;
            ibase += r->nitems;
        }
        ho[nq] = ibase;
        ln.segs.push_back({ln.hin.dev + hpos, dev_in + pl.offs, (nq + 1) * 8});
    }
    copy_segments(ln.segs.data(), ln.segs.size(), s);
    flinng_input in{};
    in.values = base + pl.in;
    in.count = nq;
    in.on_device = 1;
    if (!dense) in.offsets = reinterpret_cast<const uint64_t *>(base + pl.in + pl.offs);
    uint32_t *codes = reinterpret_cast<uint32_t *>(base + pl.codes);
    uint32_t *out = reinterpret_cast<uint32_t *>(base + pl.out);
    Arena ws{base + pl.hash, pl.total - pl.hash, 0};
    double mean_hint = dense ? -1.0 : (double)ln.nitems / (double)nq;
    if (ln.reqs[0]->text) {
        // the staged symbols become n-gram items in the hash scratch
        const Request &h = *ln.reqs[0];
        flinng_text t{};
        t.symbols = static_cast<const uint8_t *>(in.values);
        t.offsets = in.offsets;
        t.count = nq;
        t.key = h.tkey;
        t.gram = h.gram;
        t.radix = h.radix;
        t.on_device = 1;
        Scratch sc(&ws, s);
        text_to_items(t, ix.p.family, ln.nitems, s, sc, &in);
        uint64_t nwin = 0;
        for (const Request *r : ln.reqs) nwin += r->nwin;
        mean_hint = (double)nwin / (double)nq;
    }
    {
        // one index version per batch (an insert swaps arrays in between)
        std::shared_lock<std::shared_mutex> rl(ix.rw);
        hash_batch(ix, in, codes, s, nullptr, mean_hint, &ws);
        query_launch(ix, codes, nq, k, out, out + nq * k, S.cfg.persistent != 0, s,
                     reinterpret_cast<uint32_t *>(base + pl.work));
    }
    // results: requests with device outputs get their slices copied there,
    // the others share one copy of the whole batch into pinned host memory
    ln.segs.clear();
    bool to_host = false;
    uint64_t qi = 0;
    const uint64_t dout = reinterpret_cast<uint64_t>(out);
    for (Request *r : ln.reqs) {
        if (r->out_ids) {
            ln.segs.push_back({dout + qi * k * 4, reinterpret_cast<uint64_t>(r->out_ids),
                               r->nq * k * 4});
            if (r->out_scores)
                ln.segs.push_back({dout + (nq + qi) * k * 4,
                                   reinterpret_cast<uint64_t>(r->out_scores), r->nq * k * 4});
        } else {
            to_host = true;
        }
        qi += r->nq;
    }
    if (to_host) {
        ensure_pinned(&ln.hout, &ln.hout_cap, 2 * nq * k * 4);
        ln.segs.push_back({dout, ln.hout.dev, 2 * nq * k * 4});
    }
    copy_segments(ln.segs.data(), ln.segs.size(), s);
    FL_HIP(hipEventRecord(ln.done, s));
}

// Finish a completed lane (scheduler thread, lock held).
static void finish(Server &S, Lane &ln) {
    const auto now = Clock::now();
    const uint32_t *ids = reinterpret_cast<const uint32_t *>(ln.hout.host);
    const uint32_t *sc = ids + ln.nq * ln.k;
    uint64_t qi = 0;
    for (Request *r : ln.reqs) {
        if (ln.status == 0 && !r->out_ids) {
            r->ids.assign(ids + qi * ln.k, ids + (qi + r->nq) * ln.k);
            r->scores.assign(sc + qi * ln.k, sc + (qi + r->nq) * ln.k);
        }
        qi += r->nq;
        r->release_payload();
        r->status = ln.status;
        r->t_done = now;
        r->done = true;
        S.lat_ms.push_back(std::chrono::duration<double, std::milli>(now - r->t_submit).count());
        S.completed++;
    }
    S.queries += ln.nq;
    ln.reqs.clear();
    ln.busy = false;
    S.cv_done.notify_all();
}

// Completion polling period while batches are in flight (a new request
// wakes the scheduler at once).
constexpr int POLL_US = 4;

static void scheduler(Server *Sp) {
    Server &S = *Sp;
    (void)hipSetDevice(S.device);
    // Wake-ups while batches are in flight are timed waits of a few
    // microseconds; Linux lets a timed wait overshoot by the thread's timer
    // slack (50 us by default), which would delay every completion by that
    // much.  Ask for 1 us (unprivileged; ignored where unsupported).
    (void)prctl(PR_SET_TIMERSLACK, 1000UL, 0UL, 0UL, 0UL);
    std::unique_lock<std::mutex> lk(S.mu);
    for (;;) {
        // 1. retire completed batches
        bool any_busy = false;
        for (Lane &ln : S.lanes) {
            if (!ln.busy) continue;
            hipError_t e = hipEventQuery(ln.done);
            if (e == hipSuccess) {
                finish(S, ln);
            } else if (e != hipErrorNotReady) {
                ln.status = FLINNG_EDEVICE;
                (void)hipGetLastError();
                finish(S, ln);
            } else {
                any_busy = true;
            }
        }
        if (S.stop && !any_busy) break;
        // 2. admit and launch as many batches as free lanes and memory allow
        bool launched = false;
        Clock::time_point wake = Clock::time_point::max();
        while (!S.stop && !S.queue.empty()) {
            Lane *free_lane = nullptr;
            for (Lane &ln : S.lanes)
                if (!ln.busy) {
                    free_lane = &ln;
                    break;
                }
            if (!free_lane) break;
            Lane &ln = *free_lane;
            Request *head = S.queue.front();
            const Index &ix = *S.idx[head->slot];
            // device bytes this lane may hold while the other busy lanes keep theirs
            uint64_t busy_other = 0;
            for (const Lane &o : S.lanes)
                if (&o != &ln && o.busy) busy_other += o.arena_cap;
            const uint64_t allowed =
                S.cfg.mem_budget > busy_other ? S.cfg.mem_budget - busy_other : 0;
            std::vector<Request *> take;
            uint64_t nq = 0, nitems = 0;
            for (auto it = S.queue.begin(); it != S.queue.end();) {
                Request *r = *it;
                if (r->slot != head->slot || r->k != head->k || r->text != head->text ||
                    (r->text && (r->gram != head->gram || r->radix != head->radix ||
                                 r->tkey != head->tkey))) {
                    ++it;
                    continue;
                }
                if (!take.empty() && nq + r->nq > S.cfg.max_batch) break;
                if (!take.empty() &&
                    batch_device_bytes(ix, nq + r->nq, nitems + r->nitems, head->k, head->text) >
                        allowed)
                    break;
                take.push_back(r);
                nq += r->nq;
                nitems += r->nitems;
                it = S.queue.erase(it);
            }
            const BatchPlan plan = plan_batch(ix, nq, nitems, head->k, head->text);
            if (S.cfg.linger_ns && nq < S.cfg.max_batch) {
                // not full: hold it until the oldest request has lingered long enough
                const auto until = head->t_submit + std::chrono::nanoseconds(S.cfg.linger_ns);
                if (Clock::now() < until) {
                    for (auto it = take.rbegin(); it != take.rend(); ++it) S.queue.push_front(*it);
                    wake = std::min(wake, until);
                    break;
                }
            }
            if (plan.total > allowed) {
                // wait for memory: put the requests back in order
                for (auto it = take.rbegin(); it != take.rend(); ++it) S.queue.push_front(*it);
                break;
            }
            ln.reqs = take;
            ln.k = head->k;
            ln.nq = nq;
            ln.nitems = nitems;
            ln.plan = plan;
            ln.busy = true;
            ln.status = 0;
            S.batches++;
            int st = 0;
            try {
                grow_arena(S, ln, plan.total);
            } catch (const Error &e) {
                st = e.code;
            }
            if (!st) {
                lk.unlock();
                try {
                    launch(S, ln);
                } catch (const Error &e) {
                    st = e.code;
                } catch (...) {
                    st = FLINNG_EDEVICE;
                }
                lk.lock();
            }
            if (st) {
                ln.status = st;
                (void)hipStreamSynchronize(ln.stream);
                finish(S, ln);
            }
            launched = true;
        }
        if (launched) continue;
        // 3. sleep: poll briefly while batches are in flight, else wait for work
        bool busy = false;
        for (Lane &ln : S.lanes) busy |= ln.busy;
        if (busy)
            S.cv_sched.wait_for(lk, std::chrono::microseconds(POLL_US));
        else if (!S.stop && wake != Clock::time_point::max())
            S.cv_sched.wait_until(lk, wake);
        else if (!S.stop)
            S.cv_sched.wait(lk);
    }
}

// Release every lane's stream, event and buffers (no batch in flight).
static void free_lanes(Server &S) {
    for (Lane &ln : S.lanes) {
        if (ln.stream) (void)hipStreamSynchronize(ln.stream);
        if (ln.done) (void)hipEventDestroy(ln.done);
        if (ln.hin.host) (void)hipHostFree(ln.hin.host);
        if (ln.hout.host) (void)hipHostFree(ln.hout.host);
        if (ln.arena) {
            (void)hipFreeAsync(ln.arena, ln.stream);
            (void)hipStreamSynchronize(ln.stream);
        }
        if (ln.stream) (void)hipStreamDestroy(ln.stream);
        ln = Lane();
    }
}

}  // namespace flinng

using namespace flinng;

template <class F>
static int sguard(F &&f) {
    try {
        f();
        return FLINNG_OK;
    } catch (const Error &e) {
        set_last_error(e.msg);
        return e.code;
    } catch (const std::bad_alloc &) {
        set_last_error("host allocation failed");
        return FLINNG_ENOMEM;
    } catch (...) {
        set_last_error("internal error");
        return FLINNG_EDEVICE;
    }
}

extern "C" {

int flinng_serve_create(flinng_index *const *indexes, uint32_t n_idx, const flinng_serve_config *cfg,
                        flinng_server **out) {
    return sguard([&] {
        if (!indexes || !cfg || !out || n_idx == 0) fail(FLINNG_EINVAL, "NULL argument or no index");
        if (cfg->max_inflight < 1 || cfg->max_inflight > 16) fail(FLINNG_EINVAL, "max_inflight must be in 1..16");
        if (cfg->max_batch < 1) fail(FLINNG_EINVAL, "max_batch must be >= 1");
        *out = nullptr;
        std::unique_ptr<Server> S(new Server());
        S->cfg = *cfg;
        if (S->cfg.max_queue == 0) S->cfg.max_queue = 1u << 20;
        for (uint32_t i = 0; i < n_idx; ++i) {
            if (!indexes[i]) fail(FLINNG_EINVAL, "NULL index");
            S->idx.push_back(reinterpret_cast<Index *>(indexes[i]));
        }
        S->device = S->idx[0]->device;
        FL_HIP(hipSetDevice(S->device));
        S->lanes.resize(cfg->max_inflight);
        try {
            for (Lane &ln : S->lanes) {
                FL_HIP(hipStreamCreateWithFlags(&ln.stream, hipStreamNonBlocking));
                FL_HIP(hipEventCreateWithFlags(&ln.done, hipEventDisableTiming));
                // pinned buffers of a typical batch, and one round trip through
                // the copy kernel on each stream, so the first requests do not
                // pay for setting them up
                ensure_pinned(&ln.hin, &ln.hin_cap, 1 << 20);
                ensure_pinned(&ln.hout, &ln.hout_cap, 1 << 20);
                std::memset(ln.hin.host, 0, 4096);
                DevBuf probe(4096, ln.stream);
                const uint64_t pd = reinterpret_cast<uint64_t>(probe.ptr);
                const CopySeg in{ln.hin.dev, pd, 4096}, out{pd, ln.hout.dev, 4096};
                copy_segments(&in, 1, ln.stream);
                copy_segments(&out, 1, ln.stream);
                probe.release();
                FL_HIP(hipStreamSynchronize(ln.stream));
            }
        } catch (...) {
            free_lanes(*S);
            throw;
        }
        S->t0 = Clock::now();
        S->sched = std::thread(scheduler, S.get());
        *out = reinterpret_cast<flinng_server *>(S.release());
    });
}

}  // extern "C"

namespace flinng {

// Queue a request (common tail of both submit paths).
static void enqueue(Server &S, std::unique_ptr<Request> r, uint64_t *ticket) {
    std::lock_guard<std::mutex> lk(S.mu);
    if (S.stop) fail(FLINNG_ESTATE, "server is shutting down");
    if (r->mem > S.cfg.mem_budget || S.queue.size() >= S.cfg.max_queue) {
        S.rejected++;
        fail(FLINNG_EBUSY, r->mem > S.cfg.mem_budget ? "request exceeds the memory budget"
                                                     : "queue full");
    }
    Request *rp = r.release();
    rp->ticket = S.next_ticket++;
    rp->t_submit = Clock::now();
    S.tickets[rp->ticket] = rp;
    S.queue.push_back(rp);
    S.submitted++;
    *ticket = rp->ticket;
    S.cv_sched.notify_one();
}

// Submit one request (both ABI entry points).  Host inputs are copied;
// device inputs are borrowed until the request completes (set offsets are
// read back once, here, to size the batch).  out_ids/out_scores: device
// buffers the batch writes the results into, or null (kept for wait()).
static void submit_request(Server &S, uint32_t idx_slot, const flinng_input *q, uint32_t k,
                           uint32_t *out_ids, uint32_t *out_scores, uint64_t *ticket) {
    if (!q || !ticket) fail(FLINNG_EINVAL, "NULL argument");
    if (idx_slot >= S.idx.size()) fail(FLINNG_EINVAL, "bad index slot");
    if (k < 1 || k > query_max_k()) fail(FLINNG_EINVAL, "k must be in 1..4096");
    if (q->count == 0) fail(FLINNG_EINVAL, "empty request");
    if (q->reserved != 0) fail(FLINNG_EINVAL, "queries.reserved must be 0");
    if (q->on_device > 2) fail(FLINNG_EINVAL, "queries.on_device must be 0, 1 or 2");
    const Index &ix = *S.idx[idx_slot];
    std::unique_ptr<Request> r(new Request());
    r->pool = &S.pool;
    r->slot = idx_slot;
    r->k = k;
    r->nq = q->count;
    r->out_ids = out_ids;
    r->out_scores = out_ids ? out_scores : nullptr;
    if (is_dense(ix.p.family)) {
        if (!q->values) fail(FLINNG_EINVAL, "values is NULL");
        const size_t esz = ix.p.family == FLINNG_SRP_F32 ? 4 : 2;
        const size_t bytes = q->count * ix.p.dim * esz;
        if (q->on_device) {
            r->vbytes = bytes;
            r->dev_values = reinterpret_cast<uint64_t>(q->values);
        } else {
            r->set_payload(static_cast<const unsigned char *>(q->values), bytes);
        }
    } else {
        if (!q->offsets) fail(FLINNG_EINVAL, "offsets is NULL");
        if (!q->values && q->on_device) fail(FLINNG_EINVAL, "values is NULL");
        r->offsets.resize(q->count + 1);
        if (q->on_device == 1) {
            FL_HIP(hipSetDevice(S.device));
            FL_HIP(hipMemcpy(r->offsets.data(), q->offsets, (q->count + 1) * 8,
                             hipMemcpyDeviceToHost));
        } else {
            std::memcpy(r->offsets.data(), q->offsets, (q->count + 1) * 8);
        }
        const uint64_t first = r->offsets[0], last = r->offsets[q->count];
        for (uint64_t i = 0; i <= q->count; ++i) {
            if (i && r->offsets[i] < r->offsets[i - 1])
                fail(FLINNG_EINVAL, "offsets must be nondecreasing");
            r->offsets[i] -= first;
        }
        const size_t isz = ix.p.family == FLINNG_MINHASH_U64 ? 8 : 4;
        r->nitems = last - first;
        if (r->nitems && !q->values) fail(FLINNG_EINVAL, "values is NULL");
        if (q->on_device) {
            r->vbytes = r->nitems * isz;
            r->dev_values = reinterpret_cast<uint64_t>(q->values) + first * isz;
        } else {
            const unsigned char *v = static_cast<const unsigned char *>(q->values) + first * isz;
            r->set_payload(v, r->nitems * isz);
        }
    }
    r->mem = batch_device_bytes(ix, r->nq, r->nitems, k, false);
    enqueue(S, std::move(r), ticket);
}

// A request of symbol sequences: the payload is the symbols (host copy or
// borrowed device range), offsets rebased on the host.
static void submit_text_request(Server &S, uint32_t idx_slot, const flinng_text *q, uint32_t k,
                                uint32_t *out_ids, uint32_t *out_scores, uint64_t *ticket) {
    if (!ticket) fail(FLINNG_EINVAL, "NULL argument");
    if (idx_slot >= S.idx.size()) fail(FLINNG_EINVAL, "bad index slot");
    const Index &ix = *S.idx[idx_slot];
    validate_text(q, ix.p.family);
    if (k < 1 || k > query_max_k()) fail(FLINNG_EINVAL, "k must be in 1..4096");
    if (q->count == 0) fail(FLINNG_EINVAL, "empty request");
    std::unique_ptr<Request> r(new Request());
    r->pool = &S.pool;
    r->slot = idx_slot;
    r->k = k;
    r->nq = q->count;
    r->out_ids = out_ids;
    r->out_scores = out_ids ? out_scores : nullptr;
    r->text = true;
    r->gram = q->gram;
    r->radix = q->radix;
    r->tkey = q->key;
    r->offsets.resize(q->count + 1);
    if (q->on_device) {
        FL_HIP(hipSetDevice(S.device));
        FL_HIP(hipMemcpy(r->offsets.data(), q->offsets, (q->count + 1) * 8, hipMemcpyDeviceToHost));
    } else {
        std::memcpy(r->offsets.data(), q->offsets, (q->count + 1) * 8);
    }
    const uint64_t first = r->offsets[0], last = r->offsets[q->count];
    for (uint64_t i = 0; i <= q->count; ++i) {
        if (i && r->offsets[i] < r->offsets[i - 1])
            fail(FLINNG_EINVAL, "text offsets must be nondecreasing");
        r->offsets[i] -= first;
        if (i) {
            const uint64_t len = r->offsets[i] - r->offsets[i - 1];
            r->nwin += len >= q->gram ? len - q->gram + 1 : 0;
        }
    }
    r->nitems = last - first;
    if (r->nitems && !q->symbols) fail(FLINNG_EINVAL, "text.symbols is NULL");
    if (q->on_device) {
        r->vbytes = r->nitems;
        r->dev_values = reinterpret_cast<uint64_t>(q->symbols) + first;
    } else {
        r->set_payload(q->symbols + first, r->nitems);
    }
    r->mem = batch_device_bytes(ix, r->nq, r->nitems, k, true);
    enqueue(S, std::move(r), ticket);
}

}  // namespace flinng

extern "C" {

int flinng_serve_submit_text(flinng_server *srv, uint32_t idx_slot, const flinng_text *q,
                             uint32_t k, uint32_t *ids, uint32_t *scores, uint64_t *ticket) {
    return sguard([&] {
        if (!srv) fail(FLINNG_EINVAL, "NULL argument");
        if (!ids && scores) fail(FLINNG_EINVAL, "scores without ids");
        submit_text_request(*reinterpret_cast<Server *>(srv), idx_slot, q, k, ids, scores, ticket);
    });
}

int flinng_serve_submit(flinng_server *srv, uint32_t idx_slot, const flinng_input *q, uint32_t k,
                        uint64_t *ticket) {
    return sguard([&] {
        if (!srv) fail(FLINNG_EINVAL, "NULL argument");
        submit_request(*reinterpret_cast<Server *>(srv), idx_slot, q, k, nullptr, nullptr, ticket);
    });
}

int flinng_serve_submit_to(flinng_server *srv, uint32_t idx_slot, const flinng_input *q,
                           uint32_t k, uint32_t *ids, uint32_t *scores, uint64_t *ticket) {
    return sguard([&] {
        if (!srv || !ids) fail(FLINNG_EINVAL, "NULL argument");
        submit_request(*reinterpret_cast<Server *>(srv), idx_slot, q, k, ids, scores, ticket);
    });
}

int flinng_serve_poll(flinng_server *srv, uint64_t ticket) {
    if (!srv) return FLINNG_EINVAL;
    Server &S = *reinterpret_cast<Server *>(srv);
    std::lock_guard<std::mutex> lk(S.mu);
    auto it = S.tickets.find(ticket);
    if (it == S.tickets.end()) {
        set_last_error("unknown ticket");
        return FLINNG_ESTATE;
    }
    return it->second->done ? 1 : 0;
}

int flinng_serve_wait(flinng_server *srv, uint64_t ticket, uint32_t *ids, uint32_t *scores,
                      int64_t timeout_ns) {
    return sguard([&] {
        if (!srv) fail(FLINNG_EINVAL, "NULL argument");
        Server &S = *reinterpret_cast<Server *>(srv);
        std::unique_lock<std::mutex> lk(S.mu);
        auto it = S.tickets.find(ticket);
        if (it == S.tickets.end()) fail(FLINNG_ESTATE, "unknown ticket");
        Request *r = it->second;
        auto pred = [&] { return r->done; };
        if (timeout_ns < 0) {
            S.cv_done.wait(lk, pred);
        } else if (!S.cv_done.wait_for(lk, std::chrono::nanoseconds(timeout_ns), pred)) {
            fail(FLINNG_ETIMEDOUT, "request not complete");
        }
        if (!ids && !r->out_ids) fail(FLINNG_EINVAL, "ids is NULL for a request with host results");
        S.tickets.erase(it);
        const int st = r->status;
        if (st == 0 && !r->out_ids) {
            std::memcpy(ids, r->ids.data(), r->ids.size() * 4);
            if (scores) std::memcpy(scores, r->scores.data(), r->scores.size() * 4);
        }
        delete r;
        if (st) fail(st, "batch failed on the device");
    });
}

int flinng_serve_stats_get(flinng_server *srv, flinng_serve_stats *st) {
    return sguard([&] {
        if (!srv || !st) fail(FLINNG_EINVAL, "NULL argument");
        Server &S = *reinterpret_cast<Server *>(srv);
        std::lock_guard<std::mutex> lk(S.mu);
        std::memset(st, 0, sizeof(*st));
        st->submitted = S.submitted;
        st->completed = S.completed;
        st->rejected = S.rejected;
        st->batches = S.batches;
        st->queries = S.queries;
        st->wall_s = std::chrono::duration<double>(Clock::now() - S.t0).count();
        st->qps = st->wall_s > 0 ? (double)S.queries / st->wall_s : 0.0;
        st->mean_batch = S.batches ? (double)S.queries / (double)S.batches : 0.0;
        st->peak_mem_bytes = S.peak_mem;
        if (!S.lat_ms.empty()) {
            std::vector<double> v = S.lat_ms;
            std::sort(v.begin(), v.end());
            auto pct = [&](double p) {
                size_t i = (size_t)std::min<double>((double)v.size() - 1, std::ceil(p * v.size()) - 1);
                return v[i];
            };
            st->p50_ms = pct(0.50);
            st->p99_ms = pct(0.99);
            st->max_ms = v.back();
        }
    });
}

int flinng_serve_stats_reset(flinng_server *srv) {
    return sguard([&] {
        if (!srv) fail(FLINNG_EINVAL, "NULL argument");
        Server &S = *reinterpret_cast<Server *>(srv);
        std::lock_guard<std::mutex> lk(S.mu);
        S.submitted = S.completed = S.rejected = S.batches = S.queries = 0;
        S.lat_ms.clear();
        S.peak_mem = held_bytes(S);
        S.t0 = Clock::now();
    });
}

void flinng_serve_destroy(flinng_server *srv) {
    if (!srv) return;
    Server *S = reinterpret_cast<Server *>(srv);
    {
        std::lock_guard<std::mutex> lk(S->mu);
        S->stop = true;
        for (Request *r : S->queue) {
            S->tickets.erase(r->ticket);
            delete r;
        }
        S->queue.clear();
    }
    S->cv_sched.notify_all();
    if (S->sched.joinable()) S->sched.join();
    for (auto &kv : S->tickets) delete kv.second;
    free_lanes(*S);
    delete S;
}

}  // extern "C"
