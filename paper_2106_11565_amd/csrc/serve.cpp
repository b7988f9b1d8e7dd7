// Continuous-batching query server over resident FLINNG indexes.
//
// Requests (a batch of queries for one index slot) are copied at submit and
// queued.  One scheduler thread keeps up to max_inflight batches on the GPU,
// one per HIP stream (all at the default priority): whenever a stream is free
// and the memory budget admits it, it coalesces queued requests of the same
// (index, k) into one batch, stages them through a pinned buffer, enqueues
// hash + count + decode and the copy back, and records an event.  Batches of
// different indexes (hash families) run concurrently on different streams.
// Completed batches are detected by event query; each request's results are
// sliced out and its latency (completion - submit, host steady clock) is
// recorded.  Every query is decoded by its own workgroup from its own codes,
// so a request's results do not depend on what it was batched with.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <vector>

#include "flinng_internal.h"

namespace flinng {

using Clock = std::chrono::steady_clock;

uint64_t batch_device_bytes(const Index &ix, uint64_t nq, uint64_t nitems, uint32_t k) {
    const uint64_t L = ix.p.L;
    uint64_t b = nq * L * 4 + 2 * nq * (uint64_t)k * 4 + 4 + 256;
    if (is_dense(ix.p.family)) {
        const bool f32 = ix.p.family == FLINNG_SRP_F32;
        const uint64_t H = L * ix.p.K, Hw = (H + 31) / 32;
        b += nq * ix.p.dim * (f32 ? 4 : 2);                 // staged rows
        b += (f32 ? 3 : 1) * nq * (uint64_t)ix.dpad * 2;    // operand planes
        b += nq * 4 + 2 * nq * Hw * 4 + 16;                 // norms, bits, flags
    } else {
        b += nitems * (ix.p.family == FLINNG_MINHASH_U64 ? 8 : 4) + (nq + 1) * 8;
    }
    return b;
}

struct Request {
    uint64_t ticket = 0;
    uint32_t slot = 0, k = 0;
    uint64_t nq = 0, nitems = 0;
    std::vector<unsigned char> values;
    std::vector<uint64_t> offsets;  // rebased to 0 (sets)
    Clock::time_point t_submit, t_done;
    std::vector<uint32_t> ids, scores;
    int status = 0;
    bool done = false;
    uint64_t mem = 0;
};

struct Lane {  // one stream and its in-flight batch
    hipStream_t stream = nullptr;
    hipEvent_t done = nullptr;
    bool busy = false;
    std::vector<Request *> reqs;
    uint64_t nq = 0, mem = 0;
    uint32_t k = 0;
    unsigned char *hin = nullptr;
    size_t hin_cap = 0;
    uint32_t *hout = nullptr;
    size_t hout_cap = 0;
    DevBuf din, doff, dcodes, dids, dsc, dwork;
    int status = 0;
};

struct Server {
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
    uint64_t next_ticket = 1, mem_inuse = 0;
    // stats
    Clock::time_point t0;
    uint64_t submitted = 0, completed = 0, rejected = 0, batches = 0, queries = 0;
    uint64_t peak_mem = 0;
    std::vector<double> lat_ms;
};

static void ensure_pinned(unsigned char **p, size_t *cap, size_t need) {
    if (*cap >= need) return;
    if (*p) (void)hipHostFree(*p);
    *p = nullptr;
    size_t c = std::max<size_t>(need, 1 << 16);
    FL_HIP(hipHostMalloc(reinterpret_cast<void **>(p), c, hipHostMallocDefault));
    *cap = c;
}

// Launch one batch on a lane (scheduler thread, without the lock).
static void launch(Server &S, Lane &ln) {
    const Index &ix = *S.idx[ln.reqs[0]->slot];
    const bool dense = is_dense(ix.p.family);
    const uint32_t k = ln.k;
    uint64_t nq = 0, nitems = 0, vbytes = 0;
    for (Request *r : ln.reqs) {
        nq += r->nq;
        nitems += r->nitems;
        vbytes += r->values.size();
    }
    ln.nq = nq;
    const size_t obytes = dense ? 0 : (nq + 1) * 8;
    ensure_pinned(&ln.hin, &ln.hin_cap, vbytes + obytes + 8);
    // pack values, then rebased offsets
    size_t vo = 0;
    uint64_t *ho = reinterpret_cast<uint64_t *>(ln.hin + ((vbytes + 7) & ~(size_t)7));
    uint64_t qi = 0, ibase = 0;
    for (Request *r : ln.reqs) {
        std::memcpy(ln.hin + vo, r->values.data(), r->values.size());
        vo += r->values.size();
        if (!dense) {
            for (uint64_t i = 0; i < r->nq; ++i) ho[qi + i] = ibase + r->offsets[i];
            qi += r->nq;
            ibase += r->nitems;
        }
    }
    if (!dense) ho[nq] = ibase;
    hipStream_t s = ln.stream;
    ln.din = DevBuf(std::max<size_t>(vbytes, 8), s);
    FL_HIP(hipMemcpyAsync(ln.din.ptr, ln.hin, vbytes, hipMemcpyHostToDevice, s));
    flinng_input in{};
    in.values = ln.din.ptr;
    in.count = nq;
    in.on_device = 1;
    if (!dense) {
        ln.doff = DevBuf(obytes, s);
        FL_HIP(hipMemcpyAsync(ln.doff.ptr, ho, obytes, hipMemcpyHostToDevice, s));
        in.offsets = ln.doff.as<uint64_t>();
    }
    ln.dcodes = DevBuf(nq * ix.p.L * 4, s);
    hash_batch(ix, in, ln.dcodes.as<uint32_t>(), s, nullptr,
               dense ? -1.0 : (double)nitems / (double)nq);
    ln.dids = DevBuf(nq * k * 4, s);
    ln.dsc = DevBuf(nq * k * 4, s);
    ln.dwork = DevBuf(S.cfg.persistent ? 4 : 0, s);
    query_launch(ix, ln.dcodes.as<uint32_t>(), nq, k, ln.dids.as<uint32_t>(), ln.dsc.as<uint32_t>(),
                 S.cfg.persistent != 0, s, ln.dwork.as<uint32_t>());
    unsigned char *hout = reinterpret_cast<unsigned char *>(ln.hout);
    ensure_pinned(&hout, &ln.hout_cap, 2 * nq * k * 4);
    ln.hout = reinterpret_cast<uint32_t *>(hout);
    FL_HIP(hipMemcpyAsync(ln.hout, ln.dids.ptr, nq * k * 4, hipMemcpyDeviceToHost, s));
    FL_HIP(hipMemcpyAsync(ln.hout + nq * k, ln.dsc.ptr, nq * k * 4, hipMemcpyDeviceToHost, s));
    FL_HIP(hipEventRecord(ln.done, s));
}

// Finish a completed lane (scheduler thread, lock held).
static void finish(Server &S, Lane &ln) {
    const auto now = Clock::now();
    uint64_t qi = 0;
    for (Request *r : ln.reqs) {
        if (ln.status == 0) {
            r->ids.assign(ln.hout + qi * ln.k, ln.hout + (qi + r->nq) * ln.k);
            r->scores.assign(ln.hout + ln.nq * ln.k + qi * ln.k,
                             ln.hout + ln.nq * ln.k + (qi + r->nq) * ln.k);
        }
        qi += r->nq;
        r->status = ln.status;
        r->t_done = now;
        r->done = true;
        S.lat_ms.push_back(std::chrono::duration<double, std::milli>(now - r->t_submit).count());
        S.completed++;
    }
    S.queries += ln.nq;
    S.mem_inuse -= ln.mem;
    ln.reqs.clear();
    ln.busy = false;
    ln.din.release();
    ln.doff.release();
    ln.dcodes.release();
    ln.dids.release();
    ln.dsc.release();
    ln.dwork.release();
    S.cv_done.notify_all();
}

static void scheduler(Server *Sp) {
    Server &S = *Sp;
    (void)hipSetDevice(S.device);
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
        while (!S.stop && !S.queue.empty()) {
            Lane *free_lane = nullptr;
            for (Lane &ln : S.lanes)
                if (!ln.busy) {
                    free_lane = &ln;
                    break;
                }
            if (!free_lane) break;
            Request *head = S.queue.front();
            const Index &ix = *S.idx[head->slot];
            std::vector<Request *> take;
            uint64_t nq = 0, nitems = 0;
            for (auto it = S.queue.begin(); it != S.queue.end();) {
                Request *r = *it;
                if (r->slot != head->slot || r->k != head->k) {
                    ++it;
                    continue;
                }
                if (!take.empty() && nq + r->nq > S.cfg.max_batch) break;
                const uint64_t need = batch_device_bytes(ix, nq + r->nq, nitems + r->nitems, head->k);
                if (!take.empty() && S.mem_inuse + need > S.cfg.mem_budget) break;
                take.push_back(r);
                nq += r->nq;
                nitems += r->nitems;
                it = S.queue.erase(it);
            }
            const uint64_t need = batch_device_bytes(ix, nq, nitems, head->k);
            if (S.mem_inuse + need > S.cfg.mem_budget && S.mem_inuse > 0) {
                // wait for memory: put the requests back in order
                for (auto it = take.rbegin(); it != take.rend(); ++it) S.queue.push_front(*it);
                break;
            }
            Lane &ln = *free_lane;
            ln.reqs = take;
            ln.k = head->k;
            ln.mem = need;
            ln.busy = true;
            ln.status = 0;
            S.mem_inuse += need;
            S.peak_mem = std::max(S.peak_mem, S.mem_inuse);
            S.batches++;
            lk.unlock();
            int st = 0;
            try {
                launch(S, ln);
            } catch (const Error &e) {
                st = e.code;
            } catch (...) {
                st = FLINNG_EDEVICE;
            }
            lk.lock();
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
            S.cv_sched.wait_for(lk, std::chrono::microseconds(20));
        else if (!S.stop)
            S.cv_sched.wait(lk);
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
        Server *S = new Server();
        S->cfg = *cfg;
        if (S->cfg.max_queue == 0) S->cfg.max_queue = 1u << 20;
        for (uint32_t i = 0; i < n_idx; ++i) {
            if (!indexes[i]) {
                delete S;
                fail(FLINNG_EINVAL, "NULL index");
            }
            S->idx.push_back(reinterpret_cast<Index *>(indexes[i]));
        }
        S->device = S->idx[0]->device;
        (void)hipSetDevice(S->device);
        S->lanes.resize(cfg->max_inflight);
        for (Lane &ln : S->lanes) {
            FL_HIP(hipStreamCreateWithFlags(&ln.stream, hipStreamNonBlocking));
            FL_HIP(hipEventCreateWithFlags(&ln.done, hipEventDisableTiming));
        }
        S->t0 = Clock::now();
        S->sched = std::thread(scheduler, S);
        *out = reinterpret_cast<flinng_server *>(S);
    });
}

int flinng_serve_submit(flinng_server *srv, uint32_t idx_slot, const flinng_input *q, uint32_t k,
                        uint64_t *ticket) {
    return sguard([&] {
        if (!srv || !q || !ticket) fail(FLINNG_EINVAL, "NULL argument");
        Server &S = *reinterpret_cast<Server *>(srv);
        if (idx_slot >= S.idx.size()) fail(FLINNG_EINVAL, "bad index slot");
        if (k < 1 || k > query_max_k()) fail(FLINNG_EINVAL, "k must be in 1..4096");
        if (q->count == 0) fail(FLINNG_EINVAL, "empty request");
        if (q->on_device) fail(FLINNG_EINVAL, "serving takes host inputs");
        const Index &ix = *S.idx[idx_slot];
        Request *r = new Request();
        r->slot = idx_slot;
        r->k = k;
        r->nq = q->count;
        if (is_dense(ix.p.family)) {
            if (!q->values) {
                delete r;
                fail(FLINNG_EINVAL, "values is NULL");
            }
            const size_t esz = ix.p.family == FLINNG_SRP_F32 ? 4 : 2;
            const size_t bytes = q->count * ix.p.dim * esz;
            r->values.assign(static_cast<const unsigned char *>(q->values),
                             static_cast<const unsigned char *>(q->values) + bytes);
        } else {
            if (!q->offsets) {
                delete r;
                fail(FLINNG_EINVAL, "offsets is NULL");
            }
            const uint64_t first = q->offsets[0], last = q->offsets[q->count];
            const size_t isz = ix.p.family == FLINNG_MINHASH_U64 ? 8 : 4;
            r->offsets.resize(q->count + 1);
            for (uint64_t i = 0; i <= q->count; ++i) {
                if (i && q->offsets[i] < q->offsets[i - 1]) {
                    delete r;
                    fail(FLINNG_EINVAL, "offsets must be nondecreasing");
                }
                r->offsets[i] = q->offsets[i] - first;
            }
            r->nitems = last - first;
            const unsigned char *v = static_cast<const unsigned char *>(q->values) + first * isz;
            r->values.assign(v, v + r->nitems * isz);
        }
        r->mem = batch_device_bytes(ix, r->nq, r->nitems, k);
        std::lock_guard<std::mutex> lk(S.mu);
        if (S.stop) {
            delete r;
            fail(FLINNG_ESTATE, "server is shutting down");
        }
        if (r->mem > S.cfg.mem_budget || S.queue.size() >= S.cfg.max_queue) {
            S.rejected++;
            const bool big = r->mem > S.cfg.mem_budget;
            delete r;
            fail(FLINNG_EBUSY, big ? "request exceeds the memory budget" : "queue full");
        }
        r->ticket = S.next_ticket++;
        r->t_submit = Clock::now();
        S.tickets[r->ticket] = r;
        S.queue.push_back(r);
        S.submitted++;
        *ticket = r->ticket;
        S.cv_sched.notify_one();
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
        if (!srv || !ids) fail(FLINNG_EINVAL, "NULL argument");
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
        S.tickets.erase(it);
        const int st = r->status;
        if (st == 0) {
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
    for (Lane &ln : S->lanes) {
        if (ln.stream) (void)hipStreamSynchronize(ln.stream);
        if (ln.done) (void)hipEventDestroy(ln.done);
        if (ln.hin) (void)hipHostFree(ln.hin);
        if (ln.hout) (void)hipHostFree(ln.hout);
        ln.din.release();
        ln.doff.release();
        ln.dcodes.release();
        ln.dids.release();
        ln.dsc.release();
        ln.dwork.release();
        if (ln.stream) (void)hipStreamDestroy(ln.stream);
    }
    delete S;
}

}  // extern "C"
