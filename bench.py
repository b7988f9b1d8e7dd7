#!/usr/bin/env python
"""FLINNG batched-query benchmark on one MI355X.

One step = one pass of the query path over a batch of queries that is
already resident in HBM: hash (MinHash or SRP) -> per-cell counts through the
reverse index -> threshold relaxation decode -> top-k ids/scores.  The default
workload is the 1M-read genome set (MinHash K=2, L=32, R=4, B=4096, 20-bit
buckets, 10 000 queries, k=10).  Prints one JSON line.

Extras on the same line: index build time, per-stage times, the decode
kernel's roofline (algorithmic bytes from the kernel's own work counters /
its event-timed launch duration, against 8 TB/s), recall@10 against exact
Jaccard / cosine neighbours on a query sample, the served (continuous
batching) rate with p50/p99 latency under a burst and under open-loop Poisson
arrivals, and the CPU oracle timed on one host core over a bounded query
sample.

--workload c5 keeps the genome and ReLU-embedding indexes resident together
and sweeps Poisson arrival rates of mixed-family requests (1..512 queries
each) through the server, beside each family's plain batched rate.
"""
import argparse
import ctypes
import json
import os
import queue
import sys
import threading
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
COPY_BYTES = 1 << 30


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="c2", choices=["c1", "c2", "c3", "c4", "c5"])
    ap.add_argument("--scale", type=float, default=1.0)
    ap.add_argument("--persistent", action="store_true")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-serve", action="store_true")
    ap.add_argument("--no-recall", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--recall-queries", type=int, default=1000)
    ap.add_argument("--copy-calibration", action="store_true",
                    help="first copy 1 GiB device to device three times (a plain copy of known "
                         "size, for scaling the HBM byte counters of a profiled run)")
    ap.add_argument("--fixed", action="store_true",
                    help="use the workload's configured (K, L) even where a tuned setting exists")
    ap.add_argument("--pareto", action="store_true",
                    help="sweep (K, L) around the workload's and report the fastest setting "
                         "reaching R1@10 >= 0.9")
    ap.add_argument("--rates", default="", help="comma-separated Poisson arrival rates (queries/s)")
    return ap.parse_args()


def to_dev(torch, a):
    import numpy as np
    a = np.ascontiguousarray(a)
    if a.dtype == np.uint64:
        t = torch.from_numpy(a.view(np.int64))
    elif a.dtype == np.uint32:
        t = torch.from_numpy(a.view(np.int32))
    elif a.dtype == np.uint16:
        t = torch.from_numpy(a.view(np.int16))
    else:
        t = torch.from_numpy(a)
    return t.cuda()




class Workload:
    """One resident index with its queries (host copy and device copy)."""

    def __init__(self, name, scale, torch, fl, configs, keep_data=False, tuned=False):
        t = time.time()
        self.cfg, self.data, self.queries, self.qbase = configs.make(name, scale=scale)
        c = self.cfg
        log(f"generated {c['name']} N={c['N']} nq={c['nq']} in {time.time() - t:.1f}s")
        self.fam, self.K, self.L, self.R, self.B = c["family"], c["K"], c["L"], c["R"], c["B"]
        self.tuned = bool(tuned and "tuned" in c)
        if self.tuned:
            self.K, self.L = c["tuned"]["K"], c["tuned"]["L"]
        self.b, self.k = c["bucket_bits"], c["k"]
        self.dense = self.fam in (fl.SRP_F32, fl.SRP_BF16)
        # inputs resident in HBM
        if self.dense:
            data_d = to_dev(torch, self.data)
            self.q_d = to_dev(torch, self.queries)
            self.nq = self.q_d.shape[0]
        else:
            data_d = (to_dev(torch, self.data[0]), to_dev(torch, self.data[1]))
            self.q_d = (to_dev(torch, self.queries[0]), to_dev(torch, self.queries[1]))
            self.nq = self.q_d[1].shape[0] - 1
        torch.cuda.synchronize()
        t = time.perf_counter()
        self.index = fl.Index(data_d, self.fam, self.K, self.L, self.R, self.B, configs.INDEX_SEED,
                              bucket_bits=0 if self.dense else self.b)
        torch.cuda.synchronize()
        self.build_s = time.perf_counter() - t
        self.data_d = data_d if keep_data else None
        del data_d
        info = self.index.info
        log(f"built index in {self.build_s:.2f}s: entries={info.list_entries} "
            f"bytes={info.device_bytes / 2**20:.1f}MiB")

    def host_slice(self, p, n):
        """Queries p..p+n-1 as a host batch (rows, or items + rebased offsets)."""
        import numpy as np
        if self.dense:
            return self.queries[p:p + n]
        it, of = self.queries
        o = of[p:p + n + 1]
        return (it[int(o[0]):int(o[-1])], (o - o[0]).astype(np.uint64))


def plain(w, torch, steps, warmup, persistent):
    """Event-timed plain batched steps over the device-resident queries."""
    import numpy as np
    dev = torch.device("cuda:0")
    ids_d = torch.empty((w.nq, w.k), dtype=torch.int32, device=dev)
    sc_d = torch.empty((w.nq, w.k), dtype=torch.int32, device=dev)
    stream = torch.cuda.current_stream()

    def step():
        w.index.query(w.q_d, w.k, persistent=persistent, out=(ids_d, sc_d))

    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(steps):
        step()
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / steps
    ids = ids_d.cpu().numpy().view(np.uint32).copy()
    sc = sc_d.cpu().numpy().view(np.uint32).copy()
    return ms, ids, sc, (ids_d, sc_d)


def stages(w, torch, fl, steps, persistent, out):
    """Hash alone and count+decode alone, event-timed on the stream they are
    launched on, plus the decode kernel's own work counters."""
    dev = torch.device("cuda:0")
    ids_d, sc_d = out
    L_ = fl.lib()
    stream = torch.cuda.current_stream()
    codes_d = torch.empty((w.nq, w.L), dtype=torch.int32, device=dev)
    inp, keep = fl.make_input(w.q_d, w.fam)
    sptr = ctypes.c_void_p(stream.cuda_stream)

    def hash_once():
        fl.check(L_.flinng_debug_hash(w.index.handle, ctypes.byref(inp), codes_d.data_ptr(), 1, sptr))

    def decode_once(stats=None):
        fl.check(L_.flinng_query_codes(w.index.handle, codes_d.data_ptr(), w.nq, w.k,
                                       ids_d.data_ptr(), sc_d.data_ptr(), int(persistent),
                                       stats.data_ptr() if stats is not None else None, sptr))

    def timed(fn, n):
        for _ in range(2):
            fn()
        a, z = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        a.record(stream)
        for _ in range(n):
            fn()
        z.record(stream)
        torch.cuda.synchronize()
        return a.elapsed_time(z) / n

    hash_ms = timed(hash_once, steps)
    decode_ms = timed(decode_once, steps)
    stats = torch.zeros(5, dtype=torch.int64, device=dev)
    decode_once(stats)
    torch.cuda.synchronize()
    st = [int(v) for v in stats.cpu().tolist()]
    # algorithmic bytes of one decode launch: codes (L*4) and bucket offset
    # pairs (L*8) per query, every list entry read, each member id read by the
    # final decode pass (4 B), the R group ids of each candidate it gathers
    # (2R B), and k ids + scores out
    cb = w.index.info.cell_id_bytes
    alg = w.nq * w.L * 12 + st[0] * cb + st[2] * 4 + st[4] * 2 * w.R + w.nq * w.k * 8
    ach = alg / (decode_ms / 1e3) / 1e9
    roof = {"bound": "hbm", "achieved": round(ach, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(ach / HBM_PEAK_GBS, 4), "traffic": measured_traffic(w),
            "traffic_unit": "HBM bytes per launch (rocprofv3 FETCH_SIZE + WRITE_SIZE, copy-scaled)",
            "kernel": "query_kernel (count + threshold + decode)",
            "alg_bytes_per_launch": int(alg), "launch_ms": round(decode_ms, 4),
            "list_entries": st[0], "member_ids_all_passes": st[1], "member_ids_final": st[2],
            "passes": st[3], "group_rows_gathered": st[4]}
    log(f"hash {hash_ms:.3f} ms, decode {decode_ms:.3f} ms, alg {alg / 1e6:.1f} MB -> "
        f"{ach:.0f} GB/s; stats {st}")
    return hash_ms, decode_ms, roof


def measured_traffic(w):
    """HBM bytes per query_kernel launch from the committed counter summary
    (two rocprofv3 --pmc passes, scaled by a plain copy of known size), if
    it was taken for this workload and (K, L) with the current kernel
    source; None otherwise."""
    import hashlib
    src = os.path.join(ROOT, "paper_2106_11565_amd", "csrc", "query.hip")
    path = os.path.join(ROOT, "profiles", "traffic_query_kernel.md")
    if not os.path.exists(path):
        return None
    sha = hashlib.sha256(open(src, "rb").read()).hexdigest()[:16]
    for line in open(path):
        cols = [c.strip() for c in line.strip().strip("|").split("|")]
        if len(cols) >= 9 and cols[0] == w.cfg["name"] and cols[1] == str(w.K) and cols[2] == str(w.L):
            return int(cols[8]) if cols[3] == sha else None
    return None


def recall(w, fl, ids, nq_sample):
    from workloads import truth
    t = time.time()
    ns = min(nq_sample, w.nq)
    if w.dense:
        ti, _ = truth.cosine_topk_gpu(w.data, w.queries[:ns], 10, dense_bf16=(w.fam == fl.SRP_BF16))
    else:
        ji = truth.JaccardIndex(w.data[0], w.data[1])
        ti, _ = ji.topk(w.queries[0], w.queries[1][:ns + 1], 10)
    r1 = truth.recall_at(ids[:ns, :10], ti[:, 0])
    log(f"R1@10 = {r1:.4f} on {ns} queries ({time.time() - t:.1f}s)")
    return {"R1@10": round(r1, 4), "queries": ns}


def sweep_requests(w, sizes):
    """Requests (slot 0, batch, size, first query) covering the whole query
    set in order, with the given sizes (cycled) or U{1..512}."""
    import numpy as np
    rng = np.random.default_rng(4)
    out, pos, i = [], 0, 0
    while pos < w.nq:
        n = int(sizes[i % len(sizes)]) if sizes is not None else int(rng.integers(1, 513))
        n = min(n, w.nq - pos)
        out.append((0, w.host_slice(pos, n), n, pos))
        pos += n
        i += 1
    return out


def poisson_requests(workloads, n_req, seed, sizes=None):
    """n_req requests (slot, batch, size, first query): the slot uniform over
    the workloads, the size U{1..512} unless `sizes` is given (cycled); each
    workload's queries are taken in order, wrapping around."""
    import numpy as np
    rng = np.random.default_rng(seed)
    pos = [0] * len(workloads)
    out = []
    for i in range(n_req):
        s = int(rng.integers(0, len(workloads))) if len(workloads) > 1 else 0
        w = workloads[s]
        n = int(sizes[i % len(sizes)]) if sizes is not None else int(rng.integers(1, 513))
        n = min(n, w.nq)
        if pos[s] + n > w.nq:
            pos[s] = 0
        out.append((s, w.host_slice(pos[s], n), n, pos[s]))
        pos[s] += n
    return out


def serve_run(fl, workloads, reqs, rate_qps, seed, refs, persistent=False, submitters=1):
    """Submit `reqs` to a fresh server (after a warm-up burst of the first 64),
    open loop: exponential inter-arrival gaps with mean (mean request size /
    rate_qps), or all at once when rate_qps is 0.  `submitters` client
    threads share the arrivals round-robin (the library copies a request's
    payload inside the submit call, outside the Python lock, so they copy in
    parallel); one more thread waits for the tickets.  Returns the achieved
    rate (queries / time from first arrival to last completion), the server's
    latency percentiles (completion - submit) and whether every result equals
    the plain batched result for the same queries."""
    import numpy as np
    rng = np.random.default_rng(seed)
    mean = float(np.mean([r[2] for r in reqs]))
    arrivals = (np.cumsum(rng.exponential(mean / rate_qps, len(reqs))) if rate_qps > 0
                else np.zeros(len(reqs)))
    srv = fl.Server([w.index for w in workloads], mem_budget=8 << 30, max_inflight=4,
                    max_batch=4096, persistent=persistent)
    # warm-up: one burst sizes every stream's workspace and the payload pool;
    # statistics restart after it so that they describe the steady state
    warm = [srv.submit(r[0], r[1], workloads[r[0]].k) + (workloads[r[0]].k,) for r in reqs[:64]]
    for tk, n, k in warm:
        srv.wait(tk, n, k)
    srv.reset_stats()
    tq = queue.Queue()
    state = {"same": True, "t_last": 0.0, "err": None, "lag": 0.0}
    lock = threading.Lock()

    def waiter():
        try:
            while True:
                item = tq.get()
                if item is None:
                    return
                tk, n, k, (s, _, _, p) = item
                ids, sc = srv.wait(tk, n, k)
                state["t_last"] = time.perf_counter()
                ref_i, ref_s = refs[s]
                state["same"] &= bool(np.array_equal(ids, ref_i[p:p + n]) and
                                      np.array_equal(sc, ref_s[p:p + n]))
        except Exception as e:  # surfaced after join
            state["err"] = e

    def submitter(j, t0):
        try:
            lag = 0.0
            for i in range(j, len(reqs), submitters):
                r = reqs[i]
                target = t0 + arrivals[i]
                now = time.perf_counter()
                while now < target:
                    if target - now > 0.002:
                        time.sleep(target - now - 0.001)
                    now = time.perf_counter()
                lag = max(lag, now - target)
                k = workloads[r[0]].k
                tk, n = srv.submit(r[0], r[1], k)
                tq.put((tk, n, k, r))
            with lock:
                state["lag"] = max(state["lag"], lag)
        except Exception as e:
            state["err"] = e

    th = threading.Thread(target=waiter)
    th.start()
    t0 = time.perf_counter() + 0.01
    subs = [threading.Thread(target=submitter, args=(j, t0)) for j in range(submitters)]
    for t in subs:
        t.start()
    for t in subs:
        t.join()
    tq.put(None)
    th.join()
    if state["err"] is not None:
        raise state["err"]
    wall = state["t_last"] - t0
    st = srv.stats()
    srv.close()
    nq = sum(r[2] for r in reqs)
    return {"offered_qps": rate_qps if rate_qps > 0 else "burst",
            "achieved_qps": round(nq / wall, 1), "p50_ms": round(st["p50_ms"], 3),
            "p99_ms": round(st["p99_ms"], 3), "requests": len(reqs), "queries": nq,
            "batches": st["batches"], "mean_batch": round(st["mean_batch"], 1),
            "max_submit_lag_ms": round(state["lag"] * 1e3, 3), "submitters": submitters,
            "identical_to_plain": bool(state["same"])}


def cpu_baseline(w, ids, sc, seconds):
    """The oracle on one host core over the first queries of the batch."""
    import numpy as np
    import oracle
    from workloads import configs
    t = time.time()
    ofam = {0: oracle.SRP_F32, 1: oracle.SRP_BF16, 2: oracle.MINHASH_U32,
            3: oracle.MINHASH_U64}[w.fam]
    oi = oracle.OracleIndex(ofam, w.data, w.K, w.L, w.R, w.B, configs.INDEX_SEED,
                            bucket_bits=None if w.dense else w.b)
    log(f"oracle index built in {time.time() - t:.1f}s (not timed)")
    done, agree = 0, True
    t0 = time.perf_counter()
    while done < w.nq and time.perf_counter() - t0 < seconds:
        n = min(50, w.nq - done)
        wi, ws = oi.query(w.host_slice(done, n), w.k, literal=True)
        agree &= np.array_equal(wi, ids[done:done + n]) and np.array_equal(ws, sc[done:done + n])
        done += n
    cpu_s = time.perf_counter() - t0
    log(f"oracle: {done} queries in {cpu_s:.1f}s -> {done / cpu_s:.2f} q/s; agree={agree}")
    return {"value": round(done / cpu_s, 2), "unit": "queries/s", "cores": 1, "kind": "oracle",
            "sample": f"first {done} of {w.nq} queries against the full-size oracle index "
                      "(hash, reverse-index counts, literal Algorithm 3 walk; index build "
                      "not timed)",
            "gpu_matches_oracle_on_sample": bool(agree)}


METRIC = "queries/s at recall@10>=0.9, served vs plain batched; p50/p99 query latency"


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (got --gpus {args.gpus}); the query path is "
              "replicated per GPU with no exchange, so no multi-GPU figure is produced.",
              file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch
    import paper_2106_11565_amd as fl
    from workloads import configs

    assert torch.cuda.is_available(), "needs a ROCm GPU"
    torch.cuda.init()
    if args.copy_calibration:
        src = torch.ones(COPY_BYTES // 4, dtype=torch.int32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        log(f"copy calibration: {COPY_BYTES} bytes x 3")
        del src, dst
    if args.workload == "c5":
        return main_mixed(args, torch, fl, configs)
    if args.pareto:
        return main_pareto(args, torch, fl, configs)

    w = Workload(args.workload, args.scale, torch, fl, configs, keep_data=True,
                 tuned=not args.fixed)
    ms, ids, sc, out_d = plain(w, torch, args.steps, args.warmup, args.persistent)
    value = w.nq / (ms / 1e3)
    log(f"plain batched: {ms:.3f} ms/step -> {value:,.0f} q/s")
    hash_ms, decode_ms, roof = stages(w, torch, fl, args.steps, args.persistent, out_d)
    assert np.array_equal(out_d[0].cpu().numpy().view(np.uint32), ids), "decode-only != full path"

    out = {
        "metric": METRIC, "value": round(value, 1), "unit": "queries/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": ("bf16+f32acc+f64" if w.fam == fl.SRP_BF16 else "f32+f64") if w.dense else "u64",
        "data": "synthetic",
        "config": {"workload": w.cfg["name"], "N": w.cfg["N"], "nq": w.nq, "K": w.K, "L": w.L,
                   "R": w.R, "B": w.B, "bucket_bits": w.b, "k": w.k,
                   "persistent": bool(args.persistent),
                   "K_L": "tuned (R1@10 >= 0.9 by over two standard errors on 3000 queries)"
                   if w.tuned else "as configured"},
        "build_s": round(w.build_s, 3),
        "srp_rechecked_fraction": (round(w.index.info.srp_rechecked / (w.cfg["N"] * w.K * w.L), 6)
                                   if w.dense else None),
        "stages_ms": {"hash": round(hash_ms, 4), "count_decode": round(decode_ms, 4)},
        "roofline": roof,
    }
    if not args.no_recall:
        out["recall"] = recall(w, fl, ids, args.recall_queries)
    if w.tuned:
        # the configured (K, L), measured the same way on the same data
        K0, L0 = w.cfg["K"], w.cfg["L"]
        ix = fl.Index(w.data_d, w.fam, K0, L0, w.R, w.B, configs.INDEX_SEED,
                      bucket_bits=0 if w.dense else w.b)
        w2 = Workload.__new__(Workload)
        w2.__dict__.update(w.__dict__)
        w2.index, w2.K, w2.L = ix, K0, L0
        ms0, ids0, _, _ = plain(w2, torch, args.steps, args.warmup, args.persistent)
        fixed = {"K": K0, "L": L0, "qps": round(w.nq / (ms0 / 1e3), 1), "ms_per_step": round(ms0, 4)}
        if not args.no_recall:
            fixed["recall"] = recall(w2, fl, ids0, args.recall_queries)
        out["configured_K_L"] = fixed
        log(f"configured K={K0} L={L0}: {fixed}")
        ix.close()
    w.data_d = None

    if not args.no_serve:
        sizes = w.cfg.get("group_sizes")
        burst = serve_run(fl, [w], sweep_requests(w, sizes), 0, 5, [(ids, sc)], args.persistent)
        log(f"served burst: {burst}")
        rates = [float(r) for r in args.rates.split(",")] if args.rates else [1e5, 1e6]
        pois = []
        for i, rate in enumerate(rates):
            n_req = int(max(40, min(3000, rate * 1.0 / 256.5)))
            rr = poisson_requests([w], n_req, 6 + i, sizes)
            pois.append(serve_run(fl, [w], rr, rate, 7 + i, [(ids, sc)], args.persistent))
            log(f"served Poisson @ {rate:,.0f} q/s: {pois[-1]}")
        out["served"] = {"plain_qps": round(value, 1), "burst": burst, "poisson": pois}

    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(w, ids, sc, args.cpu_seconds)

    print(json.dumps(out), flush=True)


def truth_top1(w, fl, ns):
    """Exact nearest neighbour (lowest id on ties) of the first ns queries."""
    from workloads import truth
    if w.dense:
        ti, _ = truth.cosine_topk_gpu(w.data, w.queries[:ns], 1, dense_bf16=(w.fam == fl.SRP_BF16))
    else:
        ti, _ = truth.JaccardIndex(w.data[0], w.data[1]).topk(w.queries[0], w.queries[1][:ns + 1], 1)
    return ti[:, 0]


def main_pareto(args, torch, fl, configs):
    """The paper's tuning procedure, restricted to the hash parameters: with
    R and B as the workload fixes them, sweep K (hashes per table) and L
    (tables), time the plain batched query and measure R1@10 for each, and
    report the speed/recall frontier and the fastest setting with
    R1@10 >= 0.9.  For each K, L grows until two settings meet the target."""
    import numpy as np
    w = Workload(args.workload, args.scale, torch, fl, configs, keep_data=True)
    ns = min(args.recall_queries, w.nq)
    t = time.time()
    top1 = truth_top1(w, fl, ns)
    log(f"ground truth for {ns} queries in {time.time() - t:.1f}s")
    Ks = ([max(1, w.K - 4), w.K, w.K + 4, w.K + 8] if w.dense else [1, 2, 3])
    Ks = sorted(set(k for k in Ks if k <= (24 if w.dense else 32)))
    Ls = [4, 8, 12, 16, 24, 32, 48, 64, 96, 128, 192, 255]
    dev = torch.device("cuda:0")
    ids_d = torch.empty((w.nq, w.k), dtype=torch.int32, device=dev)
    sc_d = torch.empty((w.nq, w.k), dtype=torch.int32, device=dev)
    pts = []
    for K in Ks:
        for L in Ls:
            ix = fl.Index(w.data_d, w.fam, K, L, w.R, w.B, configs.INDEX_SEED,
                          bucket_bits=0 if w.dense else w.b)
            for _ in range(2):
                ix.query(w.q_d, w.k, out=(ids_d, sc_d))
            torch.cuda.synchronize()
            a, z = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record()
            for _ in range(args.steps):
                ix.query(w.q_d, w.k, out=(ids_d, sc_d))
            z.record()
            torch.cuda.synchronize()
            ms = a.elapsed_time(z) / args.steps
            ids = ids_d.cpu().numpy().view(np.uint32)
            r1 = float(np.mean(np.any(ids[:ns, :10] == top1[:, None], axis=1)))
            pt = {"K": K, "L": L, "qps": round(w.nq / (ms / 1e3), 1), "ms_per_step": round(ms, 4),
                  "R1@10": round(r1, 4), "index_bytes": int(ix.info.device_bytes)}
            pts.append(pt)
            log(f"K={K} L={L}: {pt['qps']:,.0f} q/s R1@10 {r1:.4f}")
            ix.close()
            hits = sum(1 for p in pts if p["K"] == K and p["R1@10"] >= 0.9)
            if hits >= 2:   # one setting past the first that meets the target
                break
    front = [p for p in pts if not any(o["qps"] >= p["qps"] and o["R1@10"] >= p["R1@10"] and o != p
                                       for o in pts)]
    ok = [p for p in pts if p["R1@10"] >= 0.9]
    best = max(ok, key=lambda p: p["qps"]) if ok else None
    out = {"metric": METRIC, "value": best["qps"] if best else None, "unit": "queries/s",
           "n_gpus": 1, "steps": args.steps, "warmup": 2, "ms_per_step": best["ms_per_step"] if best else None,
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
           "dtype": "u64" if not w.dense else "bf16+f32acc+f64", "data": "synthetic",
           "config": {"workload": w.cfg["name"] + " (K, L) sweep", "N": w.cfg["N"], "nq": w.nq,
                      "R": w.R, "B": w.B, "bucket_bits": w.b, "k": w.k,
                      "fixed": {"K": w.K, "L": w.L}},
           "fastest_at_R1@10>=0.9": best, "frontier": sorted(front, key=lambda p: -p["qps"]),
           "points": pts, "recall_queries": ns}
    print(json.dumps(out), flush=True)


def main_mixed(args, torch, fl, configs):
    """Genome reads (MinHash) and ReLU embeddings (SRP) resident together:
    each family's plain batched rate, then a sweep of Poisson arrival rates of
    mixed-family requests through one server, and a burst (saturation)."""
    ws = [Workload("c2", args.scale, torch, fl, configs, tuned=not args.fixed),
          Workload("c3", args.scale, torch, fl, configs)]
    plain_res, refs = [], []
    for w in ws:
        ms, ids, sc, _ = plain(w, torch, args.steps, args.warmup, False)
        plain_res.append({"workload": w.cfg["name"], "nq": w.nq, "ms_per_step": round(ms, 4),
                          "qps": round(w.nq / (ms / 1e3), 1)})
        refs.append((ids, sc))
        log(f"plain {w.cfg['name']}: {w.nq / (ms / 1e3):,.0f} q/s")
    # half the queries from each family, each family batched on its own
    mixed_plain = sum(w.nq for w in ws) / sum(r["ms_per_step"] / 1e3 for r in plain_res)
    rates = ([float(r) for r in args.rates.split(",")] if args.rates else
             [1e3, 3e3, 1e4, 3e4, 1e5, 3e5, 1e6, 2e6])
    sweep = []
    for i, rate in enumerate(rates):
        n_req = int(max(30, min(3000, rate * 1.0 / 256.5)))
        r = serve_run(fl, ws, poisson_requests(ws, n_req, 100 + i), rate, 200 + i, refs)
        sweep.append(r)
        log(f"served mixed Poisson @ {rate:,.0f} q/s: {r}")
    burst = serve_run(fl, ws, poisson_requests(ws, 200, 99), 0, 98, refs)
    log(f"served mixed burst: {burst}")
    out = {
        "metric": METRIC, "value": burst["achieved_qps"], "unit": "queries/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": None,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "u64 | bf16+f32acc+f64", "data": "synthetic",
        "config": {"workload": "mixed serving: genome_reads_1M_minhash + relu_embed_1M_d4096_bf16",
                   "requests": "Poisson arrivals, sizes U{1..512}, family 50/50, k=10",
                   "indexes": [{"workload": w.cfg["name"], "K": w.K, "L": w.L, "R": w.R, "B": w.B}
                               for w in ws]},
        "plain": plain_res, "plain_mixed_qps": round(mixed_plain, 1),
        "served_poisson": sweep, "served_burst": burst,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
