"""Benchmark: input GB/s of one Intergrams pass (n=8, k_keep=1e5, Eq. 2) on the
binary-like corpus (16,384 files, lognormal sizes, ~3.24 GB), one MI355X.

A step is one full pass over the HBM-resident corpus: scan (ingest, prefix
filter, per-file de-duplication, counting), selection of the top k_keep and the
index build for the next pass.  Passes n=1..7 run first to build the retained
set the n=8 pass filters against; each step then rewinds to that set (a pointer
swap) and runs pass 8 again.

Prints one JSON line (see the "roofline" and "cpu_baseline" objects).
"""
import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0   # MI355X HBM3E, published


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def scan_sources_digest():
    """SHA-256 over the scan kernel's sources, to tie counter records to the code they measured."""
    import hashlib
    h = hashlib.sha256()
    for f in ("ig_scan.hip", "ig_internal.h", "ig_table.hip"):
        with open(os.path.join(ROOT, "paper_2511_14955_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def profiled_record(n, launch):
    """The committed PMC record for this scan source and launch shape, and its file, else
    (None, None)."""
    import glob
    import re
    dig = scan_sources_digest()
    for path in sorted(glob.glob(os.path.join(ROOT, "profiles", "*.md"))):
        with open(path) as fh:
            text = fh.read()
        for block in re.findall(r"```json\n(.*?)\n```", text, flags=re.S):
            rec = json.loads(block)
            if (rec.get("kernel") == "k_scan" and rec.get("n") == n and rec.get("scan_sources_sha256") == dig
                    and list(rec.get("launch", [])) + list(rec.get("tables", [])) == list(launch)):
                return rec, os.path.relpath(path, ROOT)
    return None, None


def profiled_traffic(n, launch):
    """HBM bytes per scan launch from the committed PMC record for this kernel source and launch
    shape (FETCH_SIZE and WRITE_SIZE, each scaled by a copy kernel's reading), else None."""
    rec, path = profiled_record(n, launch)
    return (rec["traffic_bytes_per_launch"], path) if rec else (None, None)


def valu_issue(rec, scan_ms):
    """VALU issue time of one scan launch from the record's SQ_INSTS_VALU (wavefront instructions,
    4 cycles each on one of 256 x 4 SIMDs at 2.4 GHz), beside the measured launch time."""
    if not rec or not rec.get("sq_insts_valu") or not scan_ms:
        return None
    issue_ms = rec["sq_insts_valu"] * 4.0 / (256 * 4 * 2.4e9) * 1e3
    return {"valu_wave_instructions": rec["sq_insts_valu"], "issue_ms": round(issue_ms, 3),
            "frac_of_launch": round(issue_ms / scan_ms, 3),
            "note": "share of the scan's time its SIMDs spend issuing vector ALU instructions (SQ_INSTS_VALU of "
                    "the profiled launch); the rest is waiting on L2 and LDS"}


def recall_sample(ig, n, k_keep, corpus, zs=(1.0, 1.5, 2.0)):
    """Recall and Jaccard of the Intergrams top-k against the exact top-k (Eq. 2, same tie
    order) on the first `files` files: the exact table is one unfiltered pass at n on a fresh
    context.  Two forms: the chain n = 1..n keeping k_keep at every pass (the timed pass's
    table), and Algorithm 3 as a whole (dense 3-gram pass, ceil(z*k) kept below n) per z."""
    e = ig.Intergrams(symbol_bits=8, freq=ig.FREQ_DOC)
    e.load(corpus)
    e.pass_(n, k_keep)   # first pass after a load: every n-gram is counted
    exact = {(int(x), int(y)) for x, y in e.topk()[0]}
    e.close()

    def score(keys):
        a = {(int(x), int(y)) for x, y in keys}
        inter = len(a & exact)
        return round(inter / max(1, len(exact)), 6), round(inter / max(1, len(a | exact)), 6)

    g = ig.Intergrams(symbol_bits=8, freq=ig.FREQ_DOC)
    g.load(corpus)
    for j in range(1, n + 1):
        g.pass_(j, k_keep)
    recall, jac = score(g.topk()[0])
    sched = []
    for z in zs:
        g.intergrams(n, k_keep, z)
        r, jz = score(g.topk()[0])
        sched.append({"z": z, "recall": r, "jaccard": jz})
    g.close()
    return {"recall": recall, "jaccard": jac, "k": len(exact),
            "sample": "first %d files (%d bytes), chain n=1..%d vs one unfiltered pass at n=%d" % (
                corpus.m, corpus.nbytes, n, n),
            "algorithm3": sched}


def cpu_model():
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def cpu_baseline(n, k_keep, sample_files, threads, target_s=10.0):
    """The CPU oracle as it stands, on the first files of the same corpus: first sample_files of
    them, then, if that pass took well under target_s, as many as should take about target_s
    (at most the whole corpus)."""
    import gen
    import oracle

    def timed(files):
        corpus = gen.workload(2, m=files, nthreads=threads)
        o = oracle.Oracle(8, oracle.FREQ_DOC, nthreads=threads)
        o.load(corpus)
        for j in range(1, n):
            assert o.pass_(j, k_keep) == 0
        t0 = time.perf_counter()
        assert o.pass_(n, k_keep) == 0
        return corpus, time.perf_counter() - t0

    m_all = gen.default_m(2)
    corpus, dt = timed(sample_files)
    if dt < target_s / 2 and sample_files < m_all:
        sample_files = min(m_all, max(sample_files + 1, int(sample_files * target_s / max(dt, 1e-3))))
        log("cpu baseline: %d files took %.2f s; timing %d files" % (corpus.m, dt, sample_files))
        corpus, dt = timed(sample_files)
    # one thread on the tiny plain run (64 files x 64 KiB, n = 1..4, k = 1000)
    tiny = gen.workload(1)
    o1 = oracle.Oracle(8, oracle.FREQ_DOC, nthreads=1)
    o1.load(tiny)
    t1 = time.perf_counter()
    for j in range(1, 5):
        assert o1.pass_(j, 1000) == 0
    dt1 = time.perf_counter() - t1
    return {"value": round(corpus.nbytes / dt / 1e9, 4), "unit": "GB/s", "cores": threads, "kind": "oracle",
            "sample": "pass n=%d, k_keep=%d over the first %d files of the corpus (%d bytes), after its own passes 1..%d; "
                      "%.2f s" % (n, k_keep, sample_files, corpus.nbytes, n - 1, dt),
            "cpu_model": cpu_model(),
            "single_thread_tiny": {"GB_per_s_per_pass": round(4 * tiny.nbytes / dt1 / 1e9, 4),
                                   "sample": "1 thread, 64 files x 64 KiB, passes n=1..4, k_keep=1000, %.2f s" % dt1}}


def serve_stream(g, ig, requests, budget, n_streams, max_batch):
    """Open-loop replay of the request stream (Poisson arrivals, mean gap 0.5 ms)
    against the retained table: request i is submitted at its arrival time and
    its latency runs from that arrival to its row being on the host."""
    import gen
    import numpy as np
    from concurrent.futures import ThreadPoolExecutor
    rs = gen.RequestStream()
    t_gen = time.time()
    # every request is a pure function of its index: generated by a pool of host threads
    with ThreadPoolExecutor(max_workers=max(1, min(16, os.cpu_count() or 1))) as ex:
        files = list(ex.map(rs.file, range(requests), chunksize=64))
    gaps = np.array([rs.gap(i) for i in range(requests)])
    nbytes = int(sum(len(f) for f in files))
    log("serving: %d requests generated (%.2f GB) in %.1f s" % (requests, nbytes / 1e9, time.time() - t_gen))
    offs = [np.array([0, len(f)], np.uint64) for f in files]
    g.serve_start(max_inflight_bytes=budget, n_streams=n_streams, max_batch=max_batch, queue_capacity=1 << 20)
    t0 = g.serve_now() + 0.01
    arrive = t0 + np.cumsum(gaps)
    got = {}
    i = 0
    late = 0.0
    while len(got) < requests:
        now = g.serve_now()
        while i < requests and arrive[i] <= now:
            late = max(late, now - arrive[i])
            rc = g.submit(ig.REQ_FEATURIZE, files[i], offs[i], tag=i, t_arrival=float(arrive[i]))
            assert rc == ig.IG_OK, rc
            i += 1
            if i % 20000 == 0:
                log("serving: %d of %d requests submitted" % (i, requests))
            now = g.serve_now()
        for r in g.poll():
            got[r["tag"]] = r
        if i < requests and len(got) < requests:
            wait = arrive[i] - g.serve_now()
            if wait > 2e-4:
                time.sleep(wait - 1e-4)
    t_end = g.serve_now()
    st = g.serve_stats()
    g.serve_stop()
    bad = [t for t, r in got.items() if r["status"] != ig.IG_OK]
    assert not bad, "requests failed: %s" % bad[:5]
    lat = np.array([got[t]["t_done"] - got[t]["t_arrival"] for t in range(requests)]) * 1e3
    span = t_end - t0
    return {"requests": requests, "bytes": nbytes, "p50_ms": round(float(np.percentile(lat, 50)), 4),
            "p99_ms": round(float(np.percentile(lat, 99)), 4), "mean_ms": round(float(lat.mean()), 4),
            "max_ms": round(float(lat.max()), 4), "offered_per_s": round(requests / float(arrive[-1] - t0), 1),
            "served_GB_per_s": round(nbytes / span / 1e9, 4), "launches": st["launches"],
            "peak_running": st["peak_running"], "peak_inflight_bytes": st["peak_inflight_bytes"],
            "budget_bytes": budget, "n_streams": n_streams, "max_batch": max_batch,
            "max_submit_lateness_ms": round(late * 1e3, 4),
            "stream": "Poisson arrivals (mean gap 0.5 ms); each request one binary-like file, lognormal size "
                      "(median 64 KiB, sigma 1.5, clipped to [4 KiB, 64 MiB]) from the corpus's motif library; "
                      "table = this pass's n=%d top-k" % g.table_info()[0]}


CHAINS = {  # workload -> (symbol bits, last n, k_keep, count bits)
    1: (8, 4, 1000, 32),
    3: (8, 16, 1000000, 64),
    4: (2, 31, 1000000, 64),
}


def config_chain(ig, workload, threads, reps=3, tune_at=None, fixed=None):
    """Every pass of a workload's chain (n = 1..N, k_keep fixed, Eq. 2) on one GPU: the device
    time of each pass (median of `reps` runs, rewinding between them; graph-captured), its input
    rate and window rate.  tune_at: pass whose launch shape and table sizes the autotuner picks
    first (the rest of the chain keeps them)."""
    import gen
    bits, nmax, k, cbits = CHAINS[workload]
    t0 = time.time()
    corpus = gen.workload(workload, nthreads=threads)
    log("workload %d: %d sequences, %d bytes, generated in %.1fs" % (workload, corpus.m, corpus.nbytes, time.time() - t0))
    g = ig.Intergrams(symbol_bits=bits, freq=ig.FREQ_DOC, count_bits=cbits)
    g.load(corpus)
    if fixed:
        g.set_launch(fixed[0], fixed[1], fixed[2], wg_per_cu=fixed[3])
        g.set_tables(map_slots_log2=fixed[4], filter_max_words=fixed[5])
    rows, tune = [], None
    t_chain = time.time()
    for n in range(1, nmax + 1):
        if tune_at == n:
            tune = g.autotune(n, k)
            log("workload %d: autotune at pass %d: best %s" % (workload, n, tune["best"]))
        ms, scan = [], []
        for r in range(reps):
            if r:
                g.rewind()
            g.pass_(n, k)
            st = g.last_stats()
            ms.append(st["pass_ms"])
            scan.append(st["scan_ms"])
        med = sorted(ms)[len(ms) // 2]
        rows.append({"n": n, "pass_ms": round(med, 4), "scan_ms": round(sorted(scan)[len(scan) // 2], 4),
                     "GB_per_s": round(corpus.nbytes / (med * 1e-3) / 1e9, 3),
                     "windows_per_s": float("%.4g" % (st["windows"] / (med * 1e-3))),
                     "kept": g.table_info()[1], "distinct": st["distinct"], "records": st["records"],
                     "replays": st["replays"]})
        log("workload %d pass %d: %s" % (workload, n, rows[-1]))
    lc = g.launch()
    g.close()
    total = sum(r["pass_ms"] for r in rows)
    return {"workload": workload, "sequences": corpus.m, "bytes": corpus.nbytes, "symbol_bits": bits,
            "k_keep": k, "count_bits": cbits, "passes": rows, "chain_ms": round(total, 3),
            "chain_GB_per_s_per_pass": round(corpus.nbytes * nmax / (total * 1e-3) / 1e9, 3),
            "launch": lc, "autotune_best": tune["best"] if tune else None,
            "timing": "device time of each pass (hipEvents), median of %d runs, graph-captured" % reps,
            "wall_s": round(time.time() - t_chain, 1)}


def serve_saturation(g, ig, files, budget, n_streams, max_batch):
    """Closed loop: every request submitted at once (the queue holds them all), so the serving
    loop is never idle; served bytes over the span from the first submit to the last result."""
    import numpy as np
    offs = [np.array([0, len(f)], np.uint64) for f in files]
    g.serve_start(max_inflight_bytes=budget, n_streams=n_streams, max_batch=max_batch, queue_capacity=1 << 20)
    t0 = g.serve_now()
    for i, f in enumerate(files):
        assert g.submit(ig.REQ_FEATURIZE, f, offs[i], tag=i, t_arrival=t0) == ig.IG_OK
    got = 0
    while got < len(files):
        res = g.poll()
        assert all(r["status"] == ig.IG_OK for r in res)
        got += len(res)
        if not res:
            time.sleep(1e-4)
    span = g.serve_now() - t0
    st = g.serve_stats()
    g.serve_stop()
    nbytes = int(sum(len(f) for f in files))
    return {"requests": len(files), "bytes": nbytes, "seconds": round(span, 4),
            "GB_per_s": round(nbytes / span / 1e9, 4), "requests_per_s": round(len(files) / span, 1),
            "launches": st["launches"], "peak_running": st["peak_running"]}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--m", type=int, default=None, help="files (default: all 16,384)")
    ap.add_argument("--n", type=int, default=8)
    ap.add_argument("--k", type=int, default=100000)
    ap.add_argument("--cpu-sample-files", type=int, default=128)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-per-file", action="store_true", help="skip the one-launch-per-file comparison")
    ap.add_argument("--flags", type=int, default=0)
    ap.add_argument("--no-tune", action="store_true", help="keep the built-in launch shape")
    ap.add_argument("--launch", default=None, help="fixed scan launch shape CHUNK,BLOCK,SETCAP[,WG_PER_CU] (no autotune)")
    ap.add_argument("--tables", default=None, help="with --launch: table sizes MAP_SLOTS_LOG2,FILTER_MAX_WORDS")
    ap.add_argument("--copy-calibrate", type=int, default=0, metavar="BYTES",
                    help="only stream BYTES through a plain device copy kernel 5 times (counter calibration)")
    ap.add_argument("--serve-requests", type=int, default=100000, help="requests replayed from the stream (0: skip)")
    ap.add_argument("--recall-files", type=int, default=1024, help="files of the recall sample (0: skip)")
    ap.add_argument("--serve-budget", type=int, default=16 << 30, help="serving HBM budget in bytes")
    ap.add_argument("--serve-streams", type=int, default=4)
    ap.add_argument("--serve-batch", type=int, default=64)
    ap.add_argument("--configs", default="1,3,4",
                    help="other workloads whose whole chain is timed pass by pass (comma list; '' to skip)")
    ap.add_argument("--configs-only", action="store_true",
                    help="time only the --configs chains (for profiling them; prints their JSON, not the benchmark line)")
    ap.add_argument("--configs-launch", default=None,
                    help="with --configs-only: fixed launch shape and table sizes CHUNK,BLOCK,SETCAP,WG_PER_CU,MAP,FILTWORDS "
                         "for the chains instead of the autotuner")
    ap.add_argument("--saturation-requests", type=int, default=20000,
                    help="requests of the closed-loop serving saturation run (0: skip)")
    a = ap.parse_args()
    if a.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py runs on one GPU only: the Intergrams pass is measured on a single MI355X; "
              "--gpus %d is not supported" % a.gpus, file=sys.stderr)
        sys.exit(2)

    if a.copy_calibrate:
        # a plain streaming kernel of known size: reads BYTES and writes BYTES
        import torch
        n = a.copy_calibrate // 4
        src = torch.arange(n, dtype=torch.int32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(5):
            torch.neg(src, out=dst)
        torch.cuda.synchronize()
        print(json.dumps({"copy_calibrate_bytes": n * 4, "launches": 5, "kernel": "torch.neg int32"}), flush=True)
        return

    import gen
    import paper_2511_14955_amd as ig

    threads = min(16, os.cpu_count() or 1)
    if a.configs_only:
        fixed = [int(x) for x in a.configs_launch.split(",")] if a.configs_launch else None
        out = {str(w): config_chain(ig, w, threads, tune_at=None if fixed else {3: 8, 4: 16}.get(w), fixed=fixed)
               for w in [int(x) for x in a.configs.split(",") if x.strip()]}
        print(json.dumps({"configs": out}), flush=True)
        return
    t0 = time.time()
    corpus = gen.workload(2, m=a.m, nthreads=threads)
    log("workload 2: %d files, %d bytes, generated in %.1fs" % (corpus.m, corpus.nbytes, time.time() - t0))

    g = ig.Intergrams(symbol_bits=8, freq=ig.FREQ_DOC, flags=a.flags)
    g.load(corpus)
    if a.launch:
        g.set_launch(*[int(x) for x in a.launch.split(",")])
    for j in range(1, a.n):
        g.pass_(j, a.k)
        st = g.last_stats()
        log("pass %d: %.3f ms (scan %.3f ms, select %.3f ms), kept %d, distinct %d, records %d" % (
            j, st["pass_ms"], st["scan_ms"], st["select_ms"], g.table_info()[1], st["distinct"], st["records"]))
    if a.tables:
        ml, fw = [int(x) for x in a.tables.split(",")]
        g.set_tables(map_slots_log2=ml, filter_max_words=fw)   # re-indexes the n-1 table
    tune = None
    if not a.no_tune and not a.launch:
        t_t = time.time()
        tune = g.autotune(a.n, a.k)
        log("autotune: best %s (%d candidates, identical tables: %s, %.1fs)" % (
            tune["best"], len(tune["candidates"]), tune["identical"], time.time() - t_t))
    # first pass n (not timed) so that every step can rewind to the n-1 table
    g.pass_(a.n, a.k)
    for _ in range(a.warmup):
        g.rewind()
        g.pass_(a.n, a.k)
    scan_ms, pass_ms = [], []
    t_start = time.perf_counter()
    for _ in range(a.steps):
        g.rewind()
        g.pass_(a.n, a.k)
        st = g.last_stats()
        scan_ms.append(st["scan_ms"])
        pass_ms.append(st["pass_ms"])
    t_end = time.perf_counter()
    ms_per_step = (t_end - t_start) * 1e3 / a.steps
    st = g.last_stats()
    value = corpus.nbytes / (ms_per_step * 1e-3) / 1e9
    scan_avg = sum(scan_ms) / len(scan_ms)
    # algorithmic bytes of one scan launch: the corpus once plus the (n-1)-symbol halo of every chunk
    nchunks = int(sum(-(-int(L) // st["chunk_syms"]) for L in (corpus.offsets[1:] - corpus.offsets[:-1])))
    algo_bytes = corpus.nbytes + nchunks * (a.n - 1)
    achieved = algo_bytes / (scan_avg * 1e-3) / 1e9
    log("pass %d: %.3f ms/step wall, device pass %.3f ms, scan %.3f ms, %.1f GB/s" % (
        a.n, ms_per_step, sum(pass_ms) / len(pass_ms), scan_avg, value))

    extra = {"device_pass_ms": round(sum(pass_ms) / len(pass_ms), 4),
             "tables": {k: v for k, v in g.tables().items() if k in ("map_slots_log2", "filter_bits_per_key",
                                                                       "filter_max_words")},
             "device_pass_ms_median": round(sorted(pass_ms)[len(pass_ms) // 2], 4),
             "scan_ms": round(scan_avg, 4),
             "select_ms": round(st["select_ms"], 4), "windows": st["windows"], "distinct_counted": st["distinct"],
             "split_file_records": st["records"],
             "launch": {"chunk_syms": st["chunk_syms"], "block": st["block"], "grid": st["grid"],
                        "set_cap": g.launch()["set_cap"], "wg_per_cu": g.launch()["wg_per_cu"]},
             "graph_captured": not (a.flags & 1)}
    if tune:
        extra["autotune"] = {"identical_tables": tune["identical"],
                             "candidates": [[c["chunk_syms"], c["block"], c["set_cap"], c["wg_per_cu"],
                                             c["map_slots_log2"], c["filter_max_words"], round(c["pass_ms"], 3)]
                                            for c in tune["candidates"]]}
    # Figure 1's m x k Boolean matrix of the whole loaded corpus against this pass's table
    # (device bitmaps, then CSR copied to the host)
    t1 = time.perf_counter()
    fip, find = g.featurize_loaded()
    t2 = time.perf_counter()
    extra["featurize_corpus"] = {"ms": round((t2 - t1) * 1e3, 3), "GB_per_s": round(corpus.nbytes / (t2 - t1) / 1e9, 3),
                                 "rows": int(len(fip) - 1), "nnz": int(len(find)),
                                 "note": "whole loaded corpus, CSR on the host included"}
    log("featurize whole corpus: %s" % extra["featurize_corpus"])
    del fip, find
    serving = None
    if a.serve_requests:
        serving = serve_stream(g, ig, a.serve_requests, a.serve_budget, a.serve_streams, a.serve_batch)
        log("serving: %s" % serving)
        if a.saturation_requests:
            rs = gen.RequestStream()
            files = [rs.file(i) for i in range(a.saturation_requests)]
            serving["saturation"] = serve_saturation(g, ig, files, a.serve_budget, a.serve_streams, a.serve_batch)
            log("serving saturation: %s" % serving["saturation"])
            del files
    if not a.no_per_file:
        gp = ig.Intergrams(symbol_bits=8, freq=ig.FREQ_DOC, flags=a.flags | ig.FLAG_PER_FILE)
        lc = g.launch()
        gp.set_launch(lc["chunk_syms"], lc["block"], lc["set_cap"], lc["wg_per_cu"])
        gp.load(corpus)
        for j in range(1, a.n):
            gp.pass_(j, a.k)
        t1 = time.perf_counter()
        gp.pass_(a.n, a.k)
        t2 = time.perf_counter()
        same = bool((gp.topk()[0] == g.topk()[0]).all() and (gp.topk()[1] == g.topk()[1]).all())
        extra["per_file_form"] = {"ms_per_pass": round((t2 - t1) * 1e3, 3),
                                  "GB_per_s": round(corpus.nbytes / (t2 - t1) / 1e9, 3),
                                  "scan_ms": round(gp.last_stats()["scan_ms"], 3), "same_table": same}
        log("per-file form: %.3f ms, same table: %s" % ((t2 - t1) * 1e3, same))
        gp.close()
    g_launch = g.launch()
    g_tables = g.tables()
    # what a plain streaming read attains on this device, for comparison with the pass's rate
    extra["hbm_read_attainable"] = {"GB_per_s": round(g.measure_read_bw(4 << 30, 5), 1), "bytes": 4 << 30,
                                    "kernel": "the library's streaming-read kernel (16-byte non-temporal loads)"}
    log("attainable HBM read: %s" % extra["hbm_read_attainable"])
    g.close()
    configs = {}
    for w in [int(x) for x in a.configs.split(",") if x.strip()]:
        configs[str(w)] = config_chain(ig, w, threads, tune_at={3: 8, 4: 16}.get(w))
    extra["configs"] = configs
    quality = None
    theory_rows = None
    if a.recall_files:
        import gen
        from paper_2511_14955_amd import theory
        sample = gen.workload(2, m=a.recall_files, nthreads=threads)
        quality = recall_sample(ig, a.n, a.k, sample)
        log("recall: %s" % quality)
        # Section 4.3's quantities per step n -> n+1 on the same sample
        def fin(v):   # JSON has no NaN or infinity
            return (round(v, 6) if math.isfinite(v) else None) if isinstance(v, float) else v
        theory_rows = []
        for r in theory.diagnostics(ig, sample, list(range(2, a.n)), a.k):
            theory_rows.append({key: ([{kk: fin(vv) for kk, vv in c.items()} for c in v] if isinstance(v, list) else fin(v))
                                for key, v in r.items()})
        log("theory: %s" % theory_rows)
        del sample

    out = {
        "metric": "input GB/s per Intergrams pass (n=8,k=1e5) + %HBM roofline; p50/p99 featurize ms",
        "value": round(value, 3), "unit": "GB/s", "n_gpus": 1, "steps": a.steps, "warmup": a.warmup,
        "ms_per_step": round(ms_per_step, 4), "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "u64", "data": "synthetic",
        "config": {"workload": "binary-like corpus: %d files, lognormal sizes (median 64 KiB, sigma 1.5, cap 16 MiB), "
                               "%d bytes; one pass n=%d, k_keep=%d, Eq. 2" % (corpus.m, corpus.nbytes, a.n, a.k),
                   "files": corpus.m, "bytes": corpus.nbytes, "n": a.n, "k_keep": a.k, "freq": "doc"},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 2), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None,
                     "kernel": "k_scan (scan of pass n=%d)" % a.n, "algo_bytes_per_launch": algo_bytes,
                     "avg_launch_ms": round(scan_avg, 4)},
        "serving": serving,
        "quality": quality,
        "theory": theory_rows,
        "extra": extra,
    }
    lc = g_launch
    rec, tsrc = profiled_record(a.n, [lc["chunk_syms"], lc["block"], lc["set_cap"], lc["wg_per_cu"],
                                      g_tables["map_slots_log2"], g_tables["filter_max_words"]])
    out["roofline"]["traffic"] = rec["traffic_bytes_per_launch"] if rec else None
    out["roofline"]["traffic_source"] = tsrc
    out["roofline"]["valu_issue"] = valu_issue(rec, scan_avg)
    if not a.no_cpu:
        out["cpu_baseline"] = cpu_baseline(a.n, a.k, a.cpu_sample_files, threads)
        log("cpu baseline: %s" % out["cpu_baseline"])
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
