"""Write expected pass tables for full-size workloads, computed by the CPU oracle only.

Usage: python tests/golden/make_golden.py WORKLOAD [--threads T] [--m M] [--table-out FILE.npz]
                                          [--freq doc|occ] [--nmax N]

For each pass of the chain (n = 1..N, k_keep = K, Eq. 2 frequency by default, Eq. 1 with
--freq occ, which writes workload<W>_occ.json; --nmax cuts the chain short) it stores
the kept length, the SHA-256 of the ordered table (little-endian uint64 triples
key_lo, key_hi, count) and the first and last entries, plus the corpus digest,
in tests/golden/workload<W>.json.  With --table-out, the last pass's whole ordered table (keys as
uint64 (lo, hi) pairs and counts) also goes to a compressed .npz file.  Nothing here reads the HIP
library.
"""
import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import gen  # noqa: E402
import oracle  # noqa: E402

CHAINS = {1: (4, 1000), 2: (8, 100000), 3: (16, 1000000), 4: (31, 1000000)}


def table_digest(keys, counts):
    arr = np.zeros((len(counts), 3), np.uint64)
    if len(counts):
        arr[:, 0] = keys[:, 0]
        arr[:, 1] = keys[:, 1]
        arr[:, 2] = counts
    return hashlib.sha256(arr.astype("<u8").tobytes()).hexdigest()


def entry(keys, counts, i):
    return [str(int(keys[i, 0]) | (int(keys[i, 1]) << 64)), int(counts[i])]


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("workload", type=int)
    ap.add_argument("--threads", type=int, default=os.cpu_count())
    ap.add_argument("--m", type=int, default=None)
    ap.add_argument("--out", default=None)
    ap.add_argument("--table-out", default=None, help="npz file for the last pass's ordered table")
    ap.add_argument("--freq", choices=["doc", "occ"], default="doc")
    ap.add_argument("--nmax", type=int, default=None)
    a = ap.parse_args()
    nmax, k_keep = CHAINS[a.workload]
    nmax = min(nmax, a.nmax or nmax)
    corpus = gen.workload(a.workload, m=a.m, nthreads=a.threads)
    rec = {"workload": a.workload, "m": corpus.m, "symbol_bits": corpus.symbol_bits, "bytes": corpus.nbytes,
           "corpus_sha256": corpus.sha256(), "freq": a.freq, "k_keep": k_keep, "passes": {}}
    o = oracle.Oracle(corpus.symbol_bits, oracle.FREQ_OCC if a.freq == "occ" else oracle.FREQ_DOC,
                      nthreads=a.threads)
    o.load(corpus)
    out = a.out or os.path.join(os.path.dirname(os.path.abspath(__file__)),
                                "workload%d%s%s.json" % (a.workload, "" if a.m is None else "_m%d" % a.m,
                                                         "_occ" if a.freq == "occ" else ""))
    for n in range(1, nmax + 1):
        t0 = time.time()
        rc = o.pass_(n, k_keep)
        assert rc == 0, rc
        keys, counts = o.topk()
        k = len(counts)
        rec["passes"][str(n)] = {"kept": k, "sha256": table_digest(keys, counts),
                                 "head": [entry(keys, counts, i) for i in range(min(8, k))],
                                 "tail": [entry(keys, counts, i) for i in range(max(0, k - 4), k)]}
        print("workload %d pass %d kept %d %.1fs" % (a.workload, n, k, time.time() - t0), flush=True)
        with open(out, "w") as fh:
            json.dump(rec, fh, indent=1)
    if a.table_out:
        keys, counts = o.topk()
        np.savez_compressed(a.table_out, keys=np.ascontiguousarray(keys, np.uint64),
                            counts=np.ascontiguousarray(counts, np.uint64), n=np.uint32(nmax),
                            k_keep=np.uint64(k_keep), workload=np.uint32(a.workload))


if __name__ == "__main__":
    main()
