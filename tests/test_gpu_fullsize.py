"""Full-size workloads on the GPU, in the launch configuration the benchmark times.

- The binary-like corpus (16,384 files, ~3.24 GB, n = 1..8, k_keep = 1e5):
  every pass's ordered table equals the oracle's, by the SHA-256 digests and
  head/tail entries that tests/golden/make_golden.py wrote from the oracle;
  then 600 requests of the serving workload, featurized through the serving
  loop against that n = 8 table, equal the oracle's rows against its own
  stored table.
- The text-like (4 GiB, n = 1..16, k_keep = 1e6, 128-bit keys) and genomic
  (2-bit, n = 1..31, k_keep = 1e6) corpora take the oracle hours, so their
  expected tables are the digests make_golden.py stored (every pass equal to the
  oracle's, where the file exists); they are also checked by properties that
  hold at any size (order, Eq. 2 bounds, prefix closure and anti-monotonicity of
  the chain, the exact pass-1 table) and by exact document counts of sampled
  grams, kept and not kept, found by brute-force substring search over the files.
"""
import json
import os
import sys
import time

import numpy as np
import pytest

import gen

pytestmark = [pytest.mark.gpu, pytest.mark.slow]

ig = pytest.importorskip("paper_2511_14955_amd")

sys.path.insert(0, os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden"))
from make_golden import table_digest  # noqa: E402


def say(*a):
    print("[case]", *a, flush=True)


def test_workload2_full_chain_matches_golden(golden_dir):
    with open(os.path.join(golden_dir, "workload2.json")) as fh:
        gold = json.load(fh)
    say("workload 2 full size: generating")
    corpus = gen.workload(2, nthreads=min(16, os.cpu_count() or 1))
    assert corpus.m == gold["m"] and corpus.nbytes == gold["bytes"]
    assert corpus.sha256() == gold["corpus_sha256"]
    k = gold["k_keep"]
    g = ig.Intergrams(symbol_bits=8, freq=ig.FREQ_DOC)
    g.load(corpus)

    def check(n, what):
        keys, counts = g.topk()
        exp = gold["passes"][str(n)]
        assert len(counts) == exp["kept"], what
        for i, (key, c) in enumerate(exp["head"]):
            assert (int(keys[i, 0]) | (int(keys[i, 1]) << 64), int(counts[i])) == (int(key), c), (what, i)
        assert table_digest(keys, counts) == exp["sha256"], what

    for n in range(1, 8):
        say("workload 2 pass %d" % n)
        g.pass_(n, k)
        check(n, "pass %d" % n)
    say("workload 2: autotune pass 8, then pass 8 and two graph replays after rewinds")
    rep = g.autotune(8, k)
    assert rep["identical"]
    g.pass_(8, k)
    check(8, "pass 8")
    for r in range(2):
        g.rewind()
        g.pass_(8, k)
        check(8, "pass 8 replay %d" % r)
    _serving_rows_match_oracle(g, golden_dir, gold)
    g.close()


def _serving_rows_match_oracle(g, golden_dir, gold, requests=600):
    """The serving workload's featurize requests (the first `requests` of its stream, files
    generated like the corpus's) against this n = 8, k = 1e5 table, through the serving loop,
    equal the oracle's featurization against the oracle's own table for this pass (stored by
    make_golden.py --table-out)."""
    import oracle
    path = os.path.join(golden_dir, "workload2_n8_table.npz")
    with np.load(path, allow_pickle=False) as z:
        okeys, ocounts = z["keys"], z["counts"]
    exp = gold["passes"]["8"]
    assert table_digest(okeys, ocounts) == exp["sha256"], "stored table is not the pass-8 golden table"
    o = oracle.Oracle(8, oracle.FREQ_DOC, nthreads=min(16, os.cpu_count() or 1))
    o.set_retained(8, oracle.keys_to_int(okeys), ocounts)
    rs = gen.RequestStream()
    files = [rs.file(i) for i in range(requests)]
    say("serving: %d requests of the request stream (%d bytes) against the n=8 table" % (
        requests, sum(len(f) for f in files)))
    ip, ind = o.featurize(gen.from_files(files))
    g.serve_start(max_inflight_bytes=2 << 30, n_streams=4, max_batch=16)
    try:
        for i, f in enumerate(files):
            assert g.submit(ig.REQ_FEATURIZE, f, np.array([0, len(f)], np.uint64), tag=i) == ig.IG_OK
        got = {}
        t_end = time.time() + 120
        while len(got) < requests:
            for r in g.poll():
                got[r["tag"]] = r
            assert time.time() < t_end
    finally:
        g.serve_stop()
    for i in range(requests):
        assert got[i]["status"] == ig.IG_OK
        assert np.array_equal(got[i]["cols"], ind[int(ip[i]):int(ip[i + 1])]), "request %d" % i
    say("serving: %d rows equal the oracle's (%d entries)" % (requests, len(ind)))


# ---------------------------------------------------------------- properties

def _key_int(keys, i):
    return int(keys[i, 0]) | (int(keys[i, 1]) << 64)


def _gram(key, n, bits):
    mask = (1 << bits) - 1
    return bytes(((key >> (bits * (n - 1 - r))) & mask) for r in range(n))


def _doc_count(buf, offs, gram):
    """Files whose symbol range contains gram (one symbol per byte of buf)."""
    c = 0
    find = buf.find
    for i in range(len(offs) - 1):
        if find(gram, offs[i], offs[i + 1]) >= 0:
            c += 1
    return c


def _check_order(keys, counts, m, what):
    assert len(counts) == 0 or int(counts[0]) <= m, what
    c = counts.astype(np.uint64)
    hi, lo = keys[:, 1], keys[:, 0]
    dc = c[1:] < c[:-1]
    eq = c[1:] == c[:-1]
    kgt = (hi[1:] > hi[:-1]) | ((hi[1:] == hi[:-1]) & (lo[1:] > lo[:-1]))
    assert bool(np.all(dc | (eq & kgt))), "%s: not in (count desc, key asc) order" % what
    assert int(c[-1]) >= 1, what


def _check_prefix_closure(keys, counts, prev, bits, what):
    """Every kept n-gram's (n-1)-prefix is retained and at least as frequent (Eq. 2 is anti-monotone)."""
    pk, pc = prev
    lo, hi = keys[:, 0], keys[:, 1]
    plo = (lo >> np.uint64(bits)) | (hi << np.uint64(64 - bits))
    phi = hi >> np.uint64(bits)
    if not hi.any() and not pk[:, 1].any():
        order = np.argsort(pk[:, 0], kind="stable")
        sk = pk[order, 0]
        pos = np.minimum(np.searchsorted(sk, plo), len(sk) - 1)
        found = sk[pos] == plo
        pcount = pc[order][pos]
    else:
        allk = np.concatenate([np.stack([pk[:, 1], pk[:, 0]], 1), np.stack([phi, plo], 1)])
        _, inv = np.unique(allk, axis=0, return_inverse=True)
        inv = inv.reshape(-1)
        by_id = np.full(int(inv.max()) + 1, -1, np.int64)
        by_id[inv[:len(pk)]] = pc.astype(np.int64)
        pcount = by_id[inv[len(pk):]]
        found = pcount >= 0
    bad = np.nonzero(~found)[0]
    assert len(bad) == 0, "%s: rank %d has a prefix that was not retained" % (what, int(bad[0]))
    worse = np.nonzero(counts.astype(np.int64) > pcount.astype(np.int64))[0]
    assert len(worse) == 0, "%s: rank %d outnumbers its prefix" % (what, int(worse[0]))


def _run_chain(corpus, nmax, k):
    g = ig.Intergrams(symbol_bits=corpus.symbol_bits, freq=ig.FREQ_DOC)
    g.load(corpus)
    tables = []
    for n in range(1, nmax + 1):
        g.pass_(n, k)
        keys, counts = g.topk()
        tables.append((keys.copy(), counts.copy()))
    g.close()
    return tables


def _sampled_counts(buf, offs, tables, bits, ns, rng, what):
    """Exact Eq. 2 counts of sampled kept grams, and a completeness check on
    sampled windows: a gram that is not kept but whose prefix is retained must
    not beat the last kept gram."""
    for n in ns:
        keys, counts = tables[n - 1]
        k = len(counts)
        ranks = sorted({0, k // 2, k - 1})
        for i in ranks:
            key = _key_int(keys, i)
            got = _doc_count(buf, offs, _gram(key, n, bits))
            assert got == int(counts[i]), "%s pass %d rank %d: count %d, brute force %d" % (
                what, n, i, int(counts[i]), got)
        if n == 1:
            continue
        kept = {_key_int(keys, i) for i in range(k)}
        pk, _ = tables[n - 2]
        prev = {_key_int(pk, i) for i in range(len(pk))}
        last_c, last_key = int(counts[-1]), _key_int(keys, k - 1)
        for _ in range(400):
            f = int(rng.integers(0, len(offs) - 1))
            a, z = offs[f], offs[f + 1]
            if z - a < n:
                continue
            p = int(rng.integers(a, z - n + 1))
            gram = buf[p:p + n]
            key = 0
            for s in gram:
                key = (key << bits) | s
            if key in kept or (key >> bits) not in prev:
                continue
            c = _doc_count(buf, offs, gram)
            assert c < last_c or (c == last_c and key > last_key), \
                "%s pass %d: gram %x (count %d) beats the last kept (count %d)" % (what, n, key, c, last_c)
            break


def _symbols_as_bytes(corpus):
    if corpus.symbol_bits == 8:
        return corpus.data.tobytes(), [int(x) for x in corpus.offsets]
    syms = gen.unpack2(corpus.data, 0, int(corpus.offsets[-1]))
    return syms.tobytes(), [int(x) for x in corpus.offsets]


def _pass1_exact(buf, offs, keys, counts, k, what):
    """Pass 1 keeps every symbol: its table is the exact per-symbol document frequency."""
    df = np.zeros(256, np.int64)
    mv = np.frombuffer(buf, np.uint8)
    for i in range(len(offs) - 1):
        if offs[i + 1] > offs[i]:
            df += np.bincount(mv[offs[i]:offs[i + 1]], minlength=256) > 0
    present = [(int(df[s]), s) for s in range(256) if df[s]]
    present.sort(key=lambda t: (-t[0], t[1]))
    present = present[:k]
    assert [(int(keys[i, 0]), int(counts[i])) for i in range(len(counts))] == [(s, c) for c, s in present], what


_CORPUS = {}


def _workload(w):
    """The full-size corpus of workload w, generated once for the tests that share it."""
    if w not in _CORPUS:
        _CORPUS.clear()
        t0 = time.time()
        _CORPUS[w] = gen.workload(w, nthreads=min(16, os.cpu_count() or 1))
        say("workload %d full size: %d sequences, %d bytes (%.1fs)" % (w, _CORPUS[w].m, _CORPUS[w].nbytes,
                                                                       time.time() - t0))
    return _CORPUS[w]


def _stream_pair_counts(buf):
    """counts[a, b] = positions i of the byte stream with buf[i] = a and buf[i+1] = b (pairs that
    straddle a sequence boundary included), from the stream read as little-endian 16-bit words
    at even and then at odd offsets."""
    from concurrent.futures import ThreadPoolExecutor
    step = 1 << 24
    parts = [np.frombuffer(buf, dtype="<u2", count=(len(buf) - off) // 2, offset=off) for off in (0, 1)]
    spans = [(w, s) for w in parts for s in range(0, len(w), step)]
    with ThreadPoolExecutor(min(16, os.cpu_count() or 1)) as ex:
        cnt = sum(ex.map(lambda t: np.bincount(t[0][t[1]:t[1] + step], minlength=1 << 16), spans),
                  np.zeros(1 << 16, np.int64))
    # the word at offset i is buf[i] | buf[i + 1] << 8
    return cnt.reshape(256, 256).T


def _occ_table(counts):
    """(key, count) of every nonzero entry, in (count desc, key asc) order."""
    keys = np.nonzero(counts)[0]
    order = np.lexsort((keys, -counts[keys]))
    return [(int(keys[i]), int(counts[keys[i]])) for i in order]


def test_workload3_eq1_64bit_counters(golden_dir):
    """Eq. 1 on the full text corpus: 2^32 windows at n = 1, so 32-bit counts are refused with
    IG_EOVERFLOW and the 64-bit device counters are used.  Every pass of the stored chain (n =
    1..12, k_keep = 1e6; from n = 9 on the windows take more than 64 bits) equals the oracle's
    table by the digests make_golden.py --freq occ wrote, and passes 1 and 2 (which keep every
    gram present) equal exact occurrence counts of every byte and byte pair of the files."""
    with open(os.path.join(golden_dir, "workload3_occ.json")) as fh:
        gold = json.load(fh)
    assert gold["freq"] == "occ"
    corpus = _workload(3)
    assert corpus.m == gold["m"] and corpus.nbytes == gold["bytes"] and corpus.sha256() == gold["corpus_sha256"]
    k = gold["k_keep"]
    assert corpus.nbytes >= 1 << 32
    say("workload 3, Eq. 1: 32-bit counts refused with IG_EOVERFLOW")
    g32 = ig.Intergrams(symbol_bits=8, freq=ig.FREQ_OCC, count_bits=32)
    try:
        g32.load(corpus)
        assert g32.try_pass(1, k) == ig.IG_EOVERFLOW
        assert g32.table_info() == (0, 0)
    finally:
        g32.close()
    say("workload 3, Eq. 1 with 64-bit counters: passes 1..%d" % len(gold["passes"]))
    g = ig.Intergrams(symbol_bits=8, freq=ig.FREQ_OCC, count_bits=64)
    tables = []
    try:
        g.load(corpus)
        for n in range(1, len(gold["passes"]) + 1):
            g.pass_(n, k)
            keys, counts = g.topk()
            tables.append((keys.copy(), counts.copy()))
            exp = gold["passes"][str(n)]
            assert len(counts) == exp["kept"], "pass %d: kept %d vs %d" % (n, len(counts), exp["kept"])
            for i, (key, c) in enumerate(exp["head"]):
                assert (_key_int(keys, i), int(counts[i])) == (int(key), c), (n, i)
            assert table_digest(keys, counts) == exp["sha256"], "Eq. 1 pass %d digest" % n
    finally:
        g.close()
    t0 = time.time()
    buf = corpus.data
    pairs = _stream_pair_counts(buf)
    ones = pairs.sum(axis=1)
    ones[int(buf[-1])] += 1
    assert int(ones.sum()) == corpus.nbytes
    offs = np.asarray(corpus.offsets, np.int64)
    cut = np.unique(offs[(offs > 0) & (offs < corpus.nbytes)])
    np.subtract.at(pairs, (buf[cut - 1], buf[cut]), 1)
    assert int(pairs.sum()) == corpus.nbytes - len(cut) - 1
    for n, exact in ((1, ones), (2, pairs.reshape(-1))):
        keys, counts = tables[n - 1]
        assert int(keys[:, 1].max()) == 0
        got = [(int(keys[i, 0]), int(counts[i])) for i in range(len(counts))]
        assert got == _occ_table(exact), "Eq. 1 pass %d vs exact occurrence counts" % n
    assert int(tables[0][1][0]) < 1 << 32 <= int(tables[0][1].sum())
    say("workload 3, Eq. 1: passes 1 and 2 equal exact byte and byte-pair counts (%.1fs)" % (time.time() - t0))


@pytest.mark.parametrize("workload,nmax,k,sample_ns", [(3, 16, 1000000, [2, 16]), (4, 31, 1000000, [2, 31])])
def test_full_size_properties_and_samples(golden_dir, workload, nmax, k, sample_ns):
    t0 = time.time()
    corpus = _workload(workload)
    tables = _run_chain(corpus, nmax, k)
    say("workload %d: chain n=1..%d done (%.1fs)" % (workload, nmax, time.time() - t0))
    # the oracle's digests of every pass, where make_golden.py has written them
    gpath = os.path.join(golden_dir, "workload%d.json" % workload)
    if os.path.exists(gpath):
        with open(gpath) as fh:
            gold = json.load(fh)
        assert corpus.m == gold["m"] and corpus.nbytes == gold["bytes"] and corpus.sha256() == gold["corpus_sha256"]
        # make_golden.py writes the passes in order as the oracle finishes them: every pass the
        # file holds is compared (all of the chain once it is complete)
        ng = len(gold["passes"])
        assert gold["k_keep"] == k and 1 <= ng <= nmax and sorted(map(int, gold["passes"])) == list(range(1, ng + 1)), \
            "golden file for a different chain"
        for n in range(1, ng + 1):
            keys, counts = tables[n - 1]
            exp = gold["passes"][str(n)]
            assert len(counts) == exp["kept"], "workload %d pass %d: kept %d vs %d" % (workload, n, len(counts), exp["kept"])
            for i, (key, c) in enumerate(exp["head"]):
                assert (_key_int(keys, i), int(counts[i])) == (int(key), c), (workload, n, i)
            assert table_digest(keys, counts) == exp["sha256"], "workload %d pass %d digest" % (workload, n)
        say("workload %d: passes 1..%d of %d equal the oracle's digests (%.1fs)" % (workload, ng, nmax, time.time() - t0))
    bits = corpus.symbol_bits
    for n in range(1, nmax + 1):
        keys, counts = tables[n - 1]
        _check_order(keys, counts, corpus.m, "pass %d" % n)
        if n > 1:
            _check_prefix_closure(keys, counts, tables[n - 2], bits, "pass %d" % n)
    say("workload %d: order and prefix closure hold on every pass (%.1fs)" % (workload, time.time() - t0))
    buf, offs = _symbols_as_bytes(corpus)
    del corpus
    _CORPUS.clear()
    _pass1_exact(buf, offs, *tables[0], k, "pass 1")
    rng = np.random.default_rng(1000 + workload)
    _sampled_counts(buf, offs, tables, bits, sample_ns, rng, "workload %d" % workload)
    say("workload %d: sampled exact counts match (%.1fs)" % (workload, time.time() - t0))
