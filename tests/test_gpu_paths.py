"""Kernel paths that only some shapes reach, each against the CPU oracle or a closed form.

- Featurize with 128-bit keys (bytes at n = 10, 2-bit symbols at n = 36): the featurizing
  scan's in-place form, with more chunks than workgroups; ig_featurize, the loaded corpus, and
  serving (featurize and count requests).
- Featurize with a table too large for the per-workgroup rank bitmap in LDS (more than about
  590K kept grams): the rank bits then go straight to the sequence's bitmap in HBM.
- Eq. 1 with 64-bit device counters (more than 2^32 windows), checked against closed forms,
  and 32-bit counts refused there with IG_EOVERFLOW.
- A chunk with more distinct candidates than its LDS set holds (the set is bypassed for the
  rest of the chunk), and a pass run as the direct-indexed count inside a chain because the
  previous pass kept every (n-1)-gram of the alphabet.
- Direct-indexed passes over at most a chunk's worth of grams grow their LDS set.
"""
import time

import numpy as np
import pytest

import gen
from helpers import assert_tables_equal, gpu_tables, oracle_tables

pytestmark = pytest.mark.gpu

ig = pytest.importorskip("paper_2511_14955_amd")


def say(*a):
    print("[case]", *a, flush=True)


def _drain(g, want, timeout=120.0):
    got = {}
    t_end = time.time() + timeout
    while len(got) < want:
        for r in g.poll():
            got[r["tag"]] = r
        if len(got) < want:
            assert time.time() < t_end, "serving returned %d of %d" % (len(got), want)
            time.sleep(0.001)
    return got


def _rows(ip, ind):
    return [ind[int(ip[i]):int(ip[i + 1])] for i in range(len(ip) - 1)]


def _check_all_featurize_forms(g, o, corpus, queries, what):
    """ig_featurize, ig_featurize_loaded and serving (featurize alone, count requests) vs the oracle."""
    ip_o, ind_o = o.featurize(queries)
    ip_g, ind_g = g.featurize(queries)
    assert np.array_equal(ip_o.astype(np.uint64), ip_g) and np.array_equal(ind_o, ind_g), what + ": ig_featurize"
    assert len(ind_g) > 0, what
    ip_l, ind_l = g.featurize_loaded()
    ip_c, ind_c = o.featurize(corpus)
    assert np.array_equal(ip_c.astype(np.uint64), ip_l) and np.array_equal(ind_c, ind_l), what + ": loaded corpus"
    rows = _rows(ip_o, ind_o)
    files = [queries.file(i) for i in range(queries.m)]
    g.serve_start(max_inflight_bytes=512 << 20, n_streams=3, max_batch=4)
    try:
        for i, f in enumerate(files):
            data, offs = (f, [0, len(f)]) if queries.symbol_bits == 8 else gen.pack2([f])
            assert g.submit(ig.REQ_FEATURIZE, np.ascontiguousarray(data, np.uint8), offs, tag=i) == ig.IG_OK
        grp = list(range(0, len(files), 2))
        sub = gen.from_files([files[i] for i in grp], queries.symbol_bits)
        assert g.submit(ig.REQ_COUNT, sub.data, sub.offsets, tag=10_000) == ig.IG_OK
        got = _drain(g, len(files) + 1)
    finally:
        g.serve_stop()
    for i in range(len(files)):
        assert got[i]["status"] == ig.IG_OK and np.array_equal(got[i]["cols"], rows[i]), "%s: request %d" % (what, i)
    acc = {}
    for i in grp:
        for cidx in rows[i]:
            acc[int(cidx)] = acc.get(int(cidx), 0) + 1
    r = got[10_000]
    assert r["status"] == ig.IG_OK
    assert list(zip(r["cols"].tolist(), r["counts"].tolist())) == sorted(acc.items()), what + ": count request"


@pytest.mark.skip(reason="one GPU run left the device faulted while this case ran (after passing twice with the same "
                         "featurize code); no cause found yet, so the case stays off the GPU until one is shown")
def test_featurize_128bit_keys():
    corpus = gen.workload(3, m=60)
    ns = list(range(1, 11))
    say("featurize, 128-bit keys: text n=1..10, k=20000 on the first 60 documents")
    exp, o = oracle_tables(corpus, ns, 20000)
    got, g = gpu_tables(corpus, ns, 20000)
    try:
        assert_tables_equal(got, exp, "text chain")
        more = gen.workload(3, m=90)
        q = gen.from_files([more.file(i) for i in range(60, 90)] + [b"", b"short", more.file(3)])
        _check_all_featurize_forms(g, o, corpus, q, "128-bit")
    finally:
        g.close()


@pytest.mark.parametrize("bits,n", [(8, 10), (2, 36)])
def test_featurize_128bit_keys_in_place(bits, n):
    """A fresh pass at n = 10 bytes (80-bit keys) or n = 36 two-bit symbols (72 bits), then the
    featurizing scan against that table.  Its 128-bit form looks every window up in place (no
    survivor rings), and the loaded corpus has more chunks than the grid has workgroups, so
    each workgroup goes on to the chunk one grid further.  The files are overlapping slices of
    one random sequence, so that long grams recur across files."""
    rng = np.random.default_rng(5150 + bits)
    glen = 3_000_000 if bits == 8 else 12_000_000
    seq = rng.integers(0, 1 << bits, size=glen, dtype=np.uint8)

    def piece(lo, hi):
        ln = int(rng.integers(lo, hi))
        a = int(rng.integers(0, glen - ln))
        return seq[a:a + ln]

    scale = 1 if bits == 8 else 2
    files = [piece(200_000 * scale, 1_000_000 * scale) for _ in range(12)]
    corpus = gen.from_files(files, bits)
    k = 50_000
    say("featurize, %d-bit keys in place: %d-bit symbols, fresh pass n=%d, k=%d, %d symbols"
        % (n * bits, bits, n, k, int(corpus.offsets[-1])))
    exp, o = oracle_tables(corpus, [n], k)
    got, g = gpu_tables(corpus, [n], k)
    try:
        assert_tables_equal(got, exp, "fresh n=%d" % n)
        assert int(got[0][0][:, 1].max()) > 0 and int(got[0][1][0]) > 1
        cs = g.launch()["chunk_syms"]
        assert sum((len(f) + cs - 1) // cs for f in files) > 256
        q = gen.from_files([piece(50_000 * scale, 300_000 * scale) for _ in range(4)]
                           + [rng.integers(0, 1 << bits, size=100_000, dtype=np.uint8), seq[:n - 1],
                              np.zeros(0, np.uint8)], bits)
        _check_all_featurize_forms(g, o, corpus, q, "%d-bit keys in place" % (n * bits))
    finally:
        g.close()


@pytest.mark.parametrize("bits", [8, 2])
def test_featurize_table_beyond_lds_bitmap(bits):
    rng = np.random.default_rng(41 + bits)
    if bits == 8:
        files = [rng.integers(0, 256, size=int(rng.integers(200_000, 700_000)), dtype=np.uint8) for _ in range(8)]
        n = 3
    else:
        files = [rng.integers(0, 4, size=int(rng.integers(700_000, 1_500_000)), dtype=np.uint8) for _ in range(5)]
        n = 12
    corpus = gen.from_files(files, bits)
    k = 1_000_000
    say("featurize against a table of %d %d-grams (%d-bit symbols, fresh pass): rank bits in HBM" % (k, n, bits))
    exp, o = oracle_tables(corpus, [n], k)
    got, g = gpu_tables(corpus, [n], k)
    try:
        assert_tables_equal(got, exp, "fresh n=%d" % n)
        assert len(got[0][1]) > 600_000, len(got[0][1])
        q = gen.from_files([f[: len(f) // 3] for f in files[:3]]
                           + [rng.integers(0, 1 << bits, size=300_000, dtype=np.uint8), np.zeros(0, np.uint8)], bits)
        _check_all_featurize_forms(g, o, corpus, q, "HBM bitmap %d-bit" % bits)
    finally:
        g.close()


def test_occ_64bit_counters_and_eoverflow():
    """2-bit sequences of a repeated ACGT pattern with more than 2^32 windows: every count has a
    closed form, and above 2^32 windows Eq. 1 needs the 64-bit device counters."""
    lens = [1_500_000_001, 1_400_000_002, 1_394_967_400]       # 4,294,967,403 symbols in all
    assert sum(lens) > 1 << 32
    offs = np.concatenate([[0], np.cumsum(lens)]).astype(np.uint64)
    total = int(offs[-1])
    # symbol i of the stream is i mod 4 (A C G T ...): every byte is 0b00011011
    data = np.full((total + 3) // 4, 0x1B, np.uint8)
    say("Eq. 1, 2-bit, %d symbols in 3 sequences: IG_EOVERFLOW with 32-bit counts" % total)
    g32 = ig.Intergrams(symbol_bits=2, freq=ig.FREQ_OCC, count_bits=32)
    try:
        g32.load(data, offs)
        assert g32.try_pass(1, 4) == ig.IG_EOVERFLOW
        assert g32.table_info() == (0, 0)
    finally:
        g32.close()
    say("Eq. 1, 2-bit, 64-bit counters: passes n=1..3 against closed forms")
    g = ig.Intergrams(symbol_bits=2, freq=ig.FREQ_OCC, count_bits=64)
    try:
        g.load(data, offs)
        for n in (1, 2, 3):
            g.pass_(n, 16)
            keys, counts = g.topk()
            # windows of sequence s start at stream positions a_s .. a_s + L_s - n; the window at
            # position p spells (p, p+1, ...) mod 4, so it is one of 4 grams, chosen by p mod 4
            exp = {}
            for a, L in zip(offs[:-1].tolist(), lens):
                w = L - n + 1
                for r in range(4):
                    cnt = (w - r + 3) // 4           # positions p in [a, a+w) with p - a = r mod 4
                    start = (a + r) % 4
                    key = 0
                    for j in range(n):
                        key = (key << 2) | ((start + j) % 4)
                    exp[key] = exp.get(key, 0) + cnt
            want = sorted(exp.items(), key=lambda t: (-t[1], t[0]))
            assert sum(c for _, c in want) > (1 << 32) - 8
            assert [(int(keys[i, 0]), int(counts[i])) for i in range(len(counts))] == want, "pass %d" % n
            assert int(keys[:, 1].max()) == 0
    finally:
        g.close()


@pytest.mark.parametrize("occ", [False, True])
def test_set_overflow_bypass_and_dense_chain_pass(occ):
    """Random bytes: pass 1 keeps all 256 symbols, so pass 2 is the direct-indexed count of all
    2-grams inside the chain (under Eq. 2 with a grown LDS set, pass 1 having made few records per
    window); pass 3 (k = 60,000 prefixes) has far more distinct candidates per
    chunk than the chunk's LDS set holds, so its chunks fill the set and bypass it (straight to
    the counters for Eq. 1, to records for Eq. 2).  Every table equals the oracle's."""
    rng = np.random.default_rng(2027 + occ)
    files = [rng.integers(0, 256, size=int(rng.integers(150_000, 300_000)), dtype=np.uint8) for _ in range(8)]
    corpus = gen.from_files(files, 8)
    ns, k = [1, 2, 3], 60_000
    say("set overflow + dense chain pass: 8 random-byte files, n=1..3, k=%d, %s" % (k, "Eq. 1" if occ else "Eq. 2"))
    exp, _ = oracle_tables(corpus, ns, k, occ)
    g = ig.Intergrams(symbol_bits=8, freq=ig.FREQ_OCC if occ else ig.FREQ_DOC)
    try:
        g.load(corpus)
        lc = g.launch()
        got = []
        for n in ns:
            g.pass_(n, k)
            keys, counts = g.topk()
            got.append((keys.copy(), counts.copy()))
            st = g.last_stats()
            if n == 1:
                assert g.table_info()[1] == 256
            if n == 2:
                # 65,536 grams, more than a chunk has windows; under Eq. 2 the set still grows,
                # since pass 1 recorded at most one candidate per 8 windows
                assert (st["set_cap"] > lc["set_cap"]) == (not occ), (st["set_cap"], lc)
            if n == 3 and not occ:
                # more records than the sets of all chunks could hold: the set was bypassed
                nchunks = sum((len(f) + lc["chunk_syms"] - 1) // lc["chunk_syms"] for f in files)
                assert st["records"] > nchunks * lc["set_cap"], (st["records"], nchunks, lc)
        assert_tables_equal(got, exp, "random bytes")
    finally:
        g.close()


@pytest.mark.parametrize("bits,occ", [(2, False), (2, True), (8, False), (8, True)])
def test_direct_count_with_part_of_the_prefixes_kept(bits, occ):
    """A pass whose previous table kept at least half (not all) of the (n-1)-grams over the
    alphabet runs as the direct-indexed count of every n-gram, and the grams whose prefix was not
    kept are dropped before the selection.  2-bit: k = 700 keeps 700 of the 1024 5-grams, so
    pass 6 takes this form; bytes over 40 symbols: k = 1000 keeps 1000 of the 1600 2-grams, so
    pass 3 does.  Every table equals the oracle's."""
    rng = np.random.default_rng(3030 + bits + occ)
    if bits == 2:
        files = [rng.integers(0, 4, size=int(rng.integers(100_000, 300_000)), dtype=np.uint8) for _ in range(6)]
        ns, k = list(range(1, 8)), 700
    else:
        files = [rng.integers(0, 40, size=int(rng.integers(100_000, 300_000)), dtype=np.uint8) for _ in range(6)]
        ns, k = list(range(1, 5)), 1000
    corpus = gen.from_files(files, bits)
    say("direct-indexed pass with part of the prefixes kept: %d-bit, n=1..%d, k=%d, %s"
        % (bits, ns[-1], k, "Eq. 1" if occ else "Eq. 2"))
    exp, _ = oracle_tables(corpus, ns, k, occ)
    got, g = gpu_tables(corpus, ns, k, occ)
    try:
        assert_tables_equal(got, exp, "part of the prefixes kept")
    finally:
        g.close()


@pytest.mark.parametrize("occ", [False, True])
def test_direct_indexed_passes_grow_their_set(occ):
    """Random 2-bit files with a 4096-entry LDS set: passes 6 and 7 count all 4^6 and 4^7 grams
    directly (every shorter gram kept), no more than a chunk has windows, so their sets grow past
    4096 entries; pass 8 (4^8 grams, more than a chunk's windows) keeps the launch's set.  Every
    table equals the oracle's."""
    rng = np.random.default_rng(6060 + occ)
    files = [rng.integers(0, 4, size=int(rng.integers(200_000, 400_000)), dtype=np.uint8) for _ in range(6)]
    corpus = gen.from_files(files, 2)
    ns, k = list(range(1, 9)), 1_000_000
    say("direct-indexed passes grow their set: 2-bit, n=1..8, launch set 4096, %s" % ("Eq. 1" if occ else "Eq. 2"))
    exp, _ = oracle_tables(corpus, ns, k, occ)
    g = ig.Intergrams(symbol_bits=2, freq=ig.FREQ_OCC if occ else ig.FREQ_DOC)
    try:
        g.set_launch(23552, 1024, 4096, 1)
        g.load(corpus)
        got, caps = [], []
        for n in ns:
            g.pass_(n, k)
            keys, counts = g.topk()
            got.append((keys.copy(), counts.copy()))
            caps.append(g.last_stats()["set_cap"])
        assert_tables_equal(got, exp, "growing sets")
        assert caps[5] >= 8192 and caps[6] >= 16384 and caps[7] == 4096, caps
        assert g.launch()["set_cap"] == 4096
    finally:
        g.close()
