"""Pins of the CPU oracle against facts that do not come from the oracle.

* A chain worked by hand (tests/golden/hand_example.txt).
* The paper's Figure 4 prefix-membership example (tests/golden/fig4_trie.txt).
* Brute force on tiny random corpora (a string-based algorithm, oracle/brute.py),
  byte and 2-bit symbols, both frequencies, with empty and short files, ties
  and single-symbol runs.
* A sort-based brute force on the whole of workload 1.
* Closed forms and invariants: the window count, Lemma 1's exact identity,
  anti-monotonicity, per-sequence bounds, and that a filter holding every
  previous gram is a no-op.
* Algorithm 3 as a whole (z-oversampled schedule from the dense first pass)
  against the same schedule over brute-force passes, and, when z*k covers every
  gram, against the exact top-k.
"""
import os
import random

import numpy as np
import pytest

import gen
import oracle
from oracle import brute


def oracle_chain(corpus, ns, k_keep, occ=False, nthreads=4):
    o = oracle.Oracle(corpus.symbol_bits, oracle.FREQ_OCC if occ else oracle.FREQ_DOC, nthreads=nthreads)
    o.load(corpus)
    out = []
    for n in ns:
        assert o.pass_(n, k_keep) == 0
        out.append(o.table())
    return out


def as_strings(table, n, bits):
    return [(brute.key_to_gram(k, n, bits), c) for k, c in table]


def windows_closed_form(offsets, n):
    L = np.diff(np.asarray(offsets, np.int64))
    return int(np.maximum(0, L - n + 1).sum())


# ---------------------------------------------------------------- golden

def read_hand(golden_dir):
    files, k_keep, exp = None, None, {"doc": {}, "occ": {}}
    with open(os.path.join(golden_dir, "hand_example.txt")) as fh:
        for line in fh:
            line = line.split("#")[0].strip()
            if not line:
                continue
            w = line.split()
            if w[0] == "files":
                files = [x.encode() for x in w[1:]]
            elif w[0] == "k_keep":
                k_keep = int(w[1])
            else:
                exp[w[0]][int(w[1])] = [(g.encode(), int(c)) for g, c in (t.split(":") for t in w[2:])]
    return files, k_keep, exp


@pytest.mark.parametrize("mode", ["doc", "occ"])
def test_hand_worked_chain(golden_dir, mode):
    files, k_keep, exp = read_hand(golden_dir)
    corpus = gen.from_files(files)
    tabs = oracle_chain(corpus, [1, 2, 3], k_keep, occ=(mode == "occ"))
    for n, tab in zip([1, 2, 3], tabs):
        assert as_strings(tab, n, 8) == exp[mode][n]


def test_figure4_membership(golden_dir):
    prefixes, queries = [], []
    with open(os.path.join(golden_dir, "fig4_trie.txt")) as fh:
        for line in fh:
            line = line.split("#")[0].strip()
            if not line:
                continue
            w = line.split()
            if w[0] == "prefix":
                prefixes.append(bytes.fromhex(w[1]))
            else:
                queries.append((bytes.fromhex(w[1]), w[2] == "present"))
    # every member and every query becomes a 4-byte file: the 3-byte gram plus one byte
    grams = [p for p in prefixes] + [q for q, _ in queries]
    files = [g + bytes([0x42]) for g in grams]
    o = oracle.Oracle(8, oracle.FREQ_DOC, nthreads=1)
    o.load(gen.from_files(files))
    o.set_retained(3, [brute.gram_to_key(p, 8) for p in prefixes], [1] * len(prefixes))
    assert o.pass_(4, 1000) == 0
    surv = {brute.key_to_gram(k, 4, 8)[:3] for k, _ in o.table()}
    assert surv == set(prefixes)
    for q, present in queries:
        assert (q in surv) == present


# ---------------------------------------------------------------- brute force, tiny random

def random_files(rng, bits):
    m = rng.randint(0, 6)
    sigma = rng.choice([1, 2, 3] if bits == 2 else [1, 2, 3, 4, 256])
    sigma = min(sigma, 1 << bits)
    files = []
    for _ in range(m):
        L = rng.choice([0, 1, 2, 3, rng.randint(0, 12), rng.randint(0, 40)])
        if rng.random() < 0.15:
            files.append(bytes([rng.randrange(sigma)]) * L)          # one repeated symbol
        else:
            files.append(bytes(rng.randrange(sigma) for _ in range(L)))
    return files


@pytest.mark.parametrize("bits", [8, 2])
@pytest.mark.parametrize("occ", [False, True])
def test_oracle_equals_brute_force_tiny(bits, occ):
    rng = random.Random(1000 + bits * 10 + occ)
    for trial in range(150):
        files = random_files(rng, bits)
        ns = list(range(1, rng.randint(1, 6) + 1))
        k_keep = rng.choice([1, 2, 3, 5, 8, 20, 1000])
        corpus = gen.from_files(files, bits)
        got = oracle_chain(corpus, ns, k_keep, occ, nthreads=rng.choice([1, 3]))
        exp = brute.brute_chain(files, ns, k_keep, occ)
        for n, g, e in zip(ns, got, exp):
            assert as_strings(g, n, bits) == e, (trial, files, n, k_keep)


def test_all_256_symbols_and_ties():
    # every byte value once per file, three files: every 1-gram ties at 3, order is by byte value
    files = [bytes(range(256)), bytes(range(255, -1, -1)), bytes(range(256))]
    tab = oracle_chain(gen.from_files(files), [1, 2], 300)
    assert as_strings(tab[0], 1, 8) == [(bytes([b]), 3) for b in range(256)]
    assert as_strings(tab[1], 2, 8) == brute.brute_chain(files, [1, 2], 300)[1]


def test_2bit_boundaries_inside_bytes():
    # reads of lengths 1, 3, 5, 7 packed back to back: boundaries fall inside bytes
    rng = random.Random(7)
    files = [bytes(rng.randrange(4) for _ in range(L)) for L in (1, 3, 5, 7, 2, 9)]
    corpus = gen.from_files(files, 2)
    for i, f in enumerate(files):
        assert bytes(corpus.file(i)) == f
    got = oracle_chain(corpus, [1, 2, 3, 4], 100)
    exp = brute.brute_chain(files, [1, 2, 3, 4], 100)
    for n, g, e in zip([1, 2, 3, 4], got, exp):
        assert as_strings(g, n, 2) == e


# ---------------------------------------------------------------- workload 1, sort-based brute force

@pytest.fixture(scope="module")
def w1():
    return gen.workload(1)


@pytest.mark.parametrize("occ", [False, True])
def test_workload1_equals_sorted_brute_force(w1, occ):
    ns, k_keep = [1, 2, 3, 4], 1000
    got = oracle_chain(w1, ns, k_keep, occ, nthreads=8)
    prev = None
    for n, g in zip(ns, got):
        keys, counts = brute.sorted_pass(w1.data, w1.offsets, n, k_keep, prev, occ)
        assert [k for k, _ in g] == [int(k) for k in keys]
        assert [c for _, c in g] == [int(c) for c in counts]
        prev = keys


# ---------------------------------------------------------------- invariants

BIG = 1 << 40


def test_window_count_identity(w1):
    # Eq. 1 with no filter: the counts add up to the number of windows, and the
    # window count drops by the number of sequences of length >= n from n to n+1
    c2 = gen.workload(2, m=48)
    for corpus in (w1, c2):
        for n in (1, 2, 3, 5):
            o = oracle.Oracle(8, oracle.FREQ_OCC, nthreads=4)
            o.load(corpus)
            assert o.pass_(n, BIG) == 0
            total = sum(c for _, c in o.table())
            assert total == windows_closed_form(corpus.offsets, n)
            L = np.diff(corpus.offsets.astype(np.int64))
            assert windows_closed_form(corpus.offsets, n + 1) == total - int((L >= n).sum())


def test_lemma1_identity_occ():
    # Proof of Lemma 1: the (n+1)-grams prefixed by a retained n-gram occur
    # sum_{p in R} c_n(p) times, minus one for every sequence whose last n-gram is in R.
    corpus = gen.workload(2, m=40)
    for n, k in ((1, 20), (2, 300), (3, 1000), (4, 50)):
        o = oracle.Oracle(8, oracle.FREQ_OCC, nthreads=4)
        o.load(corpus)
        for j in range(1, n):
            assert o.pass_(j, k) == 0
        assert o.pass_(n, k) == 0
        R = o.table()
        keep = {key for key, _ in R}
        last_in_R = 0
        for i in range(corpus.m):
            f = corpus.file(i)
            if len(f) >= n and brute.gram_to_key(bytes(f[-n:]), 8) in keep:
                last_in_R += 1
        assert o.pass_(n + 1, BIG) == 0
        survivors = sum(c for _, c in o.table())
        assert survivors == sum(c for _, c in R) - last_in_R


@pytest.mark.parametrize("occ", [False, True])
def test_anti_monotone_and_bounds(occ):
    corpus = gen.workload(2, m=40)
    o = oracle.Oracle(8, oracle.FREQ_OCC if occ else oracle.FREQ_DOC, nthreads=4)
    o.load(corpus)
    prev = None
    for n in range(1, 7):
        assert o.pass_(n, 2000) == 0
        tab = o.table()
        if not occ:
            assert all(1 <= c <= corpus.m for _, c in tab)
        if prev is not None:
            for key, c in tab:
                assert (key >> 8) in prev and c <= prev[key >> 8]
        counts = [c for _, c in tab]
        assert counts == sorted(counts, reverse=True)
        prev = dict(tab)


def test_doc_vs_occ_unfiltered():
    corpus = gen.workload(2, m=24)
    for n in (1, 2, 4):
        tabs = {}
        for occ in (False, True):
            o = oracle.Oracle(8, oracle.FREQ_OCC if occ else oracle.FREQ_DOC, nthreads=4)
            o.load(corpus)
            assert o.pass_(n, BIG) == 0
            tabs[occ] = dict(o.table())
        assert tabs[False].keys() == tabs[True].keys()
        assert all(tabs[False][k] <= tabs[True][k] for k in tabs[False])
        # Eq. 2 with no filter sums the number of distinct grams per sequence
        distinct = 0
        for i in range(corpus.m):
            f = bytes(corpus.file(i))
            distinct += len({f[t:t + n] for t in range(len(f) - n + 1)})
        assert sum(tabs[False].values()) == distinct


def test_doc_equals_occ_without_repeats():
    # a de Bruijn-like walk: no 3-gram repeats inside a file, so Eq. 1 == Eq. 2
    rng = random.Random(3)
    files = []
    for _ in range(12):
        seen, f = set(), bytearray(rng.sample(range(256), 2))
        while len(f) < 200:
            nxt = rng.randrange(256)
            g = bytes(f[-2:]) + bytes([nxt])
            if g not in seen:
                seen.add(g)
                f.append(nxt)
        files.append(bytes(f))
    c = gen.from_files(files)
    a = oracle_chain(c, [1, 2, 3], BIG, occ=False)[2]
    b = oracle_chain(c, [1, 2, 3], BIG, occ=True)[2]
    assert a == b


def test_full_filter_is_noop():
    # keeping every (n-1)-gram makes pass n equal to the unfiltered count of n-grams
    corpus = gen.workload(2, m=16)
    for occ in (False, True):
        chained = oracle_chain(corpus, [1, 2, 3, 4], BIG, occ)
        for n in (2, 3, 4):
            o = oracle.Oracle(8, oracle.FREQ_OCC if occ else oracle.FREQ_DOC, nthreads=4)
            o.load(corpus)
            assert o.pass_(n, BIG) == 0          # fresh: unfiltered
            assert o.table() == chained[n - 1]


def test_thread_count_does_not_matter():
    corpus = gen.workload(2, m=64)
    a = oracle_chain(corpus, [1, 2, 3], 5000, nthreads=1)
    b = oracle_chain(corpus, [1, 2, 3], 5000, nthreads=7)
    assert a == b


def test_featurize_against_brute_force():
    rng = random.Random(11)
    files = [bytes(rng.randrange(3) for _ in range(rng.randint(0, 30))) for _ in range(10)]
    c = gen.from_files(files)
    o = oracle.Oracle(8, oracle.FREQ_DOC, nthreads=2)
    o.load(c)
    for n in (1, 2, 3):
        assert o.pass_(n, 7) == 0
    table = as_strings(o.table(), 3, 8)
    queries = [bytes(rng.randrange(3) for _ in range(rng.randint(0, 25))) for _ in range(9)]
    indptr, ind = o.featurize(gen.from_files(queries))
    rows = [list(ind[indptr[i]:indptr[i + 1]]) for i in range(len(queries))]
    assert rows == brute.brute_featurize(queries, table)


def test_argument_and_state_errors():
    o = oracle.Oracle(8, oracle.FREQ_DOC, nthreads=1)
    o.load(gen.from_files([b"abcd"]))
    assert o.pass_(0, 5) == oracle.EINVAL
    assert o.pass_(17, 5) == oracle.EINVAL            # 17 bytes do not fit 128 bits
    assert o.pass_(2, 0) == oracle.EINVAL
    assert o.pass_(2, 5) == 0                          # fresh chain: unfiltered
    assert o.pass_(4, 5) == oracle.ESTATE              # must continue at n = 3
    assert o.pass_(3, 5) == 0
    o2 = oracle.Oracle(2, oracle.FREQ_DOC, nthreads=1)
    o2.load(gen.from_files([bytes([0, 1, 2, 3])], 2))
    assert o2.pass_(64, 5) == 0                        # 64 x 2 bits = 128 bits
    assert o2.pass_(65, 5) == oracle.EINVAL


# ---------------------------------------------------------------- Algorithm 3 schedule

@pytest.mark.parametrize("bits", [8, 2])
def test_intergrams_schedule_equals_brute_force(bits):
    rng = random.Random(77 + bits)
    nmax = 6 if bits == 8 else 15          # 2-bit symbols: the dense first pass is at 12
    for trial in range(60):
        files = random_files(rng, bits)
        if bits == 2:
            files = [f + bytes(rng.randrange(4) for _ in range(rng.randint(0, 30))) for f in files]
        n = rng.randint(1, nmax)
        k = rng.choice([1, 2, 3, 5, 9, 40])
        z = rng.choice([1.0, 1.5, 2.0, 3.7])
        corpus = gen.from_files(files, bits)
        o = oracle.Oracle(bits, oracle.FREQ_DOC, nthreads=rng.choice([1, 3]))
        assert o.intergrams(corpus, n, k, z) == 0
        exp = brute.brute_intergrams(files, n, k, z, symbol_bits=bits)
        assert as_strings(o.table(), n, bits) == exp, (trial, n, k, z)


def test_intergrams_large_z_is_exact():
    # when ceil(z*k) retains every gram of every intermediate length, nothing is filtered
    # out, so the schedule returns the exact top-k of all n-grams
    rng = random.Random(5)
    for trial in range(30):
        files = [bytes(rng.randrange(3) for _ in range(rng.randint(0, 40))) for _ in range(rng.randint(1, 8))]
        n, k = rng.randint(3, 7), rng.choice([1, 4, 10])
        z = 1e6
        o = oracle.Oracle(8, oracle.FREQ_DOC, nthreads=2)
        assert o.intergrams(gen.from_files(files), n, k, z) == 0
        assert as_strings(o.table(), n, 8) == brute.brute_pass(files, n, k), trial


def test_intergrams_z_one_is_the_plain_chain():
    corpus = gen.workload(2, m=24)
    o = oracle.Oracle(8, oracle.FREQ_DOC, nthreads=4)
    assert o.intergrams(corpus, 6, 700, 1.0) == 0
    assert o.table() == oracle_chain(corpus, [3, 4, 5, 6], 700)[-1]
    with pytest.raises(ValueError):
        o.intergrams(corpus, 6, 700, 0.5)
