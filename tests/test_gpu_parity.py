"""Parity of the HIP path with the CPU oracle (bit-exact: same grams, counts, order).

Each case prints what it runs before touching the GPU.  Sizes are small enough
for the oracle to finish in seconds while spanning many chunks, multi-chunk
files, ragged tails, both symbol widths, both key widths and both frequencies.
"""
import os
import random

import numpy as np
import pytest

import gen
from helpers import assert_tables_equal, gpu_tables, oracle_tables

pytestmark = pytest.mark.gpu

ig = pytest.importorskip("paper_2511_14955_amd")


def say(*a):
    print("[case]", *a, flush=True)


@pytest.mark.parametrize("occ", [False, True])
def test_hand_worked_chain(golden_dir, occ):
    from test_oracle_pins import read_hand
    files, k_keep, exp = read_hand(golden_dir)
    say("hand example", "occ" if occ else "doc")
    got, _ = gpu_tables(gen.from_files(files), [1, 2, 3], k_keep, occ)
    mode = "occ" if occ else "doc"
    for n, (keys, counts) in zip([1, 2, 3], got):
        grams = [(bytes(((int(k) >> (8 * (n - 1 - r))) & 255) for r in range(n)), int(c)) for k, c in zip(keys[:, 0], counts)]
        assert grams == exp[mode][n]


@pytest.mark.parametrize("bits", [8, 2])
@pytest.mark.parametrize("occ", [False, True])
def test_random_tiny_corpora(bits, occ):
    rng = random.Random(77 + bits + occ)
    for trial in range(12):
        m = rng.randint(0, 7)
        sigma = rng.choice([2, 3, 4] if bits == 2 else [2, 3, 5, 256])
        files = [bytes(rng.randrange(sigma) for _ in range(rng.choice([0, 1, 3, rng.randint(0, 60)]))) for _ in range(m)]
        nmax = rng.randint(1, 8 if bits == 8 else 40)
        ns = list(range(1, nmax + 1))
        k = rng.choice([1, 3, 10, 1000])
        corpus = gen.from_files(files, bits)
        say("tiny", bits, occ, trial, m, nmax, k)
        exp, _ = oracle_tables(corpus, ns, k, occ, nthreads=2)
        got, g = gpu_tables(corpus, ns, k, occ)
        assert_tables_equal(got, exp, "tiny trial %d" % trial)
        g.close()


@pytest.mark.parametrize("occ", [False, True])
def test_workload1_full(occ):
    corpus = gen.workload(1)
    say("workload 1 full, n=1..4, k=1000", "occ" if occ else "doc")
    exp, _ = oracle_tables(corpus, [1, 2, 3, 4], 1000, occ)
    got, _ = gpu_tables(corpus, [1, 2, 3, 4], 1000, occ)
    assert_tables_equal(got, exp, "workload1")


@pytest.mark.parametrize("m,k", [(96, 100000), (160, 2000)])
def test_workload2_sample(m, k):
    corpus = gen.workload(2, m=m)
    ns = list(range(1, 9))
    say("workload 2 first %d files (%d bytes), n=1..8, k=%d" % (m, corpus.nbytes, k))
    exp, _ = oracle_tables(corpus, ns, k)
    got, _ = gpu_tables(corpus, ns, k)
    assert_tables_equal(got, exp, "workload2 m=%d" % m)


def test_workload2_occ_sample():
    corpus = gen.workload(2, m=64)
    ns = list(range(1, 9))
    say("workload 2 first 64 files, Eq. 1")
    exp, _ = oracle_tables(corpus, ns, 50000, occ=True)
    got, _ = gpu_tables(corpus, ns, 50000, occ=True)
    assert_tables_equal(got, exp, "workload2 occ")


@pytest.mark.parametrize("m,k", [(300, 1000000), (400, 3000)])
def test_workload3_sample_128bit_keys(m, k):
    corpus = gen.workload(3, m=m)
    ns = list(range(1, 17))
    say("workload 3 first %d docs (%d bytes), n=1..16, k=%d" % (m, corpus.nbytes, k))
    exp, _ = oracle_tables(corpus, ns, k)
    got, _ = gpu_tables(corpus, ns, k)
    assert_tables_equal(got, exp, "workload3 m=%d" % m)


@pytest.mark.parametrize("m,k", [(300, 1000000), (400, 3000)])
def test_workload3_occ_sample_128bit_keys(m, k):
    """Eq. 1 over bytes with windows of more than 64 bits (n = 9..16), which the scan keeps in
    place: every pass of the text sample equals the oracle's."""
    corpus = gen.workload(3, m=m)
    ns = list(range(1, 17))
    say("workload 3 first %d docs, Eq. 1, n=1..16, k=%d" % (m, k))
    exp, _ = oracle_tables(corpus, ns, k, occ=True)
    got, _ = gpu_tables(corpus, ns, k, occ=True)
    assert_tables_equal(got, exp, "workload3 occ m=%d" % m)


@pytest.mark.parametrize("m,k", [(12, 1000000), (20, 5000)])
def test_workload4_sample_2bit(m, k):
    corpus = gen.workload(4, m=m)
    ns = list(range(1, 32))
    say("workload 4 first %d reads (%d bases), n=1..31, k=%d" % (m, int(corpus.offsets[-1]), k))
    exp, _ = oracle_tables(corpus, ns, k)
    got, _ = gpu_tables(corpus, ns, k)
    assert_tables_equal(got, exp, "workload4 m=%d" % m)


def test_per_file_form_equals_persistent():
    corpus = gen.workload(2, m=48)
    ns = list(range(1, 7))
    say("per-file launch form vs persistent, workload 2 first 48 files")
    a, _ = gpu_tables(corpus, ns, 20000)
    b, _ = gpu_tables(corpus, ns, 20000, flags=ig.FLAG_PER_FILE)
    assert_tables_equal(b, a, "per-file vs persistent")


def test_fresh_unfiltered_large_n():
    # a pass right after loading is unfiltered at any n: 5-byte keys and 40-symbol DNA keys
    corpus = gen.workload(2, m=8)
    say("fresh unfiltered n=5 bytes")
    exp, _ = oracle_tables(corpus, [5], 3000)
    got, _ = gpu_tables(corpus, [5], 3000)
    assert_tables_equal(got, exp, "fresh n=5")
    c4 = gen.workload(4, m=3)
    say("fresh unfiltered n=40 DNA (80-bit keys)")
    exp, _ = oracle_tables(c4, [40, 41], 500)
    got, _ = gpu_tables(c4, [40, 41], 500)
    assert_tables_equal(got, exp, "fresh n=40 dna")


@pytest.mark.parametrize("workload,m,n,k", [(2, 96, 8, 2000), (3, 200, 12, 5000), (4, 12, 18, 3000)])
@pytest.mark.parametrize("z", [1.0, 1.5, 2.0])
def test_intergrams_schedule(workload, m, n, k, z):
    """Algorithm 3 as a whole (dense first pass, z-oversampled passes, k at n) equals the
    oracle's schedule; a chain already in progress is discarded first."""
    import oracle
    corpus = gen.workload(workload, m=m)
    say("Algorithm 3 schedule: workload %d first %d sequences, n=%d, k=%d, z=%g" % (workload, m, n, k, z))
    o = oracle.Oracle(corpus.symbol_bits, oracle.FREQ_DOC, nthreads=min(16, os.cpu_count() or 1))
    assert o.intergrams(corpus, n, k, z) == 0
    exp = o.topk()
    g = ig.Intergrams(symbol_bits=corpus.symbol_bits, freq=ig.FREQ_DOC)
    try:
        g.load(corpus)
        g.pass_(1, 10)
        g.pass_(2, 10)
        g.intergrams(n, k, z)
        assert g.table_info() == (n, len(exp[1]))
        assert_tables_equal([g.topk()], [exp], "schedule")
        g.rewind()                      # back to the z-oversampled table at n - 1
        g.pass_(n, k)
        assert_tables_equal([g.topk()], [exp], "schedule, last pass again")
        for bad in (0.5, float("nan"), float("inf")):
            with pytest.raises(ig.IGError) as e:
                g.intergrams(n, k, bad)
            assert e.value.code == ig.IG_EINVAL
    finally:
        g.close()


@pytest.mark.parametrize("workload,m,ns,k", [(2, 64, list(range(1, 7)), 4000), (4, 10, list(range(1, 15)), 2500)])
def test_featurize_loaded_corpus(workload, m, ns, k):
    """Figure 1's m x k Boolean matrix of the loaded sequences themselves equals the oracle's
    featurization of the same sequences, and the rows of the host-copy entry point."""
    corpus = gen.workload(workload, m=m)
    say("featurize the loaded corpus: workload %d first %d sequences, n=%d, k=%d" % (workload, m, ns[-1], k))
    _, o = oracle_tables(corpus, ns, k)
    _, g = gpu_tables(corpus, ns, k)
    try:
        ip, ind = g.featurize_loaded()
        eip, eind = o.featurize(corpus)
        assert np.array_equal(ip, eip) and np.array_equal(ind, eind)
        hip_, hind = g.featurize(corpus)
        assert np.array_equal(ip, hip_) and np.array_equal(ind, hind)
        assert len(ind) > 0
    finally:
        g.close()


def test_many_short_sequences():
    """More than 65535 sequences: the counting kernels' 32-bit per-candidate state (the narrow
    16-bit form covers every smaller corpus)."""
    rng = np.random.default_rng(31)
    files = [rng.integers(0, 6, size=int(rng.integers(0, 14)), dtype=np.uint8).tobytes() for _ in range(70000)]
    corpus = gen.from_files(files)
    say("70000 short sequences, n=1..5")
    exp, _ = oracle_tables(corpus, [1, 2, 3, 4, 5], 3000)
    got, g = gpu_tables(corpus, [1, 2, 3, 4, 5], 3000)
    g.close()
    assert_tables_equal(got, exp, "70000 sequences")


def test_measure_read_bw():
    g = ig.Intergrams()
    try:
        say("streaming-read bandwidth over 256 MiB")
        bw = g.measure_read_bw(256 << 20, 3)
        assert 100.0 < bw < 8000.0 * 1.05, bw   # below the HBM peak
        with pytest.raises(ig.IGError) as e:
            g.measure_read_bw(8, 1)
        assert e.value.code == ig.IG_EINVAL
    finally:
        g.close()


def test_edge_cases():
    cases = [
        ("empty corpus", [], [1, 2], 10),
        ("all files shorter than n", [b"ab", b"c", b""], [1, 2, 3], 10),
        ("one repeated symbol", [b"\x07" * 5000], [1, 2, 3, 4], 5),
        ("k_keep = 1", [b"abracadabra", b"cadabra"], [1, 2, 3], 1),
        ("16-byte grams", [bytes(range(40)) * 3, bytes(range(5, 45)) * 2], list(range(1, 17)), 100),
    ]
    for name, files, ns, k in cases:
        say("edge:", name)
        c = gen.from_files(files)
        exp, _ = oracle_tables(c, ns, k, nthreads=1)
        got, _ = gpu_tables(c, ns, k)
        assert_tables_equal(got, exp, name)


def test_featurize_matches_oracle():
    corpus = gen.workload(2, m=64)
    say("featurize against the n=6 table of workload 2 (64 files)")
    _, o = oracle_tables(corpus, list(range(1, 7)), 4000)
    _, g = gpu_tables(corpus, list(range(1, 7)), 4000)
    queries = gen.workload(2, m=80)
    qs = gen.from_files([queries.file(i) for i in range(64, 80)] + [b"", b"abc"])
    ip_o, ind_o = o.featurize(qs)
    ip_g, ind_g = g.featurize(qs)
    assert np.array_equal(ip_o.astype(np.uint64), ip_g)
    assert np.array_equal(ind_o, ind_g)


def test_errors_and_state():
    g = ig.Intergrams()
    with pytest.raises(ig.IGError) as e:
        g.pass_(1, 10)
    assert e.value.code == ig.IG_ESTATE
    g.load(gen.from_files([b"abcdef"]))
    assert g.try_pass(0, 5) == ig.IG_EINVAL
    assert g.try_pass(17, 5) == ig.IG_EINVAL
    assert g.try_pass(2, 0) == ig.IG_EINVAL
    assert g.try_pass(2, 5) == 0
    assert g.try_pass(4, 5) == ig.IG_ESTATE
    assert g.try_pass(3, 5) == 0
    assert g.table_info() == (3, 4)


def test_hbm_budget():
    """The context's HBM budget: loads and passes that would exceed it fail with IG_ENOMEM
    and leave the chain as it was; a sufficient budget gives the same table as none."""
    corpus = gen.workload(1)   # 4 MiB
    say("HBM budget: 1 MiB (the corpus does not fit), 12 MiB (a pass does not), unlimited vs 256 MiB")
    g = ig.Intergrams(hbm_budget=1 << 20)
    with pytest.raises(ig.IGError) as e:
        g.load(corpus)
    assert e.value.code == ig.IG_ENOMEM
    g.close()
    g = ig.Intergrams(hbm_budget=12 << 20)
    g.load(corpus)
    assert g.try_pass(1, 1000) == ig.IG_ENOMEM
    assert g.table_info() == (0, 0)
    with pytest.raises(ig.IGError) as e:
        g.topk()
    assert e.value.code == ig.IG_ESTATE
    g.close()
    exp, _ = gpu_tables(corpus, [1, 2, 3, 4], 1000)
    got, gb = gpu_tables(corpus, [1, 2, 3, 4], 1000, ctx=ig.Intergrams(hbm_budget=256 << 20))
    assert_tables_equal(got, exp, "budget")
    gb.close()


def test_fresh_dense_pass_with_empty_first_bucket():
    """A fresh (unfiltered, directly indexed) Eq. 2 pass on printable text: no 2-gram starts
    with a byte below 0x0A, so the lowest candidate buckets hold no record at all."""
    corpus = gen.workload(3, m=40)
    say("fresh dense n=2 and n=3 on the first 40 text documents (empty low buckets)")
    for ns in ([2], [2, 3], [3]):
        exp, _ = oracle_tables(corpus, ns, 5000)
        got, g = gpu_tables(corpus, ns, 5000)
        g.close()
        assert_tables_equal(got, exp, "fresh dense %s" % ns)


def test_2bit_kept_below_alphabet():
    """2-bit symbols with fewer kept 1-grams than symbols: the next passes filter by a one-word
    direct bitmap, and the survivor rings start right after it."""
    corpus = gen.workload(4, m=4)
    for k in (1, 2, 3):
        say("2-bit chain n=1..6 keeping %d" % k)
        exp, _ = oracle_tables(corpus, [1, 2, 3, 4, 5, 6], k)
        got, g = gpu_tables(corpus, [1, 2, 3, 4, 5, 6], k)
        g.close()
        assert_tables_equal(got, exp, "2-bit k=%d" % k)
