"""Serving loop (continuous batching) through the C ABI.

Every result must be the same whether its request runs alone or in a mix of
concurrent, batched requests under a tight HBM budget, and must equal the CPU
oracle's featurization of the same sequence against the same table (exact:
integer output).
"""
import time

import numpy as np
import pytest

import gen
from helpers import gpu_tables, oracle_tables

pytestmark = pytest.mark.gpu

ig = pytest.importorskip("paper_2511_14955_amd")


def say(*a):
    print("[case]", *a, flush=True)


def drain(g, want, timeout=120.0):
    """Poll until `want` results are in; returns {tag: result}."""
    got = {}
    t_end = time.time() + timeout
    while len(got) < want:
        for r in g.poll():
            assert r["tag"] not in got
            got[r["tag"]] = r
        if len(got) < want:
            assert time.time() < t_end, "serving loop returned %d of %d results" % (len(got), want)
            time.sleep(0.001)
    return got


def _queries(max_len=600_000, count=40):
    rs = gen.RequestStream()
    out = []
    i = 0
    while len(out) < count:
        if rs.length(i) <= max_len:
            out.append(bytes(rs.file(i)))
        i += 1
    # edge cases: empty, shorter than n, exactly n, one chunk plus one symbol
    return out + [b"", b"ab", b"abcdef", bytes(range(256)) * 64 + b"x"]


@pytest.fixture(scope="module")
def table8():
    """The n=6, k=4000 table of a 64-file binary-like corpus, on the GPU and in the oracle."""
    corpus = gen.workload(2, m=64)
    ns = list(range(1, 7))
    _, o = oracle_tables(corpus, ns, 4000)
    _, g = gpu_tables(corpus, ns, 4000)
    qs = _queries()
    ip, ind = o.featurize(gen.from_files(qs))
    rows = [ind[int(ip[i]):int(ip[i + 1])] for i in range(len(qs))]
    yield g, qs, rows
    g.close()


def _alone(g, qs):
    g.serve_start(max_inflight_bytes=64 << 20, n_streams=1, max_batch=1)
    try:
        out = []
        for i, q in enumerate(qs):
            assert g.submit(ig.REQ_FEATURIZE, np.frombuffer(q, np.uint8), [0, len(q)], tag=i) == ig.IG_OK
            out.append(drain(g, 1)[i])
    finally:
        g.serve_stop()
    return out


def test_featurize_alone_matches_oracle(table8):
    g, qs, rows = table8
    say("serving: %d featurize requests one at a time" % len(qs))
    res = _alone(g, qs)
    for i, r in enumerate(res):
        assert r["status"] == ig.IG_OK
        assert np.array_equal(r["cols"], rows[i]), "request %d" % i
        assert r["t_done"] >= r["t_arrival"]


def test_alone_vs_mix(table8):
    g, qs, rows = table8
    alone = _alone(g, qs)
    rng = np.random.default_rng(5)
    # count requests over random groups of the same sequences
    groups = [sorted(rng.choice(len(qs), size=int(rng.integers(1, 6)), replace=False)) for _ in range(12)]
    exp_counts = []
    for grp in groups:
        acc = {}
        for i in grp:
            for c in rows[i]:
                acc[int(c)] = acc.get(int(c), 0) + 1
        exp_counts.append(sorted(acc.items()))
    # a budget of a few requests, so admission waits for memory to free up
    budget = 6 << 20
    say("serving: %d featurize + %d count requests at once, 4 streams, budget %d bytes" % (len(qs), len(groups), budget))
    g.serve_start(max_inflight_bytes=budget, n_streams=4, max_batch=8)
    try:
        order = list(range(len(qs))) + [1000 + j for j in range(len(groups))]
        rng.shuffle(order)
        for t in order:
            if t < 1000:
                q = qs[t]
                rc = g.submit(ig.REQ_FEATURIZE, np.frombuffer(q, np.uint8), [0, len(q)], tag=t)
            else:
                grp = groups[t - 1000]
                data = b"".join(qs[i] for i in grp)
                offs = np.concatenate([[0], np.cumsum([len(qs[i]) for i in grp])]).astype(np.uint64)
                rc = g.submit(ig.REQ_COUNT, np.frombuffer(data, np.uint8), offs, tag=t)
            assert rc == ig.IG_OK
        got = drain(g, len(order))
        st = g.serve_stats()
    finally:
        g.serve_stop()
    for i in range(len(qs)):
        r = got[i]
        assert r["status"] == ig.IG_OK and r["kind"] == ig.REQ_FEATURIZE
        assert np.array_equal(r["cols"], alone[i]["cols"]), "request %d differs alone vs in the mix" % i
        assert np.array_equal(r["cols"], rows[i])
    for j in range(len(groups)):
        r = got[1000 + j]
        assert r["status"] == ig.IG_OK and r["kind"] == ig.REQ_COUNT
        assert list(zip(r["cols"].tolist(), r["counts"].tolist())) == exp_counts[j], "count request %d" % j
    say("stats", st)
    assert st["submitted"] == st["completed"] == len(order)
    assert st["rejected"] == 0
    assert st["launches"] < len(order)            # requests were batched
    assert 0 < st["peak_inflight_bytes"] <= budget
    assert st["peak_running"] >= 2                # launches were in flight together


def test_budget_and_queue_limits(table8):
    g, qs, rows = table8
    big = max(qs, key=len)
    say("serving: a request larger than the whole budget completes with IG_ENOMEM")
    g.serve_start(max_inflight_bytes=256 << 10, n_streams=2, max_batch=4)
    try:
        assert g.submit(ig.REQ_FEATURIZE, np.frombuffer(big, np.uint8), [0, len(big)], tag=1) == ig.IG_OK
        small = qs[-2]
        assert g.submit(ig.REQ_FEATURIZE, np.frombuffer(small, np.uint8), [0, len(small)], tag=2) == ig.IG_OK
        got = drain(g, 2)
        assert got[1]["status"] == ig.IG_ENOMEM and got[1]["n"] == 0
        assert got[2]["status"] == ig.IG_OK and np.array_equal(got[2]["cols"], rows[len(qs) - 2])
        assert g.serve_stats()["rejected"] == 1
    finally:
        g.serve_stop()
    say("serving: queue capacity 4, one stream, one request per launch")
    g.serve_start(max_inflight_bytes=64 << 20, n_streams=1, max_batch=1, queue_capacity=4)
    try:
        q = qs[0]
        acc, busy = [], 0
        for t in range(200):
            rc = g.submit(ig.REQ_FEATURIZE, np.frombuffer(q, np.uint8), [0, len(q)], tag=t)
            if rc == ig.IG_OK:
                acc.append(t)
            else:
                assert rc == ig.IG_EBUSY
                busy += 1
        got = drain(g, len(acc))
        assert busy > 0
        for t in acc:
            assert np.array_equal(got[t]["cols"], rows[0])
    finally:
        g.serve_stop()


def test_state_errors(table8):
    g, qs, _ = table8
    with pytest.raises(ig.IGError) as e:
        g.submit(ig.REQ_FEATURIZE, np.zeros(4, np.uint8), [0, 4], tag=0)
    assert e.value.code == ig.IG_ESTATE
    g.serve_start()
    try:
        with pytest.raises(ig.IGError) as e:
            g.serve_start()
        assert e.value.code == ig.IG_ESTATE
        assert g.try_pass(7, 100) == ig.IG_ESTATE
        with pytest.raises(ig.IGError) as e:
            g.featurize(gen.from_files([b"abcdefgh"]))
        assert e.value.code == ig.IG_ESTATE
        with pytest.raises(ig.IGError) as e:   # featurize takes exactly one sequence
            g.submit(ig.REQ_FEATURIZE, np.zeros(8, np.uint8), [0, 4, 8], tag=0)
        assert e.value.code == ig.IG_EINVAL
        with pytest.raises(ig.IGError) as e:
            g.submit(7, np.zeros(8, np.uint8), [0, 8], tag=0)
        assert e.value.code == ig.IG_EINVAL
        with pytest.raises(ig.IGError) as e:   # data shorter than the offsets say
            g.submit(ig.REQ_COUNT, np.zeros(8, np.uint8), [0, 4, 9], tag=0)
        assert e.value.code == ig.IG_EINVAL
    finally:
        g.serve_stop()
    fresh = ig.Intergrams()
    with pytest.raises(ig.IGError) as e:
        fresh.serve_start()
    assert e.value.code == ig.IG_ESTATE
    fresh.close()


def test_two_bit_serving():
    """2-bit symbols: each request is re-packed at an arbitrary symbol offset of its batch."""
    corpus = gen.workload(4, m=24)
    ns = list(range(1, 11))
    say("serving 2-bit: n=10 table of 24 sequences, 30 requests of ragged lengths")
    _, o = oracle_tables(corpus, ns, 3000)
    _, g = gpu_tables(corpus, ns, 3000)
    rng = np.random.default_rng(9)
    seqs = []
    for j in range(30):
        src = corpus.file(int(rng.integers(0, corpus.m)))
        a = int(rng.integers(0, max(1, len(src) - 10)))
        seqs.append(src[a:a + int(rng.integers(0, 40000))])
    seqs += [np.zeros(0, np.uint8), np.array([1, 2, 3], np.uint8)]
    q = gen.from_files(seqs, symbol_bits=2)
    ip, ind = o.featurize(q)
    g.serve_start(max_inflight_bytes=8 << 20, n_streams=3, max_batch=5)
    try:
        for i, s in enumerate(seqs):
            data, offs = gen.pack2([s])
            assert g.submit(ig.REQ_FEATURIZE, data, offs, tag=i) == ig.IG_OK
        got = drain(g, len(seqs))
    finally:
        g.serve_stop()
    for i in range(len(seqs)):
        assert got[i]["status"] == ig.IG_OK
        assert np.array_equal(got[i]["cols"], ind[int(ip[i]):int(ip[i + 1])]), "sequence %d" % i
    g.close()
