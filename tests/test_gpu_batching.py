"""Batching: graph-captured passes, launch shapes and the autotuner never change results.

A captured pass is replayed several times with eager work (featurize, table
reads) and synchronizations in between; every replay must equal the eagerly
launched pass, which itself equals the CPU oracle.
"""
import numpy as np
import pytest

import gen
from helpers import assert_tables_equal, gpu_tables, oracle_tables

pytestmark = pytest.mark.gpu
ig = pytest.importorskip("paper_2511_14955_amd")


def say(*a):
    print("[case]", *a, flush=True)


def test_graph_replays_match_eager_and_oracle():
    corpus = gen.workload(2, m=72)
    ns = list(range(1, 7))
    say("graph replays vs eager, workload 2 first 72 files, n=1..6")
    exp, _ = oracle_tables(corpus, ns, 30000)
    eager, _ = gpu_tables(corpus, ns, 30000, flags=ig.FLAG_NO_GRAPH)
    assert_tables_equal(eager, exp, "eager")
    graphed, g = gpu_tables(corpus, ns, 30000)
    assert_tables_equal(graphed, exp, "graph")
    q = gen.from_files([corpus.file(i) for i in range(5)])
    for r in range(4):
        g.rewind()
        g.pass_(6, 30000)                      # same captured graph again (or its twin for the other table set)
        keys, counts = g.topk()
        assert np.array_equal(keys, exp[-1][0]) and np.array_equal(counts, exp[-1][1]), "replay %d" % r
        g.featurize(q)                         # eager work between replays


@pytest.mark.parametrize("shape", [(8192, 256, 4096), (16384, 1024, 8192), (32768, 512, 8192), (4096, 512, 1024),
                                   (16384, 1024, 4096, 2), (12288, 1024, 4096, 2)])
def test_launch_shapes_same_result(shape):
    corpus = gen.workload(2, m=40)
    ns = list(range(1, 6))
    say("launch shape", shape)
    exp, _ = oracle_tables(corpus, ns, 20000)
    g = ig.Intergrams()
    g.set_launch(*shape)
    if len(shape) == 4 and shape[3] == 2:
        g.set_tables(filter_max_words=1024)   # two workgroups per CU: the Bloom image stays in L2
    got, _ = gpu_tables(corpus, ns, 20000, ctx=g)
    assert_tables_equal(got, exp, "shape %s" % (shape,))


def test_shape_too_large_for_a_pass_runs_with_a_smaller_set():
    """A launch shape whose LDS set does not fit some pass runs that pass with the set halved; the
    set size in use is reported, and every table is the oracle's.  With 31744-symbol chunks and a
    16384-entry set, pass 4 (k = 60,000 retained 3-grams: a 64 KB Bloom image in LDS) does not fit
    even without the survivor rings, while passes 1 and 2 (direct-indexed) do."""
    corpus = gen.workload(2, m=40)
    ns, k = list(range(1, 5)), 60_000
    exp, _ = oracle_tables(corpus, ns, k)
    g = ig.Intergrams()
    try:
        g.set_launch(31744, 1024, 16384)
        g.set_tables(filter_max_words=16384, filter_bits_per_key=12)
        g.load(corpus)
        got, caps = [], []
        for n in ns:
            g.pass_(n, k)
            keys, counts = g.topk()
            got.append((keys.copy(), counts.copy()))
            caps.append(g.last_stats()["set_cap"])
        say("LDS set in use per pass:", caps)
        assert all(c in (1024, 2048, 4096, 8192, 16384) for c in caps), caps
        assert caps[0] == 16384 and caps[3] < 16384, caps
        assert_tables_equal(got, exp, "set fallback")
        assert g.launch()["set_cap"] == 16384   # the launch shape itself is unchanged
    finally:
        g.close()


def test_autotune_skips_shapes_that_need_a_smaller_set():
    """At pass 4 with k = 60,000 (a 64 KB Bloom image), the 16384-symbol, 16384-entry candidate
    fits only with a smaller set: it is reported unusable, and the chain is left as it was."""
    corpus = gen.workload(2, m=40)
    k = 60_000
    exp, _ = oracle_tables(corpus, [1, 2, 3, 4], k)
    g = ig.Intergrams()
    try:
        g.load(corpus)
        for n in (1, 2, 3):
            g.pass_(n, k)
        rep = g.autotune(4, k)
        assert rep["identical"]
        assert g.table_info() == (3, len(exp[2][1]))
        bad = [(c["chunk_syms"], c["block"], c["set_cap"]) for c in rep["candidates"] if c["pass_ms"] < 0]
        say("autotune at pass 4, unusable shapes:", bad)
        assert (16384, 1024, 16384) in bad
        g.pass_(4, k)
        keys, counts = g.topk()
        assert np.array_equal(keys, exp[3][0]) and np.array_equal(counts, exp[3][1])
    finally:
        g.close()


def test_autotune_is_deterministic_and_keeps_state():
    corpus = gen.workload(2, m=48)
    say("autotune on pass 5, workload 2 first 48 files")
    exp, _ = oracle_tables(corpus, list(range(1, 6)), 20000)
    g = ig.Intergrams()
    g.load(corpus)
    for n in range(1, 5):
        g.pass_(n, 20000)
    rep = g.autotune(5, 20000)
    assert rep["identical"]
    assert g.table_info() == (4, len(exp[3][1]))   # chain state unchanged
    g.pass_(5, 20000)
    keys, counts = g.topk()
    assert np.array_equal(keys, exp[4][0]) and np.array_equal(counts, exp[4][1])
    axes = {(c["map_slots_log2"], c["filter_max_words"]) for c in rep["candidates"]}
    assert {(1, 8192), (2, 8192), (2, 16384), (1, 16384)} <= axes     # table sizes were searched too
    tables = g.tables()
    assert (tables["map_slots_log2"], tables["filter_max_words"]) == (rep["best"]["map_slots_log2"],
                                                                      rep["best"]["filter_max_words"])


@pytest.mark.parametrize("shape", [dict(map_slots_log2=3, filter_bits_per_key=4, filter_max_words=1024),
                                   dict(map_slots_log2=2, filter_bits_per_key=32, filter_max_words=4096),
                                   dict(map_slots_log2=1, filter_bits_per_key=20, filter_max_words=16384)])
def test_table_shapes_same_result(shape):
    """Map load and filter sizes change speed only; a change between passes re-indexes the current
    table, so the next pass already filters with the new sizes."""
    corpus = gen.workload(2, m=40)
    ns = list(range(1, 7))
    say("table shape", shape)
    exp, _ = oracle_tables(corpus, ns, 20000)
    g = ig.Intergrams()
    g.set_tables(**shape)
    got = gpu_tables(corpus, ns[:3], 20000, ctx=g)[0]
    g.set_tables(map_slots_log2=1, filter_bits_per_key=12, filter_max_words=16384)   # mid-chain
    for n in ns[3:5]:
        g.pass_(n, 20000)
        got.append(g.topk())
    g.set_tables(**shape)
    g.pass_(6, 20000)
    got.append(g.topk())
    assert_tables_equal(got, exp, "table shape %s" % shape)
    g.close()


def test_forced_table_overflows_replay():
    """Starting capacities far too small: the sparse key table of a fresh large-n pass and the
    Eq. 2 record arrays overflow, the pass is replayed with larger ones, and the tables are the
    oracle's."""
    corpus = gen.workload(2, m=8)
    say("fresh n=5 pass with a 16K-slot key table")
    exp, _ = oracle_tables(corpus, [5], 3000)
    g = ig.Intergrams()
    g.set_tables(sparse_slots=1 << 14)
    got = gpu_tables(corpus, [5], 3000, ctx=g)[0]
    assert_tables_equal(got, exp, "sparse overflow")
    assert g.last_stats()["replays"] >= 1
    assert g.tables()["sparse_slots"] > 1 << 14
    g.close()
    corpus = gen.workload(2, m=48)
    ns = list(range(1, 6))
    say("chain n=1..5 with the record capacity reset to its floor before passes 3 and 5")
    exp, _ = oracle_tables(corpus, ns, 20000)
    g = ig.Intergrams()
    got = gpu_tables(corpus, ns[:2], 20000, ctx=g)[0]
    replays = []
    for n in ns[2:]:
        if n != 4:
            g.set_tables(record_capacity=1)
        g.pass_(n, 20000)
        replays.append(g.last_stats()["replays"])
        got.append(g.topk())
    assert_tables_equal(got, exp, "record overflow")
    assert replays[0] >= 1 and replays[2] >= 1, replays
    with pytest.raises(ig.IGError) as e:
        g.set_tables(map_slots_log2=4)
    assert e.value.code == ig.IG_EINVAL
    with pytest.raises(ig.IGError) as e:
        g.set_tables(sparse_slots=3000)
    assert e.value.code == ig.IG_EINVAL
    g.close()
