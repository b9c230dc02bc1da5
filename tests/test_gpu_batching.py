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


@pytest.mark.parametrize("shape", [(8192, 256, 4096), (16384, 1024, 8192), (32768, 512, 8192), (4096, 512, 1024)])
def test_launch_shapes_same_result(shape):
    corpus = gen.workload(2, m=40)
    ns = list(range(1, 6))
    say("launch shape", shape)
    exp, _ = oracle_tables(corpus, ns, 20000)
    g = ig.Intergrams()
    g.set_launch(*shape)
    got, _ = gpu_tables(corpus, ns, 20000, ctx=g)
    assert_tables_equal(got, exp, "shape %s" % (shape,))


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
