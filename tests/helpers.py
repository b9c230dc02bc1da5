"""Shared helpers of the test suite (no method arithmetic here)."""
import os

import numpy as np

import gen
import oracle


def oracle_tables(corpus, ns, k_keep, occ=False, nthreads=None):
    """The CPU oracle's ordered table after each pass of the chain ns."""
    o = oracle.Oracle(corpus.symbol_bits, oracle.FREQ_OCC if occ else oracle.FREQ_DOC,
                      nthreads=nthreads or min(16, os.cpu_count() or 1))
    o.load(corpus)
    out = []
    for n in ns:
        rc = o.pass_(n, k_keep)
        assert rc == 0, rc
        keys, counts = o.topk()
        out.append((keys.copy(), counts.copy()))
    return out, o


def gpu_tables(corpus, ns, k_keep, occ=False, flags=0, ctx=None):
    import paper_2511_14955_amd as ig
    g = ctx or ig.Intergrams(symbol_bits=corpus.symbol_bits, freq=ig.FREQ_OCC if occ else ig.FREQ_DOC, flags=flags)
    g.load(corpus)
    out = []
    for n in ns:
        g.pass_(n, k_keep)
        keys, counts = g.topk()
        out.append((keys.copy(), counts.copy()))
    return out, g


def assert_tables_equal(got, exp, what=""):
    for j, ((gk, gc), (ek, ec)) in enumerate(zip(got, exp)):
        assert len(gc) == len(ec), "%s pass %d: kept %d vs oracle %d" % (what, j, len(gc), len(ec))
        if not (np.array_equal(gk, ek) and np.array_equal(gc, ec)):
            bad = np.nonzero((gk != ek).any(axis=1) | (gc != ec))[0]
            i = int(bad[0])
            raise AssertionError("%s pass %d: first difference at rank %d: gpu (%x,%x,%d) oracle (%x,%x,%d); %d differ" % (
                what, j, i, int(gk[i, 1]), int(gk[i, 0]), int(gc[i]), int(ek[i, 1]), int(ek[i, 0]), int(ec[i]), len(bad)))
