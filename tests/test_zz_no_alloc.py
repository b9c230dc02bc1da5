"""ig_featurize_noalloc (device buffers carved from the library's fixed scratch array, nothing
allocated) against ig_featurize on the same table: identical rows on two calls in a row, the
second with a smaller batch; a batch larger than the scratch is refused with IG_EINVAL."""
import numpy as np
import pytest

import gen
from helpers import gpu_tables

pytestmark = pytest.mark.gpu

ig = pytest.importorskip("paper_2511_14955_amd")


def say(*a):
    print("[case]", *a, flush=True)


def test_noalloc_matches_featurize():
    corpus = gen.workload(2, m=64)
    say("no-allocation featurize: workload 2 first 64 files, n=1..6, k=4000")
    _, g = gpu_tables(corpus, list(range(1, 7)), 4000)
    try:
        more = gen.workload(2, m=96)
        batches = [gen.from_files([more.file(i) for i in range(64, 96)] + [b"", b"abc"]),   # 34 sequences
                   gen.from_files([more.file(i) for i in range(70, 73)])]                   # then 3 smaller
        for j, q in enumerate(batches):
            say("batch %d: %d sequences, %d bytes" % (j, q.m, q.nbytes))
            ip_a, ind_a = g.featurize(q)
            ip_b, ind_b = g.featurize(q, noalloc=True)
            assert np.array_equal(ip_a, ip_b) and np.array_equal(ind_a, ind_b), "batch %d" % j
            assert len(ind_b) > 0
        # a second context on the same device shares the scratch array
        _, g2 = gpu_tables(corpus, list(range(1, 5)), 1500)
        try:
            q = batches[1]
            assert all(np.array_equal(x, y) for x, y in zip(g2.featurize(q), g2.featurize(q, noalloc=True)))
            assert all(np.array_equal(x, y) for x, y in zip(g.featurize(q), g.featurize(q, noalloc=True)))
        finally:
            g2.close()
        # larger than the scratch: refused, and the context stays usable
        big = np.zeros(ig.NOALLOC_SCRATCH_BYTES + 4096, np.uint8)
        say("batch of %d bytes (over the scratch)" % big.nbytes)
        with pytest.raises(ig.IGError) as e:
            g.featurize(big, np.array([0, big.nbytes], np.uint64), noalloc=True)
        assert e.value.code == ig.IG_EINVAL
        ip_b, ind_b = g.featurize(batches[1], noalloc=True)
        ip_a, ind_a = g.featurize(batches[1])
        assert np.array_equal(ip_a, ip_b) and np.array_equal(ind_a, ind_b)
    finally:
        g.close()
