"""The caller's device allocator (ig_config.alloc / free): every device buffer of a context comes
from it and goes back to it, results are unchanged, and an allocator that refuses gives IG_ENOMEM."""
import ctypes

import numpy as np
import pytest

import gen
from helpers import assert_tables_equal, gpu_tables, oracle_tables

pytestmark = pytest.mark.gpu

ig = pytest.importorskip("paper_2511_14955_amd")


def say(*a):
    print("[case]", *a, flush=True)


def _hip():
    ig.load_library()
    hip = ctypes.CDLL("libamdhip64.so.7")   # the HIP runtime libintergrams.so is linked against
    hip.hipMalloc.argtypes = [ctypes.POINTER(ctypes.c_void_p), ctypes.c_size_t]
    hip.hipFree.argtypes = [ctypes.c_void_p]
    return hip


def test_caller_allocator_holds_every_buffer():
    hip = _hip()
    live, log = {}, {"alloc": 0, "free": 0, "bytes": 0}

    def alloc(n, stream):
        p = ctypes.c_void_p()
        if hip.hipMalloc(ctypes.byref(p), n) != 0:
            return 0
        live[p.value] = n
        log["alloc"] += 1
        log["bytes"] += n
        return p.value

    def free(p, stream):
        assert p in live, "a pointer the allocator never gave out"
        del live[p]
        log["free"] += 1
        assert hip.hipFree(ctypes.c_void_p(p)) == 0

    corpus = gen.workload(2, m=48)
    ns = list(range(1, 7))
    say("caller's allocator: workload 2 first 48 files, n=1..6, k=20000, featurize and serving")
    exp, o = oracle_tables(corpus, ns, 20000)
    g = ig.Intergrams(allocator=(alloc, free))
    got = gpu_tables(corpus, ns, 20000, ctx=g)[0]
    assert_tables_equal(got, exp, "caller's allocator")
    q = gen.from_files([corpus.file(i) for i in range(6)] + [b"abc"])
    ip_o, ind_o = o.featurize(q)
    ip_g, ind_g = g.featurize(q)
    assert np.array_equal(ip_o.astype(np.uint64), ip_g) and np.array_equal(ind_o, ind_g)
    g.serve_start(max_inflight_bytes=32 << 20, n_streams=2, max_batch=4)
    try:
        f = corpus.file(3)
        assert g.submit(ig.REQ_FEATURIZE, np.ascontiguousarray(f), [0, len(f)], tag=1) == ig.IG_OK
        got_rows = []
        while not got_rows:
            got_rows = g.poll()
        assert np.array_equal(got_rows[0]["cols"], ind_o[int(ip_o[3]):int(ip_o[4])])
    finally:
        g.serve_stop()
    assert log["alloc"] > 10 and live
    g.close()
    assert not live, "%d buffers were not given back" % len(live)
    assert log["free"] == log["alloc"]


def test_allocator_that_refuses():
    say("an allocator that returns no memory, and one that refuses only large requests")
    with pytest.raises(ig.IGError) as e:                   # the context's own small buffers
        ig.Intergrams(allocator=(lambda n, s: 0, lambda p, s: None))
    assert e.value.code == ig.IG_ENOMEM
    hip = _hip()
    live = {}

    def alloc(n, stream):
        if n > 1 << 20:
            return 0
        p = ctypes.c_void_p()
        assert hip.hipMalloc(ctypes.byref(p), n) == 0
        live[p.value] = n
        return p.value

    def free(p, stream):
        del live[p]
        hip.hipFree(ctypes.c_void_p(p))

    g = ig.Intergrams(allocator=(alloc, free))
    with pytest.raises(ig.IGError) as e:
        g.load(gen.from_files([bytes(range(256)) * 8192]))   # 2 MiB of corpus
    assert e.value.code == ig.IG_ENOMEM
    g.close()
    assert not live
