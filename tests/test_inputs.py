"""The seeded input generators: every file and request is a pure function of its seed and index,
so runs repeat exactly and a pool of host threads produces the same stream as one thread."""
from concurrent.futures import ThreadPoolExecutor

import numpy as np

import gen


def test_request_stream_is_a_function_of_the_index():
    a, b = gen.RequestStream(), gen.RequestStream()
    idx = [7, 0, 123, 5, 7]
    for i in idx:
        fa, fb = a.file(i), b.file(i)
        assert fa.dtype == np.uint8 and len(fa) == a.length(i)
        assert np.array_equal(fa, fb)
        assert a.gap(i) == b.gap(i) > 0.0
    # sizes stay inside the stated clip [4 KiB, 64 MiB]
    assert all(4096 <= a.length(i) <= (64 << 20) for i in range(200))


def test_request_stream_threads_match_one_thread():
    rs = gen.RequestStream()
    seq = [rs.file(i) for i in range(96)]
    with ThreadPoolExecutor(max_workers=8) as ex:
        par = list(ex.map(rs.file, range(96)))
    assert all(np.array_equal(x, y) for x, y in zip(seq, par))


def test_workload_is_reproducible():
    c1 = gen.workload(2, m=24)
    c2 = gen.workload(2, m=24)
    assert c1.m == c2.m == 24
    assert np.array_equal(c1.offsets, c2.offsets)
    assert np.array_equal(c1.data, c2.data)
