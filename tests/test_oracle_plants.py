"""Planted mistakes: each plausible slip in the oracle must fail a pin.

Each case copies ``oracle/ig_oracle.cpp`` to a temporary directory, applies one
textual mutation (a dropped window, a missing de-duplication, a reversed tie
order, a filter on the wrong end of the gram, windows across file boundaries,
LSB-first 2-bit symbols, a reversed key, the filter ignored), compiles the
copy, and runs a battery of the independent checks.  The committed oracle is
never modified.
"""
import os
import random
import subprocess

import numpy as np
import pytest

import gen
import oracle
from oracle import brute

SRC = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "oracle", "ig_oracle.cpp")

PLANTS = {
    "last_window_dropped": ("for (uint64_t t = 0; t + n <= L; t++) {", "for (uint64_t t = 0; t + n < L; t++) {"),
    "no_per_sequence_dedup": ("if (!o->occ) {", "if (false) {"),
    "ties_key_descending": ("return a.first < b.first;", "return a.first > b.first;"),
    "filter_on_suffix": ("P.find(x >> o->bits)", "P.find(x & ((((u128)1) << (o->bits * (n - 1))) - 1))"),
    "windows_cross_files": ("uint64_t a = c.off[f], L = c.off[f + 1] - a;", "uint64_t a = c.off[f], L = c.off.back() - a;"),
    "lsb_first_2bit": ("uint32_t shift = 8 - (uint32_t)bits * (uint32_t)(g % per + 1);",
                       "uint32_t shift = (uint32_t)bits * (uint32_t)(g % per);"),
    "key_reversed": ("x = (x << bits) | (u128)symbol(data, bits, g + r);", "x = (x << bits) | (u128)symbol(data, bits, g + n - 1 - r);"),
    "filter_ignored": ("const bool filtered = !(n == 1 || o->fresh);", "const bool filtered = false;"),
}


def _build_variant(tmpdir, name):
    with open(SRC) as fh:
        src = fh.read()
    old, new = PLANTS[name]
    assert src.count(old) == 1, "mutation pattern must match exactly once: %s" % name
    path = os.path.join(tmpdir, "%s.cpp" % name)
    with open(path, "w") as fh:
        fh.write(src.replace(old, new))
    so = os.path.join(tmpdir, "lib_%s.so" % name)
    subprocess.check_call(["g++", "-O1", "-std=c++17", "-shared", "-fPIC", "-pthread", path, "-o", so])
    return so


def _chain(lib, corpus, ns, k_keep, occ):
    o = oracle.Oracle(corpus.symbol_bits, oracle.FREQ_OCC if occ else oracle.FREQ_DOC, nthreads=2, lib_path=lib)
    o.load(corpus)
    out = []
    for n in ns:
        if o.pass_(n, k_keep) != 0:
            return None
        out.append(o.table())
    return out


def battery(lib):
    """Names of the checks that fail for the oracle built at ``lib``."""
    failed = []
    rng = random.Random(5)
    # brute force on tiny random corpora, both symbol widths and frequencies
    for bits in (8, 2):
        for occ in (False, True):
            ok = True
            for _ in range(25):
                m = rng.randint(1, 5)
                files = [bytes(rng.randrange(3) for _ in range(rng.randint(0, 14))) for _ in range(m)]
                ns = [1, 2, 3, 4]
                k = rng.choice([2, 3, 6, 100])
                got = _chain(lib, gen.from_files(files, bits), ns, k, occ)
                exp = brute.brute_chain(files, ns, k, occ)
                if got is None or any([(brute.key_to_gram(key, n, bits), c) for key, c in g] != e
                                      for n, g, e in zip(ns, got, exp)):
                    ok = False
                    break
            if not ok:
                failed.append("brute_%d_%s" % (bits, "occ" if occ else "doc"))
    # closed-form window count (Eq. 1, unfiltered)
    c = gen.workload(2, m=12)
    for n in (1, 3):
        got = _chain(lib, c, [n], 1 << 40, True)
        L = np.diff(c.offsets.astype(np.int64))
        if got is None or sum(x for _, x in got[0]) != int(np.maximum(0, L - n + 1).sum()):
            failed.append("window_count_%d" % n)
    return failed


@pytest.fixture(scope="module")
def tmpdir_plants(tmp_path_factory):
    return str(tmp_path_factory.mktemp("plants"))


def test_unmutated_copy_passes(tmpdir_plants):
    so = os.path.join(tmpdir_plants, "lib_clean.so")
    subprocess.check_call(["g++", "-O1", "-std=c++17", "-shared", "-fPIC", "-pthread", SRC, "-o", so])
    assert battery(so) == []


@pytest.mark.parametrize("name", sorted(PLANTS))
def test_planted_mistake_is_caught(tmpdir_plants, name):
    so = _build_variant(tmpdir_plants, name)
    assert battery(so), "planted mistake %s passed every pin" % name
