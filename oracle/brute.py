"""Brute-force checkers for the oracle (TEST INFRASTRUCTURE ONLY).

These use a different algorithm from ``ig_oracle.cpp`` so that the two can
pin each other:

* ``brute_pass`` works on the symbol strings themselves (Python ``bytes``),
  never on packed integer keys: an n-gram is the slice ``s[t:t+n]`` and grams
  are ordered as strings.  Equal-length strings order lexicographically, which
  is the order of the most-significant-first packed key the oracle uses.
* ``sorted_pass`` enumerates every window with numpy, de-duplicates per file by
  sorting (``np.unique``), filters by binary search in the sorted previous
  table, and counts by sorting again (the textbook dictionary count of the
  paper's Related Work section, done with sorts instead of a dictionary).

Both follow Eq. 1 (occurrences) / Eq. 2 (sequences containing the gram) and
one pass of Algorithm 3 with the (count desc, key asc) order.
"""
from collections import Counter

import numpy as np


def brute_pass(files, n, k_keep, prev=None, occ=False):
    """files: list of bytes-like symbol strings.  prev: set of (n-1)-strings or
    None (unfiltered).  Returns the ordered list of (gram_bytes, count)."""
    cnt = Counter()
    for f in files:
        f = bytes(f)
        grams = [f[t:t + n] for t in range(len(f) - n + 1)]
        if prev is not None:
            grams = [g for g in grams if g[:-1] in prev]
        if not occ:
            grams = set(grams)
        cnt.update(grams)
    items = sorted(cnt.items(), key=lambda kv: (-kv[1], kv[0]))
    return items[:k_keep]


def brute_intergrams(files, n, k, z, symbol_bits=8, occ=False):
    """Algorithm 3 with z-oversampling on symbol strings: the top ceil(z*k) n0-grams
    (n0 = min(n, 24 // symbol_bits)), then each longer gram length filtered by the
    previous table, ceil(z*k) kept below n and k at n.  Returns the last table."""
    import math
    kz = math.ceil(z * float(k))
    n0 = min(n, 24 // symbol_bits)
    table = brute_pass(files, n0, kz if n0 < n else k, occ=occ)
    for j in range(n0 + 1, n + 1):
        table = brute_pass(files, j, kz if j < n else k, prev={g for g, _ in table}, occ=occ)
    return table


def brute_chain(files, ns, k_keep, occ=False):
    """Passes over consecutive n (the first one unfiltered); returns one table per n."""
    out, prev = [], None
    for j, n in enumerate(ns):
        tab = brute_pass(files, n, k_keep, prev if j > 0 else None, occ)
        out.append(tab)
        prev = set(g for g, _ in tab)
    return out


def brute_featurize(files, table):
    """Row per file: sorted ranks of table grams that occur in the file."""
    rank = {g: i for i, (g, _) in enumerate(table)}
    n = len(table[0][0]) if table else 0
    rows = []
    for f in files:
        f = bytes(f)
        r = set()
        for t in range(len(f) - n + 1):
            g = f[t:t + n]
            if g in rank:
                r.add(rank[g])
        rows.append(sorted(r))
    return rows


def gram_to_key(gram, bits):
    """Pack a symbol string most significant first (used only to compare with the oracle)."""
    k = 0
    for s in gram:
        k = (k << bits) | int(s)
    return k


def key_to_gram(key, n, bits):
    mask = (1 << bits) - 1
    return bytes(((key >> (bits * (n - 1 - r))) & mask) for r in range(n))


def sorted_pass(data, offsets, n, k_keep, prev_keys=None, occ=False):
    """Byte corpus (8-bit symbols, n <= 8) with numpy sorts.  prev_keys: uint64
    array of the previous table's keys or None.  Returns (keys uint64, counts)."""
    assert n <= 8
    keys_all = []
    prev_sorted = None if prev_keys is None else np.sort(np.asarray(prev_keys, np.uint64))
    offs = np.asarray(offsets, np.int64)
    for i in range(len(offs) - 1):
        a, b = int(offs[i]), int(offs[i + 1])
        L = b - a
        if L < n:
            continue
        w = L - n + 1
        x = np.zeros(w, np.uint64)
        for r in range(n):
            x = (x << np.uint64(8)) | data[a + r:a + r + w].astype(np.uint64)
        if prev_sorted is not None:
            p = x >> np.uint64(8)
            j = np.searchsorted(prev_sorted, p)
            j[j >= len(prev_sorted)] = 0
            x = x[prev_sorted[j] == p] if len(prev_sorted) else x[:0]
        if not occ:
            x = np.unique(x)
        keys_all.append(x)
    if not keys_all:
        return np.zeros(0, np.uint64), np.zeros(0, np.int64)
    k, c = np.unique(np.concatenate(keys_all), return_counts=True)
    order = np.lexsort((k, -c))          # count desc, then key asc
    order = order[:k_keep]
    return k[order], c[order]
