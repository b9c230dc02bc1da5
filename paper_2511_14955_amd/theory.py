"""The paper's theory (Section 4.3: Lemma 1, Theorem 1, Lemma 2, Theorem 2) against measured counts.

Formulas (host arithmetic on the printed expressions, nothing fitted into them):

* Lemma 1: if the top-k' n-grams hold a share beta of all N n-gram occurrences over m
  sequences, the (n+1)-grams whose n-prefix is one of them hold at least
  beta' = beta - m / (N - m) of all (n+1)-gram occurrences.
* Theorem 1 (Zipf exponent a != 1, |D| distinct (n+1)-grams): the most frequent (n+1)-gram found
  ranks at most U = ((|D|^(1-a) - a)(1 - beta') + 1)^(1/(1-a)) - 1, and the recalled share of the
  top-k mass is at least 1 - (u^(1-a) - a) / ((k+1)^(1-a) - 1) at u = U.  The theorem prints the
  substituted form with (|D|^(1-a) - a)(1 - beta') - a in the numerator; substituting
  U^(1-a) <= (U+1)^(1-a) (a < 1; the inequality turns with the sign of 1-a for a > 1, and so does
  the division) gives (|D|^(1-a) - a)(1 - beta') + 1 - a instead: the proof's u / u+1 slip.
  Both are returned; the corrected one is the bound.
* Lemma 2: with probability 1 - delta the empirical top-k mass is within
  Delta = 4 sqrt(k^2 ln(2|D_n| / delta) / (2N)) of the true one; Theorem 2 uses
  beta'' = beta' - Delta in Theorem 1.

``diagnostics`` measures, for each step n -> n+1 on a loaded corpus (every count from the
library's kernels):

* beta (Eq. 1 share of the top-k' n-grams) and Lemma 1's bound next to the measured share of
  (n+1)-gram occurrences whose prefix is retained (a filtered Eq. 1 pass keeping everything);
* Figure 3's quantity: the fraction of the exact top-k (n+1)-grams (Eq. 2) whose n-prefix is
  among the exact top-ceil(z k) n-grams, per z.  That fraction is also the recall of one filtered
  step, since an exact top-k gram that passes the filter keeps its rank among the candidates;
* a least-squares Zipf exponent of the top-k (n+1)-gram occurrence counts, and Theorem 1's and
  Theorem 2's recall bounds at that exponent, next to the measured one-step recall.
"""
import math

import numpy as np


def lemma1_bound(beta, m, N):
    """beta' = beta - m / (N - m)."""
    return beta - m / (N - m) if N > m else float("-inf")


def lemma2_delta(k, D, N, delta):
    """Delta(delta) = 4 sqrt(k^2 ln(2 D / delta) / (2 N))."""
    return 4.0 * math.sqrt(k * k * math.log(2.0 * D / delta) / (2.0 * N))


def thm1_u_bound(D, a, beta_p):
    """Rank bound of the most frequent (n+1)-gram found (Theorem 1, part 1), a != 1."""
    base = (D ** (1.0 - a) - a) * (1.0 - beta_p) + 1.0
    if base <= 0:
        return float("nan")
    return base ** (1.0 / (1.0 - a)) - 1.0


def thm1_recall_bound_printed(D, a, beta_p, k):
    """Theorem 1, part 3, as printed (a != 1)."""
    return 1.0 - ((D ** (1.0 - a) - a) * (1.0 - beta_p) - a) / ((k + 1.0) ** (1.0 - a) - 1.0)


def thm1_recall_bound(D, a, beta_p, k):
    """Theorem 1, part 3, with the proof's substitution of u <= U carried out (a != 1); NaN where
    the rank bound U is undefined (a > 1 and (|D|^(1-a) - a)(1 - beta') + 1 <= 0)."""
    if (D ** (1.0 - a) - a) * (1.0 - beta_p) + 1.0 <= 0:
        return float("nan")
    return 1.0 - ((D ** (1.0 - a) - a) * (1.0 - beta_p) + 1.0 - a) / ((k + 1.0) ** (1.0 - a) - 1.0)


def zipf_fit(counts):
    """Least-squares slope of log(count) against log(rank) over the given (descending) counts."""
    c = np.asarray(counts, np.float64)
    c = c[c > 0]
    if len(c) < 2:
        return float("nan")
    x = np.log(np.arange(1, len(c) + 1, dtype=np.float64))
    y = np.log(c)
    slope = np.polyfit(x, y, 1)[0]
    return float(-slope)


def _keys(t):
    keys = t[0]
    return keys[:, 0].astype(object) | (keys[:, 1].astype(object) << 64)


def diagnostics(ig, corpus, ns, k, zs=(1.0, 1.5, 2.0, 3.0), delta=0.05):
    """One row per step n -> n+1 for n in ns (see the module docstring); k' = k."""
    b = corpus.symbol_bits
    m = int(corpus.m)
    rows = []

    def fresh(freq):
        g = ig.Intergrams(symbol_bits=b, freq=freq)
        g.load(corpus)
        return g

    for n in ns:
        row = {"n": n}
        # Eq. 1: beta of the top-k n-grams, then the share of (n+1)-grams they prefix
        g = fresh(ig.FREQ_OCC)
        try:
            g.pass_(n, k)
            st = g.last_stats()
            N, Dn = int(st["windows"]), int(st["distinct"])
            _, c = g.topk()
            kept = len(c)
            beta = float(c.sum(dtype=np.uint64)) / N if N else 0.0
            g.pass_(n + 1, max(1, kept * (1 << b)))        # every candidate kept
            st1 = g.last_stats()
            N1 = int(st1["windows"])
            _, c1 = g.topk()
            share = float(c1.sum(dtype=np.uint64)) / N1 if N1 else 0.0
        finally:
            g.close()
        row.update({"N": N, "distinct_n": Dn, "beta": beta, "lemma1_bound": lemma1_bound(beta, m, N),
                    "prefixed_share": share})
        # exact Eq. 1 top-k (n+1)-grams: Zipf exponent and |D_{n+1}|
        g = fresh(ig.FREQ_OCC)
        try:
            g.pass_(n + 1, k)
            D1 = int(g.last_stats()["distinct"])
            a = zipf_fit(g.topk()[1])
        finally:
            g.close()
        # exact Eq. 2 top-k (n+1)-grams and top-ceil(z k) n-grams: Figure 3's coverage
        g = fresh(ig.FREQ_DOC)
        try:
            g.pass_(n + 1, k)
            top1 = _keys(g.topk())
            g.load(corpus)
            g.pass_(n, int(math.ceil(max(zs) * k)))
            topn = _keys(g.topk())
        finally:
            g.close()
        pref = np.array([int(x) >> b for x in top1], dtype=object)
        cover = []
        for z in zs:
            P = set(int(x) for x in topn[:int(math.ceil(z * k))])
            cover.append({"z": z, "coverage": float(sum(1 for x in pref if int(x) in P)) / max(1, len(pref))})
        one_step = cover[0]["coverage"] if zs[0] == 1.0 else None
        row.update({"distinct_n1": D1, "zipf_a": a, "figure3": cover, "one_step_recall_z1": one_step})
        if a == a and abs(a - 1.0) > 1e-9:
            row["thm1_recall_bound"] = thm1_recall_bound(D1, a, row["lemma1_bound"], k)
            row["thm1_recall_bound_printed"] = thm1_recall_bound_printed(D1, a, row["lemma1_bound"], k)
            row["thm1_u_bound"] = thm1_u_bound(D1, a, row["lemma1_bound"])
            dl = lemma2_delta(k, max(Dn, 1), N, delta)
            row["lemma2_delta"] = dl
            row["thm2_recall_bound"] = thm1_recall_bound(D1, a, row["lemma1_bound"] - dl, k)
        rows.append(row)
    return rows
