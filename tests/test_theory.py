"""The theory diagnostics (Section 4.3): formulas on the CPU, measured quantities on the GPU.

CPU: the Zipf fit returns the exponent of exact power-law counts, Lemma 1's and Lemma 2's
closed forms at hand-computed points, Theorem 1's rank and (corrected) recall bounds against exact
Zipf sums in the theorem's own model, and that the bound rises with beta'.
GPU: on a sample of the binary-like corpus, Lemma 1 holds (the measured share of prefixed
(n+1)-grams is at least the bound), Figure 3's coverage never falls as z grows and reaches 1 once
ceil(z k) keeps every n-gram, the coverage at z = 1 equals the recall of one filtered pass, and
beta agrees with the oracle's Eq. 1 table.
"""
import math
import os

import numpy as np
import pytest

import gen


def _theory():
    from paper_2511_14955_amd import theory
    return theory


def test_zipf_fit_recovers_the_exponent():
    th = _theory()
    for a in (0.6, 1.0, 1.3):
        c = 1e9 * np.arange(1, 5001, dtype=np.float64) ** (-a)
        assert abs(th.zipf_fit(c) - a) < 1e-9


def test_lemma_closed_forms():
    th = _theory()
    assert th.lemma1_bound(0.5, 10, 110) == pytest.approx(0.4)
    # 4 sqrt(2^2 ln(2*4/0.5) / (2*8)) = 4 sqrt(ln 16 / 4) = 2 sqrt(ln 16)
    assert th.lemma2_delta(2, 4, 8, 0.5) == pytest.approx(2 * math.sqrt(math.log(16)))


def _zipf_prefix_sums(D, a):
    return np.concatenate([[0.0], np.cumsum(np.arange(1, D + 1, dtype=np.float64) ** (-a))])


@pytest.mark.parametrize("a", [0.6, 0.9, 1.2, 1.6])
@pytest.mark.parametrize("beta_p", [0.3, 0.7, 0.95])
def test_theorem1_against_exact_zipf_sums(a, beta_p):
    """In the theorem's own model (exact Zipf masses, no noise): the largest u with
    M_u / M_D <= 1 - beta' is at most the rank bound U, and the true share 1 - M_u / M_k is at least
    the corrected recall bound.  Exact sums, not the integral approximations the proof uses."""
    th = _theory()
    D, k = 200000, 500
    U = th.thm1_u_bound(D, a, beta_p)
    if math.isnan(U):
        # a > 1 with a small beta': the rank bound (and the recall bound built on it) is undefined
        assert a > 1 and math.isnan(th.thm1_recall_bound(D, a, beta_p, k))
        return
    M = _zipf_prefix_sums(D, a)
    u = int(np.searchsorted(M / M[D], 1.0 - beta_p, side="right")) - 1   # largest u with M_u/M_D <= 1-beta'
    assert u <= U + 1e-9
    if u < k:
        true_share = 1.0 - M[u] / M[k]
        assert th.thm1_recall_bound(D, a, beta_p, k) <= true_share + 1e-12


def test_theorem1_printed_form_can_leave_the_unit_interval():
    # the printed numerator drops the +1 of the substitution: at these values it claims more than all
    th = _theory()
    assert th.thm1_recall_bound_printed(4.49e7, 0.958, 0.6913, 100000) > 1.0
    assert th.thm1_recall_bound(4.49e7, 0.958, 0.6913, 100000) < 1.0


def test_theorem1_bound_rises_with_beta():
    th = _theory()
    for a in (0.5, 0.8, 1.5):
        vals = [th.thm1_recall_bound(1e7, a, bp, 1000) for bp in (0.5, 0.9, 0.99, 0.999)]
        assert all(x < y for x, y in zip(vals, vals[1:])), (a, vals)


@pytest.mark.gpu
def test_measured_diagnostics():
    ig = pytest.importorskip("paper_2511_14955_amd")
    from paper_2511_14955_amd import theory
    import oracle
    corpus = gen.workload(2, m=48)
    k = 30000
    print("[case] theory diagnostics: workload 2 first 48 files, n=2..4, k=%d" % k, flush=True)
    rows = theory.diagnostics(ig, corpus, [2, 3, 4], k, zs=(1.0, 1.5, 2.0, 3.0))
    for r in rows:
        assert 0.0 < r["beta"] <= 1.0
        assert r["prefixed_share"] >= r["lemma1_bound"] - 1e-12, r
        cov = [c["coverage"] for c in r["figure3"]]
        assert all(x <= y for x, y in zip(cov, cov[1:])), r
        if math.ceil(3.0 * k) >= r["distinct_n"]:
            assert cov[-1] == 1.0, r
    # 3 * 30000 >= 65536 possible 2-grams: full coverage at n = 2
    assert rows[0]["figure3"][-1]["coverage"] == 1.0
    # coverage at z = 1 is the recall of one filtered pass after the exact top-k n-grams
    for r in rows:
        n = r["n"]
        g = ig.Intergrams(symbol_bits=8, freq=ig.FREQ_DOC)
        g.load(corpus)
        g.pass_(n + 1, k)
        exact = {int(a) | (int(b) << 64) for a, b in g.topk()[0]}
        g.load(corpus)
        g.pass_(n, k)
        g.pass_(n + 1, k)
        got = {int(a) | (int(b) << 64) for a, b in g.topk()[0]}
        g.close()
        assert r["one_step_recall_z1"] == pytest.approx(len(exact & got) / len(exact), abs=1e-12)
    # beta from the oracle's Eq. 1 table
    o = oracle.Oracle(8, oracle.FREQ_OCC, nthreads=min(16, os.cpu_count() or 1))
    o.load(corpus)
    assert o.pass_(3, k) == 0
    _, c = o.topk()
    assert rows[1]["beta"] == pytest.approx(float(c.sum()) / rows[1]["N"], rel=0, abs=1e-15)
