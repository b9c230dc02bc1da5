// CPU oracle for the Intergrams per-pass scan.
//
// TEST INFRASTRUCTURE ONLY.  Nothing in the product path may link, load or
// call this file; only the tests, the smoke check and the benchmark's CPU
// baseline do.  It shares no code, header or table with the HIP library.
//
// It is deliberately plain: every window's key is rebuilt from its symbols,
// membership uses std::unordered_set, a sequence's grams are made distinct by
// sorting them (Eq. 2), counts use std::unordered_map, and selection is one
// std::sort.  Threads only split the files between private maps that are
// summed afterwards (sums commute, so the result does not depend on the split).
//
// What it computes (arXiv 2511.14955):
//  * Problem statement (Section "Problem Formalization and Notation"):
//    m sequences over an alphabet; an n-gram is n consecutive symbols of one
//    sequence, so no n-gram crosses a sequence boundary.  Frequency is either
//    Eq. 1 (every occurrence, "OCC") or Eq. 2 (number of sequences that contain
//    the gram, "DOC"; the paper's focus and our default).
//  * One pass of Intergrams (Algorithm 3): count every n-gram whose
//    (n-1)-gram prefix is in the set P retained by the previous pass, once per
//    sequence in DOC mode; then retain the k_keep most frequent.  A pass with
//    no retained set (n = 1, or the first pass after loading data) counts
//    every n-gram: that is the unfiltered start the paper obtains from
//    Algorithm 2.
//  * The k-argmax is made unique by ordering (count descending, key
//    ascending); only grams with a positive count are eligible, and fewer
//    than k_keep grams are all kept.  The paper leaves the tie order open.
//  * Keys: the n symbols packed most significant first,
//    key = sum_r s[t+r] * 2^(b(n-1-r)), so numeric key order is the
//    lexicographic order of the symbol strings.
//  * Featurize (Figure 1, the Boolean m x k feature matrix): row i lists the
//    ranks (0-based positions in the retained order) of the retained grams
//    that occur in sequence i, ascending.
//
// Parity pins live in tests/test_oracle_pins.py.
#include <algorithm>
#include <atomic>
#include <cstdint>
#include <cstring>
#include <new>
#include <thread>
#include <unordered_map>
#include <unordered_set>
#include <utility>
#include <vector>

namespace {

typedef unsigned __int128 u128;

// return codes (same meaning as the library's, defined here independently)
enum { OK = 0, EINVAL_ = -1, ESTATE_ = -2, ENOMEM_ = -3, ETRUNC_ = -4 };

struct KeyHash {
  size_t operator()(u128 x) const {
    uint64_t h = (uint64_t)x ^ ((uint64_t)(x >> 64) * 0x9E3779B97F4A7C15ull);
    h = (h ^ (h >> 30)) * 0xBF58476D1CE4E5B9ull;
    h = (h ^ (h >> 27)) * 0x94D049BB133111EBull;
    return (size_t)(h ^ (h >> 31));
  }
};

typedef std::unordered_set<u128, KeyHash> KeySet;
typedef std::unordered_map<u128, uint64_t, KeyHash> CountMap;

struct Corpus {
  std::vector<uint8_t> data;
  std::vector<uint64_t> off;   // m+1 symbol offsets
};

struct Oracle {
  int bits = 8;                // symbol width b: 8 (bytes) or 2 (ACGT)
  int occ = 0;                 // 0: Eq. 2 (once per sequence), 1: Eq. 1 (every occurrence)
  int nthreads = 1;
  Corpus c;
  bool fresh = true;           // no retained set since the last load
  uint32_t n_prev = 0;         // gram length of the retained set
  std::vector<std::pair<u128, uint64_t>> R;   // retained (key, count), ordered
};

// symbol t of a stream: a byte, or 2 bits taken most significant first
inline uint32_t symbol(const uint8_t *data, int bits, uint64_t g) {
  if (bits == 8) return data[g];
  const uint64_t per = 4;      // bits == 2 (the only other width igo_create accepts)
  uint32_t shift = 8 - (uint32_t)bits * (uint32_t)(g % per + 1);
  return (data[g / per] >> shift) & ((1u << bits) - 1);
}

// key of the n-gram starting at symbol g: n symbols, first one most significant
inline u128 key_at(const uint8_t *data, int bits, uint64_t g, uint32_t n) {
  u128 x = 0;
  for (uint32_t r = 0; r < n; r++) x = (x << bits) | (u128)symbol(data, bits, g + r);
  return x;
}

// (count desc, key asc)
inline bool ranks_before(const std::pair<u128, uint64_t> &a, const std::pair<u128, uint64_t> &b) {
  if (a.second != b.second) return a.second > b.second;
  return a.first < b.first;
}

// Files in order of decreasing length so that threads finish together.
std::vector<uint64_t> file_order(const Corpus &c) {
  uint64_t m = c.off.size() - 1;
  std::vector<uint64_t> ord(m);
  for (uint64_t i = 0; i < m; i++) ord[i] = i;
  std::stable_sort(ord.begin(), ord.end(), [&](uint64_t a, uint64_t b) {
    return c.off[a + 1] - c.off[a] > c.off[b + 1] - c.off[b];
  });
  return ord;
}

int do_pass(Oracle *o, uint32_t n, uint64_t k_keep) {
  if (n == 0 || (uint64_t)n * (uint64_t)o->bits > 128 || k_keep == 0) return EINVAL_;
  const bool filtered = !(n == 1 || o->fresh);
  if (filtered && o->n_prev != n - 1) return ESTATE_;

  KeySet P;                                      // prefixes retained by the previous pass
  if (filtered) for (auto &e : o->R) P.insert(e.first);

  const Corpus &c = o->c;
  const std::vector<uint64_t> ord = file_order(c);
  std::atomic<uint64_t> next(0);
  const int T = std::max(1, o->nthreads);
  // part[t][q]: what thread t counted of the grams in share q (a share is a slice of the hash
  // range), so that the sums over threads can be taken one share per thread
  std::vector<std::vector<CountMap>> part(T, std::vector<CountMap>(T));
  auto share = [&](const u128 &x) { return (int)((KeyHash()(x) >> 40) % (uint64_t)T); };
  auto worker = [&](int tid) {
    std::vector<CountMap> &cnt = part[tid];
    std::vector<u128> grams;
    for (;;) {
      uint64_t j = next.fetch_add(1);
      if (j >= ord.size()) break;
      uint64_t f = ord[j];
      uint64_t a = c.off[f], L = c.off[f + 1] - a;
      if (L < n) continue;                       // no window fits in this sequence
      grams.clear();                             // the accepted grams of this sequence, one per window
      for (uint64_t t = 0; t + n <= L; t++) {
        u128 x = key_at(c.data.data(), o->bits, a + t, n);
        if (filtered && P.find(x >> o->bits) == P.end()) continue;
        grams.push_back(x);
      }
      if (!o->occ) {                             // Eq. 2: a gram counts once per sequence
        std::sort(grams.begin(), grams.end());
        grams.erase(std::unique(grams.begin(), grams.end()), grams.end());
      }
      for (const u128 &x : grams) cnt[share(x)][x] += 1;
    }
  };
  std::vector<std::thread> th;
  for (int t = 1; t < T; t++) th.emplace_back(worker, t);
  worker(0);
  for (auto &x : th) x.join();
  th.clear();

  // c(x) = the sum over threads of their counts of x; thread q sums share q
  std::vector<std::vector<std::pair<u128, uint64_t>>> sums(T);
  auto summer = [&](int q) {
    CountMap total;
    for (int t = 0; t < T; t++) {
      for (auto &kv : part[t][q]) total[kv.first] += kv.second;
      CountMap().swap(part[t][q]);
    }
    sums[q].assign(total.begin(), total.end());
  };
  for (int q = 1; q < T; q++) th.emplace_back(summer, q);
  summer(0);
  for (auto &x : th) x.join();
  std::vector<std::pair<u128, uint64_t>> all;
  for (auto &v : sums) {
    all.insert(all.end(), v.begin(), v.end());
    std::vector<std::pair<u128, uint64_t>>().swap(v);
  }
  std::sort(all.begin(), all.end(), ranks_before);
  if (all.size() > k_keep) all.resize(k_keep);
  o->R.swap(all);
  o->n_prev = n;
  o->fresh = false;
  return OK;
}

}  // namespace

extern "C" {

void *igo_create(int symbol_bits, int occ, int nthreads) {
  if (symbol_bits != 8 && symbol_bits != 2) return nullptr;
  Oracle *o = new (std::nothrow) Oracle();
  if (!o) return nullptr;
  o->bits = symbol_bits;
  o->occ = occ ? 1 : 0;
  o->nthreads = nthreads > 0 ? nthreads : 1;
  return o;
}

void igo_destroy(void *h) { delete (Oracle *)h; }

int igo_set_threads(void *h, int nthreads) { ((Oracle *)h)->nthreads = nthreads > 0 ? nthreads : 1; return OK; }

// Copy m sequences; offsets are symbol offsets (m+1 of them, non-decreasing, offs[0] = 0).
int igo_load(void *h, const uint8_t *data, uint64_t nbytes, const uint64_t *offs, uint64_t m) {
  Oracle *o = (Oracle *)h;
  if (!offs || offs[0] != 0) return EINVAL_;
  for (uint64_t i = 0; i < m; i++) if (offs[i + 1] < offs[i]) return EINVAL_;
  uint64_t need = o->bits == 8 ? offs[m] : (offs[m] * (uint64_t)o->bits + 7) / 8;
  if (nbytes < need) return EINVAL_;
  o->c.data.assign(data, data + need);
  o->c.off.assign(offs, offs + m + 1);
  o->fresh = true;
  o->n_prev = 0;
  o->R.clear();
  return OK;
}

int igo_pass(void *h, uint32_t n, uint64_t k_keep) { return do_pass((Oracle *)h, n, k_keep); }

uint64_t igo_kept(void *h) { return ((Oracle *)h)->R.size(); }
uint32_t igo_last_n(void *h) { return ((Oracle *)h)->n_prev; }

// First min(k, kept) entries: keys as (lo, hi) 64-bit pairs, counts.
int igo_topk(void *h, uint64_t k, uint64_t *keys_lohi, uint64_t *counts, uint64_t *k_out) {
  Oracle *o = (Oracle *)h;
  if (o->fresh) return ESTATE_;
  uint64_t cnt = std::min<uint64_t>(k, o->R.size());
  for (uint64_t i = 0; i < cnt; i++) {
    keys_lohi[2 * i] = (uint64_t)o->R[i].first;
    keys_lohi[2 * i + 1] = (uint64_t)(o->R[i].first >> 64);
    counts[i] = o->R[i].second;
  }
  *k_out = cnt;
  return OK;
}

// Install a retained set for gram length n (for tests that fix P directly, and for resuming a chain).
// Entries are stored in the given order.
int igo_set_retained(void *h, uint32_t n, const uint64_t *keys_lohi, const uint64_t *counts, uint64_t len) {
  Oracle *o = (Oracle *)h;
  if (n == 0 || (uint64_t)n * (uint64_t)o->bits > 128) return EINVAL_;
  o->R.clear();
  for (uint64_t i = 0; i < len; i++) {
    u128 k = ((u128)keys_lohi[2 * i + 1] << 64) | keys_lohi[2 * i];
    o->R.emplace_back(k, counts[i]);
  }
  o->n_prev = n;
  o->fresh = false;
  return OK;
}

// Boolean rows of m new sequences against the retained table: indptr[m+1], indices[cap].
int igo_featurize(void *h, const uint8_t *data, uint64_t nbytes, const uint64_t *offs, uint64_t m,
                  uint64_t *indptr, int32_t *indices, uint64_t cap, uint64_t *nnz_out) {
  Oracle *o = (Oracle *)h;
  if (o->fresh) return ESTATE_;
  if (!offs || offs[0] != 0) return EINVAL_;
  for (uint64_t i = 0; i < m; i++) if (offs[i + 1] < offs[i]) return EINVAL_;
  uint64_t need = o->bits == 8 ? offs[m] : (offs[m] * (uint64_t)o->bits + 7) / 8;
  if (nbytes < need) return EINVAL_;
  const uint32_t n = o->n_prev;
  std::unordered_map<u128, int32_t, KeyHash> rank;
  for (uint64_t i = 0; i < o->R.size(); i++) rank.emplace(o->R[i].first, (int32_t)i);
  uint64_t nnz = 0;
  indptr[0] = 0;
  for (uint64_t f = 0; f < m; f++) {
    uint64_t a = offs[f], L = offs[f + 1] - a;
    std::vector<int32_t> row;
    for (uint64_t t = 0; L >= n && t + n <= L; t++) {
      auto it = rank.find(key_at(data, o->bits, a + t, n));
      if (it != rank.end()) row.push_back(it->second);
    }
    std::sort(row.begin(), row.end());
    row.erase(std::unique(row.begin(), row.end()), row.end());
    for (int32_t r : row) { if (nnz < cap) indices[nnz] = r; nnz++; }
    indptr[f + 1] = nnz;
  }
  *nnz_out = nnz;
  return nnz > cap ? ETRUNC_ : OK;
}

}  // extern "C"
