/*
 * Seeded synthetic corpora for the Intergrams hot path.
 *
 * This module holds no part of the method's arithmetic: it only writes symbol
 * streams and file boundaries.  Both the CPU oracle and the HIP path read its
 * output; neither shares anything else.
 *
 * Randomness: SplitMix64 (Steele, Lea, Flood, "Fast splittable pseudorandom
 * number generators", OOPSLA 2014), one independent stream per
 * (workload seed, stream tag, index).  A file's bytes depend only on the seed
 * and its index, never on thread count or scheduling.
 *
 * Workloads (stand-ins for the paper's datasets, Section "Experiments",
 * Table 2; no dataset item is reproduced):
 *   1  64 files x 65,536 B; order-1 Markov chain over 256 byte symbols whose
 *      stationary law is Zipf(1.1) over ranks (bytes = seeded permutation).
 *   2  16,384 binary-like files, lognormal sizes (median 64 KiB, sigma 1.5,
 *      clipped to [1 B, 16 MiB]); chain background with injected copies of
 *      65,536 motifs (length 4..64) picked with probability ~ j^-1.2.
 *   3  200,000 text documents totalling 4 GiB over {\n} U [0x20,0x7e];
 *      tokens from a 50,000-word synthetic vocabulary, Zipf(1.0).
 *   4  100,000 DNA reads, lengths uniform in [1000, 100000] bases,
 *      GC 0.41, 5% of reads with one 31..300 bp segment copied 2..10x;
 *      packed 2 bits per base, MSB first, A=0 C=1 G=2 T=3.
 *   5  request stream: exponential inter-arrival (mean 0.5 ms), one file per
 *      request, lognormal(ln 64 KiB, 1.5) clipped to [4 KiB, 64 MiB], content
 *      as workload 2 with the same motif library.
 */
#include <math.h>
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define GOLDEN 0x9E3779B97F4A7C15ull

static inline uint64_t sm_mix(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}
typedef struct { uint64_t s; } rng_t;
static inline uint64_t rng_next(rng_t *r) { r->s += GOLDEN; return sm_mix(r->s); }
/* uniform double in [0, 1) with 53 random bits */
static inline double rng_unif(rng_t *r) { return (double)(rng_next(r) >> 11) * 0x1.0p-53; }
/* uniform integer in [lo, hi] (inclusive); modulo bias is < 2^-40 here */
static inline uint64_t rng_range(rng_t *r, uint64_t lo, uint64_t hi) { return lo + rng_next(r) % (hi - lo + 1); }
static rng_t rng_stream(uint64_t seed, uint64_t tag, uint64_t idx) {
  rng_t r;
  r.s = sm_mix(seed ^ sm_mix(tag * 0xD1B54A32D192ED03ull + sm_mix(idx + GOLDEN)));
  return r;
}
static double rng_normal(rng_t *r) {
  /* Box-Muller, one value per call */
  double u1 = rng_unif(r), u2 = rng_unif(r);
  if (u1 < 1e-300) u1 = 1e-300;
  return sqrt(-2.0 * log(u1)) * cos(6.283185307179586476925 * u2);
}

enum { TAG_SIZES = 1, TAG_MOTIFS = 2, TAG_FILE = 3, TAG_VOCAB = 4, TAG_PERM = 5, TAG_REQ = 6, TAG_ARRIVAL = 7 };

/* ---------------- byte chain (workloads 1, 2, 5) ---------------- */
typedef struct {
  double cdf[256];      /* cdf of Zipf(1.1) over ranks 1..256 */
  double acc_up[257];   /* Metropolis acceptance of r -> r+1: (r/(r+1))^1.1 */
  uint8_t perm[256];    /* rank r (1-based) -> byte perm[r-1] */
} chain_t;

static void chain_init(chain_t *c, uint64_t seed) {
  double tot = 0.0;
  for (int r = 1; r <= 256; r++) tot += pow((double)r, -1.1);
  double acc = 0.0;
  for (int r = 1; r <= 256; r++) { acc += pow((double)r, -1.1) / tot; c->cdf[r - 1] = acc; }
  c->cdf[255] = 1.0;
  for (int r = 1; r < 256; r++) c->acc_up[r] = pow((double)r / (double)(r + 1), 1.1);
  c->acc_up[256] = 0.0;
  rng_t pr = rng_stream(seed, TAG_PERM, 0);
  for (int i = 0; i < 256; i++) c->perm[i] = (uint8_t)i;
  for (int i = 255; i > 0; i--) {
    int j = (int)rng_range(&pr, 0, (uint64_t)i);
    uint8_t t = c->perm[i]; c->perm[i] = c->perm[j]; c->perm[j] = t;
  }
}
static inline int cdf_search(const double *cdf, int n, double u) {
  int lo = 0, hi = n - 1;           /* smallest i with cdf[i] > u */
  while (lo < hi) { int mid = (lo + hi) >> 1; if (cdf[mid] > u) hi = mid; else lo = mid + 1; }
  return lo;
}
static inline int chain_fresh(const chain_t *c, rng_t *r) { return 1 + cdf_search(c->cdf, 256, rng_unif(r)); }
static inline int chain_step(const chain_t *c, rng_t *r, int rank) {
  if (rng_unif(r) < 0.5) return chain_fresh(c, r);
  if (rng_unif(r) < 0.5) return rank > 1 ? rank - 1 : rank;            /* proposal down: always accepted */
  if (rank == 256) return rank;                                          /* proposal up off the end */
  return rng_unif(r) < c->acc_up[rank] ? rank + 1 : rank;               /* proposal up */
}

/* ---------------- motif library (workloads 2, 5) ---------------- */
#define N_MOTIFS 65536
typedef struct {
  chain_t chain;
  uint8_t *bytes;                 /* concatenated motif bytes */
  uint32_t off[N_MOTIFS + 1];
  double *cdf;                    /* pick law ~ j^-1.2 over j = 1..N_MOTIFS */
} motifs_t;

static int motifs_init(motifs_t *m, uint64_t lib_seed) {
  chain_init(&m->chain, lib_seed);
  rng_t r = rng_stream(lib_seed, TAG_MOTIFS, 0);
  uint32_t tot = 0;
  uint8_t lens[N_MOTIFS];
  for (int j = 0; j < N_MOTIFS; j++) { lens[j] = (uint8_t)rng_range(&r, 4, 64); tot += lens[j]; }
  m->bytes = (uint8_t *)malloc(tot);
  m->cdf = (double *)malloc(sizeof(double) * N_MOTIFS);
  if (!m->bytes || !m->cdf) return -1;
  uint32_t o = 0;
  for (int j = 0; j < N_MOTIFS; j++) {
    m->off[j] = o;
    rng_t mr = rng_stream(lib_seed, TAG_MOTIFS, 1 + (uint64_t)j);
    int rank = chain_fresh(&m->chain, &mr);
    for (int t = 0; t < lens[j]; t++) {
      m->bytes[o++] = m->chain.perm[rank - 1];
      rank = chain_step(&m->chain, &mr, rank);
    }
  }
  m->off[N_MOTIFS] = o;
  double s = 0.0;
  for (int j = 1; j <= N_MOTIFS; j++) s += pow((double)j, -1.2);
  double a = 0.0;
  for (int j = 1; j <= N_MOTIFS; j++) { a += pow((double)j, -1.2) / s; m->cdf[j - 1] = a; }
  m->cdf[N_MOTIFS - 1] = 1.0;
  return 0;
}
static void motifs_free(motifs_t *m) { free(m->bytes); free(m->cdf); }

/* workload-1 file: the chain only */
static void fill_chain_file(const chain_t *c, rng_t *r, uint8_t *dst, uint64_t len) {
  if (!len) return;
  int rank = chain_fresh(c, r);
  for (uint64_t t = 0; t < len; t++) { dst[t] = c->perm[rank - 1]; rank = chain_step(c, r, rank); }
}
/* workload-2 file: chain background runs (geometric, mean 100 B) alternating with motif copies */
static void fill_binary_file(const motifs_t *m, rng_t *r, uint8_t *dst, uint64_t len) {
  const chain_t *c = &m->chain;
  uint64_t pos = 0;
  int rank = chain_fresh(c, r);
  const double lq = log(1.0 - 0.01);
  while (pos < len) {
    double u = rng_unif(r);
    uint64_t run = 1 + (uint64_t)floor(log(1.0 - u) / lq);
    for (uint64_t t = 0; t < run && pos < len; t++) { dst[pos++] = c->perm[rank - 1]; rank = chain_step(c, r, rank); }
    if (pos >= len) break;
    int j = cdf_search(m->cdf, N_MOTIFS, rng_unif(r));
    for (uint32_t t = m->off[j]; t < m->off[j + 1] && pos < len; t++) dst[pos++] = m->bytes[t];
  }
}

/* ---------------- text (workload 3) ---------------- */
#define N_WORDS 50000
typedef struct {
  char *chars;                 /* concatenated words */
  uint32_t off[N_WORDS + 1];
  double *cdf;                 /* Zipf(1.0) over word rank */
} vocab_t;

static uint64_t str_hash(const char *s, int n) { uint64_t h = 1469598103934665603ull; for (int i = 0; i < n; i++) { h ^= (uint8_t)s[i]; h *= 1099511628211ull; } return h; }

static int vocab_init(vocab_t *v, uint64_t seed) {
  v->chars = (char *)malloc((size_t)N_WORDS * 16);
  v->cdf = (double *)malloc(sizeof(double) * N_WORDS);
  uint32_t cap = 1u << 17;
  int32_t *slots = (int32_t *)malloc(sizeof(int32_t) * cap);
  if (!v->chars || !v->cdf || !slots) return -1;
  for (uint32_t i = 0; i < cap; i++) slots[i] = -1;
  rng_t r = rng_stream(seed, TAG_VOCAB, 0);
  uint32_t o = 0;
  int nw = 0;
  char w[16];
  while (nw < N_WORDS) {
    /* length 1 + Poisson(4.5), capped at 15 (Knuth's product method) */
    double L = exp(-4.5), p = 1.0; int k = 0;
    do { k++; p *= rng_unif(&r); } while (p > L);
    int len = 1 + (k - 1); if (len > 15) len = 15;
    for (int i = 0; i < len; i++) w[i] = (char)('a' + rng_range(&r, 0, 25));
    uint64_t h = str_hash(w, len);
    uint32_t s = (uint32_t)h & (cap - 1);
    int dup = 0;
    while (slots[s] >= 0) {
      int q = slots[s]; int ql = (int)(v->off[q + 1] - v->off[q]);
      if (ql == len && memcmp(v->chars + v->off[q], w, (size_t)len) == 0) { dup = 1; break; }
      s = (s + 1) & (cap - 1);
    }
    if (dup) continue;
    slots[s] = nw;
    v->off[nw] = o; memcpy(v->chars + o, w, (size_t)len); o += (uint32_t)len; v->off[nw + 1] = o;
    nw++;
  }
  free(slots);
  double tot = 0.0;
  for (int j = 1; j <= N_WORDS; j++) tot += 1.0 / j;
  double a = 0.0;
  for (int j = 1; j <= N_WORDS; j++) { a += 1.0 / j / tot; v->cdf[j - 1] = a; }
  v->cdf[N_WORDS - 1] = 1.0;
  return 0;
}
static void vocab_free(vocab_t *v) { free(v->chars); free(v->cdf); }

static void fill_text_file(const vocab_t *v, rng_t *r, uint8_t *dst, uint64_t len) {
  static const char punct[6] = {'.', ',', ';', ':', '!', '?'};
  uint64_t pos = 0, col = 0;
  int cap_next = 1;
  while (pos < len) {
    int j = cdf_search(v->cdf, N_WORDS, rng_unif(r));
    for (uint32_t t = v->off[j]; t < v->off[j + 1] && pos < len; t++) {
      char ch = v->chars[t];
      if (cap_next && t == v->off[j]) ch = (char)(ch - 'a' + 'A');
      dst[pos++] = (uint8_t)ch; col++;
    }
    cap_next = 0;
    if (pos >= len) break;
    if (rng_unif(r) < 0.08) {
      char p = punct[rng_range(r, 0, 5)];
      dst[pos++] = (uint8_t)p; col++;
      if (p == '.' || p == '!' || p == '?') cap_next = 1;
      if (pos >= len) break;
    }
    if (col >= 80) { dst[pos++] = '\n'; col = 0; }
    else { dst[pos++] = ' '; col++; }
  }
}

/* ---------------- DNA (workload 4) ---------------- */
static inline void put2(uint8_t *data, uint64_t g, uint8_t sym, uint64_t lo_byte, uint64_t hi_byte) {
  uint64_t b = g >> 2;
  uint8_t v = (uint8_t)(sym << (6 - 2 * (g & 3)));
  if (b == lo_byte || b == hi_byte) __atomic_fetch_or(&data[b], v, __ATOMIC_RELAXED);
  else data[b] |= v;
}
static void fill_dna_read(rng_t *r, uint8_t *sym, uint64_t len) {
  for (uint64_t t = 0; t < len; t++) {
    double u = rng_unif(r);   /* A .295, C .205, G .205, T .295 */
    sym[t] = u < 0.295 ? 0 : u < 0.500 ? 1 : u < 0.705 ? 2 : 3;
  }
  if (rng_unif(r) < 0.05) {
    uint64_t seg = rng_range(r, 31, 300);
    if (seg > len) seg = len;
    uint64_t src = rng_range(r, 0, len - seg);
    int copies = (int)rng_range(r, 2, 10);
    for (int c = 0; c < copies; c++) {
      uint64_t d = rng_range(r, 0, len - seg);
      memmove(sym + d, sym + src, seg);
    }
  }
}

/* ---------------- sizes ---------------- */
static const uint64_t DEFAULT_M[6] = {0, 64, 16384, 200000, 100000, 0};

int iggen_default_m(int cfg) { return (cfg >= 1 && cfg <= 4) ? (int)DEFAULT_M[cfg] : -1; }
int iggen_symbol_bits(int cfg) { return cfg == 4 ? 2 : 8; }

static uint64_t lognormal_size(rng_t *r, double median, double sigma, uint64_t lo, uint64_t hi) {
  double x = median * exp(sigma * rng_normal(r));
  double f = floor(x + 0.5);
  if (f < (double)lo) return lo;
  if (f > (double)hi) return hi;
  return (uint64_t)f;
}

/* Fills sym_offsets[0..m]; returns 0, or -1 for a bad workload. Offsets count symbols. */
int iggen_offsets(int cfg, uint64_t seed, uint64_t m, uint64_t *sym_offsets) {
  rng_t r = rng_stream(seed, TAG_SIZES, 0);
  sym_offsets[0] = 0;
  if (cfg == 1) {
    for (uint64_t i = 0; i < m; i++) sym_offsets[i + 1] = sym_offsets[i] + 65536;
  } else if (cfg == 2) {
    for (uint64_t i = 0; i < m; i++) sym_offsets[i + 1] = sym_offsets[i] + lognormal_size(&r, 65536.0, 1.5, 1, 16ull << 20);
  } else if (cfg == 3) {
    /* lognormal(sigma 1) weights rescaled so that the full 200,000-document corpus totals 4 GiB */
    double *w = (double *)malloc(sizeof(double) * (m ? m : 1));
    if (!w) return -1;
    double s = 0.0;
    for (uint64_t i = 0; i < m; i++) { w[i] = exp(rng_normal(&r)); s += w[i]; }
    uint64_t total = (uint64_t)((double)(4ull << 30) * (double)m / 200000.0);
    uint64_t acc = 0;
    for (uint64_t i = 0; i < m; i++) {
      uint64_t L = (uint64_t)floor(w[i] / s * (double)total);
      sym_offsets[i + 1] = sym_offsets[i] + L; acc += L;
    }
    uint64_t rem = total - acc;             /* < m: one more symbol to the first rem documents */
    uint64_t add = 0;
    for (uint64_t i = 0; i < m; i++) { if (i < rem) add++; sym_offsets[i + 1] += add; }
    free(w);
  } else if (cfg == 4) {
    for (uint64_t i = 0; i < m; i++) sym_offsets[i + 1] = sym_offsets[i] + rng_range(&r, 1000, 100000);
  } else {
    return -1;
  }
  return 0;
}

/* bytes needed to hold the symbol stream */
uint64_t iggen_data_bytes(int cfg, uint64_t total_syms) { return cfg == 4 ? (total_syms + 3) / 4 : total_syms; }

typedef struct {
  int cfg; uint64_t seed; uint64_t m; const uint64_t *off; uint8_t *data;
  const chain_t *chain; const motifs_t *motifs; const vocab_t *vocab;
  uint64_t f0, f1;
} job_t;

static void *fill_worker(void *arg) {
  job_t *j = (job_t *)arg;
  uint8_t *tmp = NULL;
  uint64_t tmpcap = 0;
  uint64_t lo_byte = 0, hi_byte = 0;
  if (j->cfg == 4 && j->f1 > j->f0) { lo_byte = j->off[j->f0] >> 2; hi_byte = (j->off[j->f1] + 3) / 4 - 1; }
  for (uint64_t f = j->f0; f < j->f1; f++) {
    uint64_t len = j->off[f + 1] - j->off[f];
    rng_t r = rng_stream(j->seed, TAG_FILE, f);
    if (j->cfg == 1) fill_chain_file(j->chain, &r, j->data + j->off[f], len);
    else if (j->cfg == 2) fill_binary_file(j->motifs, &r, j->data + j->off[f], len);
    else if (j->cfg == 3) fill_text_file(j->vocab, &r, j->data + j->off[f], len);
    else if (j->cfg == 4) {
      if (len > tmpcap) { free(tmp); tmp = (uint8_t *)malloc(len); tmpcap = len; }
      if (!tmp) return (void *)1;
      fill_dna_read(&r, tmp, len);
      for (uint64_t t = 0; t < len; t++) put2(j->data, j->off[f] + t, tmp[t], lo_byte, hi_byte);
    }
  }
  free(tmp);
  return NULL;
}

/* Fill data (iggen_data_bytes(...) bytes) for files [0, m) with the given offsets. */
int iggen_fill(int cfg, uint64_t seed, uint64_t m, const uint64_t *sym_offsets, uint8_t *data, int nthreads) {
  if (cfg < 1 || cfg > 4) return -1;
  if (nthreads < 1) nthreads = 1;
  if (nthreads > 256) nthreads = 256;
  chain_t chain; motifs_t *motifs = NULL; vocab_t *vocab = NULL;
  chain_init(&chain, seed);
  if (cfg == 2) { motifs = (motifs_t *)malloc(sizeof(motifs_t)); if (!motifs || motifs_init(motifs, seed)) return -2; }
  if (cfg == 3) { vocab = (vocab_t *)malloc(sizeof(vocab_t)); if (!vocab || vocab_init(vocab, seed)) return -2; }
  if (cfg == 4) memset(data, 0, iggen_data_bytes(cfg, sym_offsets[m]));
  /* split files by symbol count so that threads get similar work */
  job_t jobs[256]; pthread_t th[256];
  uint64_t total = sym_offsets[m], f = 0;
  for (int t = 0; t < nthreads; t++) {
    uint64_t target = total / (uint64_t)nthreads * (uint64_t)(t + 1);
    uint64_t f0 = f;
    if (t == nthreads - 1) f = m;
    else while (f < m && sym_offsets[f + 1] <= target) f++;
    jobs[t] = (job_t){cfg, seed, m, sym_offsets, data, &chain, motifs, vocab, f0, f};
  }
  int rc = 0;
  for (int t = 0; t < nthreads; t++) pthread_create(&th[t], NULL, fill_worker, &jobs[t]);
  for (int t = 0; t < nthreads; t++) { void *ret; pthread_join(th[t], &ret); if (ret) rc = -3; }
  if (motifs) { motifs_free(motifs); free(motifs); }
  if (vocab) { vocab_free(vocab); free(vocab); }
  return rc;
}

/* ---------------- request stream (workload 5) ---------------- */
typedef struct { motifs_t motifs; uint64_t seed; } reqgen_t;

void *iggen_req_open(uint64_t seed, uint64_t lib_seed) {
  reqgen_t *g = (reqgen_t *)malloc(sizeof(reqgen_t));
  if (!g) return NULL;
  if (motifs_init(&g->motifs, lib_seed)) { free(g); return NULL; }
  g->seed = seed;
  return g;
}
void iggen_req_close(void *h) { reqgen_t *g = (reqgen_t *)h; if (g) { motifs_free(&g->motifs); free(g); } }
/* gap (seconds) before request i arrives, exponential with mean 0.5 ms */
double iggen_req_gap(void *h, uint64_t i) {
  reqgen_t *g = (reqgen_t *)h;
  rng_t r = rng_stream(g->seed, TAG_ARRIVAL, i);
  return -0.0005 * log(1.0 - rng_unif(&r));
}
uint64_t iggen_req_len(void *h, uint64_t i) {
  reqgen_t *g = (reqgen_t *)h;
  rng_t r = rng_stream(g->seed, TAG_REQ, i);
  return lognormal_size(&r, 65536.0, 1.5, 4096, 64ull << 20);
}
/* writes request i's file (iggen_req_len bytes) */
int iggen_req_fill(void *h, uint64_t i, uint8_t *dst) {
  reqgen_t *g = (reqgen_t *)h;
  uint64_t len = iggen_req_len(h, i);
  rng_t r = rng_stream(g->seed, TAG_FILE, i);
  fill_binary_file(&g->motifs, &r, dst, len);
  return 0;
}
