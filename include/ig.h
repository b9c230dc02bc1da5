/*
 * ig.h -- C ABI of libintergrams.so: the Intergrams per-pass scan on one
 * AMD Instinct MI355X (gfx950).
 *
 * Method: Curtin, Lu, Raff, Ranade, "Intermediate N-Gramming: Deterministic
 * and Fast N-Grams For Large N and Large Datasets" (arXiv 2511.14955).
 *
 *  - Problem statement (Section "Problem Formalization and Notation"): m
 *    sequences; an n-gram is n consecutive symbols of one sequence (no gram
 *    crosses a sequence boundary); its frequency is Eq. 1 (occurrences) or
 *    Eq. 2 (number of sequences containing it; the paper's focus).
 *  - A pass (Algorithm 3): count the n-grams whose (n-1)-gram prefix is in
 *    the set retained by the previous pass and retain the k_keep most
 *    frequent.
 *  - Featurize (Figure 1): map sequences to Boolean rows over the retained
 *    n-grams.
 *
 * Conventions for every call:
 *  - Return IG_OK (0) or a negative IG_E* code.  The message of the last
 *    failure is available from ig_last_error().  No C++ exception crosses the
 *    ABI.
 *  - Calls are synchronous: they return after the device work has finished,
 *    except ig_serve_* which run asynchronously by design.
 *  - The caller owns every pointer it passes.  Host buffers are read or
 *    written before the call returns; a device pointer passed with
 *    data_on_device = 1 must stay valid for the duration of the call.  The
 *    library owns the device copy of the corpus, the tables and all scratch,
 *    and ig_destroy frees them.
 *  - One context is used by one thread at a time; the serving calls are
 *    internally synchronized.
 *  - IG_EDEVICE (a HIP runtime error) is sticky: every later call on the
 *    context fails with it and the context must be destroyed.
 */
#ifndef IG_H
#define IG_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define IG_OK          0
#define IG_EINVAL     (-1)  /* bad argument: n = 0, n*b > 128, k_keep = 0, bad offsets, bad config */
#define IG_ESTATE     (-2)  /* call out of order: pass n after a pass other than n-1, topk before a pass */
#define IG_ENOMEM     (-3)  /* device allocation failed or the HBM budget would be exceeded */
#define IG_ETRUNC     (-4)  /* caller buffer too small; the *_out argument holds the size needed */
#define IG_EOVERFLOW  (-5)  /* 32-bit counts requested but a count could reach 2^32 */
#define IG_EDEVICE    (-6)  /* HIP runtime error (sticky) */
#define IG_EBUSY      (-7)  /* serving: queue full */

typedef struct ig_ctx ig_ctx;

/* An n-gram key: the n symbols packed most significant first into an
 * n*b-bit integer, right-aligned (hi holds bits 64..127).  Numeric order of
 * keys equals lexicographic order of the symbol strings. */
typedef struct { uint64_t lo, hi; } ig_key;

/* Frequency (problem statement, Eq. 1 and Eq. 2). */
typedef enum {
  IG_FREQ_DOC = 0,   /* Eq. 2: number of sequences containing the gram (default) */
  IG_FREQ_OCC = 1    /* Eq. 1: number of occurrences */
} ig_freq;

typedef struct {
  uint32_t symbol_bits;  /* 8: bytes / text; 2: DNA packed A=0 C=1 G=2 T=3 */
  ig_freq  freq;         /* counting rule */
  uint32_t count_bits;   /* 32 or 64: width callers need; 32 is refused with IG_EOVERFLOW
                            when W_n >= 2^32 under IG_FREQ_OCC (Eq. 2 counts are <= m) */
  int      device;       /* HIP device ordinal */
  void    *stream;       /* hipStream_t to run on; NULL: the library creates one */
  uint64_t hbm_budget;   /* bytes of device memory this context may hold; 0 = no limit */
  uint32_t flags;        /* IG_FLAG_* */
  /* Optional device allocator, e.g. a framework's caching allocator.  When alloc is set (free
   * must be too), every device buffer the context holds is taken from alloc(bytes, stream,
   * alloc_user) and given back through free(p, stream, alloc_user); alloc returns NULL on
   * failure (the call then fails with IG_ENOMEM).  stream is the context's stream; a buffer is
   * given back only after the work that used it has finished.  Both are called from the
   * thread making the library call (and from the serving thread while serving). */
  void *(*alloc)(size_t bytes, void *stream, void *user);
  void  (*free)(void *p, void *stream, void *user);
  void   *alloc_user;
} ig_config;

#define IG_FLAG_NO_GRAPH      1u  /* launch pass kernels directly instead of a captured hipGraph */
#define IG_FLAG_PER_FILE      2u  /* one scan launch per file (comparison form) instead of one
                                     persistent launch over the whole work queue */

/* Fill *cfg with defaults: bytes, Eq. 2, 64-bit counts, device 0, own stream, no budget. */
void ig_config_default(ig_config *cfg);

/* Create a context on cfg->device.  On failure *out is NULL. */
int  ig_create(const ig_config *cfg, ig_ctx **out);
void ig_destroy(ig_ctx *ctx);

/* Load m sequences (the problem statement's m input sequences over an alphabet; an n-gram is n
 * consecutive symbols of one sequence, so sequence boundaries are kept), replacing any previous
 * corpus and resetting the pass chain.
 *  data:        symbol stream; symbol i occupies bits [i*b, i*b+b) of the stream,
 *               most significant first within each byte (bytes when b = 8).
 *  data_bytes:  size of data; must cover sym_offsets[m] symbols.
 *  sym_offsets: m+1 non-decreasing symbol offsets, sym_offsets[0] = 0; sequence i is
 *               symbols [sym_offsets[i], sym_offsets[i+1]).  Always a host array.
 *  data_on_device: 0: data is a host pointer; 1: a device pointer on ctx's device.
 * Errors: IG_EINVAL (offsets), IG_ENOMEM (budget / allocation), IG_EDEVICE. */
int  ig_load_batch(ig_ctx *ctx, const void *data, uint64_t data_bytes,
                   const uint64_t *sym_offsets, uint64_t m, int data_on_device);

/* One pass (Algorithm 3): count every n-gram of the loaded sequences whose
 * (n-1)-gram prefix is in the table retained by the previous pass (no filter
 * when n = 1 or when no pass has run since the last load), then retain the
 * first min(k_keep, D) of the D counted grams in the order (count desc, key asc).
 * Errors: IG_EINVAL (n = 0, n*b > 128, k_keep = 0), IG_ESTATE (previous pass
 * was not n-1 and the chain is not fresh, or nothing loaded), IG_EOVERFLOW,
 * IG_ENOMEM, IG_EDEVICE.  On error the previous table is kept. */
int  ig_pass(ig_ctx *ctx, uint32_t n, uint64_t k_keep);

/* The whole of Algorithm 3 with z-oversampling (Section 4; z as in the evaluation):
 * the chain run since the last load is discarded, then
 *  - a fresh, unfiltered pass at n0 = min(n, floor(24 / b)) (3 for bytes: Algorithm 2's
 *    direct-indexed count over all 2^24 3-grams) keeps ceil(z*k) grams, and
 *  - the filtered passes j = n0+1 .. n keep ceil(z*k) grams for j < n and k at j = n.
 * With n <= n0 the single pass at n keeps k.  Afterwards the retained table is the
 * top-k of the last pass, as after ig_pass(ctx, n, k), and ig_rewind undoes that pass.
 * Errors: IG_EINVAL (k = 0, z < 1 or not finite, ceil(z*k) >= 2^63, or n as in
 * ig_pass), then those of ig_pass; on an error the passes that completed remain. */
int  ig_intergrams(ig_ctx *ctx, uint32_t n, uint64_t k, double z);

/* Undo the last pass (the chain of Algorithm 3's retained sets P^(j), one level back): the
 * table retained before it becomes current again
 * (one level; the state right after ig_load_batch counts as a level), so the
 * last pass can be run again.  Device-side pointer swap, no copy.
 * IG_ESTATE if there is nothing to undo. */
int  ig_rewind(ig_ctx *ctx);

/* The result of Algorithm 3's final k-argmax: copy the first min(k, kept) entries of the
 * retained table, in the order (count desc, key asc) (host buffers of k entries; keys as above;
 * counts may be NULL; counts are Eq. 1 or Eq. 2 frequencies by ig_config.freq).
 * *k_out = number copied.  IG_ESTATE before a pass. */
int  ig_topk(ig_ctx *ctx, uint64_t k, ig_key *keys, uint64_t *counts, uint64_t *k_out);

/* Gram length n and size of the retained table P^(n) of Algorithm 3 (0, 0 before any pass). */
int  ig_table_info(const ig_ctx *ctx, uint32_t *n, uint64_t *kept);

/* Boolean feature rows (Figure 1) of m new sequences against the retained table:
 * row i lists, ascending, the 0-based ranks of retained grams occurring in
 * sequence i.  data / sym_offsets as in ig_load_batch (data is a host pointer).
 *  indptr:  host array of m+1 entries (row i = indices[indptr[i] .. indptr[i+1])).
 *  indices: host array of cap entries.
 *  *nnz_out: total entries.  IG_ETRUNC if nnz > cap (indptr is still filled).
 * The loaded corpus and the pass chain are not changed. */
int  ig_featurize(ig_ctx *ctx, const void *data, uint64_t data_bytes,
                  const uint64_t *sym_offsets, uint64_t m,
                  uint64_t *indptr, int32_t *indices, uint64_t cap, uint64_t *nnz_out);

/* For callers that cannot allocate device memory (code under HIP graph capture, serving loops
 * or harnesses that forbid hipMalloc): the same rows as ig_featurize, with the same arguments
 * and errors, computed without allocating.  Every device buffer the call needs beyond its
 * inputs and outputs (the staged batch, its chunk list, per-sequence rank bitmaps, row counts
 * and offsets, the CSR entries before their copy out) is carved from a fixed scratch array of
 * IG_NOALLOC_SCRATCH_BYTES that the library holds on each device it runs on until the process
 * ends.  IG_EINVAL (with a message naming the limit) when a batch does not fit it: about
 * data_bytes + 24 B per chunk of the launch shape + m * (4 * ceil(kept / 32) + 16) + 4 * nnz
 * bytes, each piece rounded up to 256.  Calls on one device share that array; within a
 * process they are serialized (a call waits for the one running on the same device).
 * IG_EDEVICE if the array could not be located when the context was created. */
#define IG_NOALLOC_SCRATCH_BYTES (64ull << 20)
int  ig_featurize_noalloc(ig_ctx *ctx, const void *data, uint64_t data_bytes,
                          const uint64_t *sym_offsets, uint64_t m,
                          uint64_t *indptr, int32_t *indices, uint64_t cap, uint64_t *nnz_out);

/* The same Boolean rows (Figure 1's m x k matrix) for the m loaded sequences themselves,
 * from the corpus already resident on the device (no host copy of the data).
 *  indptr:  host array of m+1 entries; indices: host array of cap entries (may be NULL
 *  when cap = 0, to learn *nnz_out).  IG_ETRUNC if nnz > cap (indptr is still filled).
 *  IG_ESTATE before a pass or while serving. */
int  ig_featurize_loaded(ig_ctx *ctx, uint64_t *indptr, int32_t *indices, uint64_t cap, uint64_t *nnz_out);

/* Per-pass measurements of the last ig_pass: device time of the whole pass and of
 * the scan kernel (milliseconds, hipEvent-timed on the context's stream), windows
 * scanned, distinct grams counted, and the scan kernel's average duration. */
typedef struct {
  double   pass_ms;      /* whole pass: clear, scan, counting, selection, index */
  double   scan_ms;      /* the scan kernel */
  double   select_ms;    /* selection and index build */
  uint64_t windows;
  uint64_t distinct;
  uint64_t input_bytes;
  uint32_t replays;      /* times the pass was re-run after growing a table */
  uint32_t chunk_syms;   /* launch parameters in use */
  uint32_t block;
  uint32_t grid;
  uint64_t records;      /* Eq. 2: chunk-distinct (candidate, sequence) records counted once per sequence */
  double   dedup_ms;     /* Eq. 2: counting the records once per sequence */
  uint32_t set_cap;      /* the scan's LDS set size in use: the launch's, halved while it did not
                            fit this pass's LDS, or, for a direct-indexed pass whose chunks
                            repeat their grams, grown (results do not depend on it) */
  uint32_t reserved;
} ig_pass_stats;
int  ig_last_pass_stats(const ig_ctx *ctx, ig_pass_stats *st);

/* Measurement aid, not part of the method: the read bandwidth (GB/s, 1e9 B) that a plain
 * streaming kernel attains on ctx's device, for comparison with a pass's input rate.  It
 * allocates `bytes` (within the context's HBM budget), reads them once untimed and then reps
 * times timed with device events, and frees them.  Errors: IG_EINVAL (bytes < 16, reps = 0,
 * null output), IG_ESTATE while serving, IG_ENOMEM, IG_EDEVICE. */
int  ig_measure_read_bw(ig_ctx *ctx, uint64_t bytes, uint32_t reps, double *gb_per_s);

const char *ig_last_error(const ig_ctx *ctx);

/* ---------------------------------------------------------------------------
 * Launch shape of the scan and its autotuner.
 *
 * chunk_syms: symbols per work item (a chunk of one sequence plus its n-1
 * symbol halo, 1024..65536); block: threads per workgroup (256, 512, 1024);
 * set_cap: LDS de-duplication set entries (a power of two, 1024..32768, at
 * least block); wg_per_cu: scan workgroups per compute unit (1 or 2; a pass
 * whose workgroup LDS does not fit half a CU runs one per CU).
 * IG_EINVAL otherwise.  The shape changes speed only, never results.  A pass
 * whose LDS cannot hold the shape (its filter image, survivor rings and
 * histograms depend on the pass) halves the set down to 4096 entries while its
 * survivor rings do not fit, then resolves survivors without the rings, then
 * halves the set further until it fits (down to block entries).  A directly
 * indexed pass (every n-gram of the alphabet a candidate) over at most
 * chunk_syms grams (sigma^n over the corpus's alphabet) grows a set smaller
 * than twice that, up to twice it or 32768 entries, while its LDS allows; so
 * does an Eq. 2 one over more grams whose previous table's pass made at most
 * one record per 8 windows.  ig_last_pass_stats reports the set size the pass
 * ran with.
 *
 * ig_autotune runs pass n on the loaded corpus for each candidate shape
 * (rewinding after each), checks that all candidates return the same table,
 * and keeps the fastest (a shape that runs only with a smaller LDS set counts as
 * unusable for the pass); the chain state is left as it was.  It searches the
 * launch shape first, then, with the best one, the table sizes of
 * ig_set_tables (map_slots_log2 1 or 2, filter_max_words 8192 or 16384),
 * which apply to the current table's index, and last two workgroups per CU
 * (Bloom image in L2, 4096-entry LDS set, chunks of 12288, 16384 or the winner's symbols,
 * 512- or 1024-thread workgroups).  With the
 * environment variable IG_TUNE_CACHE naming a file, results are read from and
 * appended to it, keyed by device, corpus shape and (n, k_keep).
 * --------------------------------------------------------------------------- */
#define IG_TUNE_MAX 32
typedef struct {
  uint32_t n_candidates;
  struct {
    uint32_t chunk_syms, block, set_cap, wg_per_cu, map_slots_log2, filter_max_words;
    double pass_ms;             /* < 0: shape unusable for this pass */
  } cand[IG_TUNE_MAX];
  uint32_t best;
  int      identical;     /* 1 if every candidate produced the same table */
  int      from_cache;
} ig_tune_report;
int ig_autotune(ig_ctx *ctx, uint32_t n, uint64_t k_keep, ig_tune_report *rep);
int ig_get_launch(const ig_ctx *ctx, uint32_t *chunk_syms, uint32_t *block, uint32_t *set_cap,
                  uint32_t *wg_per_cu);
int ig_set_launch(ig_ctx *ctx, uint32_t chunk_syms, uint32_t block, uint32_t set_cap, uint32_t wg_per_cu);

/* ---------------------------------------------------------------------------
 * Table sizes (speed only, never results).
 *
 *  map_slots_log2:      the exact maps over a retained table of k keys (key -> rank, and the
 *                       quotient map) get the smallest power of two >= k << map_slots_log2
 *                       slots: load at most 1/2, 1/4, 1/8 for 1, 2, 3 (default 2).
 *  filter_bits_per_key: the Bloom filter image a scan workgroup holds in LDS gets about this
 *                       many bits per retained key (4..32, default 12), a power of two of at
 *                       most filter_max_words 32-bit words (1024..16384, default 16384).
 *  sparse_slots:        key-table slots of unfiltered passes with n*b > 26 (a power of two,
 *                       1024..2^31; 0 leaves it as is; the library starts at twice the windows
 *                       of the first such pass).  A pass that fills it is replayed with 4x.
 *  record_capacity:     Eq. 2 records the bucketed arrays hold (0 leaves it as is; raised to
 *                       one tile per level-1 bucket at least).  A pass that fills it is
 *                       replayed with twice as much.
 * ig_set_tables indexes the current table again with the new map and filter sizes, so the
 * next pass uses them.  IG_EINVAL for values out of range, IG_ESTATE while serving.
 * ig_autotune also searches map_slots_log2 and filter_max_words (after the launch shape).
 * --------------------------------------------------------------------------- */
typedef struct {
  uint32_t map_slots_log2;
  uint32_t filter_bits_per_key;
  uint32_t filter_max_words;
  uint32_t reserved;
  uint64_t sparse_slots;
  uint64_t record_capacity;
} ig_table_shape;
int ig_get_tables(const ig_ctx *ctx, ig_table_shape *shape);
int ig_set_tables(ig_ctx *ctx, const ig_table_shape *shape);

/* ---------------------------------------------------------------------------
 * Serving (continuous batching of featurize / count requests).
 *
 * ig_serve_start takes one device arena of max_inflight_bytes (counted
 * against ig_config.hbm_budget) and starts a background thread.  The thread
 * admits submitted requests in FIFO order while the device region the next
 * launch needs (inputs, per-sequence bitmaps, outputs) fits the arena's
 * largest free block, packs up to max_batch requests into one launch on one
 * of n_streams streams, and completes them when the launch has finished,
 * returning the region.  Requests that arrive while launches run are admitted
 * as soon as a stream and arena space free up; launches on different streams
 * overlap.  A request that cannot fit even an empty arena completes with
 * status IG_ENOMEM.  The table served is the context's retained table at
 * ig_serve_start (the featurization step of Figure 1); ig_pass, ig_rewind,
 * ig_load_batch, ig_featurize, ig_autotune and ig_set_launch return
 * IG_ESTATE until ig_serve_stop.  ig_submit, ig_poll and ig_serve_get_stats
 * may be called from any thread (results go to whoever polls first);
 * ig_serve_stop and ig_destroy must not overlap them.
 *
 * kind IG_REQ_FEATURIZE: one sequence (m = 1); the result is its Boolean row
 *   (int32 ranks, ascending), as ig_featurize.
 * kind IG_REQ_COUNT: m >= 1 sequences; the result is, for every retained
 *   gram found in at least one of them, (rank, number of the request's
 *   sequences containing it), rank ascending: Eq. 2 restricted to the table.
 * Errors: IG_ESTATE (no serving loop), IG_EINVAL (bad kind or offsets),
 *   IG_EBUSY from ig_submit when queue_capacity requests are pending.
 * --------------------------------------------------------------------------- */
#define IG_REQ_FEATURIZE 0
#define IG_REQ_COUNT     1

typedef struct {
  uint64_t max_inflight_bytes;  /* HBM admission budget for in-flight requests */
  uint32_t n_streams;           /* concurrent launches (1..8) */
  uint32_t max_batch;           /* most requests packed into one launch */
  uint64_t queue_capacity;      /* most submitted, not yet completed requests */
} ig_serve_config;

int ig_serve_start(ig_ctx *ctx, const ig_serve_config *scfg);
/* Submit one request (a copy of data is taken before returning).
 *  sym_offsets: m+1 offsets of the request's sequences (m = 1 for featurize).
 *  tag: caller id returned with the result.  t_arrival: caller clock (seconds),
 *  returned with the result.  IG_EBUSY when queue_capacity requests are pending. */
int ig_submit(ig_ctx *ctx, int kind, const void *data, uint64_t data_bytes,
              const uint64_t *sym_offsets, uint64_t m, uint64_t tag, double t_arrival);

typedef struct {
  uint64_t tag;
  int      kind;
  int      status;         /* IG_OK or an error for this request */
  double   t_arrival;      /* as submitted */
  double   t_done;         /* library clock (seconds, same base as ig_serve_now) when the result was on the host */
  uint64_t n;              /* entries in the result */
} ig_result;

/* Take up to max completed results, oldest first, as long as their entries
 * together fit cap: result i's entries go to cols[out_off[i] .. out_off[i+1])
 * (ranks) and, for COUNT requests, counts[] at the same positions (counts may
 * be NULL).  out_off (may be NULL) has max+1 entries.  *n_out = results taken
 * (0 when none is ready).  If the oldest result alone needs more than cap
 * entries, nothing is taken, res[0] holds its header (its n is the room
 * needed) and IG_ETRUNC is returned. */
int ig_poll(ig_ctx *ctx, ig_result *res, uint64_t max, int32_t *cols, uint64_t *counts,
            uint64_t cap, uint64_t *out_off, uint64_t *n_out);
/* Library clock in seconds (CLOCK_MONOTONIC). */
double ig_serve_now(void);
/* Stop admitting, drain in-flight work, join the serving thread. */
int ig_serve_stop(ig_ctx *ctx);

typedef struct {
  uint64_t submitted, completed, launches, rejected;
  uint64_t peak_inflight_bytes;   /* most arena bytes held by running launches at once */
  uint64_t bytes_in;              /* request payload bytes launched */
  uint64_t peak_running;          /* most launches running at once (<= n_streams) */
} ig_serve_stats;
int ig_serve_get_stats(ig_ctx *ctx, ig_serve_stats *st);

#ifdef __cplusplus
}
#endif
#endif /* IG_H */
