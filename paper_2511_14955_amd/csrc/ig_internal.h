// Internal declarations shared by the HIP sources of libintergrams.so.
//
// Data layout in HBM (all buffers owned by the context):
//  * corpus: the symbol stream as loaded (bytes, or 2-bit symbols MSB first),
//    padded with 64 zero bytes; file offsets in symbols (m+1 x u64).
//  * work items ("chunks"): each covers at most chunk_syms symbols of one file;
//    a chunk owns the windows that start inside it and reads the n-1 symbols
//    after it (the halo) from the same file.  Chunks are kept in file order (for
//    the one-launch-per-file form) and in decreasing length (the LPT order of
//    the persistent work queue).
//  * candidate space: a pass counts into a dense array indexed by a candidate id
//      filtered pass:      cid = rank(prefix) * sigma + code(last symbol)
//                          (the paper's C in N^{256 zk}, Algorithm 3, with the
//                          alphabet compacted to the sigma symbols present)
//      small unfiltered:   cid = key                       (n*b <= 26)
//      large unfiltered:   cid = slot of the key in a device hash table
//  * retained table: keys (lo/hi u64 arrays) and counts (u64), in the order
//    (count desc, key asc); a hash map key -> rank (32-bit slots with a hash
//    fingerprint, confirmed against the keys) and a compact filter image over
//    the same keys serve both the next pass (prefix test) and featurize.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/ig.h"

namespace ig {

// ------------------------------------------------------------------ device helpers
__host__ __device__ __forceinline__ uint64_t mix64(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}
// Hash of an n-gram key (lo, hi): xor-shift, one 64-bit multiply, xor-shift (the first half of
// the murmur3 finalizer).  Keys of at most 64 bits have hi = 0, and the hi term folds away.
// The filter image takes its word from the high half and its bits from the low bits, map
// slots take the low bits and fingerprints the top bits.
__host__ __device__ __forceinline__ uint64_t hash_key(uint64_t lo, uint64_t hi) {
  uint64_t x = lo ^ (hi * 0x9E3779B97F4A7C15ull);
  x ^= x >> 33;
  x *= 0xFF51AFD7ED558CCDull;
  return x ^ (x >> 29);
}
// Index keys.  The maps and filter images over a retained table are keyed by a gram's stream
// form: its n symbols with the FIRST symbol in the LOWEST b bits (symbol r at bits [b r, b r + b)),
// the order in which symbols sit in the little-endian bit stream that the scan stages (bytes as
// stored; 2-bit symbols with the four of each byte reversed).  A window's stream form is then a
// funnel shift of two staged words and its prefix a mask.  The retained table itself keeps the
// canonical form (first symbol most significant, numeric order = lexicographic order).
__host__ __device__ __forceinline__ uint64_t rev_pairs64(uint64_t x) {   // 2-bit digits of x in reverse order
  x = ((x >> 2) & 0x3333333333333333ull) | ((x & 0x3333333333333333ull) << 2);
  x = ((x >> 4) & 0x0F0F0F0F0F0F0F0Full) | ((x & 0x0F0F0F0F0F0F0F0Full) << 4);
  return __builtin_bswap64(x);
}
__host__ __device__ __forceinline__ void stream_form(uint64_t lo, uint64_t hi, uint32_t n, uint32_t b, uint64_t *olo,
                                                     uint64_t *ohi) {
  const uint32_t nb = n * b;
  if (nb == 0) { *olo = 0; *ohi = 0; return; }
  if (nb <= 64) {
    const uint64_t r = b == 8 ? __builtin_bswap64(lo) : rev_pairs64(lo);
    *olo = r >> (64 - nb);
    *ohi = 0;
    return;
  }
  // 64 < nb <= 128: digit j of the canonical key (from the top) goes to digit j of the result
  // (from the bottom)
  const uint64_t dm = (1ull << b) - 1;
  uint64_t rlo = 0, rhi = 0;
  for (uint32_t j = 0; j < n; j++) {
    const uint32_t src = nb - b * (j + 1);   // canonical position of digit j
    const uint64_t d = (src >= 64 ? (hi >> (src - 64)) : (lo >> src) | (src ? (hi << (64 - src)) : 0ull)) & dm;
    const uint32_t dst = b * j;
    if (dst >= 64) rhi |= d << (dst - 64);
    else rlo |= d << dst;
  }
  *olo = rlo;
  *ohi = rhi;
}
// The stream form's low 32 bits folded with its high bits (a filter image's hash input).
__host__ __device__ __forceinline__ uint32_t fold_le(uint64_t lo, uint64_t hi) {
  const uint32_t a = (uint32_t)lo, c = (uint32_t)(lo >> 32);
  return a ^ ((c >> 13) | (c << 19)) ^ (uint32_t)hi ^ (uint32_t)(hi >> 32) * 0x85EBCA6Bu;
}
// Quotient map over keys of w <= 64 bits.  qmix is a bijection of w-bit values (xor-shifts and
// odd multiplies modulo 2^w); the top sbits of the mix choose the home slot and the low qbits are
// stored in the slot, above the displacement from home (dbits) and rank+1 (rbits).  A slot's
// home and stored bits give back the whole mix, hence the key: one 8-byte read identifies it.
struct QMapShape {
  uint32_t w, sbits, qbits, rbits, dbits;
};
__host__ __device__ __forceinline__ uint64_t qmix(uint64_t x, uint32_t w) {
  // one round: the multiply carries every bit into the top bits (the home slot), the last
  // xor-shift folds the top bits into the stored low bits
  const uint64_t m = w >= 64 ? ~0ull : ((1ull << w) - 1);
  const uint32_t s = (w + 1) >> 1;
  x ^= x >> s;
  x = (x * 0xFF51AFD7ED558CCDull) & m;
  return x ^ (x >> s);
}
// Quotient map with 16-byte slots, for tables whose 8-byte slots cannot hold remainder,
// displacement and rank: prefixes of more than 64 bits (up to 128), or of up to 64 bits with many
// keys.  qmix2 is a bijection of w-bit values, lo the first 64 bits and hi the other w - 64:
//   w <= 64: qmix of lo (as above);
//   w > 64:  a = mix64(lo); b = hi xor (a times an odd constant), cut to w - 64 bits;
//            a' = mix64(a xor (b times an odd constant)).
// Each step is invertible (mix64, the finalizer above, is xor-shifts and odd multiplies; an xor of
// a function of the other half is undone by the same xor), so (a', b) gives back the key.  The home slot is the
// top sbits of the mix (of a' for w > 64) and the remainder the rest of it, (a' below the home,
// then b) for w > 64.  A slot holds rank+1 in its low rbits, the displacement from home in the
// next dbits, and the remainder above them: one 16-byte read identifies its key.
// home slot and remainder (rl: its low 64 bits, rh: the rest) of a w-bit key in 2^sbits slots
__host__ __device__ __forceinline__ void qmix2(uint64_t lo, uint64_t hi, uint32_t w, uint32_t sbits, uint64_t *home,
                                               uint64_t *rl, uint64_t *rh) {
  if (w <= 64) {
    const uint64_t x = qmix(lo, w);
    const uint32_t qb = w - sbits;   // 1 <= qb <= 54 (sbits >= 10, and w > sbits for such tables)
    *home = x >> qb;
    *rl = x & ((1ull << qb) - 1);
    *rh = 0;
    return;
  }
  const uint32_t bw = w - 64;
  const uint64_t bm = bw >= 64 ? ~0ull : ((1ull << bw) - 1);
  const uint64_t a = mix64(lo);
  const uint64_t b = (hi ^ (a * 0x9E3779B97F4A7C15ull)) & bm;
  const uint64_t a2 = mix64(a ^ (b * 0xC2B2AE3D27D4EB4Full));
  const uint32_t lb = 64 - sbits;   // bits of a' below the home (10 <= sbits <= 40)
  *home = a2 >> lb;
  *rl = (a2 & ((1ull << lb) - 1)) | (b << lb);
  *rh = b >> (64 - lb);
}

// Blocked Bloom filter position of a key's 32-bit fold (filter of `words` 32-bit words, a power
// of two): one 32 x 32 -> 64-bit multiply; the word and the three bits come from the product's
// high word.  (Folding only adds collisions of about k / 2^32 per query; a filter has no false
// negatives either way.)
__host__ __device__ __forceinline__ void bloom_pos(uint32_t v, uint32_t words, uint32_t *word, uint32_t *mask) {
  const uint32_t t = (uint32_t)(((uint64_t)v * 0x9E3779B1ull) >> 32);
  *word = t & (words - 1);
  *mask = (1u << ((t >> 14) & 31)) | (1u << ((t >> 19) & 31)) | (1u << ((t >> 24) & 31));
}

// Lanes of this wavefront whose `key` (its low `nbits` bits) equals this lane's, among the
// valid lanes (the wavefront's analogue of a match instruction: one ballot per key bit).
// Invalid lanes get the mask of valid lanes sharing their bits, which callers ignore.
__device__ __forceinline__ uint64_t wave_match(uint32_t key, uint32_t nbits, bool valid) {
  const uint64_t vm = __ballot(valid);
  // per bit: the lanes with that bit set, complemented where this lane's bit is clear (an
  // xor with an all-ones word, so each step is a few plain VALU operations on the ballot)
  uint32_t lo = (uint32_t)vm, hi = (uint32_t)(vm >> 32);
  for (uint32_t q = 0; q < nbits; q++) {
    const uint32_t bit = (key >> q) & 1u;
    const uint64_t bq = __ballot(bit != 0u);
    const uint32_t flip = bit - 1u;   // 0 where the bit is set, all ones where it is clear
    lo &= (uint32_t)bq ^ flip;
    hi &= (uint32_t)(bq >> 32) ^ flip;
  }
  return ((uint64_t)hi << 32) | lo;
}

// Key -> rank map: one 32-bit slot per entry, holding rank+1 in its low rank_bits bits and a
// fingerprint of the key's hash in the rest (empty = 0).  A probe compares fingerprints and
// only on a match reads the key itself from the table's keys (stored in rank order) to confirm.
__device__ __forceinline__ uint32_t map_fp(uint64_t h, uint32_t rank_bits) {
  return rank_bits >= 32 ? 0u : (uint32_t)(h >> (32 + rank_bits));
}

// Exclusive scan of a[0, len) in place by one workgroup of 1024 threads (16 wavefronts): blocks
// of 4096 elements, 4 consecutive per thread (coalesced), wavefront scans by shuffles, the
// wavefront sums scanned in LDS, and a carry between blocks.  *total_out (if given) = the sum.
template <typename T> __device__ __forceinline__ T shfl_up_t(T x, uint32_t d) {
  if constexpr (sizeof(T) == 8) {
    const uint32_t lo = __shfl_up((unsigned)(x & 0xFFFFFFFFull), d), hi = __shfl_up((unsigned)(x >> 32), d);
    return ((T)hi << 32) | (T)lo;
  } else {
    return (T)__shfl_up((unsigned)x, d);
  }
}
template <typename T> __device__ void wg_exclusive_scan(T *a, uint64_t len, T *total_out) {
  __shared__ T wsum[16];
  __shared__ T carry;
  const uint32_t t = threadIdx.x, lane = t & 63, w = t >> 6;
  if (t == 0) carry = 0;
  __syncthreads();
  for (uint64_t base = 0; base < len; base += 4096) {
    T v[4], sum = 0;
#pragma unroll
    for (int q = 0; q < 4; q++) {
      const uint64_t i = base + (uint64_t)t * 4 + q;
      v[q] = i < len ? a[i] : (T)0;
      sum += v[q];
    }
    T x = sum;
    for (uint32_t off = 1; off < 64; off <<= 1) {
      const T y = shfl_up_t(x, off);
      if (lane >= off) x += y;
    }
    if (lane == 63) wsum[w] = x;
    __syncthreads();
    if (t < 64) {
      T ws = lane < 16 ? wsum[lane] : (T)0;
      for (uint32_t off = 1; off < 16; off <<= 1) {
        const T y = shfl_up_t(ws, off);
        if (lane >= off) ws += y;
      }
      if (lane < 16) wsum[lane] = ws;   // inclusive over the wavefronts
    }
    __syncthreads();
    T run = carry + (w ? wsum[w - 1] : (T)0) + x - sum;
#pragma unroll
    for (int q = 0; q < 4; q++) {
      const uint64_t i = base + (uint64_t)t * 4 + q;
      if (i < len) a[i] = run;
      run += v[q];
    }
    __syncthreads();   // carry and wsum have been read
    if (t == 0) carry += wsum[15];
    __syncthreads();
  }
  if (t == 0 && total_out) *total_out = carry;
}

// ------------------------------------------------------------------ shared structs
struct Chunk {
  uint64_t s0;      // first symbol (absolute) whose window this chunk owns
  uint32_t file;
  uint32_t nsym;    // symbols owned (windows start in [s0, s0 + nsym))
  uint32_t multi;   // the file has more than one chunk
  uint32_t fci;     // index of this chunk in file order (records and histograms are kept in that order)
};

enum PassMode { MODE_DENSE = 0, MODE_FILTERED = 1, MODE_SPARSE = 2 };
// FILT_GBLOOM: a Bloom filter image too large for LDS (more than about 131K retained keys), read
// from global memory, where it stays in L2; the others are copied into LDS.
enum FilterKind { FILT_NONE = 0, FILT_DIRECT = 1, FILT_BLOOM = 2, FILT_GBLOOM = 3 };
// 32-bit words of a table's filter image that a workgroup copies into LDS
__host__ __device__ __forceinline__ uint32_t filt_lds_words(uint32_t kind, uint32_t words) {
  return (kind == FILT_DIRECT || kind == FILT_BLOOM) ? words : 0u;
}
enum StatusBits { ST_TABLE_OVF = 2u, ST_REC_OVF = 4u };

static constexpr uint32_t LDS_EMPTY = 0xFFFFFFFFu;
static constexpr uint32_t SCAN_QCAP = 128;   // filter survivors queued per wavefront (power of two, >= 127)

// Parameters of one scan (ingest + prefix filter + per-sequence dedup + count) launch.
struct ScanParams {
  const uint8_t *data;
  const uint64_t *offs;          // m+1 symbol offsets
  const Chunk *chunks;
  uint32_t nchunks;              // chunks of this launch
  uint32_t chunk_base;           // non-persistent launches: first chunk index
  uint32_t *qctr;                // persistent launches: work-queue counter
  uint32_t persistent;           // 0: one chunk per workgroup, 1: work queue (qctr), 2: strided by the grid
  uint32_t n;                    // gram length
  uint32_t sigma;                // compacted alphabet size
  const uint8_t *code;           // symbol -> code (256 entries)
  // compact filter over the previous table's keys (copied into LDS)
  const uint32_t *filt;
  uint32_t filt_words;           // power of two
  uint32_t filt_kind;
  // exact map previous key -> rank (fingerprinted slots; keys confirmed against the table)
  const uint32_t *map;
  uint64_t mmask;
  uint32_t rank_bits;            // low bits of a slot holding rank+1
  const uint64_t *tkeys_lo, *tkeys_hi;   // previous table's keys (stream forms), in rank order
  const uint64_t *qmap;          // quotient map of the previous table (null: none)
  const uint64_t *qmap2;         // its 16-byte-slot quotient map (null: none; survivor-ring drains only)
  const uint32_t *qflag;         // non-zero: a key of that table did not fit its displacement field (lookups
                                 // then use the fingerprinted map and the table's keys)
  QMapShape qs, qs2;
  // large unfiltered passes: key table
  uint64_t *tkey_lo, *tkey_hi;
  uint32_t *tstate;
  uint64_t tmask;
  // counts (Eq. 1), or chunk-distinct records for once-per-sequence counting (Eq. 2)
  void *cnt;
  uint32_t *rec;                 // Eq. 2: one u32 slot per symbol; a chunk writes its records at [s0, s0 + nrec)
  uint32_t *nrec;                // Eq. 2: records per chunk (file-order index)
  uint32_t *hist1;               // Eq. 2: [chunk][bucket] counts of the records' top bits
  uint32_t nct;                  // chunks in file order (histogram row length)
  uint32_t low1;                 // level-1 bucket = cid >> low1
  uint32_t nb1;                  // level-1 buckets (<= 256)
  uint32_t b1bits;               // log2(nb1)
  uint32_t hist_words;           // Eq. 2: LDS words of the per-wavefront level-1 histograms
  uint32_t *status;
  uint32_t set_cap;              // LDS de-duplication set entries (power of two)
  uint32_t stage_bytes;          // LDS staging bytes
  uint32_t qbytes;               // LDS bytes of the per-wavefront survivor rings (keys + displacements)
  // featurize form: per-sequence rank bitmaps of fwords 32-bit words; lds_bitmap: a chunk
  // collects its bits in LDS first
  uint32_t *bitmaps;
  uint32_t fwords, lds_bitmap;
};

// Once-per-sequence counting from chunk records (see ig_dedup.hip).
struct DedupShape {
  uint32_t nb1, nb2;             // level-1 and level-2 bucket counts (powers of two)
  uint32_t low1, low2;           // candidate bits below the level-1 / final bucket
  uint32_t w1, w2;               // record bytes at level 1 / level 2 (4 or 8)
};
struct DedupParams {
  const Chunk *chunks;           // file order
  uint32_t nct;
  uint32_t nb1, nb2, low1, low2, w1, w2;
  uint32_t b1bits, b2bits;       // log2(nb1), log2(nb2)
  const uint32_t *rec0;          // the scan's slab
  const uint32_t *nrec;
  const uint32_t *hist1;         // [nct][nb1]
  uint64_t *g1;                  // [nct][nb1]: records before (bucket, chunk) in bucket-major order
  uint64_t *scan_tmp;            // column partials [nb1][ncol] + total; later the hist2 scan's partials
  uint32_t ncol;                 // chunk groups of the column scan
  uint64_t *base1;               // nb1 + 1 tile-aligned bucket starts
  uint64_t *bend;                // nb1 bucket ends
  uint64_t *bshift;              // nb1: base1[b] - (records before bucket b), modulo 2^64
  uint64_t *dscal;               // [0] records, [1] tiles, [2] padded records
  void *l1;
  void *l2;
  uint64_t cap;                  // capacity of l1 and l2 (records, multiple of the tile)
  uint64_t ntmax;                // tile slots (cap / tile)
  uint32_t *hist2;               // ntmax * nb2
  uint64_t *g2;                  // scan of hist2 (ntmax*nb2 + 1)
  uint64_t *fin;                 // nb1*nb2 + 1 final bucket starts in l2
  uint32_t *nseg;                // nb1*nb2 counting segments per final bucket
  uint64_t *seg0;                // nb1*nb2 + 1: scan of nseg
  void *cnt;                     // u32 counts, nc entries
  uint64_t nc;
  uint32_t narrow;               // fewer than 65535 sequences: 16-bit per-candidate state in k_count
  uint32_t *status;
};
DedupShape dedup_shape(uint64_t nc, uint64_t m);
uint64_t dedup_tile();
uint64_t dedup_scan_tmp_entries(uint64_t n);
uint32_t dedup_ncol(uint32_t nct);
size_t count_lds_bytes(uint32_t low2);
hipError_t dedup_enqueue(const DedupParams &d, int n_cu, hipStream_t s);
hipError_t prepare_dedup(uint32_t low2);

// Parameters of the selection of the k_keep best candidates.
struct SelectParams {
  const void *cnt;
  uint64_t nc;                   // candidate ids [0, nc)
  int count64;                   // count array is u64
  int mode;
  uint32_t bits;                 // symbol bits
  uint32_t sigma;
  const uint8_t *sym_of_code;
  const uint64_t *pk_lo, *pk_hi; // previous table keys (filtered mode)
  const uint64_t *tk_lo, *tk_hi; // key table (sparse mode)
};

// ------------------------------------------------------------------ device buffers
struct DevBuf {
  void *p = nullptr;
  size_t bytes = 0;
};

// One retained table and its index (exact map key -> rank+1, compact filter image).
struct TableSet {
  DevBuf lo, hi, cnt;
  DevBuf le_lo, le_hi;            // the keys' stream forms, in rank order (probes confirm against them)
  DevBuf map, filt;               // map: 32-bit fingerprinted slots (rank+1 in the low rank_bits)
  DevBuf qmap, qflag;             // quotient map (keys of at most 64 bits) and its overflow flag
  DevBuf qmap2;                   // the 16-byte-slot quotient map, where 8-byte slots do not fit
  uint64_t kept = 0, map_mask = 0;
  uint32_t rank_bits = 32;
  uint32_t n = 0, filt_words = 0, filt_kind = 0;
  bool has_qmap = false, has_qmap2 = false;
  QMapShape qs{}, qs2{};
  // the pass that made the table: its windows and (Eq. 2) chunk-distinct records
  uint64_t made_windows = 0, made_records = 0;
};

struct LaunchCfg {
  uint32_t chunk_syms = 23552;       // 23 x 1024: per-thread runs of 23 windows (batches of 8, 8, 7)
  uint32_t block = 1024;
  uint32_t grid_per_cu = 1;
  uint32_t set_cap = 8192;
  uint32_t filt_max_words = 16384;   // 64 KB of LDS
  uint32_t map_log2 = 2;             // map slots >= kept << map_log2 (load <= 1/4)
  uint32_t bloom_bits = 12;          // Bloom filter image: bits per retained key (within filt_max_words)
};

}  // namespace ig

// ------------------------------------------------------------------ context
struct ig_ctx {
  ig_config cfg{};
  hipStream_t stream = nullptr;
  bool own_stream = false;
  int n_cu = 256;
  std::string err;
  int sticky = 0;
  uint64_t held_bytes = 0;

  // corpus
  ig::DevBuf data, offs, chunks_lpt, chunks_file, code, sym_of_code, qctr, status, kdev, zero;
  std::vector<uint64_t> h_offs;
  std::vector<uint32_t> file_chunk0;   // first chunk (file order) of each file, m+1 entries
  uint64_t m = 0, total_syms = 0, data_bytes = 0, nchunks = 0;
  uint32_t sigma = 0;
  uint8_t h_code[256]{}, h_sym_of_code[256]{};
  bool loaded = false;
  ig::LaunchCfg lc;

  // pass state: three rotating table sets (current, previous, next)
  ig::TableSet ts[3];
  int cur = 0, prev = 1, nxt = 2;
  bool fresh = true;            // no retained table since the last load
  bool prev_fresh = true;       // state before the last pass (for ig_rewind)
  bool can_rewind = false;
  uint32_t n_prev = 0;
  uint64_t kept = 0;
  ig::TableSet &T() { return ts[cur]; }

  // pass scratch
  ig::DevBuf cnt, tkey_lo, tkey_hi, tstate;
  uint64_t tkey_slots = 0;
  // once-per-sequence counting: slab, per-chunk counts and histograms, bucketed records
  ig::DevBuf rec0, nrec, hist1, g1, scan_tmp, base1, bend, bshift, dscal, l1, l2, hist2, g2, fin, nsegs, seg0;
  uint64_t rec_cap = 0;         // records the bucketed arrays hold (multiple of the tile)
  bool rec_floor = false;       // a caller set rec_cap: raise it only to the per-pass floor, not to the size guess
  ig::DevBuf sel_cid, sel_cnt, sel_klo, sel_khi, tie_a, tie_b, sort_tmp, hist, selstate, thist;
  ig::DevBuf pmask;   // kept (n-1)-grams as bits, for a direct-indexed pass with part of the prefixes kept

  ig_pass_stats last{};
  hipEvent_t ev[5]{};

  // captured passes: one executable graph per (pass shape, buffers)
  struct GraphEntry {
    std::string key;          // bytes of every argument baked into the captured stages
    hipGraphExec_t exec[4];   // clear, scan, once-per-sequence counting, select + index
  };
  std::vector<GraphEntry> graphs;
  uint64_t alloc_gen = 0;     // bumped whenever a device buffer is (re)allocated

  // featurize / serving
  void *server = nullptr;
};

namespace ig {
// chunk list for the current launch shape (ig_api.hip)
int rebuild_chunks(ig_ctx *c);
// serving loop teardown (ig_serve.hip)
void serve_teardown(ig_ctx *c);
// allocation helpers (ig_api.hip)
int dev_reserve(ig_ctx *c, DevBuf &b, size_t bytes);
void dev_release(ig_ctx *c, DevBuf &b);
int set_error(ig_ctx *c, int code, const char *fmt, ...);
int check_hip(ig_ctx *c, hipError_t e, const char *what);

// kernels' host launchers
hipError_t launch_fill_u32(uint32_t *p, uint64_t n, uint32_t v, hipStream_t s);
hipError_t launch_fill_u64(uint64_t *p, uint64_t n, uint64_t v, hipStream_t s);
hipError_t launch_scan(const ScanParams &p, int bits, int kw, int mode, int occ, int count64,
                       uint32_t grid, uint32_t block, hipStream_t s);
// set the kernel's LDS limit outside of any stream capture
hipError_t prepare_scan(int bits, int kw, int mode, int occ, int count64);
size_t scan_lds_bytes(const ScanParams &p, int mode, int occ, int feat = 0);
hipError_t launch_scan_feat(const ScanParams &p, int bits, int kw, uint32_t grid, uint32_t block, hipStream_t s);
// selection: reserve scratch, enqueue kernels (no host sync), read the kept length afterwards
int select_reserve(ig_ctx *c, uint64_t nc, uint64_t k_keep);
hipError_t select_enqueue(ig_ctx *c, const SelectParams &sp, uint64_t k_keep, uint32_t key_bits, uint32_t count_bits);
const unsigned long long *select_kept_ptr(ig_ctx *c);
// zero the counts of grams whose (n-1)-prefix the previous table did not keep (ig_select.hip)
hipError_t prefix_mask_enqueue(ig_ctx *c, const uint64_t *prev_keys, uint64_t prev_kept, uint32_t prefix_bits, void *cnt,
                               int c64, uint64_t nc, uint32_t b, uint32_t *bits, hipStream_t s);
int select_read(ig_ctx *c, uint64_t *kept, uint64_t *distinct);
// map + filter over a table set (sizes bounded by k_max; the length is read on the device)
int index_reserve(ig_ctx *c, TableSet &t, uint32_t n, uint64_t k_max);
hipError_t index_enqueue(ig_ctx *c, TableSet &t, uint64_t k_max, const unsigned long long *kept_dev);
// rebuild the current table's map and filter with the context's table shape (ig_table.hip)
int reindex_current(ig_ctx *c);
// featurize a device-resident batch into per-file rank bitmaps and CSR
struct FeatBatch {
  const uint8_t *data;       // device
  const uint64_t *offs;      // device, m+1
  uint64_t m;
  const Chunk *chunks;       // device
  uint32_t nchunks;
  uint32_t *bitmaps;         // device, m * words
  uint32_t words;
};
hipError_t launch_featurize(ig_ctx *c, const FeatBatch &fb, hipStream_t s);
// A device region that buffers are carved from instead of allocated (256-byte aligned pieces).
struct Carve {
  uint8_t *base = nullptr;
  size_t size = 0, used = 0;
  void *take(size_t bytes) {
    const size_t at = (used + 255) & ~(size_t)255;
    if (bytes > size || at > size - bytes) return nullptr;
    used = at + bytes;
    return base + at;
  }
};
// the no-allocation scratch's device address for c's device, taken once per device (ig_noalloc.hip)
int noalloc_setup(ig_ctx *c);
// ig_featurize of a host batch; device buffers come from `arena` when it is not null (ig_api.hip)
int featurize_host(ig_ctx *c, const void *data, uint64_t data_bytes, const uint64_t *sym_offsets, uint64_t m,
                   uint64_t *indptr, int32_t *indices, uint64_t cap, uint64_t *nnz_out, Carve *arena);
hipError_t launch_rows(const uint32_t *bitmaps, uint64_t m, uint32_t words, uint64_t *nnz_per_row,
                       const uint64_t *indptr, int32_t *indices, uint64_t cap, int count_only, hipStream_t s);
hipError_t launch_col_counts(const uint32_t *bitmaps, uint64_t m, uint32_t words, uint32_t kept,
                             uint32_t *col_counts, hipStream_t s);
}  // namespace ig
