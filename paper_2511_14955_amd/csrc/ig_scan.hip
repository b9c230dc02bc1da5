// Scan kernel: one pass over the corpus (Algorithm 3's inner loops).
//
// For every window t of every sequence (windows never cross a sequence end):
//   key      = the n symbols at t, first symbol most significant     (ingest)
//   survive  = n = 1, no previous table, or (key >> b) in the table  (prefix filter)
//   count    = once per sequence (Eq. 2) or once per occurrence (Eq. 1)
//
// Work items are chunks of one file; a workgroup stages a chunk (plus the
// n-1-symbol halo read from the same file) into LDS with 16-byte coalesced
// loads, then each thread rolls a key across a contiguous run of windows.
// The prefix test first consults a compact filter image held in LDS (a direct
// bitmap when the prefix space is small, otherwise a blocked Bloom filter with
// no false negatives); only filter hits probe the exact key -> rank map.  For keys
// of at most 64 bits the hits are first compacted into a per-wavefront LDS ring and
// resolved 64 at a time, one lane each (one 8-byte quotient-map read when the table
// has one); the others are resolved in place.
// Survivors become dense candidate ids, de-duplicated per chunk in an LDS hash
// set.  For Eq. 1 the set also holds per-candidate counts that are added to the
// count array at the end of the chunk.  For Eq. 2 the chunk writes its distinct
// candidates ("records") into its own slot range of a slab, with a histogram of
// their top bits; the records are counted once per sequence afterwards without
// device-scope atomics (ig_dedup.hip).  A candidate that finds the LDS set full
// is recorded directly (a duplicate record within one sequence is harmless).
#include <type_traits>

#include "ig_internal.h"

namespace ig {

template <int KW> struct KeyT;
template <> struct KeyT<1> {
  uint64_t lo;
  __device__ __forceinline__ void clear() { lo = 0; }
  template <int B> __device__ __forceinline__ void push(uint32_t s, uint64_t mlo, uint64_t) { lo = ((lo << B) | s) & mlo; }
  // stream form: the new symbol enters at the top (bit `top` = (n-1) b), the first leaves at the bottom
  template <int B> __device__ __forceinline__ void push_le(uint32_t s, uint32_t top) { lo = (lo >> B) | ((uint64_t)s << top); }
  template <int B> __device__ __forceinline__ uint64_t pre_lo() const { return lo >> B; }
  template <int B> __device__ __forceinline__ uint64_t pre_hi() const { return 0; }
  static constexpr uint64_t hi = 0;
};
template <> struct KeyT<2> {
  uint64_t lo, hi;
  __device__ __forceinline__ void clear() { lo = 0; hi = 0; }
  template <int B> __device__ __forceinline__ void push(uint32_t s, uint64_t, uint64_t mhi) {
    hi = ((hi << B) | (lo >> (64 - B))) & mhi;
    lo = (lo << B) | s;
  }
  template <int B> __device__ __forceinline__ void push_le(uint32_t s, uint32_t top) {
    lo = (lo >> B) | (hi << (64 - B));
    hi >>= B;
    if (top >= 64) hi |= (uint64_t)s << (top - 64);
    else lo |= (uint64_t)s << top;
  }
  template <int B> __device__ __forceinline__ uint64_t pre_lo() const { return (lo >> B) | (hi << (64 - B)); }
  template <int B> __device__ __forceinline__ uint64_t pre_hi() const { return hi >> B; }
};

template <typename CT> __device__ __forceinline__ void cnt_add(void *cnt, uint32_t cid, CT v) {
  __hip_atomic_fetch_add(reinterpret_cast<CT *>(cnt) + cid, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Insert-or-find in the key table of large unfiltered passes; returns the slot,
// or 0xFFFFFFFF after flagging an overflow.  A slot is claimed (state 0 -> 1),
// its key words written, then published (state 2); readers wait on state 1.
__device__ __forceinline__ uint32_t table_insert(const ScanParams &p, uint64_t lo, uint64_t hi) {
  uint64_t slot = hash_key(lo, hi) & p.tmask;
  uint32_t probes = 0;
  for (uint32_t iter = 0; iter < (1u << 22); iter++) {
    uint32_t st = __hip_atomic_load(p.tstate + slot, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
    if (st == 0) {
      uint32_t expect = 0;
      if (__hip_atomic_compare_exchange_strong(p.tstate + slot, &expect, 1u, __ATOMIC_ACQ_REL, __ATOMIC_ACQUIRE,
                                               __HIP_MEMORY_SCOPE_AGENT)) {
        __hip_atomic_store(p.tkey_lo + slot, lo, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __hip_atomic_store(p.tkey_hi + slot, hi, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __hip_atomic_store(p.tstate + slot, 2u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
        return (uint32_t)slot;
      }
      continue;
    }
    if (st == 1) continue;  // being published by another thread
    const uint64_t klo = __hip_atomic_load(p.tkey_lo + slot, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    const uint64_t khi = __hip_atomic_load(p.tkey_hi + slot, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (klo == lo && khi == hi) return (uint32_t)slot;
    slot = (slot + 1) & p.tmask;
    if (++probes > 4096) break;
  }
  atomicOr(p.status, ST_TABLE_OVF);
  return 0xFFFFFFFFu;
}

// LDS open-addressing set of candidate ids: 1 = newly inserted, 0 = present, -1 = full (no
// free slot within 32 probes).
// The home slot is the top bits of a 24 x 24-bit product (a full-rate multiply): the candidate
// ids of a chunk are dense ranks times sigma plus a code, and the product spreads them over the
// top bits; ids of 24 bits and more fold their high bits in first.  HIP's __umul24 returns a
// signed int: the product is shifted as unsigned, or a set top bit would make the slot negative.
__device__ __forceinline__ int lds_insert(uint32_t *s_set, uint32_t capmask, uint32_t capshift, uint32_t cid,
                                          uint32_t *slot_out) {
  uint32_t h = static_cast<uint32_t>(__umul24(cid ^ (cid >> 20), 0x9E3779u)) >> capshift;
  for (int i = 0; i < 32; i++) {
    const uint32_t cur = atomicCAS(s_set + h, LDS_EMPTY, cid);
    if (cur == LDS_EMPTY) { *slot_out = h; return 1; }
    if (cur == cid) { *slot_out = h; return 0; }
    h = (h + 1) & capmask;
  }
  return -1;
}

template <int B>
__device__ __forceinline__ uint32_t stage_sym(const uint8_t *s_stage, uint64_t g, uint64_t a0) {
  if (B == 8) return s_stage[g - a0];
  const uint32_t byte = s_stage[(g >> 2) - a0];
  return (byte >> (6 - 2 * (uint32_t)(g & 3))) & 3u;
}

// CMP: filter survivors are compacted into per-wavefront rings (filtered 64-bit keys only).
// FEAT: featurize instead of count (Figure 1's Boolean rows): the whole window is looked up in
// the current table (n-grams), and a hit sets bit rank(window) of its sequence's bitmap (in LDS
// for the chunk when it fits, else straight in HBM).  Filtered mode, Eq. 2 layout, no counts.
template <int B, int KW, int MODE, int OCC, typename CT, int CMP, int FEAT>
__global__ void __launch_bounds__(1024) k_scan(ScanParams p) {
  extern __shared__ __align__(16) uint8_t lds[];
  __shared__ uint32_t s_nrec;          // Eq. 2: records written by this chunk
  __shared__ uint32_t s_full;          // the chunk's LDS set refused an insert: bypass it
  uint8_t *s_stage = lds;
  uint32_t *s_filt = reinterpret_cast<uint32_t *>(lds + p.stage_bytes);
  // the filter image is padded to 16 bytes, so that the 8-byte ring entries below stay aligned
  const uint32_t filt_lds = MODE == MODE_FILTERED ? filt_lds_words(p.filt_kind, p.filt_words) : 0u;
  uint32_t *s_set = s_filt + ((filt_lds + 3u) & ~3u);
  uint32_t *s_bm = s_set;                              // FEAT: the chunk's rank bitmap, in place of the set
  const uint32_t bm_lds = FEAT && p.lds_bitmap ? (p.fwords + 3u) & ~3u : 0u;
  uint32_t *s_cnt = s_set + (FEAT ? bm_lds : p.set_cap);   // OCC only
  uint8_t *s_code = reinterpret_cast<uint8_t *>(s_cnt + (OCC ? p.set_cap : 0));
  // Eq. 2: histogram of this chunk's records over the level-1 buckets, one copy per
  // wavefront (a few hot buckets take most records; a shared copy would serialize them)
  // filtered 64-bit keys: one ring of SCAN_QCAP filter survivors per wavefront
  uint64_t *s_q = reinterpret_cast<uint64_t *>(s_code + 256);
  // and, after the keys, 16 bits per ring entry: the next displacement to probe (the quotient
  // map's displacement field has at most 16 bits)
  uint16_t *s_qd = reinterpret_cast<uint16_t *>(s_q + (size_t)(blockDim.x >> 6) * SCAN_QCAP * KW);
  uint32_t *s_h1w = reinterpret_cast<uint32_t *>(s_code + 256 + p.qbytes);
  __shared__ uint32_t s_chunk, s_next;

  const uint32_t tid = threadIdx.x, bs = blockDim.x;
  const uint32_t n = p.n;
  // Eq. 2 with survivor rings: each drain records its candidates new to the chunk as it inserts them
  constexpr bool EAI = CMP != 0 && !OCC && !FEAT;
  const uint32_t nb = n * B;
  const uint64_t mlo = (KW == 1) ? (nb >= 64 ? ~0ull : ((1ull << nb) - 1)) : ~0ull;
  const uint64_t mhi = (KW == 2) ? (nb >= 128 ? ~0ull : ((1ull << (nb - 64)) - 1)) : 0ull;
  // the LDS set's buckets (set_cap / 4, a power of two)
  const uint32_t capmask = p.set_cap - 1;
  const uint32_t capshift = 32u - (uint32_t)__builtin_ctz(p.set_cap);
  const uint32_t fmask = p.filt_words - 1;

  if (MODE == MODE_FILTERED)
    for (uint32_t i = tid; i < filt_lds; i += bs) s_filt[i] = p.filt[i];
  if (FEAT) {
    for (uint32_t i = tid; i < bm_lds; i += bs) s_bm[i] = 0;
  } else {
    for (uint32_t i = tid; i < p.set_cap; i += bs) {
      s_set[i] = LDS_EMPTY;
      if (OCC) s_cnt[i] = 0;
    }
  }
  for (uint32_t i = tid; i < 256; i += bs) s_code[i] = p.code[i];
  for (uint32_t i = tid; i < p.hist_words; i += bs) s_h1w[i] = 0;
  if (tid == 0) {
    s_nrec = 0;
    s_full = 0;
  }
  __syncthreads();
  const uint32_t lane = tid & 63, nwaves = bs >> 6;
  const uint64_t lanes_below = (1ull << lane) - 1;
  uint32_t *my_h1 = s_h1w + (tid >> 6) * p.nb1;
  // Eq. 2: append one record of this chunk (slot c.s0 + k, k < windows of the chunk);
  // used by threads whose insert found the LDS set full
  auto emit = [&](uint64_t s0, uint32_t cid) {
    const uint32_t k = atomicAdd(&s_nrec, 1u);
    p.rec[s0 + k] = cid;
    atomicAdd(my_h1 + (p.low1 >= 32 ? 0u : (cid >> p.low1)), 1u);
  };

  constexpr uint32_t END = 0xFFFFFFFFu;
  auto valid_chunk = [&](uint32_t ci) {
    return ci != END && (p.persistent ? ci < p.nchunks : ci < p.chunk_base + p.nchunks);
  };
  // a chunk's windows [wbeg, wend) and the 16-byte words [a0, a0 + 16 nw) of the corpus it stages
  struct Span {
    Chunk c;
    uint64_t wbeg, wend, a0;
    uint32_t nw;
  };
  auto span_of = [&](uint32_t ci) {
    Span sp;
    sp.c = p.chunks[ci];
    const uint64_t fend = p.offs[sp.c.file + 1];
    const uint64_t flen = fend - p.offs[sp.c.file];
    sp.wbeg = sp.c.s0;
    sp.wend = sp.c.s0 + sp.c.nsym;
    if (flen < n) sp.wend = sp.wbeg;
    else if (sp.wend > fend - n + 1) sp.wend = fend - n + 1;
    sp.a0 = 0;
    sp.nw = 0;
    if (sp.wbeg < sp.wend) {
      const uint64_t byte_lo = (B == 8) ? sp.wbeg : (sp.wbeg >> 2);
      const uint64_t byte_hi = (B == 8) ? (sp.wend + n - 1) : ((sp.wend + n - 2) >> 2) + 1;
      sp.a0 = byte_lo & ~15ull;
      sp.nw = (uint32_t)((((byte_hi + 15) & ~15ull) - sp.a0) / 16);
    }
    return sp;
  };
  // The corpus streams through once per pass: non-temporal loads keep it from evicting the
  // key -> rank map from L2.
  typedef uint32_t u32x4_t __attribute__((ext_vector_type(4)));
  auto word_at = [&](const Span &sp, uint32_t i) {
    return __builtin_nontemporal_load(reinterpret_cast<const u32x4_t *>(p.data + sp.a0) + i);
  };
  // Persistent launches of the compacted kernel run their chunks as a pipeline: the next chunk
  // is known one chunk ahead (thread 0 claims the one after it while the current chunk runs),
  // the first PF 16-byte words per thread of its stage load into registers while the current
  // chunk's windows run, and go to the stage once those are done.
  constexpr uint32_t PF = CMP != 0 ? 4u : 0u;
  u32x4_t pf[PF ? PF : 1];
  if (tid == 0) {
    uint32_t c0 = END, c1 = END;
    if (p.persistent == 2) {   // strided: chunks blockIdx.x, + gridDim.x, ...
      c0 = blockIdx.x;
      if (PF) c1 = blockIdx.x + gridDim.x;
    } else if (p.persistent) {
      c0 = atomicAdd(p.qctr, 1u);
      if (PF) c1 = atomicAdd(p.qctr, 1u);
    } else {
      c0 = p.chunk_base + blockIdx.x;
    }
    // a table overflowed: this launch will be replayed with larger tables, stop early
    if (__hip_atomic_load(p.status, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) c0 = c1 = END;
    s_chunk = c0;
    s_next = c1;
  }
  __syncthreads();
  Span nx{};             // the next chunk's span (when have_nx)
  bool have_nx = false;
  uint32_t staged = 0;   // words of the current chunk already in the stage
  for (;;) {
    const uint32_t ci = __builtin_amdgcn_readfirstlane(s_chunk);
    const uint32_t cn = __builtin_amdgcn_readfirstlane(s_next);
    if (!valid_chunk(ci)) break;
    uint32_t claim = END;   // thread 0: the chunk after cn
    if (PF && tid == 0 && valid_chunk(cn)) claim = p.persistent == 2 ? cn + gridDim.x : atomicAdd(p.qctr, 1u);
    const Span cur = have_nx ? nx : span_of(ci);
    const Chunk c = cur.c;
    const uint64_t wbeg = cur.wbeg, wend = cur.wend;
    // the rest of this chunk's stage (all of it unless loaded ahead), then the next chunk's
    // first words into registers
    for (uint32_t i = staged + tid; i < cur.nw; i += bs) reinterpret_cast<u32x4_t *>(s_stage)[i] = word_at(cur, i);
    have_nx = false;
    if (PF && valid_chunk(cn)) {
      nx = span_of(cn);
      have_nx = true;
#pragma unroll
      for (uint32_t q = 0; q < PF; q++)
        if (q * bs + tid < nx.nw) pf[q] = word_at(nx, q * bs + tid);
    }
    __syncthreads();
    if (wbeg < wend) {
      const uint64_t nwin = wend - wbeg;
      const uint64_t a0 = cur.a0;

      // each thread rolls its key over a contiguous run of windows; an odd run length puts
      // neighbouring lanes' staged symbols in different LDS banks
      const uint32_t per = (uint32_t)((nwin + bs - 1) / bs) | 1u;
      const uint64_t t_lo = (uint64_t)tid * per;
      const uint64_t t_hi = t_lo + per < nwin ? t_lo + per : nwin;
      const uint64_t sbase = a0;
      uint32_t *gbm = FEAT ? p.bitmaps + (uint64_t)c.file * p.fwords : nullptr;
      // one surviving candidate: de-duplicate in the chunk's LDS set (FEAT: cid is the rank, whose
      // bit is set in the sequence's bitmap)
      // (returns the set insert's result: 1 when cid is new to the chunk)
      auto handle = [&](uint32_t cid) -> int {
        if constexpr (FEAT) {
          if (p.lds_bitmap) atomicOr(s_bm + (cid >> 5), 1u << (cid & 31));
          else atomicOr(gbm + (cid >> 5), 1u << (cid & 31));
          return 0;
        }
        // A chunk with more distinct candidates than the set holds would probe a full set for
        // every later window: once an insert has failed, the rest of the chunk goes straight to
        // the counters (Eq. 1) or to records (Eq. 2; a record may repeat one of the set's, which
        // the once-per-sequence count allows).
        uint32_t slot;
        int ins = -1;
        if (!__hip_atomic_load(&s_full, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP)) {
          ins = lds_insert(s_set, capmask, capshift, cid, &slot);
          if (ins < 0) __hip_atomic_store(&s_full, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
        }
        if (OCC) {
          if (ins >= 0) atomicAdd(s_cnt + slot, 1u);
          else cnt_add<CT>(p.cnt, cid, (CT)1);
        } else if (ins < 0) {
          emit(wbeg, cid);
        }
        return ins;
      };
      if constexpr (CMP != 0) {
        // About a third of the windows pass the filter, so nearly every wavefront has a
        // survivor at each step: resolving survivors in place would run the probe on all 64
        // lanes for a few live ones.  Survivors' keys are compacted into the wavefront's
        // LDS ring instead (ballot + prefix count) and resolved 64 at a time, one per lane.
        //
        // Keys are stream forms (first symbol lowest): the stage is read one 32-bit word at a
        // time, and the 64 bits that start at a window are a funnel shift of two neighbouring
        // words (v_alignbit); the prefix is a mask of them, the last symbol a bit field.
        constexpr int RBC = 4;
        constexpr uint32_t SPD = 32 / B;   // symbols per stage word
        // ring entries: the window's first 64 bits (KW 2: its first 128, as two words)
        uint64_t *q = s_q + (tid >> 6) * SCAN_QCAP * KW;
        uint16_t *qd = s_qd + (tid >> 6) * SCAN_QCAP;
        const uint32_t rmask = p.rank_bits >= 32 ? 0xFFFFFFFFu : ((1u << p.rank_bits) - 1);
        const uint64_t rmask64 = rmask;
        uint32_t head = 0, tail = 0;   // ring positions, the same in every lane of the wavefront
        const uint32_t pb = (FEAT ? n : n - 1) * B;   // bits looked up: the prefix (FEAT: the whole window)
        const uint32_t pm_lo = pb >= 32 ? 0xFFFFFFFFu : ((1u << pb) - 1);
        const uint32_t pm_hi = pb <= 32 ? 0u : (pb >= 64 ? 0xFFFFFFFFu : ((1u << (pb - 32)) - 1));
        const uint64_t pmask = ((uint64_t)pm_hi << 32) | pm_lo;
        // KW 2: the prefix's bits in the window's second 64 (pb >= 64 there)
        const uint64_t pmask2 = KW == 2 ? (pb >= 128 ? ~0ull : ((1ull << (pb - 64)) - 1)) : 0ull;
        // Exact rank of each queued key's prefix.  With the quotient map one 8-byte slot read
        // decides (home and stored bits give back the key); otherwise the fingerprinted map and
        // the table's keys are probed.  An empty slot ends either probe.
        const bool useq = p.qmap != nullptr && *p.qflag == 0u;
        // the 16-byte-slot quotient map (tables whose 8-byte slots do not fit: the host builds it
        // for prefixes of more than 64 bits, or of 64 with many keys, whose windows take this
        // kernel's 128-bit form): the same probe, with 32-byte reads of two slots
        const bool useq2 = KW == 2 && !useq && p.qmap2 != nullptr && *p.qflag == 0u;
        const uint64_t dmax2 = (1ull << p.qs2.dbits) - 1;
        const uint32_t sh2 = p.qs2.rbits + p.qs2.dbits;
        const uint64_t rmask2 = p.qs2.rbits >= 64 ? ~0ull : ((1ull << p.qs2.rbits) - 1);
        const uint64_t dmax = (1ull << p.qs.dbits) - 1;
        const uint32_t rsh = p.qs.rbits + p.qs.dbits;
        const uint64_t qmaskq = p.qs.qbits ? ((1ull << p.qs.qbits) - 1) : 0ull;
        // Each dequeued key takes exactly one probe step (two neighbouring slots).  Slots that hold
        // other keys send the key back into the ring with the next displacement (a later drain
        // takes it), so a few displaced keys never hold up the other lanes of the wavefront.
        auto drain = [&](uint32_t cnt) {
          __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
          bool again = false;
          uint64_t key = 0, key2 = 0;   // (key2: KW 2's second word)
          uint32_t dnext = 0;
          uint32_t newcid = LDS_EMPTY;   // Eq. 2: a candidate new to the chunk, recorded below
          if (lane < cnt) {
            key = q[((head + lane) & (SCAN_QCAP - 1)) * KW];
            if (KW == 2) key2 = q[((head + lane) & (SCAN_QCAP - 1)) * KW + 1];
            const uint32_t d = qd[(head + lane) & (SCAN_QCAP - 1)];
            const uint64_t plo = key & pmask;
            const uint64_t phi = key2 & pmask2;
            // the window's last symbol sits right above its prefix (counting passes: pb < 64 for
            // KW 1, 64 <= pb < 128 for KW 2)
            const uint32_t code =
                FEAT ? 0u : s_code[(KW == 2 ? (uint32_t)(key2 >> (pb - 64)) : (uint32_t)(key >> pb)) & ((1u << B) - 1)];
            uint32_t cid = LDS_EMPTY;   // not found
            if (useq) {
              // one 16-byte read covers displacements d and d+1 (the slot past the last mirrors
              // slot 0); a key further out comes back with d+2.  A slot holds the key whose
              // stored bits and displacement are exactly the wanted ones (rank+1 >= 1 below them).
              const uint64_t x = qmix(plo, p.qs.w);
              const uint64_t slot = ((x >> p.qs.qbits) + d) & p.mmask;
              typedef unsigned long long u64x2_t __attribute__((ext_vector_type(2), aligned(8)));
              const u64x2_t e2 = *reinterpret_cast<const u64x2_t *>(p.qmap + slot);
              const uint64_t e0 = e2.x, e1 = e2.y;
              const uint64_t want0 = ((x & qmaskq) << rsh) | ((uint64_t)d << p.qs.rbits);
              const uint64_t want1 = want0 + (1ull << p.qs.rbits);
              const bool m0 = (e0 & rmask64) != 0 && (e0 & ~rmask64) == want0;
              const bool m1 = (e1 & rmask64) != 0 && (e1 & ~rmask64) == want1 && d + 1 <= dmax;
              if (m0 || m1) cid = (((uint32_t)(m0 ? e0 : e1) & rmask) - 1) * p.sigma + code;
              again = !(m0 || m1) && (e0 & rmask64) != 0 && (e1 & rmask64) != 0 && d + 2 <= dmax;
              dnext = d + 2;
            } else if (KW == 2 && useq2) {
              // slots d and d+1 (the slot past the last mirrors slot 0) in one 32-byte read; a slot
              // holds the key whose remainder and displacement are exactly the wanted ones
              uint64_t home, rl, rh;
              qmix2(plo, phi, p.qs2.w, p.qs2.sbits, &home, &rl, &rh);
              const uint64_t slot = (home + d) & p.mmask;
              typedef unsigned long long u64x4_t __attribute__((ext_vector_type(4), aligned(16)));
              const u64x4_t e4 = *reinterpret_cast<const u64x4_t *>(p.qmap2 + 2 * slot);
              const uint64_t wlo = (rl << sh2) | ((uint64_t)d << p.qs2.rbits);
              const uint64_t whi = (rl >> (64 - sh2)) | (rh << sh2);
              const bool m0 = (e4.x & rmask2) != 0 && (e4.x & ~rmask2) == wlo && e4.y == whi;
              const bool m1 = (e4.z & rmask2) != 0 && (e4.z & ~rmask2) == wlo + (1ull << p.qs2.rbits) && e4.w == whi &&
                              d + 1 <= dmax2;
              if (m0 || m1) cid = (((uint32_t)(m0 ? e4.x : e4.z) & rmask) - 1) * p.sigma + code;
              again = !(m0 || m1) && (e4.x & rmask2) != 0 && (e4.z & rmask2) != 0 && d + 2 <= dmax2;
              dnext = d + 2;
            } else {
              // the fingerprinted map, confirmed against the table's key (KW 2: both words)
              const uint64_t h = hash_key(plo, phi);
              const uint32_t fp = map_fp(h, p.rank_bits);
              uint64_t slot = h & p.mmask;
              uint32_t v = p.map[slot];
              while (v != 0) {
                if (p.rank_bits >= 32 || (v >> p.rank_bits) == fp) {
                  const uint32_t r = (v & rmask) - 1;
                  if (p.tkeys_lo[r] == plo && (KW == 1 || p.tkeys_hi[r] == phi)) {
                    cid = r * p.sigma + code;
                    break;
                  }
                }
                slot = (slot + 1) & p.mmask;
                v = p.map[slot];
              }
            }
            if (cid != LDS_EMPTY && handle(cid) == 1) newcid = cid;
          }
          head += cnt;
          if constexpr (EAI) {
            // the drain's new candidates become records at once, at consecutive slots (one LDS
            // atomic per wavefront), so the chunk's end only clears the set
            const uint64_t nm = __ballot(newcid != LDS_EMPTY);
            if (nm) {
              const uint32_t leader = (uint32_t)__ffsll((unsigned long long)nm) - 1;
              uint32_t base = 0;
              if (lane == leader) base = atomicAdd(&s_nrec, (uint32_t)__popcll(nm));
              base = __shfl(base, leader);
              if (newcid != LDS_EMPTY) {
                __builtin_nontemporal_store(newcid, p.rec + wbeg + base + (uint32_t)__popcll(nm & lanes_below));
                atomicAdd(my_h1 + (p.low1 >= 32 ? 0u : (newcid >> p.low1)), 1u);
              }
            }
          }
          // requeue behind the live entries: at most 63 + cnt <= 127 entries are live afterwards
          const uint64_t m = __ballot(again);
          if (again) {   // (quotient map only: keys of at most 64 bits)
            const uint32_t at = (tail + (uint32_t)__popcll(m & lanes_below)) & (SCAN_QCAP - 1);
            q[at * KW] = key;
            if (KW == 2) q[at * KW + 1] = key2;
            qd[at] = (uint16_t)dnext;
          }
          tail += (uint32_t)__popcll(m);
          __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        };
        // Thread runs: stage symbol positions [p0, p0 + run) with run a multiple of SPD, so a run
        // starts on a stage word.  The chunk's windows sit at positions [ofirst, ofirst + nwin);
        // vbits marks the run's positions that are windows of this chunk (run <= 64, checked by
        // the host before it picks this kernel).  Runs past the chunk read clamped stage words and
        // keep no window.
        const uint32_t ofirst = (uint32_t)(wbeg - (B == 8 ? sbase : 4 * sbase));
        const uint32_t span = ofirst + (uint32_t)nwin;
        const uint32_t run = SPD * ((span + SPD * bs - 1) / (SPD * bs));
        const uint32_t p0 = tid * run;
        const uint32_t vlo = ofirst > p0 ? (ofirst - p0 < run ? ofirst - p0 : run) : 0u;
        const uint32_t vhi = span > p0 ? (span - p0 < run ? span - p0 : run) : 0u;
        const uint64_t vbits = vhi > vlo ? ((vhi >= 64 ? ~0ull : ((1ull << vhi) - 1)) & ~((1ull << vlo) - 1)) : 0ull;
        const uint32_t vb_lo = (uint32_t)vbits, vb_hi = (uint32_t)(vbits >> 32);
        const uint32_t *st32 = reinterpret_cast<const uint32_t *>(s_stage);
        // a stage word with its symbols in stream order (2-bit: each byte's four reversed)
        const uint32_t jcap = p.stage_bytes / 4 - 1;
        auto rd = [&](uint32_t j) -> uint32_t {
          uint32_t w = st32[j < jcap ? j : jcap];
          if (B == 2) {
            w = ((w >> 2) & 0x33333333u) | ((w & 0x33333333u) << 2);
            w = ((w >> 4) & 0x0F0F0F0Fu) | ((w & 0x0F0F0F0Fu) << 4);
          }
          return w;
        };
        // one copy of the loop per filter kind, so that no window branches on it
        auto windows = [&](auto kind) {
          constexpr int FK = decltype(kind)::value;
          uint32_t j = p0 / SPD;
          uint32_t D0 = rd(j), D1 = rd(j + 1);
          // KW 2 (byte windows of up to 16 symbols): five words hold a window at any of the four
          // byte offsets of the first; D2c and D3c carry the third and fourth across words
          uint32_t D2c = KW == 2 ? rd(j + 2) : 0u, D3c = KW == 2 ? rd(j + 3) : 0u;
          for (uint32_t it = 0; it < run; it += SPD, j++) {
            const uint32_t D2 = KW == 2 ? D2c : rd(j + 2);
            const uint32_t D3 = D3c;
            const uint32_t D4 = KW == 2 ? rd(j + 4) : 0u;
#pragma unroll 1
            for (uint32_t e0 = 0; e0 < SPD; e0 += RBC) {
              // the RBC windows at run positions it + e0 + u: keys, filter positions, then the
              // RBC filter reads issued together
              uint32_t widx[RBC], bm[RBC], w[RBC];
              uint32_t pass = 0;
#pragma unroll
              for (int u = 0; u < RBC; u++) {
                const uint32_t sh = B * (e0 + u);
                const uint32_t pl = __builtin_amdgcn_alignbit(D1, D0, sh) & pm_lo;
                const uint32_t ph = __builtin_amdgcn_alignbit(D2, D1, sh) & pm_hi;
                if constexpr (KW == 2) {
                  // the prefix's first 64 bits are (ph, pl) unmasked (pb >= 64); its rest is the
                  // next 64 masked to pb - 64 bits.  (A direct bitmap never serves such keys.)
                  const uint64_t phi = (((uint64_t)__builtin_amdgcn_alignbit(D4, D3, sh) << 32) |
                                        __builtin_amdgcn_alignbit(D3, D2, sh)) & pmask2;
                  if constexpr (FK == FILT_BLOOM || FK == FILT_GBLOOM)
                    bloom_pos(fold_le(((uint64_t)ph << 32) | pl, phi), p.filt_words, &widx[u], &bm[u]);
                  else if constexpr (FK == FILT_DIRECT) {
                    widx[u] = 0;
                    bm[u] = 0;
                  }
                } else if constexpr (FK == FILT_BLOOM || FK == FILT_GBLOOM) {
                  bloom_pos(pl ^ ((ph >> 13) | (ph << 19)), p.filt_words, &widx[u], &bm[u]);
                } else if constexpr (FK == FILT_DIRECT) {
                  widx[u] = (pl >> 5) & fmask;
                  bm[u] = 1u << (pl & 31);
                }
              }
              if constexpr (FK != FILT_NONE) {
#pragma unroll
                for (int u = 0; u < RBC; u++) w[u] = FK == FILT_GBLOOM ? p.filt[widx[u]] : s_filt[widx[u]];
#pragma unroll
                for (int u = 0; u < RBC; u++) pass |= (uint32_t)((w[u] & bm[u]) == bm[u]) << u;
              } else {
                pass = (1u << RBC) - 1;
              }
              // the windows of this batch that belong to the chunk
              const uint32_t rel = it + e0;
              pass &= (rel & 32u ? vb_hi : vb_lo) >> (rel & 31u);
              // a rolled loop keeps a single copy of the drain in the loop body; the survivor's
              // 64 key bits are shifted out of the stage words again
#pragma unroll 1
              for (uint32_t u = 0; u < (uint32_t)RBC; u++) {
                const bool sv = pass & 1u;
                const uint64_t m = __ballot(sv);
                if (sv) {
                  const uint32_t below =
                      __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
                  const uint32_t at = (tail + below) & (SCAN_QCAP - 1);
                  const uint32_t sh = B * (e0 + u);
                  q[at * KW] = ((uint64_t)__builtin_amdgcn_alignbit(D2, D1, sh) << 32) | __builtin_amdgcn_alignbit(D1, D0, sh);
                  if (KW == 2)
                    q[at * KW + 1] =
                        ((uint64_t)__builtin_amdgcn_alignbit(D4, D3, sh) << 32) | __builtin_amdgcn_alignbit(D3, D2, sh);
                  qd[at] = 0;
                }
                tail += (uint32_t)__popcll(m);
                while (tail - head >= 64) drain(64);
                pass >>= 1;
              }
            }
            D0 = D1;
            D1 = D2;
            D2c = D3;
            D3c = D4;
          }
        };
        if (p.filt_kind == FILT_BLOOM) windows(std::integral_constant<int, FILT_BLOOM>{});
        else if (p.filt_kind == FILT_GBLOOM) windows(std::integral_constant<int, FILT_GBLOOM>{});
        else if (p.filt_kind == FILT_DIRECT) windows(std::integral_constant<int, FILT_DIRECT>{});
        else windows(std::integral_constant<int, FILT_NONE>{});
        while (tail != head) drain(tail - head < 64 ? tail - head : 64u);
      } else if (t_lo < t_hi) {
        KeyT<KW> k;
        k.clear();
        const uint64_t g0 = wbeg + t_lo;   // absolute symbol of the first window
        // filtered passes look prefixes up by their stream form (first symbol lowest); the
        // unfiltered ones count canonical keys
        const uint32_t top = (n - 1) * B;
        for (uint32_t r = 0; r + 1 < n; r++) {
          const uint32_t sym = stage_sym<B>(s_stage, g0 + r, sbase);
          if (MODE == MODE_FILTERED) k.template push_le<B>(sym, top);
          else k.template push<B>(sym, mlo, mhi);
        }
        if (MODE == MODE_FILTERED) {
          const uint32_t lb = FEAT ? top + B : top;   // bits looked up (FEAT: the whole window)
          const uint64_t pmlo = lb >= 64 ? ~0ull : ((1ull << lb) - 1);
          const uint64_t pmhi = lb <= 64 ? 0ull : (lb >= 128 ? ~0ull : ((1ull << (lb - 64)) - 1));
          // Windows are taken RB at a time: every window's key is rolled and filtered and the
          // first map slot of each survivor is read; then the keys of fingerprint matches are
          // read from the table; then the probes are resolved.  Up to RB independent reads
          // per thread are in flight at each step.
          constexpr int RB = KW == 2 ? 4 : 8;   // 128-bit keys: half the batch, no register spills
          const uint32_t rmask = p.rank_bits >= 32 ? 0xFFFFFFFFu : ((1u << p.rank_bits) - 1);
          for (uint64_t t0 = t_lo; t0 < t_hi; t0 += RB) {
            // q_*[u] are only read where bit u of `live` (or `hit`) is set
            uint64_t q_lo[RB], q_hi[RB], q_klo[RB], q_khi[RB], q_slot[RB];
            uint32_t q_v[RB], q_fp[RB], q_code[RB];
            uint32_t live = 0, hit = 0;
#pragma unroll
            for (int u = 0; u < RB; u++) {
              if (t0 + u >= t_hi) continue;
              const uint64_t g = wbeg + t0 + u;
              const uint32_t sym = stage_sym<B>(s_stage, g + n - 1, sbase);
              k.template push_le<B>(sym, top);
              const uint64_t plo = k.lo & pmlo, phi = k.hi & pmhi;
              uint64_t h = 0;
              if (p.filt_kind == FILT_DIRECT) {
                if (!((s_filt[(uint32_t)(plo >> 5) & fmask] >> (plo & 31)) & 1u)) continue;
              } else if (p.filt_kind == FILT_BLOOM || p.filt_kind == FILT_GBLOOM) {
                uint32_t wi, bm;
                bloom_pos(fold_le(plo, phi), p.filt_words, &wi, &bm);
                const uint32_t w = p.filt_kind == FILT_GBLOOM ? p.filt[wi] : s_filt[wi];
                if ((w & bm) != bm) continue;
              }
              h = hash_key(plo, phi);
              const uint64_t slot = h & p.mmask;
              q_slot[u] = slot;
              q_v[u] = p.map[slot];
              q_fp[u] = map_fp(h, p.rank_bits);
              q_lo[u] = plo;
              q_hi[u] = phi;
              q_code[u] = FEAT ? 0u : s_code[sym];
              live |= 1u << u;
            }
#pragma unroll
            for (int u = 0; u < RB; u++) {
              if (!((live >> u) & 1u)) continue;
              const uint32_t v = q_v[u];
              if (v != 0 && (p.rank_bits >= 32 || (v >> p.rank_bits) == q_fp[u])) {
                const uint32_t r = (v & rmask) - 1;
                q_klo[u] = p.tkeys_lo[r];
                if (KW == 2) q_khi[u] = p.tkeys_hi[r];
                hit |= 1u << u;
              }
            }
#pragma unroll
            for (int u = 0; u < RB; u++) {
              if (!((live >> u) & 1u)) continue;
              uint64_t slot = q_slot[u];
              uint32_t v = q_v[u];
              int64_t r = -1;
              if (((hit >> u) & 1u) && q_klo[u] == q_lo[u] && (KW == 1 || q_khi[u] == q_hi[u])) {
                r = (int64_t)(v & rmask) - 1;
              } else {
                // rare: the first slot was another key's; continue the linear probe
                while (v != 0) {
                  slot = (slot + 1) & p.mmask;
                  v = p.map[slot];
                  if (v == 0) break;
                  if (p.rank_bits < 32 && (v >> p.rank_bits) != q_fp[u]) continue;
                  const uint32_t rr = (v & rmask) - 1;
                  if (p.tkeys_lo[rr] == q_lo[u] && (KW == 1 || p.tkeys_hi[rr] == q_hi[u])) {
                    r = rr;
                    break;
                  }
                }
              }
              if (r < 0) continue;
              handle((uint32_t)r * p.sigma + q_code[u]);
            }
          }
        } else {
          for (uint64_t t = t_lo; t < t_hi; t++) {
            const uint64_t g = wbeg + t;
            k.template push<B>(stage_sym<B>(s_stage, g + n - 1, sbase), mlo, mhi);
            uint32_t cid;
            if (MODE == MODE_DENSE) {
              cid = (uint32_t)k.lo;
            } else {
              cid = table_insert(p, k.lo, k.hi);
              if (cid == 0xFFFFFFFFu) continue;
            }
            handle(cid);
          }
        }
      }
    }
    __syncthreads();
    // the stage is free: the next chunk's loaded words go in
    staged = 0;
    if (PF && have_nx) {
#pragma unroll
      for (uint32_t q = 0; q < PF; q++)
        if (q * bs + tid < nx.nw) reinterpret_cast<u32x4_t *>(s_stage)[q * bs + tid] = pf[q];
      staged = nx.nw < PF * bs ? nx.nw : PF * bs;
    }
    // FEAT: the chunk's bitmap words that are set go into the sequence's bitmap
    if (FEAT) {
      uint32_t *gbm = p.bitmaps + (uint64_t)c.file * p.fwords;
      for (uint32_t i = tid; i < bm_lds; i += bs) {
        const uint32_t v = s_bm[i];
        if (v) {
          atomicOr(gbm + i, v);
          s_bm[i] = 0;
        }
      }
    }
    // records made at insert time: the set is only cleared
    if (EAI) {
      typedef uint32_t u32x4e_t __attribute__((ext_vector_type(4)));
      for (uint32_t i = tid; i < p.set_cap / 4; i += bs)
        reinterpret_cast<u32x4e_t *>(s_set)[i] = u32x4e_t{LDS_EMPTY, LDS_EMPTY, LDS_EMPTY, LDS_EMPTY};
    }
    // set_cap is a multiple of the block, so every lane of a wavefront runs the same iterations
    for (uint32_t i = tid; !FEAT && !EAI && i < p.set_cap; i += bs) {
      const uint32_t cid = s_set[i];
      const bool full = cid != LDS_EMPTY;
      if (OCC) {
        if (full) {
          cnt_add<CT>(p.cnt, cid, (CT)s_cnt[i]);
          s_cnt[i] = 0;
          s_set[i] = LDS_EMPTY;
        }
        continue;
      }
      // one LDS atomic per wavefront reserves the wavefront's consecutive record slots
      const uint64_t mask = __ballot(full);
      if (!mask) continue;
      const uint32_t leader = (uint32_t)__ffsll((unsigned long long)mask) - 1;
      uint32_t base = 0;
      if (lane == leader) base = atomicAdd(&s_nrec, (uint32_t)__popcll(mask));
      base = __shfl(base, leader);
      if (full) {
        __builtin_nontemporal_store(cid, p.rec + wbeg + base + (uint32_t)__popcll(mask & lanes_below));
        atomicAdd(my_h1 + (p.low1 >= 32 ? 0u : (cid >> p.low1)), 1u);
        s_set[i] = LDS_EMPTY;
      }
    }
    __syncthreads();
    if (tid == 0) s_full = 0;
    if (!OCC && !FEAT) {
      if (tid == 0) {
        p.nrec[c.fci] = s_nrec;
        s_nrec = 0;
      }
      for (uint32_t b = tid; b < p.nb1; b += bs) {
        uint32_t sum = 0;
        for (uint32_t w = 0; w < nwaves; w++) {
          sum += s_h1w[w * p.nb1 + b];
          s_h1w[w * p.nb1 + b] = 0;
        }
        p.hist1[(uint64_t)c.fci * p.nb1 + b] = sum;
      }
    }
    if (tid == 0) {
      uint32_t c0 = END, c1 = END;
      if (PF) {
        c0 = cn;
        c1 = claim;
      } else if (p.persistent == 2) {   // strided (no queue counter is passed in this form)
        c0 = ci + gridDim.x;
      } else if (p.persistent) {
        c0 = atomicAdd(p.qctr, 1u);
      }
      if (__hip_atomic_load(p.status, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) c0 = c1 = END;
      s_chunk = c0;
      s_next = c1;
    }
    __syncthreads();
  }
}

size_t scan_lds_bytes(const ScanParams &p, int mode, int occ, int feat) {
  size_t b = p.stage_bytes;
  if (mode == MODE_FILTERED) b += (size_t)((filt_lds_words(p.filt_kind, p.filt_words) + 3u) & ~3u) * 4;
  if (feat) b += p.lds_bitmap ? (size_t)((p.fwords + 3u) & ~3u) * 4 : 0;
  else b += (size_t)p.set_cap * 4 * (occ ? 2 : 1);
  b += 256;
  b += p.qbytes;
  b += (size_t)p.hist_words * 4;
  return b;
}

template <int B, int KW, int MODE, int OCC, typename CT, int FEAT = 0>
static hipError_t launch_t(const ScanParams &p, uint32_t grid, uint32_t block, hipStream_t s) {
  const size_t lds = scan_lds_bytes(p, MODE, OCC, FEAT);
  // survivor rings: filtered passes with keys of at most 64 bits, and Eq. 2 passes over bytes with
  // keys of up to 128 (their windows take five stage words); featurize keeps 128-bit keys in place
  constexpr int can_cmp = (MODE == MODE_FILTERED && (KW == 1 || (B == 8 && !OCC && !FEAT))) ? 1 : 0;
  auto fn0 = k_scan<B, KW, MODE, OCC, CT, 0, FEAT>;
  auto fn1 = k_scan<B, KW, MODE, OCC, CT, can_cmp, FEAT>;
  if (grid == 0) {   // preparation call: allow the whole LDS of a CU (never issued during a capture)
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(fn0), hipFuncAttributeMaxDynamicSharedMemorySize,
                                       160 * 1024 - 4096);
    if (e == hipSuccess && can_cmp)
      e = hipFuncSetAttribute(reinterpret_cast<const void *>(fn1), hipFuncAttributeMaxDynamicSharedMemorySize,
                              160 * 1024 - 4096);
    return e;
  }
  hipLaunchKernelGGL((can_cmp && p.qbytes) ? fn1 : fn0, dim3(grid), dim3(block), lds, s, p);
  return hipGetLastError();
}

template <int B, int KW, int MODE>
static hipError_t launch_m(const ScanParams &p, int occ, int count64, uint32_t grid, uint32_t block, hipStream_t s) {
  if (!occ) return launch_t<B, KW, MODE, 0, uint32_t>(p, grid, block, s);
  if (!count64) return launch_t<B, KW, MODE, 1, uint32_t>(p, grid, block, s);
  return launch_t<B, KW, MODE, 1, unsigned long long>(p, grid, block, s);
}

// The featurizing form of the scan (FEAT): filtered mode against the current table.  grid = 0
// prepares the kernels' LDS limit.
hipError_t launch_scan_feat(const ScanParams &p, int bits, int kw, uint32_t grid, uint32_t block, hipStream_t s) {
  if (bits == 8)
    return kw == 1 ? launch_t<8, 1, MODE_FILTERED, 0, uint32_t, 1>(p, grid, block, s)
                   : launch_t<8, 2, MODE_FILTERED, 0, uint32_t, 1>(p, grid, block, s);
  return kw == 1 ? launch_t<2, 1, MODE_FILTERED, 0, uint32_t, 1>(p, grid, block, s)
                 : launch_t<2, 2, MODE_FILTERED, 0, uint32_t, 1>(p, grid, block, s);
}

hipError_t launch_scan(const ScanParams &p, int bits, int kw, int mode, int occ, int count64, uint32_t grid,
                       uint32_t block, hipStream_t s) {
  if (bits == 8) {
    if (mode == MODE_DENSE) return launch_m<8, 1, MODE_DENSE>(p, occ, count64, grid, block, s);
    if (kw == 1) {
      if (mode == MODE_FILTERED) return launch_m<8, 1, MODE_FILTERED>(p, occ, count64, grid, block, s);
      return launch_m<8, 1, MODE_SPARSE>(p, occ, count64, grid, block, s);
    }
    if (mode == MODE_FILTERED) return launch_m<8, 2, MODE_FILTERED>(p, occ, count64, grid, block, s);
    return launch_m<8, 2, MODE_SPARSE>(p, occ, count64, grid, block, s);
  }
  if (mode == MODE_DENSE) return launch_m<2, 1, MODE_DENSE>(p, occ, count64, grid, block, s);
  if (kw == 1) {
    if (mode == MODE_FILTERED) return launch_m<2, 1, MODE_FILTERED>(p, occ, count64, grid, block, s);
    return launch_m<2, 1, MODE_SPARSE>(p, occ, count64, grid, block, s);
  }
  if (mode == MODE_FILTERED) return launch_m<2, 2, MODE_FILTERED>(p, occ, count64, grid, block, s);
  return launch_m<2, 2, MODE_SPARSE>(p, occ, count64, grid, block, s);
}

hipError_t prepare_scan(int bits, int kw, int mode, int occ, int count64) {
  ScanParams p{};
  return launch_scan(p, bits, kw, mode, occ, count64, 0, 0, nullptr);
}

// ------------------------------------------------------------------ fills (graph-safe, no memset nodes)
__global__ void k_fill_u32(uint32_t *p, uint64_t n, uint32_t v) {
  for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x)
    p[i] = v;
}
__global__ void k_fill_u64(uint64_t *p, uint64_t n, uint64_t v) {
  for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x)
    p[i] = v;
}
hipError_t launch_fill_u32(uint32_t *p, uint64_t n, uint32_t v, hipStream_t s) {
  if (!n) return hipSuccess;
  uint64_t g = (n + 255) / 256;
  if (g > 4096) g = 4096;
  hipLaunchKernelGGL(k_fill_u32, dim3((uint32_t)g), dim3(256), 0, s, p, n, v);
  return hipGetLastError();
}
hipError_t launch_fill_u64(uint64_t *p, uint64_t n, uint64_t v, hipStream_t s) {
  if (!n) return hipSuccess;
  uint64_t g = (n + 255) / 256;
  if (g > 4096) g = 4096;
  hipLaunchKernelGGL(k_fill_u64, dim3((uint32_t)g), dim3(256), 0, s, p, n, v);
  return hipGetLastError();
}

}  // namespace ig
