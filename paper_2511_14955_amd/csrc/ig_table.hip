// Index over the retained table, and featurization against it.
//
// After a pass (Algorithm 3's selection of P^(j)) the retained keys are indexed:
//  * an exact open-addressing map key -> rank+1 (capacity a power of two, at
//    least twice the table), probed only by filter hits;
//  * for keys of at most 64 bits, a quotient map of the same capacity whose 8-byte
//    slots identify their key without a second read (see QMapShape);
//  * a compact filter image that a scan workgroup copies into LDS: a direct
//    bitmap over the whole key space when it is small enough (exact), else a
//    blocked Bloom filter (three bits in one 32-bit word chosen by the key hash;
//    no false negatives).
// The same index answers the prefix test of the next pass (the prefix of an
// (n+1)-window is an n-gram) and the lookups of featurize (Figure 1's Boolean
// m x k matrix).
//
// Featurize: each workgroup takes a chunk of one sequence, rolls n-gram keys
// over it, and sets bit rank(key) in an LDS bitmap of kept bits; at the end of
// the chunk the non-zero words are OR-ed into the sequence's bitmap in HBM
// (word-contiguous, so the atomics coalesce).  A sequence's row is then the set
// bits of its bitmap in increasing order: de-duplicated and sorted by
// construction.
#include "ig_internal.h"

namespace ig {

// The retained keys' stream forms (the form every index below is keyed by).
__global__ void k_le_keys(const uint64_t *tlo, const uint64_t *thi, const unsigned long long *kept_p, uint32_t n,
                          uint32_t b, uint64_t *llo, uint64_t *lhi) {
  const uint64_t kept = *kept_p;
  for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < kept; i += (uint64_t)gridDim.x * blockDim.x) {
    uint64_t a, c;
    stream_form(tlo[i], thi[i], n, b, &a, &c);
    llo[i] = a;
    lhi[i] = c;
  }
}

// Slot: rank+1 in the low rank_bits bits, a fingerprint of the key's hash above them.
__global__ void k_map_insert(const uint64_t *tlo, const uint64_t *thi, const unsigned long long *kept_p, uint32_t *map,
                             uint64_t mmask, uint32_t rank_bits) {
  const uint64_t kept = *kept_p;
  for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < kept; i += (uint64_t)gridDim.x * blockDim.x) {
    const uint64_t h = hash_key(tlo[i], thi[i]);
    const uint32_t v = (uint32_t)(i + 1) | (rank_bits >= 32 ? 0u : (map_fp(h, rank_bits) << rank_bits));
    uint64_t slot = h & mmask;
    while (atomicCAS(map + slot, 0u, v) != 0u) slot = (slot + 1) & mmask;
  }
}

// Quotient map insert of ranks [r0, min(r1, kept)): linear probing from the home slot.  The
// ranks go in by increasing batches, so that the most frequent keys, which take most lookups,
// find their home slot free.  A key whose displacement would not fit its field raises the
// table's flag (lookups then use the fingerprinted map and the table's keys).
__global__ void k_qmap_insert(const uint64_t *tlo, const unsigned long long *kept_p, uint64_t r0, uint64_t r1,
                              unsigned long long *qmap, uint32_t *qflag, uint64_t mmask, QMapShape qs) {
  const uint64_t kept = *kept_p < r1 ? *kept_p : r1;
  const uint64_t dmax = (1ull << qs.dbits) - 1;
  for (uint64_t i = r0 + blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < kept; i += (uint64_t)gridDim.x * blockDim.x) {
    const uint64_t x = qmix(tlo[i], qs.w);
    uint64_t slot = x >> qs.qbits;
    const uint64_t rem = qs.qbits ? (x & ((1ull << qs.qbits) - 1)) : 0ull;
    for (uint64_t d = 0;; d++) {
      if (d > dmax) {
        atomicOr(qflag, 1u);
        break;
      }
      const uint64_t e = (rem << (qs.rbits + qs.dbits)) | (d << qs.rbits) | (i + 1);
      if (atomicCAS(qmap + slot, 0ull, (unsigned long long)e) == 0ull) break;
      slot = (slot + 1) & mmask;
    }
  }
}

__global__ void k_qmap_mirror(unsigned long long *qmap, uint64_t mmask) {
  if (threadIdx.x == 0) qmap[mmask + 1] = qmap[0];
}

__global__ void k_filter_build(const uint64_t *tlo, const uint64_t *thi, const unsigned long long *kept_p, uint32_t *filt,
                               uint32_t words, uint32_t kind) {
  const uint64_t kept = *kept_p;
  for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < kept; i += (uint64_t)gridDim.x * blockDim.x) {
    const uint64_t lo = tlo[i], hi = thi[i];
    if (kind == FILT_DIRECT) {
      atomicOr(filt + (lo >> 5), 1u << (lo & 31));
    } else {
      uint32_t w, bm;
      bloom_pos(fold_le(lo, hi), words, &w, &bm);
      atomicOr(filt + w, bm);
    }
  }
}

// Sizes come from k_max (an upper bound of the table length known on the host);
// the kernels read the actual length from device memory.
int index_reserve(ig_ctx *c, TableSet &ts, uint32_t n, uint64_t k_max) {
  uint64_t cap = 1024;
  while (cap < (k_max << c->lc.map_log2)) cap <<= 1;
  const uint32_t nbits = n * c->cfg.symbol_bits;
  const uint64_t maxw = c->lc.filt_max_words;
  uint32_t kind, words;
  if (nbits <= 40 && (1ull << nbits) <= maxw * 32) {
    kind = FILT_DIRECT;
    words = (uint32_t)(((1ull << nbits) + 31) / 32);
  } else {
    kind = FILT_BLOOM;
    uint64_t w = 64;   // about bloom_bits bits per key, a power of two within [64, maxw]
    while (w < (k_max * c->lc.bloom_bits + 31) / 32 && w < maxw) w <<= 1;
    words = (uint32_t)w;
  }
  uint32_t rb = 1;
  while (rb < 32 && (1ull << rb) <= k_max) rb++;   // rank+1 <= k_max fits
  if (dev_reserve(c, ts.map, cap * 4) || dev_reserve(c, ts.filt, (uint64_t)words * 4) ||
      dev_reserve(c, ts.le_lo, std::max<uint64_t>(k_max, 1) * 8) || dev_reserve(c, ts.le_hi, std::max<uint64_t>(k_max, 1) * 8))
    return IG_ENOMEM;
  ts.has_qmap = false;
  if (nbits <= 64) {
    QMapShape qs{};
    qs.w = nbits;
    while ((1ull << qs.sbits) < cap) qs.sbits++;
    qs.qbits = nbits > qs.sbits ? nbits - qs.sbits : 0;
    qs.rbits = rb;
    const int room = 64 - (int)qs.qbits - (int)qs.rbits;
    if (room >= 6) {
      qs.dbits = room < 16 ? (uint32_t)room : 16u;
      // one slot past the end mirrors slot 0, so that a probe can read two neighbouring slots
      if (dev_reserve(c, ts.qmap, (cap + 1) * 8) || dev_reserve(c, ts.qflag, 64)) return IG_ENOMEM;
      ts.qs = qs;
      ts.has_qmap = true;
    }
  }
  ts.n = n;   // (the stream forms are computed for this gram length)
  ts.map_mask = cap - 1;
  ts.rank_bits = rb;
  ts.filt_words = words;
  ts.filt_kind = kind;
  return IG_OK;
}

hipError_t index_enqueue(ig_ctx *c, TableSet &ts, uint64_t k_max, const unsigned long long *kept_dev) {
  hipStream_t s = c->stream;
  hipError_t e = launch_fill_u32(reinterpret_cast<uint32_t *>(ts.map.p), ts.map_mask + 1, 0, s);
  if (e == hipSuccess) e = launch_fill_u32(reinterpret_cast<uint32_t *>(ts.filt.p), ts.filt_words, 0, s);
  if (e != hipSuccess) return e;
  uint64_t g = (k_max + 255) / 256;
  if (g > 4096) g = 4096;
  if (g < 1) g = 1;
  const uint64_t *llo = reinterpret_cast<const uint64_t *>(ts.le_lo.p), *lhi = reinterpret_cast<const uint64_t *>(ts.le_hi.p);
  hipLaunchKernelGGL(k_le_keys, dim3((uint32_t)g), dim3(256), 0, s, reinterpret_cast<const uint64_t *>(ts.lo.p),
                     reinterpret_cast<const uint64_t *>(ts.hi.p), kept_dev, ts.n, c->cfg.symbol_bits,
                     reinterpret_cast<uint64_t *>(ts.le_lo.p), reinterpret_cast<uint64_t *>(ts.le_hi.p));
  hipLaunchKernelGGL(k_map_insert, dim3((uint32_t)g), dim3(256), 0, s, llo, lhi, kept_dev,
                     reinterpret_cast<uint32_t *>(ts.map.p), ts.map_mask, ts.rank_bits);
  hipLaunchKernelGGL(k_filter_build, dim3((uint32_t)g), dim3(256), 0, s, llo, lhi, kept_dev,
                     reinterpret_cast<uint32_t *>(ts.filt.p), ts.filt_words, ts.filt_kind);
  if (ts.has_qmap) {
    if ((e = hipGetLastError()) == hipSuccess) e = launch_fill_u64(reinterpret_cast<uint64_t *>(ts.qmap.p), ts.map_mask + 2, 0, s);
    if (e == hipSuccess) e = launch_fill_u32(reinterpret_cast<uint32_t *>(ts.qflag.p), 1, 0, s);
    if (e != hipSuccess) return e;
    // ranks [0, 256), [256, 1024), [1024, 4096), ... then the rest
    uint64_t r0 = 0;
    for (uint64_t r1 = 256; r0 < k_max; r1 = r1 < (1ull << 14) ? r1 * 4 : k_max) {
      uint64_t gb = (r1 - r0 + 255) / 256;
      if (gb > 4096) gb = 4096;
      hipLaunchKernelGGL(k_qmap_insert, dim3((uint32_t)gb), dim3(256), 0, s, llo, kept_dev, r0, r1, reinterpret_cast<unsigned long long *>(ts.qmap.p),
                         reinterpret_cast<uint32_t *>(ts.qflag.p), ts.map_mask, ts.qs);
      r0 = r1;
    }
    hipLaunchKernelGGL(k_qmap_mirror, dim3(1), dim3(64), 0, s, reinterpret_cast<unsigned long long *>(ts.qmap.p),
                       ts.map_mask);
  }
  return hipGetLastError();
}

// ------------------------------------------------------------------ featurize
struct FeatParams {
  const uint8_t *data;
  const uint64_t *offs;
  const Chunk *chunks;
  uint32_t nchunks;
  uint32_t n;
  const uint32_t *filt;
  uint32_t filt_words, filt_kind;
  const uint32_t *map;
  uint64_t mmask;
  uint32_t rank_bits;
  const uint64_t *tkeys_lo, *tkeys_hi;
  uint32_t *bitmaps;
  uint32_t words;        // per-sequence bitmap words (ceil(kept / 32))
  uint32_t lds_bitmap;   // the bitmap fits in LDS
  uint32_t stage_bytes;
};

template <int B, int KW>
__global__ void __launch_bounds__(512) k_featurize(FeatParams p) {
  extern __shared__ __align__(16) uint8_t lds[];
  uint8_t *s_stage = lds;
  uint32_t *s_filt = reinterpret_cast<uint32_t *>(lds + p.stage_bytes);
  uint32_t *s_bm = s_filt + p.filt_words;
  const uint32_t tid = threadIdx.x, bs = blockDim.x, n = p.n;
  for (uint32_t i = tid; i < p.filt_words; i += bs) s_filt[i] = p.filt[i];
  if (p.lds_bitmap)
    for (uint32_t i = tid; i < p.words; i += bs) s_bm[i] = 0;
  __syncthreads();
  for (uint32_t ci = blockIdx.x; ci < p.nchunks; ci += gridDim.x) {
    const Chunk c = p.chunks[ci];
    const uint64_t fend = p.offs[c.file + 1], flen = fend - p.offs[c.file];
    uint32_t *gbm = p.bitmaps + (uint64_t)c.file * p.words;
    const uint64_t wbeg = c.s0;
    uint64_t wend = c.s0 + c.nsym;
    if (flen < n) wend = wbeg;
    else if (wend > fend - n + 1) wend = fend - n + 1;
    if (wbeg < wend) {
      const uint64_t nwin = wend - wbeg;
      const uint64_t byte_lo = (B == 8) ? wbeg : (wbeg >> 2);
      const uint64_t byte_hi = (B == 8) ? (wend + n - 1) : ((wend + n - 2) >> 2) + 1;
      const uint64_t a0 = byte_lo & ~15ull, a1 = (byte_hi + 15) & ~15ull;
      const uint4 *src = reinterpret_cast<const uint4 *>(p.data + a0);
      for (uint64_t i = tid; i < (a1 - a0) / 16; i += bs) reinterpret_cast<uint4 *>(s_stage)[i] = src[i];
      __syncthreads();
      const uint32_t per = (uint32_t)((nwin + bs - 1) / bs) | 1u;   // odd: lanes in different LDS banks
      const uint64_t t_lo = (uint64_t)tid * per, t_hi = t_lo + per < nwin ? t_lo + per : nwin;
      if (t_lo < t_hi) {
        uint64_t klo = 0, khi = 0;
        auto sym = [&](uint64_t g) -> uint32_t {
          if (B == 8) return s_stage[g - a0];
          return (s_stage[(g >> 2) - a0] >> (6 - 2 * (uint32_t)(g & 3))) & 3u;
        };
        // the window's stream form (first symbol lowest), the form the table's index is keyed by
        const uint32_t top = (n - 1) * B;
        auto push = [&](uint32_t sv) {
          if (KW == 2) {
            klo = (klo >> B) | (khi << (64 - B));
            khi >>= B;
            if (top >= 64) khi |= (uint64_t)sv << (top - 64);
            else klo |= (uint64_t)sv << top;
          } else {
            klo = (klo >> B) | ((uint64_t)sv << top);
          }
        };
        for (uint32_t r = 0; r + 1 < n; r++) push(sym(wbeg + t_lo + r));
        for (uint64_t t = t_lo; t < t_hi; t++) {
          push(sym(wbeg + t + n - 1));
          if (p.filt_kind == FILT_DIRECT) {
            if (!((s_filt[klo >> 5] >> (klo & 31)) & 1u)) continue;
          } else {
            uint32_t wi, bm;
            bloom_pos(fold_le(klo, khi), p.filt_words, &wi, &bm);
            const uint32_t w = s_filt[wi];
            if ((w & bm) != bm) continue;
          }
          const uint64_t h = hash_key(klo, khi);
          uint64_t slot = h & p.mmask;
          int64_t r = -1;
          const uint32_t fp = map_fp(h, p.rank_bits);
          const uint32_t rmask = p.rank_bits >= 32 ? 0xFFFFFFFFu : ((1u << p.rank_bits) - 1);
          for (;;) {
            const uint32_t v = p.map[slot];
            if (!v) break;
            if (p.rank_bits >= 32 || (v >> p.rank_bits) == fp) {
              const uint32_t rr = (v & rmask) - 1;
              if (p.tkeys_lo[rr] == klo && p.tkeys_hi[rr] == khi) { r = rr; break; }
            }
            slot = (slot + 1) & p.mmask;
          }
          if (r < 0) continue;
          if (p.lds_bitmap) atomicOr(s_bm + (r >> 5), 1u << (r & 31));
          else atomicOr(gbm + (r >> 5), 1u << (r & 31));
        }
      }
      __syncthreads();
      if (p.lds_bitmap) {
        for (uint32_t i = tid; i < p.words; i += bs) {
          const uint32_t v = s_bm[i];
          if (v) { atomicOr(gbm + i, v); s_bm[i] = 0; }
        }
      }
    }
    __syncthreads();
  }
}

hipError_t launch_featurize(ig_ctx *c, const FeatBatch &fb, hipStream_t s) {
  FeatParams p{};
  p.data = fb.data;
  p.offs = fb.offs;
  p.chunks = fb.chunks;
  p.nchunks = fb.nchunks;
  const TableSet &ts = c->ts[c->cur];
  p.n = ts.n;
  p.filt = reinterpret_cast<const uint32_t *>(ts.filt.p);
  p.filt_words = ts.filt_words;
  p.filt_kind = ts.filt_kind;
  p.map = reinterpret_cast<const uint32_t *>(ts.map.p);
  p.mmask = ts.map_mask;
  p.rank_bits = ts.rank_bits;
  p.tkeys_lo = reinterpret_cast<const uint64_t *>(ts.le_lo.p);   // stream forms, rank order
  p.tkeys_hi = reinterpret_cast<const uint64_t *>(ts.le_hi.p);
  p.bitmaps = fb.bitmaps;
  p.words = fb.words;
  const uint32_t bits = c->cfg.symbol_bits;
  p.stage_bytes = (uint32_t)(((uint64_t)c->lc.chunk_syms * bits / 8 + 64 + 32) & ~15ull);
  const size_t base = p.stage_bytes + (size_t)p.filt_words * 4;
  const size_t limit = 160 * 1024 - 512;
  p.lds_bitmap = base + (size_t)p.words * 4 <= limit ? 1u : 0u;
  const size_t lds = base + (p.lds_bitmap ? (size_t)p.words * 4 : 0);
  if (!fb.nchunks) return hipSuccess;
  uint32_t grid = fb.nchunks < (uint32_t)c->n_cu * 2 ? fb.nchunks : (uint32_t)c->n_cu * 2;
  const bool kw2 = (uint64_t)p.n * bits > 64;
  const void *fn;
  if (bits == 8) fn = kw2 ? reinterpret_cast<const void *>(k_featurize<8, 2>) : reinterpret_cast<const void *>(k_featurize<8, 1>);
  else fn = kw2 ? reinterpret_cast<const void *>(k_featurize<2, 2>) : reinterpret_cast<const void *>(k_featurize<2, 1>);
  hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  if (bits == 8) {
    if (kw2) hipLaunchKernelGGL((k_featurize<8, 2>), dim3(grid), dim3(512), lds, s, p);
    else hipLaunchKernelGGL((k_featurize<8, 1>), dim3(grid), dim3(512), lds, s, p);
  } else {
    if (kw2) hipLaunchKernelGGL((k_featurize<2, 2>), dim3(grid), dim3(512), lds, s, p);
    else hipLaunchKernelGGL((k_featurize<2, 1>), dim3(grid), dim3(512), lds, s, p);
  }
  return hipGetLastError();
}

// one workgroup per row: popcount (count_only) or write the set-bit positions in order
__global__ void __launch_bounds__(256) k_rows(const uint32_t *bitmaps, uint64_t m, uint32_t words, uint64_t *nnz,
                                              const uint64_t *indptr, int32_t *indices, uint64_t cap, int count_only) {
  __shared__ uint32_t part[256];
  const uint32_t t = threadIdx.x;
  for (uint64_t f = blockIdx.x; f < m; f += gridDim.x) {
    const uint32_t *bm = bitmaps + f * words;
    const uint32_t per = (words + 255) / 256;
    const uint32_t lo = t * per, hi = lo + per < words ? lo + per : words;
    uint32_t cntl = 0;
    for (uint32_t w = lo; w < hi; w++) cntl += __popc(bm[w]);
    part[t] = cntl;
    __syncthreads();
    for (uint32_t off = 1; off < 256; off <<= 1) {
      const uint32_t v = t >= off ? part[t - off] : 0;
      __syncthreads();
      part[t] += v;
      __syncthreads();
    }
    if (count_only) {
      if (t == 255) nnz[f] = part[255];
    } else {
      uint64_t pos = indptr[f] + part[t] - cntl;
      for (uint32_t w = lo; w < hi; w++) {
        uint32_t v = bm[w];
        while (v) {
          const uint32_t b = __ffs(v) - 1;
          v &= v - 1;
          if (pos < cap) indices[pos] = (int32_t)(w * 32 + b);
          pos++;
        }
      }
    }
    __syncthreads();
  }
}

hipError_t launch_rows(const uint32_t *bitmaps, uint64_t m, uint32_t words, uint64_t *nnz_per_row, const uint64_t *indptr,
                       int32_t *indices, uint64_t cap, int count_only, hipStream_t s) {
  if (!m) return hipSuccess;
  const uint32_t grid = m < 4096 ? (uint32_t)m : 4096;
  hipLaunchKernelGGL(k_rows, dim3(grid), dim3(256), 0, s, bitmaps, m, words, nnz_per_row, indptr, indices, cap,
                     count_only);
  return hipGetLastError();
}

// number of the m sequences whose bitmap has each bit set (count requests)
__global__ void k_col_counts(const uint32_t *bitmaps, uint64_t m, uint32_t words, uint32_t kept, uint32_t *out) {
  for (uint64_t w = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; w < words; w += (uint64_t)gridDim.x * blockDim.x) {
    uint32_t acc[32];
    for (int b = 0; b < 32; b++) acc[b] = 0;
    for (uint64_t f = 0; f < m; f++) {
      const uint32_t v = bitmaps[f * words + w];
      for (int b = 0; b < 32; b++) acc[b] += (v >> b) & 1u;
    }
    for (int b = 0; b < 32; b++)
      if (w * 32 + b < kept) out[w * 32 + b] = acc[b];
  }
}

hipError_t launch_col_counts(const uint32_t *bitmaps, uint64_t m, uint32_t words, uint32_t kept, uint32_t *col_counts,
                             hipStream_t s) {
  if (!words) return hipSuccess;
  const uint32_t grid = (words + 255) / 256;
  hipLaunchKernelGGL(k_col_counts, dim3(grid), dim3(256), 0, s, bitmaps, m, words, kept, col_counts);
  return hipGetLastError();
}

// The current table indexed again (map, quotient map, filter image) with the context's table
// shape; the table's keys and order are unchanged.
int reindex_current(ig_ctx *c) {
  if (c->fresh || !c->kept) return IG_OK;
  TableSet &t = c->T();
  int rc = index_reserve(c, t, t.n, t.kept);
  if (rc) return rc;
  const unsigned long long kept = t.kept;
  hipStream_t s = c->stream;
  hipError_t e = hipMemcpyAsync(c->kdev.p, &kept, sizeof kept, hipMemcpyHostToDevice, s);
  if (e == hipSuccess) e = index_enqueue(c, t, t.kept, reinterpret_cast<const unsigned long long *>(c->kdev.p));
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  return check_hip(c, e, "re-index") ? IG_EDEVICE : IG_OK;
}

}  // namespace ig
