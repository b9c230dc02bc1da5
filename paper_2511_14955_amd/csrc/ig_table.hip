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
#include <cstring>
#include <mutex>

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

// The same for the 16-byte-slot quotient map (keys of up to 128 bits, stream forms lo and hi): a
// slot is claimed by a compare-and-swap of its first word (rank+1, displacement and the
// remainder's low bits: never zero), and its second word (the rest of the remainder) is stored
// after; the scan reads the map only once the build has finished.
__global__ void k_qmap2_insert(const uint64_t *tlo, const uint64_t *thi, const unsigned long long *kept_p, uint64_t r0,
                               uint64_t r1, unsigned long long *qmap2, uint32_t *qflag, uint64_t mmask, QMapShape qs) {
  const uint64_t kept = *kept_p < r1 ? *kept_p : r1;
  const uint64_t dmax = (1ull << qs.dbits) - 1;
  const uint32_t sh = qs.rbits + qs.dbits;
  for (uint64_t i = r0 + blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < kept; i += (uint64_t)gridDim.x * blockDim.x) {
    uint64_t home, rl, rh;
    qmix2(tlo[i], qs.w > 64 ? thi[i] : 0ull, qs.w, qs.sbits, &home, &rl, &rh);
    const uint64_t w1 = (rl >> (64 - sh)) | (rh << sh);
    uint64_t slot = home & mmask;
    for (uint64_t d = 0;; d++) {
      if (d > dmax) {
        atomicOr(qflag, 1u);
        break;
      }
      const uint64_t w0 = (rl << sh) | (d << qs.rbits) | (i + 1);
      if (atomicCAS(qmap2 + 2 * slot, 0ull, (unsigned long long)w0) == 0ull) {
        qmap2[2 * slot + 1] = w1;
        break;
      }
      slot = (slot + 1) & mmask;
    }
  }
}

__global__ void k_qmap2_mirror(unsigned long long *qmap2, uint64_t mmask) {
  if (threadIdx.x < 2) qmap2[2 * (mmask + 1) + threadIdx.x] = qmap2[threadIdx.x];
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
    // about bloom_bits bits per key, a power of two of at least 64 words; in LDS while that cap
    // still leaves 4 bits per key, else in global memory (L2) at the full size (up to 64 MB)
    const uint64_t want = (k_max * c->lc.bloom_bits + 31) / 32;
    kind = maxw * 32 >= k_max * 4 ? FILT_BLOOM : FILT_GBLOOM;
    const uint64_t cap = kind == FILT_BLOOM ? maxw : (1ull << 24);
    uint64_t w = 64;
    while (w < want && w < cap) w <<= 1;
    words = (uint32_t)w;
  }
  uint32_t rb = 1;
  while (rb < 32 && (1ull << rb) <= k_max) rb++;   // rank+1 <= k_max fits
  if (dev_reserve(c, ts.map, cap * 4) || dev_reserve(c, ts.filt, (uint64_t)words * 4) ||
      dev_reserve(c, ts.le_lo, std::max<uint64_t>(k_max, 1) * 8) || dev_reserve(c, ts.le_hi, std::max<uint64_t>(k_max, 1) * 8))
    return IG_ENOMEM;
  ts.has_qmap = false;
  ts.has_qmap2 = false;
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
  if (!ts.has_qmap && nbits <= 128 && nbits + c->cfg.symbol_bits > 64) {
    // 16-byte slots: 128 bits hold the remainder (nbits - sbits), rank+1 and the displacement.
    // (Only for a table whose next pass has windows of more than 64 bits: the scan's 128-bit form
    // is the one that reads it.)
    QMapShape qs{};
    qs.w = nbits;
    while ((1ull << qs.sbits) < cap) qs.sbits++;
    qs.qbits = nbits > qs.sbits ? nbits - qs.sbits : 0;
    qs.rbits = rb;
    const int room = 128 - (int)qs.qbits - (int)qs.rbits;
    if (nbits > qs.sbits && room >= 6) {
      qs.dbits = room < 16 ? (uint32_t)room : 16u;
      if (dev_reserve(c, ts.qmap2, (cap + 1) * 16) || dev_reserve(c, ts.qflag, 64)) return IG_ENOMEM;
      ts.qs2 = qs;
      ts.has_qmap2 = true;
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
  if (ts.has_qmap2) {
    if ((e = hipGetLastError()) == hipSuccess)
      e = launch_fill_u64(reinterpret_cast<uint64_t *>(ts.qmap2.p), 2 * (ts.map_mask + 2), 0, s);
    if (e == hipSuccess) e = launch_fill_u32(reinterpret_cast<uint32_t *>(ts.qflag.p), 1, 0, s);
    if (e != hipSuccess) return e;
    uint64_t r0 = 0;
    for (uint64_t r1 = 256; r0 < k_max; r1 = r1 < (1ull << 14) ? r1 * 4 : k_max) {
      uint64_t gb = (r1 - r0 + 255) / 256;
      if (gb > 4096) gb = 4096;
      hipLaunchKernelGGL(k_qmap2_insert, dim3((uint32_t)gb), dim3(256), 0, s, llo, lhi, kept_dev, r0, r1,
                         reinterpret_cast<unsigned long long *>(ts.qmap2.p), reinterpret_cast<uint32_t *>(ts.qflag.p),
                         ts.map_mask, ts.qs2);
      r0 = r1;
    }
    hipLaunchKernelGGL(k_qmap2_mirror, dim3(1), dim3(64), 0, s, reinterpret_cast<unsigned long long *>(ts.qmap2.p),
                       ts.map_mask);
  }
  return hipGetLastError();
}

// ------------------------------------------------------------------ featurize
// Figure 1's Boolean rows run on the scan kernel in its featurizing form: the same staging,
// filter image, survivor rings and quotient-map probes as a pass, with the whole window looked
// up in the current table and each hit setting bit rank(window) in its sequence's bitmap.
// Workgroups take the batch's chunks strided by the grid.
hipError_t launch_featurize(ig_ctx *c, const FeatBatch &fb, hipStream_t s) {
  if (!fb.nchunks || !fb.words) return hipSuccess;
  const TableSet &ts = c->ts[c->cur];
  const uint32_t b = c->cfg.symbol_bits;
  ScanParams p;
  std::memset(&p, 0, sizeof p);
  p.data = fb.data;
  p.offs = fb.offs;
  p.chunks = fb.chunks;
  p.nchunks = fb.nchunks;
  p.persistent = 2;
  p.n = ts.n;
  p.sigma = 1;   // a hit's id is its rank
  p.code = reinterpret_cast<const uint8_t *>(c->code.p);
  p.filt = reinterpret_cast<const uint32_t *>(ts.filt.p);
  p.filt_words = ts.filt_words;
  p.filt_kind = ts.filt_kind;
  p.map = reinterpret_cast<const uint32_t *>(ts.map.p);
  p.mmask = ts.map_mask;
  p.rank_bits = ts.rank_bits;
  p.tkeys_lo = reinterpret_cast<const uint64_t *>(ts.le_lo.p);
  p.tkeys_hi = reinterpret_cast<const uint64_t *>(ts.le_hi.p);
  if (ts.has_qmap) {
    p.qmap = reinterpret_cast<const uint64_t *>(ts.qmap.p);
    p.qflag = reinterpret_cast<const uint32_t *>(ts.qflag.p);
    p.qs = ts.qs;
  }
  p.status = reinterpret_cast<uint32_t *>(c->zero.p);
  p.set_cap = 1024;   // (no set in this form)
  p.stage_bytes = (uint32_t)(((uint64_t)c->lc.chunk_syms * b / 8 + 64 + 32) & ~15ull);
  p.bitmaps = fb.bitmaps;
  p.fwords = fb.words;
  const uint32_t block = 1024;
  const int kw = (uint64_t)ts.n * b > 64 ? 2 : 1;
  const size_t limit = 160 * 1024 - 8192;
  // survivor rings when the window fits 64 bits and thread runs stay within 64 windows; then
  // the chunk's LDS bitmap if there is room left
  if (kw == 1) {
    const uint64_t spd = 32 / b, span_max = c->lc.chunk_syms + 128 / b - 1;
    if (spd * ((span_max + spd * block - 1) / (spd * block)) <= 64) p.qbytes = (block / 64) * SCAN_QCAP * 10u;
  }
  if (scan_lds_bytes(p, MODE_FILTERED, 0, 1) > limit) p.qbytes = 0;
  p.lds_bitmap = 1;
  if (scan_lds_bytes(p, MODE_FILTERED, 0, 1) > limit) p.lds_bitmap = 0;
  if (scan_lds_bytes(p, MODE_FILTERED, 0, 1) > limit) return hipErrorInvalidValue;
  static std::once_flag prepared[2][2];
  hipError_t e = hipSuccess;
  std::call_once(prepared[b == 8][kw - 1], [&]() { e = launch_scan_feat(p, (int)b, kw, 0, 0, nullptr); });
  if (e != hipSuccess) return e;
  const uint32_t grid = fb.nchunks < (uint32_t)c->n_cu ? fb.nchunks : (uint32_t)c->n_cu;
  return launch_scan_feat(p, (int)b, kw, grid, block, s);
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
