// C ABI of libintergrams.so: contexts, corpus load, passes, table access, featurize.
#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <new>

#include "ig_internal.h"

namespace ig {

int set_error(ig_ctx *c, int code, const char *fmt, ...) {
  if (!c) return code;
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  c->err = buf;
  if (code == IG_EDEVICE) c->sticky = 1;
  return code;
}

int check_hip(ig_ctx *c, hipError_t e, const char *what) {
  if (e == hipSuccess) return 0;
  set_error(c, IG_EDEVICE, "%s: %s", what, hipGetErrorString(e));
  return 1;
}

// a device buffer back to where it came from (the caller's allocator, or HIP)
static void free_device(ig_ctx *c, void *p) {
  if (c->cfg.alloc) c->cfg.free(p, reinterpret_cast<void *>(c->stream), c->cfg.alloc_user);
  else (void)hipFree(p);
}

int dev_reserve(ig_ctx *c, DevBuf &b, size_t bytes) {
  if (bytes == 0) bytes = 16;
  if (b.p && b.bytes >= bytes) return 0;
  size_t want = bytes + bytes / 8;
  if (b.p) {
    // the stream may still use the old buffer
    if (check_hip(c, hipStreamSynchronize(c->stream), "sync before realloc")) return IG_EDEVICE;
    free_device(c, b.p);
    c->held_bytes -= b.bytes;
    b.p = nullptr;
    b.bytes = 0;
  }
  if (c->cfg.hbm_budget && c->held_bytes + want > c->cfg.hbm_budget) {
    want = bytes;
    if (c->held_bytes + want > c->cfg.hbm_budget) {
      set_error(c, IG_ENOMEM, "HBM budget exceeded: holding %llu, need %llu more, budget %llu",
                (unsigned long long)c->held_bytes, (unsigned long long)want, (unsigned long long)c->cfg.hbm_budget);
      return IG_ENOMEM;
    }
  }
  void *p = nullptr;
  if (c->cfg.alloc) {
    p = c->cfg.alloc(want, reinterpret_cast<void *>(c->stream), c->cfg.alloc_user);
    if (!p) {
      set_error(c, IG_ENOMEM, "the caller's allocator returned no memory for %llu bytes", (unsigned long long)want);
      return IG_ENOMEM;
    }
  } else {
    hipError_t e = hipMalloc(&p, want);
    if (e != hipSuccess) {
      (void)hipGetLastError();
      set_error(c, IG_ENOMEM, "hipMalloc(%llu) failed: %s", (unsigned long long)want, hipGetErrorString(e));
      return IG_ENOMEM;
    }
  }
  b.p = p;
  b.bytes = want;
  c->held_bytes += want;
  c->alloc_gen++;
  return 0;
}

void dev_release(ig_ctx *c, DevBuf &b) {
  if (b.p) {
    free_device(c, b.p);
    c->held_bytes -= b.bytes;
  }
  b.p = nullptr;
  b.bytes = 0;
}

// symbol histogram over [0, total_syms) of the stream
__global__ void k_sym_hist(const uint8_t *data, uint64_t total_syms, uint32_t bits, unsigned long long *hist) {
  __shared__ uint32_t h[256];
  h[threadIdx.x] = 0;
  __syncthreads();
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  if (bits == 8) {
    for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < total_syms / 16; i += stride) {
      const uint4 v = reinterpret_cast<const uint4 *>(data)[i];
      const uint32_t w[4] = {v.x, v.y, v.z, v.w};
      for (int j = 0; j < 4; j++)
        for (int k = 0; k < 4; k++) atomicAdd(&h[(w[j] >> (8 * k)) & 255], 1u);
    }
    for (uint64_t i = (total_syms / 16) * 16 + blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < total_syms; i += stride)
      atomicAdd(&h[data[i]], 1u);
  } else {
    for (uint64_t g = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; g < total_syms; g += stride)
      atomicAdd(&h[(data[g >> 2] >> (6 - 2 * (g & 3))) & 3], 1u);
  }
  __syncthreads();
  if (h[threadIdx.x]) atomicAdd(&hist[threadIdx.x], (unsigned long long)h[threadIdx.x]);
}

static int count_bits_for(uint64_t maxv) {
  int b = 1;
  while (b < 64 && (maxv >> b)) b++;
  return b;
}

static uint64_t windows_of(const ig_ctx *c, uint32_t n) {
  uint64_t w = 0;
  for (uint64_t i = 0; i < c->m; i++) {
    const uint64_t L = c->h_offs[i + 1] - c->h_offs[i];
    if (L >= n) w += L - n + 1;
  }
  return w;
}

int rebuild_chunks(ig_ctx *c) {
  c->alloc_gen++;   // captured passes refer to the chunk list
  std::vector<Chunk> ch;
  c->file_chunk0.assign(c->m + 1, 0);
  const uint64_t CH = c->lc.chunk_syms;
  for (uint64_t f = 0; f < c->m; f++) {
    c->file_chunk0[f] = (uint32_t)ch.size();
    const uint64_t a = c->h_offs[f], L = c->h_offs[f + 1] - a;
    for (uint64_t s = 0; s < L; s += CH) {
      Chunk k{};
      k.s0 = a + s;
      k.file = (uint32_t)f;
      k.nsym = (uint32_t)std::min<uint64_t>(CH, L - s);
      k.multi = L > CH ? 1u : 0u;
      k.fci = (uint32_t)ch.size();
      ch.push_back(k);
    }
  }
  c->file_chunk0[c->m] = (uint32_t)ch.size();
  c->nchunks = ch.size();
  std::vector<Chunk> lpt(ch);
  std::stable_sort(lpt.begin(), lpt.end(), [](const Chunk &x, const Chunk &y) { return x.nsym > y.nsym; });
  const size_t bytes = std::max<size_t>(1, ch.size()) * sizeof(Chunk);
  if (dev_reserve(c, c->chunks_file, bytes) || dev_reserve(c, c->chunks_lpt, bytes)) return IG_ENOMEM;
  if (!ch.empty()) {
    if (check_hip(c, hipMemcpyAsync(c->chunks_file.p, ch.data(), ch.size() * sizeof(Chunk), hipMemcpyHostToDevice, c->stream),
                  "chunk upload") ||
        check_hip(c, hipMemcpyAsync(c->chunks_lpt.p, lpt.data(), lpt.size() * sizeof(Chunk), hipMemcpyHostToDevice, c->stream),
                  "chunk upload") ||
        check_hip(c, hipStreamSynchronize(c->stream), "chunk upload sync"))
      return IG_EDEVICE;
  }
  return IG_OK;
}

}  // namespace ig

using namespace ig;

extern "C" {

void ig_config_default(ig_config *cfg) {
  if (!cfg) return;
  std::memset(cfg, 0, sizeof *cfg);
  cfg->symbol_bits = 8;
  cfg->freq = IG_FREQ_DOC;
  cfg->count_bits = 64;
  cfg->device = 0;
  cfg->stream = nullptr;
  cfg->hbm_budget = 0;
  cfg->flags = 0;
}

int ig_create(const ig_config *cfg, ig_ctx **out) {
  if (!out) return IG_EINVAL;
  *out = nullptr;
  if (!cfg || (cfg->symbol_bits != 8 && cfg->symbol_bits != 2) || (cfg->count_bits != 32 && cfg->count_bits != 64) ||
      (cfg->freq != IG_FREQ_DOC && cfg->freq != IG_FREQ_OCC) || (!cfg->alloc != !cfg->free))
    return IG_EINVAL;
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || cfg->device < 0 || cfg->device >= ndev) {
    (void)hipGetLastError();
    return IG_EDEVICE;
  }
  ig_ctx *c = new (std::nothrow) ig_ctx();
  if (!c) return IG_ENOMEM;
  c->cfg = *cfg;
  if (hipSetDevice(cfg->device) != hipSuccess) { delete c; return IG_EDEVICE; }
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, cfg->device) == hipSuccess && prop.multiProcessorCount > 0)
    c->n_cu = prop.multiProcessorCount;
  if (cfg->stream) {
    c->stream = reinterpret_cast<hipStream_t>(cfg->stream);
  } else {
    if (hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking) != hipSuccess) { delete c; return IG_EDEVICE; }
    c->own_stream = true;
  }
  for (auto &e : c->ev)
    if (hipEventCreate(&e) != hipSuccess) { delete c; return IG_EDEVICE; }
  if (noalloc_setup(c) != IG_OK) {
    ig_destroy(c);
    return IG_EDEVICE;
  }
  if (dev_reserve(c, c->qctr, 64) || dev_reserve(c, c->status, 64) || dev_reserve(c, c->kdev, 64) ||
      dev_reserve(c, c->zero, 64) || dev_reserve(c, c->code, 256) ||
      dev_reserve(c, c->sym_of_code, 256)) {
    ig_destroy(c);
    return IG_ENOMEM;
  }
  // a word that stays zero: the featurizing scan's "stop early" status
  if (launch_fill_u32(reinterpret_cast<uint32_t *>(c->zero.p), 16, 0, c->stream) != hipSuccess ||
      hipStreamSynchronize(c->stream) != hipSuccess) {
    ig_destroy(c);
    return IG_EDEVICE;
  }
  *out = c;
  return IG_OK;
}

void ig_destroy(ig_ctx *c) {
  if (!c) return;
  serve_teardown(c);
  if (c->stream) (void)hipStreamSynchronize(c->stream);
  for (auto &g : c->graphs)
    for (auto &x : g.exec)
      if (x) (void)hipGraphExecDestroy(x);
  c->graphs.clear();
  DevBuf *bufs[] = {&c->data, &c->offs, &c->chunks_lpt, &c->chunks_file, &c->code, &c->sym_of_code, &c->qctr,
                    &c->status, &c->kdev, &c->zero, &c->cnt, &c->rec0, &c->nrec, &c->hist1, &c->g1, &c->scan_tmp, &c->base1, &c->bend, &c->bshift, &c->dscal, &c->l1, &c->l2, &c->hist2, &c->g2, &c->fin, &c->nsegs, &c->seg0, &c->tkey_lo, &c->tkey_hi, &c->tstate, &c->sel_cid, &c->sel_cnt, &c->sel_klo,
                    &c->sel_khi, &c->tie_a, &c->tie_b, &c->sort_tmp, &c->hist, &c->selstate, &c->thist, &c->pmask};
  for (DevBuf *b : bufs) dev_release(c, *b);
  for (TableSet &t : c->ts) {
    DevBuf *tb[] = {&t.lo, &t.hi, &t.cnt, &t.le_lo, &t.le_hi, &t.map, &t.filt, &t.qmap, &t.qflag, &t.qmap2};
    for (DevBuf *b : tb) dev_release(c, *b);
  }
  for (auto &e : c->ev)
    if (e) (void)hipEventDestroy(e);
  if (c->own_stream && c->stream) (void)hipStreamDestroy(c->stream);
  delete c;
}

const char *ig_last_error(const ig_ctx *c) { return c ? c->err.c_str() : "null context"; }

int ig_load_batch(ig_ctx *c, const void *data, uint64_t data_bytes, const uint64_t *sym_offsets, uint64_t m,
                  int data_on_device) {
  if (!c) return IG_EINVAL;
  if (c->sticky) return set_error(c, IG_EDEVICE, "context has a sticky device error: %s", c->err.c_str());
  if (c->server) return set_error(c, IG_ESTATE, "serving loop is running");
  if (!sym_offsets || sym_offsets[0] != 0) return set_error(c, IG_EINVAL, "sym_offsets[0] must be 0");
  if (m >= 0xFFFFFFFEull) return set_error(c, IG_EINVAL, "too many sequences");
  for (uint64_t i = 0; i < m; i++)
    if (sym_offsets[i + 1] < sym_offsets[i]) return set_error(c, IG_EINVAL, "sym_offsets not monotone at %llu", (unsigned long long)i);
  const uint32_t b = c->cfg.symbol_bits;
  const uint64_t total = sym_offsets[m];
  const uint64_t need = (total * b + 7) / 8;
  if (data_bytes < need) return set_error(c, IG_EINVAL, "data_bytes %llu < %llu needed", (unsigned long long)data_bytes, (unsigned long long)need);
  if (need && !data) return set_error(c, IG_EINVAL, "null data");
  if (hipSetDevice(c->cfg.device) != hipSuccess) return set_error(c, IG_EDEVICE, "hipSetDevice");
  c->loaded = false;
  c->fresh = true;
  c->can_rewind = false;
  c->n_prev = 0;
  c->kept = 0;
  const uint64_t alloc = ((need + 15) & ~15ull) + 64;
  if (dev_reserve(c, c->data, alloc) || dev_reserve(c, c->offs, (m + 1) * 8)) return IG_ENOMEM;
  hipStream_t s = c->stream;
  if (need) {
    if (check_hip(c, hipMemcpyAsync(c->data.p, data, need, data_on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice, s),
                  "corpus copy"))
      return IG_EDEVICE;
  }
  // zero the tail so that 16-byte staging past the last symbol reads zeros
  if (check_hip(c, hipMemsetAsync(reinterpret_cast<uint8_t *>(c->data.p) + need, 0, alloc - need, s), "tail zero"))
    return IG_EDEVICE;
  c->h_offs.assign(sym_offsets, sym_offsets + m + 1);
  c->m = m;
  c->total_syms = total;
  c->data_bytes = need;
  if (check_hip(c, hipMemcpyAsync(c->offs.p, sym_offsets, (m + 1) * 8, hipMemcpyHostToDevice, s), "offsets copy"))
    return IG_EDEVICE;
  // alphabet actually present (the candidate space uses the compacted alphabet)
  if (dev_reserve(c, c->hist, 512 * 8)) return IG_ENOMEM;
  if (launch_fill_u64(reinterpret_cast<uint64_t *>(c->hist.p), 256, 0, s) != hipSuccess) return set_error(c, IG_EDEVICE, "fill");
  if (total) {
    uint64_t g = (total / 16 + 255) / 256;
    g = std::max<uint64_t>(1, std::min<uint64_t>(g, (uint64_t)c->n_cu * 8));
    hipLaunchKernelGGL(k_sym_hist, dim3((uint32_t)g), dim3(256), 0, s, reinterpret_cast<const uint8_t *>(c->data.p), total, b,
                       reinterpret_cast<unsigned long long *>(c->hist.p));
  }
  unsigned long long hh[256];
  if (check_hip(c, hipMemcpyAsync(hh, c->hist.p, sizeof hh, hipMemcpyDeviceToHost, s), "hist copy") ||
      check_hip(c, hipStreamSynchronize(s), "hist sync"))
    return IG_EDEVICE;
  uint32_t sigma = 0;
  std::memset(c->h_code, 0, 256);
  std::memset(c->h_sym_of_code, 0, 256);
  for (int v = 0; v < (1 << b); v++)
    if (hh[v]) {
      c->h_code[v] = (uint8_t)sigma;
      c->h_sym_of_code[sigma] = (uint8_t)v;
      sigma++;
    }
  c->sigma = sigma ? sigma : 1;
  if (check_hip(c, hipMemcpyAsync(c->code.p, c->h_code, 256, hipMemcpyHostToDevice, s), "code copy") ||
      check_hip(c, hipMemcpyAsync(c->sym_of_code.p, c->h_sym_of_code, 256, hipMemcpyHostToDevice, s), "code copy"))
    return IG_EDEVICE;
  int rc = rebuild_chunks(c);
  if (rc) return rc;
  c->loaded = true;
  return IG_OK;
}

int ig_table_info(const ig_ctx *c, uint32_t *n, uint64_t *kept) {
  if (!c) return IG_EINVAL;
  if (n) *n = c->fresh ? 0 : c->n_prev;
  if (kept) *kept = c->fresh ? 0 : c->kept;
  return IG_OK;
}

int ig_last_pass_stats(const ig_ctx *c, ig_pass_stats *st) {
  if (!c || !st) return IG_EINVAL;
  *st = c->last;
  return IG_OK;
}

int ig_pass(ig_ctx *c, uint32_t n, uint64_t k_keep) {
  if (!c) return IG_EINVAL;
  if (c->sticky) return set_error(c, IG_EDEVICE, "context has a sticky device error: %s", c->err.c_str());
  if (c->server) return set_error(c, IG_ESTATE, "serving loop is running");
  const uint32_t b = c->cfg.symbol_bits;
  if (n == 0 || (uint64_t)n * b > 128 || k_keep == 0) return set_error(c, IG_EINVAL, "bad n=%u or k_keep", n);
  if (!c->loaded) return set_error(c, IG_ESTATE, "no corpus loaded");
  const bool filtered = !(n == 1 || c->fresh);
  if (filtered && c->n_prev != n - 1) return set_error(c, IG_ESTATE, "pass %u must follow pass %u", n, n - 1);
  const uint64_t W = windows_of(c, n);
  const bool occ = c->cfg.freq == IG_FREQ_OCC;
  if (occ && c->cfg.count_bits == 32 && W >= (1ull << 32))
    return set_error(c, IG_EOVERFLOW, "W_n = %llu windows need 64-bit counts", (unsigned long long)W);
  if (hipSetDevice(c->cfg.device) != hipSuccess) return set_error(c, IG_EDEVICE, "hipSetDevice");
  hipStream_t s = c->stream;
  int mode = filtered ? MODE_FILTERED : ((uint64_t)n * b <= 26 ? MODE_DENSE : MODE_SPARSE);
  // The previous pass kept every (n-1)-gram over the alphabet (kept = sigma^(n-1)): every window
  // passes Algorithm 3's prefix test, so the pass is the unfiltered count of all n-grams, and it
  // is direct-indexed when its keys fit (no prefix lookup per window).  When it kept at least
  // half of them, the direct-indexed count of all n-grams is still cheaper than looking every
  // window's prefix up: the grams whose prefix was not kept are then made ineligible before the
  // selection (mask_prefix), which leaves the filtered pass's counts exactly.
  bool mask_prefix = false;
  if (filtered && (uint64_t)n * b <= 26) {
    uint64_t space = 1;   // sigma^(n-1) <= 2^((n-1) b) <= 2^26
    for (uint32_t j = 0; j + 1 < n; j++) space *= c->sigma;
    if (space <= c->kept) {
      mode = MODE_DENSE;
    } else if (space <= 2 * c->kept) {
      mode = MODE_DENSE;
      mask_prefix = true;
    }
  }
  const int kw = (uint64_t)n * b > 64 ? 2 : 1;
  const int count64 = occ && W >= 0xFFFFFFFFull ? 1 : 0;
  const uint32_t cbits = (uint32_t)count_bits_for(occ ? std::max<uint64_t>(W, 1) : std::max<uint64_t>(c->m, 1));
  c->last = ig_pass_stats{};
  c->last.windows = W;
  c->last.input_bytes = c->data_bytes;

  // candidate space
  uint64_t nc = 0;
  if (mode == MODE_DENSE) nc = 1ull << (n * b);
  else if (mode == MODE_FILTERED) nc = c->kept * c->sigma;
  else {
    if (!c->tkey_slots) {
      uint64_t want = std::min<uint64_t>(std::max<uint64_t>(W, 1), 1ull << 26) * 2;
      uint64_t cap = 1ull << 16;
      while (cap < want) cap <<= 1;
      c->tkey_slots = cap;
    }
    nc = c->tkey_slots;
  }
  if (nc >= 0xFFFFFFFFull) return set_error(c, IG_ENOMEM, "candidate space %llu too large", (unsigned long long)nc);

  ScanParams p;
  std::memset(&p, 0, sizeof p);   // padding too: the bytes key captured graphs
  p.data = reinterpret_cast<const uint8_t *>(c->data.p);
  p.offs = reinterpret_cast<const uint64_t *>(c->offs.p);
  p.n = n;
  p.sigma = c->sigma;
  p.code = reinterpret_cast<const uint8_t *>(c->code.p);
  p.status = reinterpret_cast<uint32_t *>(c->status.p);
  p.qctr = reinterpret_cast<uint32_t *>(c->qctr.p);
  if (mode == MODE_FILTERED) {
    const TableSet &t = c->T();
    p.filt = reinterpret_cast<const uint32_t *>(t.filt.p);
    p.filt_words = t.filt_words;
    p.filt_kind = t.filt_kind;
    p.map = reinterpret_cast<const uint32_t *>(t.map.p);
    p.mmask = t.map_mask;
    p.rank_bits = t.rank_bits;
    p.tkeys_lo = reinterpret_cast<const uint64_t *>(t.le_lo.p);   // stream forms, rank order
    p.tkeys_hi = reinterpret_cast<const uint64_t *>(t.le_hi.p);
    if (t.has_qmap) {
      p.qmap = reinterpret_cast<const uint64_t *>(t.qmap.p);
      p.qflag = reinterpret_cast<const uint32_t *>(t.qflag.p);
      p.qs = t.qs;
    } else if (t.has_qmap2) {
      p.qmap2 = reinterpret_cast<const uint64_t *>(t.qmap2.p);
      p.qflag = reinterpret_cast<const uint32_t *>(t.qflag.p);
      p.qs2 = t.qs2;
    }
  }
  p.set_cap = c->lc.set_cap;
  p.stage_bytes = (uint32_t)(((uint64_t)c->lc.chunk_syms * b / 8 + 64 + 32) & ~15ull);
  // level-1 histogram: a filtered pass knows its bucket count now (its candidate space is fixed);
  // the other passes assume the largest (256 buckets per wavefront)
  p.hist_words = occ ? 0u : (c->lc.block / 64) * (mode == MODE_FILTERED ? dedup_shape(nc, c->m).nb1 : 256u);
  // survivor rings (8 or 16 B of window per entry + a 2 B step): keys of at most 64 bits, and
  // byte Eq. 2 passes with keys of up to 128 (the scan kernel's compacted forms)
  const bool rings = mode == MODE_FILTERED && (kw == 1 || (b == 8 && !occ));
  p.qbytes = rings ? (c->lc.block / 64) * SCAN_QCAP * (8u * kw + 2u) : 0u;
  // LDS a workgroup may take: all of a CU's (less static use and slack) with one workgroup per
  // CU, half of it with two.  Two per CU is a request: a pass whose LDS does not fit half a CU
  // (with the survivor rings, when it would have them) runs one per CU.
  const size_t lds_one = 160 * 1024 - 8192, lds_two = 80 * 1024 - 1024;
  uint32_t wpc = c->lc.grid_per_cu > 1 ? 2u : 1u;
  if (wpc == 2 && scan_lds_bytes(p, mode, occ) > lds_two) wpc = 1;
  const size_t lds_budget = wpc == 2 ? lds_two : lds_one;
  // the survivor rings need thread runs of whole stage words, at most 64 windows long; without
  // them the scan resolves survivors in place, as it also does when the previous table holds
  // every (n-1)-gram over the alphabet (every window survives)
  if (p.qbytes) {
    const uint64_t spd = 32 / b, span_max = c->lc.chunk_syms + 128 / b - 1;
    if (spd * ((span_max + spd * c->lc.block - 1) / (spd * c->lc.block)) > 64) p.qbytes = 0;
  }
  if (p.qbytes) {
    uint64_t space = 1;
    for (uint32_t j = 0; j + 1 < n && space <= c->kept; j++) space *= c->sigma;
    if (space <= c->kept) p.qbytes = 0;
  }
  // A shape whose LDS does not fit this pass (say a shape tuned for a later pass, whose filter
  // image, rings and histograms differ) keeps the rings first: the LDS set is halved, down to 4096
  // entries, while they do not fit (the rings take the probes' divergence out; the set's size only
  // changes how many duplicates a chunk merges, not the result); then the rings go; then the set
  // is halved further, down to one entry per thread.  The pass's statistics report the set size.
  const uint32_t set_floor = std::min<uint32_t>(p.set_cap, std::max<uint32_t>(4096u, c->lc.block));
  while (p.qbytes && scan_lds_bytes(p, mode, occ) > lds_budget && p.set_cap > set_floor) p.set_cap >>= 1;
  if (p.qbytes && scan_lds_bytes(p, mode, occ) > lds_budget) p.qbytes = 0;
  while (scan_lds_bytes(p, mode, occ) > lds_budget && p.set_cap > c->lc.block) p.set_cap >>= 1;
  if (scan_lds_bytes(p, mode, occ) > lds_budget)
    return set_error(c, IG_EINVAL, "launch configuration needs %llu bytes of LDS",
                     (unsigned long long)scan_lds_bytes(p, mode, occ));
  // A direct-indexed pass over at most sigma^n distinct grams, no more than a chunk has windows,
  // repeats candidates within every full chunk; a set that cannot hold them twice over would fill
  // and then count (Eq. 1) or record (Eq. 2) the rest of the chunk once per window.  Its set grows
  // instead, up to twice sigma^n (at most 32768 entries), while the pass's LDS budget allows.  So
  // does an Eq. 2 pass over more grams when the pass that made the previous table recorded at
  // most one candidate per 8 windows: its chunks then repeated their (n-1)-grams, and their
  // n-grams likely repeat too.  (Over a larger space whose chunks hold mostly distinct grams, a
  // larger set only costs.)
  uint64_t grams = 1;   // sigma^n, capped
  for (uint32_t j = 0; j < n && grams <= c->lc.chunk_syms; j++) grams *= c->sigma;
  const bool repeats_prev = !occ && filtered && c->T().made_windows > 0 &&
                            c->T().made_records * 8 <= c->T().made_windows;
  if (mode == MODE_DENSE && (grams <= c->lc.chunk_syms || repeats_prev))
    while (p.set_cap < 2 * grams && p.set_cap < 32768u) {
      p.set_cap <<= 1;
      if (scan_lds_bytes(p, mode, occ) > lds_budget) {
        p.set_cap >>= 1;
        break;
      }
    }
  const uint32_t block = c->lc.block;
  const uint32_t grid = (uint32_t)c->n_cu * wpc;
  c->last.set_cap = p.set_cap;
  c->last.chunk_syms = c->lc.chunk_syms;
  c->last.block = block;
  c->last.grid = grid;

  if (check_hip(c, prepare_scan(b, kw, mode, occ, count64), "scan attributes")) return IG_EDEVICE;
  const uint64_t T = dedup_tile();
  const uint32_t nct = (uint32_t)c->nchunks;
  const bool per_file = (c->cfg.flags & IG_FLAG_PER_FILE) != 0;
  const bool use_graph = !per_file && !(c->cfg.flags & IG_FLAG_NO_GRAPH);
  uint32_t replays = 0;
  const uint64_t kmax0 = k_keep;
  for (;;) {
    // every buffer of the pass is reserved before anything is enqueued
    if (mode == MODE_SPARSE) {
      if (dev_reserve(c, c->tkey_lo, c->tkey_slots * 8) || dev_reserve(c, c->tkey_hi, c->tkey_slots * 8) ||
          dev_reserve(c, c->tstate, c->tkey_slots * 4))
        return IG_ENOMEM;
      nc = c->tkey_slots;
    }
    if (dev_reserve(c, c->cnt, nc * (count64 ? 8 : 4))) return IG_ENOMEM;
    // Eq. 2: records of every chunk, bucketed and counted once per sequence
    DedupShape sh{};
    DedupParams dp;
    std::memset(&dp, 0, sizeof dp);
    if (!occ) {
      sh = dedup_shape(nc, c->m);
      const uint64_t floor_cap = ((uint64_t)sh.nb1 + 1) * T;
      if (c->rec_cap < floor_cap && c->rec_floor) {
        c->rec_cap = (floor_cap + T - 1) / T * T;
      } else if (c->rec_cap < floor_cap) {
        const uint64_t guess = std::min<uint64_t>(std::max<uint64_t>(W, 1), std::max<uint64_t>(1ull << 22, W / 4));
        c->rec_cap = (guess + floor_cap + T - 1) / T * T;
      }
      const uint64_t cap = c->rec_cap, ntmax = cap / T;
      const uint32_t ncol = dedup_ncol(nct);
      const uint64_t n1 = (uint64_t)sh.nb1 * nct, n2 = ntmax * sh.nb2;
      const uint64_t tmp = std::max<uint64_t>(std::max<uint64_t>((uint64_t)sh.nb1 * ncol + 1, dedup_scan_tmp_entries(n2)),
                                              dedup_scan_tmp_entries((uint64_t)sh.nb1 * sh.nb2));
      if (dev_reserve(c, c->rec0, (c->total_syms + 16) * 4) || dev_reserve(c, c->nrec, std::max<uint64_t>(nct, 1) * 4) ||
          dev_reserve(c, c->hist1, std::max<uint64_t>(n1, 1) * 4) || dev_reserve(c, c->g1, std::max<uint64_t>(n1, 1) * 8) ||
          dev_reserve(c, c->scan_tmp, tmp * 8) || dev_reserve(c, c->base1, ((uint64_t)sh.nb1 + 1) * 8) ||
          dev_reserve(c, c->bend, (uint64_t)sh.nb1 * 8) || dev_reserve(c, c->bshift, (uint64_t)sh.nb1 * 8) ||
          dev_reserve(c, c->dscal, 64) ||
          dev_reserve(c, c->l1, cap * sh.w1) || dev_reserve(c, c->l2, cap * sh.w2) ||
          dev_reserve(c, c->hist2, n2 * 4) || dev_reserve(c, c->g2, (n2 + 1) * 8) ||
          dev_reserve(c, c->fin, ((uint64_t)sh.nb1 * sh.nb2 + 1) * 8) ||
          dev_reserve(c, c->nsegs, (uint64_t)sh.nb1 * sh.nb2 * 4) || dev_reserve(c, c->seg0, ((uint64_t)sh.nb1 * sh.nb2 + 1) * 8))
        return IG_ENOMEM;
      dp.chunks = reinterpret_cast<const Chunk *>(c->chunks_file.p);
      dp.nct = nct;
      dp.nb1 = sh.nb1;
      dp.nb2 = sh.nb2;
      dp.low1 = sh.low1;
      dp.low2 = sh.low2;
      dp.w1 = sh.w1;
      dp.w2 = sh.w2;
      dp.rec0 = reinterpret_cast<const uint32_t *>(c->rec0.p);
      dp.nrec = reinterpret_cast<const uint32_t *>(c->nrec.p);
      dp.hist1 = reinterpret_cast<const uint32_t *>(c->hist1.p);
      dp.g1 = reinterpret_cast<uint64_t *>(c->g1.p);
      dp.scan_tmp = reinterpret_cast<uint64_t *>(c->scan_tmp.p);
      dp.ncol = ncol;
      dp.base1 = reinterpret_cast<uint64_t *>(c->base1.p);
      dp.bend = reinterpret_cast<uint64_t *>(c->bend.p);
      dp.bshift = reinterpret_cast<uint64_t *>(c->bshift.p);
      dp.dscal = reinterpret_cast<uint64_t *>(c->dscal.p);
      dp.l1 = c->l1.p;
      dp.l2 = c->l2.p;
      dp.cap = cap;
      dp.ntmax = ntmax;
      dp.hist2 = reinterpret_cast<uint32_t *>(c->hist2.p);
      dp.g2 = reinterpret_cast<uint64_t *>(c->g2.p);
      dp.fin = reinterpret_cast<uint64_t *>(c->fin.p);
      dp.nseg = reinterpret_cast<uint32_t *>(c->nsegs.p);
      dp.seg0 = reinterpret_cast<uint64_t *>(c->seg0.p);
      dp.cnt = c->cnt.p;
      dp.nc = nc;
      dp.narrow = c->m < 65535 ? 1u : 0u;
      dp.status = reinterpret_cast<uint32_t *>(c->status.p);
      p.rec = reinterpret_cast<uint32_t *>(c->rec0.p);
      p.nrec = reinterpret_cast<uint32_t *>(c->nrec.p);
      p.hist1 = reinterpret_cast<uint32_t *>(c->hist1.p);
      p.nct = nct;
      p.low1 = sh.low1;
      p.nb1 = sh.nb1;
      p.hist_words = (c->lc.block / 64) * sh.nb1;
      p.b1bits = (uint32_t)__builtin_ctz(sh.nb1);
      dp.b1bits = p.b1bits;
      dp.b2bits = (uint32_t)__builtin_ctz(sh.nb2);
      if (check_hip(c, prepare_dedup(sh.low2), "counting attributes")) return IG_EDEVICE;
    }
    const uint64_t kmax = std::min<uint64_t>(kmax0, nc);
    int rc = select_reserve(c, nc, k_keep);
    if (rc) return rc;
    if (mask_prefix && dev_reserve(c, c->pmask, ((1ull << ((n - 1) * b)) + 31) / 32 * 4)) return IG_ENOMEM;
    TableSet &nt = c->ts[c->nxt];
    rc = index_reserve(c, nt, n, kmax);
    if (rc) return rc;
    p.cnt = c->cnt.p;
    if (mode == MODE_SPARSE) {
      p.tkey_lo = reinterpret_cast<uint64_t *>(c->tkey_lo.p);
      p.tkey_hi = reinterpret_cast<uint64_t *>(c->tkey_hi.p);
      p.tstate = reinterpret_cast<uint32_t *>(c->tstate.p);
      p.tmask = c->tkey_slots - 1;
    }
    SelectParams sp;
    std::memset(&sp, 0, sizeof sp);
    sp.cnt = c->cnt.p;
    sp.nc = nc;
    sp.count64 = count64;
    sp.mode = mode;
    sp.bits = b;
    sp.sigma = c->sigma;
    sp.sym_of_code = reinterpret_cast<const uint8_t *>(c->sym_of_code.p);
    sp.pk_lo = reinterpret_cast<const uint64_t *>(c->T().lo.p);
    sp.pk_hi = reinterpret_cast<const uint64_t *>(c->T().hi.p);
    sp.tk_lo = reinterpret_cast<const uint64_t *>(c->tkey_lo.p);
    sp.tk_hi = reinterpret_cast<const uint64_t *>(c->tkey_hi.p);
    const uint32_t sel_count_bits = count64 ? 64 : cbits;

    // the pass in four stages: clear, scan, count once per sequence (Eq. 2), select and
    // index the new table.  Timing events are recorded between the stages (outside any capture).
    auto stage = [&](int k) -> hipError_t {
      hipError_t e = hipSuccess;
      if (k == 0) {
        // counters start at zero (Eq. 2 buckets counted in segments add into them)
        e = count64 ? launch_fill_u64(reinterpret_cast<uint64_t *>(p.cnt), nc, 0, s)
                    : launch_fill_u32(reinterpret_cast<uint32_t *>(p.cnt), nc, 0, s);
        if (e == hipSuccess && mode == MODE_SPARSE) e = launch_fill_u32(p.tstate, c->tkey_slots, 0, s);
        if (e == hipSuccess) e = launch_fill_u32(p.status, 16, 0, s);
        if (e == hipSuccess) e = launch_fill_u32(p.qctr, 16, 0, s);
      } else if (k == 1) {
        if (per_file) {
          p.persistent = 0;
          p.chunks = reinterpret_cast<const Chunk *>(c->chunks_file.p);
          for (uint64_t f = 0; f < c->m && e == hipSuccess; f++) {
            const uint32_t c0 = c->file_chunk0[f], c1 = c->file_chunk0[f + 1];
            if (c1 == c0) continue;
            p.chunk_base = c0;
            p.nchunks = c1 - c0;
            e = launch_scan(p, b, kw, mode, occ, count64, c1 - c0, block, s);
          }
        } else {
          p.persistent = 1;
          p.chunks = reinterpret_cast<const Chunk *>(c->chunks_lpt.p);
          p.chunk_base = 0;
          p.nchunks = (uint32_t)c->nchunks;
          if (c->nchunks) e = launch_scan(p, b, kw, mode, occ, count64, grid, block, s);
        }
      } else if (k == 2) {
        if (!occ) e = dedup_enqueue(dp, c->n_cu, s);
      } else {
        if (mask_prefix)
          e = prefix_mask_enqueue(c, reinterpret_cast<const uint64_t *>(c->T().lo.p), c->T().kept, (n - 1) * b, p.cnt,
                                  count64, nc, b, reinterpret_cast<uint32_t *>(c->pmask.p), s);
        if (e == hipSuccess) e = select_enqueue(c, sp, k_keep, n * b, sel_count_bits);
        if (e == hipSuccess) e = index_enqueue(c, nt, kmax, select_kept_ptr(c));
      }
      return e;
    };
    const int NST = 4;

    hipError_t e = hipSuccess;
    hipGraphExec_t execs[4] = {nullptr, nullptr, nullptr, nullptr};
    if (use_graph) {
      // a captured stage bakes in every launch argument: key the graphs by their exact bytes
      if (!per_file) {
        p.persistent = 1;
        p.chunks = reinterpret_cast<const Chunk *>(c->chunks_lpt.p);
        p.chunk_base = 0;
        p.nchunks = (uint32_t)c->nchunks;
      }
      const uint64_t extra[] = {n, k_keep, kmax, nc, (uint64_t)mode, (uint64_t)kw, (uint64_t)occ, (uint64_t)count64,
                                sel_count_bits, grid, block, c->rec_cap, c->tkey_slots, c->alloc_gen,
                                (uint64_t)mask_prefix, mask_prefix ? c->T().kept : 0ull, (uint64_t)(uintptr_t)c->pmask.p,
                                nt.map_mask, nt.filt_words, nt.filt_kind,
                                (uint64_t)(uintptr_t)nt.lo.p, (uint64_t)(uintptr_t)nt.map.p, (uint64_t)(uintptr_t)nt.filt.p};
      std::string key(reinterpret_cast<const char *>(&p), sizeof p);
      key.append(reinterpret_cast<const char *>(&sp), sizeof sp);
      key.append(reinterpret_cast<const char *>(&dp), sizeof dp);
      key.append(reinterpret_cast<const char *>(extra), sizeof extra);
      for (auto &g : c->graphs)
        if (g.key == key) std::copy(g.exec, g.exec + NST, execs);
      if (!execs[0]) {
        for (int k = 0; k < NST && e == hipSuccess; k++) {
          if (k == 2 && occ) continue;   // no counting stage for Eq. 1
          hipGraph_t graph = nullptr;
          e = hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal);
          if (e == hipSuccess) {
            hipError_t e1 = stage(k);
            e = hipStreamEndCapture(s, &graph);
            if (e1 != hipSuccess) e = e1;
          }
          if (e == hipSuccess) e = hipGraphInstantiate(&execs[k], graph, nullptr, nullptr, 0);
          if (graph) (void)hipGraphDestroy(graph);
        }
        if (check_hip(c, e, "pass graph capture")) {
          for (auto &x : execs)
            if (x) (void)hipGraphExecDestroy(x);
          return IG_EDEVICE;
        }
        // up to 32 captured passes: a whole chain (n <= 31 for 2-bit symbols) replays from the cache
        if (c->graphs.size() >= 32) {
          for (auto &x : c->graphs.front().exec)
            if (x) (void)hipGraphExecDestroy(x);
          c->graphs.erase(c->graphs.begin());
        }
        ig_ctx::GraphEntry ge;
        ge.key = key;
        std::copy(execs, execs + NST, ge.exec);
        c->graphs.push_back(ge);
      }
    }
    for (int k = 0; k < NST && e == hipSuccess; k++) {
      e = hipEventRecord(c->ev[k], s);
      if (e == hipSuccess && !(k == 2 && occ)) e = use_graph ? hipGraphLaunch(execs[k], s) : stage(k);
    }
    if (e == hipSuccess) e = hipEventRecord(c->ev[NST], s);
    if (check_hip(c, e, "pass launch")) return IG_EDEVICE;
    uint32_t status = 0;
    uint64_t dsc[3] = {0, 0, 0};
    if (check_hip(c, hipMemcpyAsync(&status, p.status, 4, hipMemcpyDeviceToHost, s), "status copy") ||
        (!occ && check_hip(c, hipMemcpyAsync(dsc, c->dscal.p, sizeof dsc, hipMemcpyDeviceToHost, s), "record count copy")) ||
        check_hip(c, hipStreamSynchronize(s), "pass sync"))
      return IG_EDEVICE;
    c->last.records = dsc[0];
    if (!status) break;
    // a table overflowed: grow it and run the pass again (the result does not depend on the sizes)
    if (status & ST_TABLE_OVF) c->tkey_slots <<= 2;
    if (status == ST_REC_OVF) {   // (after a table overflow the record totals are stale)
      const uint64_t need = dsc[2] + ((uint64_t)sh.nb1 + 1) * T;
      c->rec_cap = std::max<uint64_t>(c->rec_cap * 2, (need + T - 1) / T * T);
    }
    if (++replays > 8) return set_error(c, IG_ENOMEM, "tables kept overflowing (status %u)", status);
  }
  uint64_t kept = 0, distinct = 0;
  int rc = select_read(c, &kept, &distinct);
  if (rc) return rc;
  float scan_ms = 0.f, dd_ms = 0.f, sel_ms = 0.f, total_ms = 0.f;
  (void)hipEventElapsedTime(&scan_ms, c->ev[1], c->ev[2]);
  (void)hipEventElapsedTime(&dd_ms, c->ev[2], c->ev[3]);    // once-per-sequence counting
  (void)hipEventElapsedTime(&sel_ms, c->ev[3], c->ev[4]);   // selection and index build
  (void)hipEventElapsedTime(&total_ms, c->ev[0], c->ev[4]);
  c->last.replays = replays;
  c->last.scan_ms = scan_ms;
  c->last.dedup_ms = dd_ms;
  c->last.select_ms = sel_ms;
  c->last.pass_ms = total_ms;
  c->last.distinct = distinct;
  // commit: the new table (set nxt) becomes current; the old current is kept for ig_rewind
  TableSet &nt = c->ts[c->nxt];
  nt.kept = kept;
  nt.n = n;
  nt.made_windows = W;
  nt.made_records = occ ? 0 : c->last.records;
  {
    const int old_prev = c->prev;
    c->prev = c->cur;
    c->cur = c->nxt;
    c->nxt = old_prev;
  }
  c->prev_fresh = c->fresh;
  c->can_rewind = true;
  c->kept = kept;
  c->n_prev = n;
  c->fresh = false;
  return IG_OK;
}

// Algorithm 3 as a whole: the dense first pass of Algorithm 2 generalized to b-bit symbols
// (the largest gram length whose keys fit 24 bits), z-oversampled intermediate passes, k at n.
int ig_intergrams(ig_ctx *c, uint32_t n, uint64_t k, double z) {
  if (!c) return IG_EINVAL;
  if (c->sticky) return set_error(c, IG_EDEVICE, "context has a sticky device error: %s", c->err.c_str());
  if (c->server) return set_error(c, IG_ESTATE, "serving loop is running");
  const uint32_t b = c->cfg.symbol_bits;
  if (n == 0 || (uint64_t)n * b > 128 || k == 0) return set_error(c, IG_EINVAL, "bad n=%u or k", n);
  if (!(z >= 1.0) || !std::isfinite(z)) return set_error(c, IG_EINVAL, "z must be finite and >= 1");
  const double zk = std::ceil(z * (double)k);
  if (zk >= 9223372036854775808.0) return set_error(c, IG_EINVAL, "ceil(z*k) too large");
  if (!c->loaded) return set_error(c, IG_ESTATE, "no corpus loaded");
  const uint64_t kz = (uint64_t)zk;
  uint32_t n0 = 24 / b;
  if (n0 > n) n0 = n;
  // a fresh chain: the next pass counts every n0-gram
  c->fresh = true;
  c->n_prev = 0;
  c->kept = 0;
  c->can_rewind = false;
  for (uint32_t j = n0; j <= n; j++) {
    const int rc = ig_pass(c, j, j < n ? kz : k);
    if (rc) return rc;
  }
  return IG_OK;
}

int ig_rewind(ig_ctx *c) {
  if (!c) return IG_EINVAL;
  if (c->sticky) return set_error(c, IG_EDEVICE, "context has a sticky device error: %s", c->err.c_str());
  if (c->server) return set_error(c, IG_ESTATE, "serving loop is running");
  if (!c->can_rewind) return set_error(c, IG_ESTATE, "nothing to rewind");
  std::swap(c->cur, c->prev);
  c->fresh = c->prev_fresh;
  c->n_prev = c->fresh ? 0 : c->T().n;
  c->kept = c->fresh ? 0 : c->T().kept;
  c->can_rewind = false;
  return IG_OK;
}

int ig_topk(ig_ctx *c, uint64_t k, ig_key *keys, uint64_t *counts, uint64_t *k_out) {
  if (!c) return IG_EINVAL;
  if (c->sticky) return set_error(c, IG_EDEVICE, "context has a sticky device error: %s", c->err.c_str());
  if (c->fresh || !c->loaded) return set_error(c, IG_ESTATE, "no pass has run");
  const uint64_t cnt = std::min(k, c->kept);
  if (k_out) *k_out = cnt;
  if (!cnt) return IG_OK;
  if (!keys && !counts) return IG_OK;
  std::vector<uint64_t> lo(cnt), hi(cnt);
  hipStream_t s = c->stream;
  if (keys) {
    if (check_hip(c, hipMemcpyAsync(lo.data(), c->T().lo.p, cnt * 8, hipMemcpyDeviceToHost, s), "topk copy") ||
        check_hip(c, hipMemcpyAsync(hi.data(), c->T().hi.p, cnt * 8, hipMemcpyDeviceToHost, s), "topk copy"))
      return IG_EDEVICE;
  }
  if (counts && check_hip(c, hipMemcpyAsync(counts, c->T().cnt.p, cnt * 8, hipMemcpyDeviceToHost, s), "topk copy"))
    return IG_EDEVICE;
  if (check_hip(c, hipStreamSynchronize(s), "topk sync")) return IG_EDEVICE;
  if (keys)
    for (uint64_t i = 0; i < cnt; i++) keys[i] = ig_key{lo[i], hi[i]};
  return IG_OK;
}

}  // extern "C"

namespace ig {

static int arena_full(ig_ctx *c, const Carve &a, const char *what) {
  return set_error(c, IG_EINVAL, "%s does not fit the %llu-byte no-allocation scratch (%llu bytes in use)", what,
                   (unsigned long long)a.size, (unsigned long long)a.used);
}

// Boolean rows of a batch already on the device (corpus, offsets, chunks): per-sequence bitmaps
// of kept ranks, then CSR.  Device buffers come from dev_reserve, or (arena != nullptr) are carved
// from a region the caller provides, in which case nothing is allocated.
static int featurize_rows(ig_ctx *c, const FeatBatch &in, uint64_t *indptr, int32_t *indices, uint64_t cap,
                          uint64_t *nnz_out, Carve *arena) {
  hipStream_t s = c->stream;
  const uint64_t m = in.m;
  const uint32_t words = (uint32_t)((c->kept + 31) / 32);
  DevBuf d_bm, d_nnz, d_ind, d_ptr;
  auto cleanup = [&]() {
    (void)hipStreamSynchronize(s);
    dev_release(c, d_bm); dev_release(c, d_nnz); dev_release(c, d_ind); dev_release(c, d_ptr);
  };
  const size_t bm_bytes = std::max<uint64_t>(1, m * words) * 4;
  if (arena) {
    d_bm.p = arena->take(bm_bytes);
    d_nnz.p = arena->take(std::max<uint64_t>(1, m) * 8);
    d_ptr.p = arena->take((m + 1) * 8);
    if (!d_bm.p || !d_nnz.p || !d_ptr.p) return arena_full(c, *arena, "the row bitmaps");
  } else if (dev_reserve(c, d_bm, bm_bytes) || dev_reserve(c, d_nnz, std::max<uint64_t>(1, m) * 8) ||
             dev_reserve(c, d_ptr, (m + 1) * 8)) {
    cleanup();
    return IG_ENOMEM;
  }
  FeatBatch fb = in;
  fb.bitmaps = reinterpret_cast<uint32_t *>(d_bm.p);
  fb.words = words;
  hipError_t e = launch_fill_u32(fb.bitmaps, std::max<uint64_t>(1, m * words), 0, s);
  if (e == hipSuccess && words && fb.nchunks) e = launch_featurize(c, fb, s);
  if (e == hipSuccess && words)
    e = launch_rows(fb.bitmaps, m, words, reinterpret_cast<uint64_t *>(d_nnz.p), nullptr, nullptr, 0, 1, s);
  std::vector<uint64_t> nnz(m, 0);
  if (e == hipSuccess && m && words) e = hipMemcpyAsync(nnz.data(), d_nnz.p, m * 8, hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (check_hip(c, e, "featurize")) { cleanup(); return IG_EDEVICE; }
  indptr[0] = 0;
  for (uint64_t i = 0; i < m; i++) indptr[i + 1] = indptr[i] + nnz[i];
  const uint64_t total = indptr[m];
  if (nnz_out) *nnz_out = total;
  if (total > cap) { cleanup(); return set_error(c, IG_ETRUNC, "need %llu indices", (unsigned long long)total); }
  if (total) {
    if (!indices) { cleanup(); return set_error(c, IG_EINVAL, "null indices"); }
    if (arena) {
      d_ind.p = arena->take(total * 4);
      if (!d_ind.p) return arena_full(c, *arena, "the row entries");
    } else if (dev_reserve(c, d_ind, total * 4)) {
      cleanup();
      return IG_ENOMEM;
    }
    e = hipMemcpyAsync(d_ptr.p, indptr, (m + 1) * 8, hipMemcpyHostToDevice, s);
    if (e == hipSuccess)
      e = launch_rows(fb.bitmaps, m, words, nullptr, reinterpret_cast<const uint64_t *>(d_ptr.p),
                      reinterpret_cast<int32_t *>(d_ind.p), total, 0, s);
    if (e == hipSuccess) e = hipMemcpyAsync(indices, d_ind.p, total * 4, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (check_hip(c, e, "featurize rows")) { cleanup(); return IG_EDEVICE; }
  }
  if (arena) return IG_OK;   // nothing was reserved
  cleanup();
  return IG_OK;
}

// ig_featurize's body: stage the host batch on the device (from dev_reserve, or carved from
// `arena`), then the rows.
int featurize_host(ig_ctx *c, const void *data, uint64_t data_bytes, const uint64_t *sym_offsets, uint64_t m,
                   uint64_t *indptr, int32_t *indices, uint64_t cap, uint64_t *nnz_out, Carve *arena) {
  if (!c) return IG_EINVAL;
  if (c->sticky) return set_error(c, IG_EDEVICE, "context has a sticky device error: %s", c->err.c_str());
  if (c->server) return set_error(c, IG_ESTATE, "serving loop is running");
  if (c->fresh || !c->loaded) return set_error(c, IG_ESTATE, "no pass has run");
  if (!sym_offsets || sym_offsets[0] != 0 || !indptr) return set_error(c, IG_EINVAL, "bad offsets");
  for (uint64_t i = 0; i < m; i++)
    if (sym_offsets[i + 1] < sym_offsets[i]) return set_error(c, IG_EINVAL, "sym_offsets not monotone");
  const uint32_t b = c->cfg.symbol_bits;
  const uint64_t need = (sym_offsets[m] * b + 7) / 8;
  if (data_bytes < need || (need && !data)) return set_error(c, IG_EINVAL, "data too small");
  if (hipSetDevice(c->cfg.device) != hipSuccess) return set_error(c, IG_EDEVICE, "hipSetDevice");
  hipStream_t s = c->stream;
  // chunks of the batch
  std::vector<Chunk> ch;
  const uint64_t CH = c->lc.chunk_syms;
  for (uint64_t f = 0; f < m; f++) {
    const uint64_t a = sym_offsets[f], L = sym_offsets[f + 1] - a;
    for (uint64_t q = 0; q < L; q += CH) ch.push_back(Chunk{a + q, (uint32_t)f, (uint32_t)std::min<uint64_t>(CH, L - q), L > CH ? 1u : 0u, 0u});
  }
  DevBuf d_data, d_offs, d_ch;
  auto cleanup = [&]() {
    (void)hipStreamSynchronize(s);
    dev_release(c, d_data); dev_release(c, d_offs); dev_release(c, d_ch);
  };
  // whole 16-byte words plus 64 zero bytes, so that staging past the last symbol reads zeros
  const uint64_t alloc = ((need + 15) & ~15ull) + 64;
  const size_t ch_bytes = std::max<size_t>(1, ch.size()) * sizeof(Chunk);
  if (arena) {
    d_data.p = arena->take(alloc);
    d_offs.p = arena->take((m + 1) * 8);
    d_ch.p = arena->take(ch_bytes);
    if (!d_data.p || !d_offs.p || !d_ch.p) return arena_full(c, *arena, "the batch");
  } else if (dev_reserve(c, d_data, alloc) || dev_reserve(c, d_offs, (m + 1) * 8) || dev_reserve(c, d_ch, ch_bytes)) {
    cleanup();
    return IG_ENOMEM;
  }
  // the zero tail by a fill kernel (the region's last whole word onward; the copy rewrites its head)
  const uint64_t tail0 = need & ~3ull;
  hipError_t e = launch_fill_u32(reinterpret_cast<uint32_t *>(reinterpret_cast<uint8_t *>(d_data.p) + tail0),
                                 (alloc - tail0) / 4, 0, s);
  if (e == hipSuccess && need) e = hipMemcpyAsync(d_data.p, data, need, hipMemcpyHostToDevice, s);
  if (e == hipSuccess) e = hipMemcpyAsync(d_offs.p, sym_offsets, (m + 1) * 8, hipMemcpyHostToDevice, s);
  if (e == hipSuccess && !ch.empty()) e = hipMemcpyAsync(d_ch.p, ch.data(), ch.size() * sizeof(Chunk), hipMemcpyHostToDevice, s);
  if (check_hip(c, e, "featurize staging")) { cleanup(); return IG_EDEVICE; }
  FeatBatch fb{reinterpret_cast<const uint8_t *>(d_data.p), reinterpret_cast<const uint64_t *>(d_offs.p), m,
               reinterpret_cast<const Chunk *>(d_ch.p), (uint32_t)ch.size(), nullptr, 0};
  const int rc = featurize_rows(c, fb, indptr, indices, cap, nnz_out, arena);
  if (arena) {
    (void)hipStreamSynchronize(s);
    return rc;
  }
  cleanup();
  return rc;
}

}  // namespace ig

extern "C" {

int ig_featurize(ig_ctx *c, const void *data, uint64_t data_bytes, const uint64_t *sym_offsets, uint64_t m,
                 uint64_t *indptr, int32_t *indices, uint64_t cap, uint64_t *nnz_out) {
  return featurize_host(c, data, data_bytes, sym_offsets, m, indptr, indices, cap, nnz_out, nullptr);
}

int ig_featurize_loaded(ig_ctx *c, uint64_t *indptr, int32_t *indices, uint64_t cap, uint64_t *nnz_out) {
  if (!c) return IG_EINVAL;
  if (c->sticky) return set_error(c, IG_EDEVICE, "context has a sticky device error: %s", c->err.c_str());
  if (c->server) return set_error(c, IG_ESTATE, "serving loop is running");
  if (c->fresh || !c->loaded) return set_error(c, IG_ESTATE, "no pass has run");
  if (!indptr) return set_error(c, IG_EINVAL, "null indptr");
  if (hipSetDevice(c->cfg.device) != hipSuccess) return set_error(c, IG_EDEVICE, "hipSetDevice");
  // the corpus, its offsets and its chunk list are resident since the load
  FeatBatch fb{reinterpret_cast<const uint8_t *>(c->data.p), reinterpret_cast<const uint64_t *>(c->offs.p), c->m,
               reinterpret_cast<const Chunk *>(c->chunks_file.p), (uint32_t)c->nchunks, nullptr, 0};
  return featurize_rows(c, fb, indptr, indices, cap, nnz_out, nullptr);
}

}  // extern "C"
