// Deterministic selection of the k_keep best candidates (Algorithm 3's
// zk-argmax), in the total order (count desc, key asc), and the sort of the
// winners in that order.
//
//  1. Radix select on the count, most significant 8-bit digit first, over the
//     dense count array: each level histograms the entries whose higher digits
//     match the prefix chosen so far (LDS histograms, merged with coalesced
//     atomics) and one workgroup picks the digit.  The result is the threshold
//     count T and how many entries with count T are still needed.
//  2. Entries with count > T are kept; entries with count T are ties.
//  3. If there are more ties than needed, radix select on the key (most
//     significant digit first, smallest wins) among the ties, compacting the
//     candidate list level by level.
//  4. LSD radix sort of the kept entries: key digits first, then the digits of
//     (max - count), with a stable scatter (ballot-based ranking per wave).
// Every kernel reads its element counts from device memory, so the sequence of
// launches is fixed for a given (k_keep, key bits, count bits) and can be
// captured in a graph.
#include "ig_internal.h"

namespace ig {

struct SelState {
  unsigned long long total, kprime, need, prefix, T;
  unsigned long long nsel, ntie, ncand, nnext;
  unsigned int done, bstar, cur, pad;
};

__device__ __forceinline__ void key_of(const SelectParams &sp, uint32_t cid, uint64_t &lo, uint64_t &hi) {
  if (sp.mode == MODE_DENSE) {
    lo = cid;
    hi = 0;
  } else if (sp.mode == MODE_FILTERED) {
    const uint32_t r = cid / sp.sigma, code = cid - r * sp.sigma;
    const uint64_t plo = sp.pk_lo[r], phi = sp.pk_hi[r];
    const uint32_t B = sp.bits;
    hi = (phi << B) | (plo >> (64 - B));
    lo = (plo << B) | sp.sym_of_code[code];
  } else {
    lo = sp.tk_lo[cid];
    hi = sp.tk_hi[cid];
  }
}

__device__ __forceinline__ uint64_t load_cnt(const void *cnt, int c64, uint64_t i) {
  return c64 ? reinterpret_cast<const uint64_t *>(cnt)[i] : (uint64_t)reinterpret_cast<const uint32_t *>(cnt)[i];
}

// wave-aggregated append: returns the slot for this lane (valid only if pred)
__device__ __forceinline__ unsigned long long wave_append(unsigned long long *ctr, bool pred) {
  const unsigned long long mask = __ballot(pred);
  if (!mask) return 0;
  const uint32_t lane = threadIdx.x & 63;
  const int leader = __ffsll((long long)mask) - 1;
  unsigned long long base = 0;
  if ((int)lane == leader) base = atomicAdd(ctr, (unsigned long long)__popcll(mask));
  base = __shfl(base, leader);
  return base + __popcll(mask & ((1ull << lane) - 1));
}

__global__ void k_sel_reset(SelState *st) {
  if (threadIdx.x == 0) {
    SelState z{};
    *st = z;
  }
}

__global__ void k_cnt_hist(SelectParams sp, uint32_t shift, const SelState *st, unsigned long long *hist) {
  __shared__ uint32_t h[256];
  h[threadIdx.x] = 0;
  __syncthreads();
  const uint64_t pre_hi = (shift + 8 >= 64) ? 0 : (st->prefix >> (shift + 8));
  for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < sp.nc; i += (uint64_t)gridDim.x * blockDim.x) {
    const uint64_t c = load_cnt(sp.cnt, sp.count64, i);
    if (!c) continue;
    if (shift + 8 < 64 && (c >> (shift + 8)) != pre_hi) continue;
    atomicAdd(&h[(c >> shift) & 255], 1u);
  }
  __syncthreads();
  if (h[threadIdx.x]) atomicAdd(&hist[threadIdx.x], (unsigned long long)h[threadIdx.x]);
}

// pick the count digit: largest b with (#above b) < need <= (#above b) + hist[b]
__global__ void k_cnt_pick(SelState *st, unsigned long long *hist, uint32_t shift, int level0, uint64_t k_keep) {
  if (threadIdx.x == 0) {
    if (level0) {
      unsigned long long tot = 0;
      for (int d = 0; d < 256; d++) tot += hist[d];
      st->total = tot;
      st->kprime = tot < k_keep ? tot : k_keep;
      st->need = st->kprime;
    }
    if (st->kprime) {
      unsigned long long above = 0;
      int b = 255;
      for (; b > 0; b--) {
        if (above + hist[b] >= st->need) break;
        above += hist[b];
      }
      st->need -= above;
      st->prefix |= (unsigned long long)b << shift;
    }
    if (shift == 0) st->T = st->prefix;
  }
  __syncthreads();
  hist[threadIdx.x] = 0;
}

// Candidates above the threshold T go to sel_*, those equal to T to tie.  Each workgroup takes a
// contiguous range: it counts its hits per thread, scans the counts in LDS, reserves its output
// with one device atomic per list, then re-reads the range and writes at the scanned positions.
// (Output order is irrelevant: the selection is sorted by count and key afterwards.)
__global__ void __launch_bounds__(256) k_collect(SelectParams sp, SelState *st, uint32_t *sel_cid,
                                                 unsigned long long *sel_cnt, uint32_t *tie) {
  __shared__ uint32_t s_gt[256], s_eq[256];
  __shared__ unsigned long long s_base[2];
  if (!st->kprime) return;
  const uint32_t tid = threadIdx.x, bs = blockDim.x;
  const uint64_t T = st->T;
  const uint64_t per = ((sp.nc + gridDim.x - 1) / gridDim.x + bs - 1) / bs * bs;
  const uint64_t lo = (uint64_t)blockIdx.x * per, hi = lo + per < sp.nc ? lo + per : sp.nc;
  uint32_t ngt = 0, neq = 0;
  for (uint64_t i = lo + tid; i < hi; i += bs) {
    const uint64_t c = load_cnt(sp.cnt, sp.count64, i);
    ngt += c > T ? 1u : 0u;
    neq += (c != 0 && c == T) ? 1u : 0u;
  }
  s_gt[tid] = ngt;
  s_eq[tid] = neq;
  __syncthreads();
  // inclusive scan over the threads (Hillis-Steele in LDS)
  for (uint32_t off = 1; off < bs; off <<= 1) {
    const uint32_t a = tid >= off ? s_gt[tid - off] : 0u, e = tid >= off ? s_eq[tid - off] : 0u;
    __syncthreads();
    s_gt[tid] += a;
    s_eq[tid] += e;
    __syncthreads();
  }
  if (tid == 0) {
    s_base[0] = s_gt[bs - 1] ? atomicAdd(&st->nsel, (unsigned long long)s_gt[bs - 1]) : 0ull;
    s_base[1] = s_eq[bs - 1] ? atomicAdd(&st->ntie, (unsigned long long)s_eq[bs - 1]) : 0ull;
  }
  __syncthreads();
  if (s_gt[bs - 1] == 0 && s_eq[bs - 1] == 0) return;
  unsigned long long pg = s_base[0] + s_gt[tid] - ngt, pe = s_base[1] + s_eq[tid] - neq;
  for (uint64_t i = lo + tid; i < hi && (ngt | neq); i += bs) {
    const uint64_t c = load_cnt(sp.cnt, sp.count64, i);
    if (c > T) {
      sel_cid[pg] = (uint32_t)i;
      sel_cnt[pg] = c;
      pg++;
      ngt--;
    } else if (c != 0 && c == T) {
      tie[pe++] = (uint32_t)i;
      neq--;
    }
  }
}

__global__ void k_tie_init(SelState *st) {
  if (threadIdx.x == 0) {
    st->ncand = st->ntie;
    st->cur = 0;
    st->done = (st->kprime == 0 || st->need == st->ntie || st->need == 0) ? 1u : 0u;
  }
}

__device__ __forceinline__ uint32_t key_digit(uint64_t lo, uint64_t hi, uint32_t shift) {
  return shift >= 64 ? (uint32_t)((hi >> (shift - 64)) & 255) : (uint32_t)((lo >> shift) & 255);
}

__global__ void k_key_hist(SelectParams sp, uint32_t shift, const SelState *st, const uint32_t *ta, const uint32_t *tb,
                           unsigned long long *hist) {
  if (st->done) return;
  __shared__ uint32_t h[256];
  h[threadIdx.x] = 0;
  __syncthreads();
  const uint32_t *src = st->cur ? tb : ta;
  for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < st->ncand; i += (uint64_t)gridDim.x * blockDim.x) {
    uint64_t lo, hi;
    key_of(sp, src[i], lo, hi);
    atomicAdd(&h[key_digit(lo, hi, shift)], 1u);
  }
  __syncthreads();
  if (h[threadIdx.x]) atomicAdd(&hist[threadIdx.x], (unsigned long long)h[threadIdx.x]);
}

// smallest b with (#below b) < need <= (#below b) + hist[b]
__global__ void k_key_pick(SelState *st, unsigned long long *hist) {
  if (threadIdx.x == 0 && !st->done) {
    unsigned long long below = 0;
    int b = 0;
    for (; b < 255; b++) {
      if (below + hist[b] >= st->need) break;
      below += hist[b];
    }
    st->bstar = (unsigned)b;
    st->nnext = 0;
  }
  __syncthreads();
  hist[threadIdx.x] = 0;
}

__global__ void k_key_route(SelectParams sp, uint32_t shift, SelState *st, uint32_t *ta, uint32_t *tb,
                            uint32_t *sel_cid, unsigned long long *sel_cnt) {
  if (st->done) return;
  const uint32_t *src = st->cur ? tb : ta;
  uint32_t *dst = st->cur ? ta : tb;
  const uint32_t bstar = st->bstar;
  const uint64_t T = st->T;
  const uint64_t nr = (st->ncand + 63) & ~63ull;
  for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < nr; i += (uint64_t)gridDim.x * blockDim.x) {
    uint32_t cid = 0, d = 256;
    if (i < st->ncand) {
      uint64_t lo, hi;
      cid = src[i];
      key_of(sp, cid, lo, hi);
      d = key_digit(lo, hi, shift);
    }
    const bool take = d < bstar, keep = d == bstar;
    const unsigned long long a = wave_append(&st->nsel, take);
    if (take) { sel_cid[a] = cid; sel_cnt[a] = T; }
    const unsigned long long b = wave_append(&st->nnext, keep);
    if (keep) dst[b] = cid;
  }
}

__global__ void k_key_next(SelState *st, unsigned long long *hist) {
  if (threadIdx.x == 0 && !st->done) {
    unsigned long long below = 0;
    for (uint32_t b = 0; b < st->bstar; b++) below += hist[256 + b];   // histogram copy kept at hist[256..]
    st->need -= below;
    st->ncand = st->nnext;
    st->cur ^= 1u;
    if (st->need == st->ncand || st->need == 0) st->done = 1;
  }
}

// keep a copy of the level histogram (k_key_pick clears the working one)
__global__ void k_hist_copy(unsigned long long *hist, const SelState *st) {
  if (!st->done) hist[256 + threadIdx.x] = hist[threadIdx.x];
}

__global__ void k_tie_final(SelState *st, const uint32_t *ta, const uint32_t *tb, uint32_t *sel_cid,
                            unsigned long long *sel_cnt) {
  if (!st->kprime || st->need == 0) return;
  const uint32_t *src = st->cur ? tb : ta;
  const uint64_t n = st->ncand;
  const uint64_t base = st->nsel;   // no other appends run concurrently
  for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x) {
    sel_cid[base + i] = src[i];
    sel_cnt[base + i] = st->T;
  }
}

__global__ void k_materialize(SelectParams sp, const SelState *st, const uint32_t *sel_cid, uint64_t *klo,
                              uint64_t *khi) {
  for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < st->kprime; i += (uint64_t)gridDim.x * blockDim.x) {
    uint64_t lo, hi;
    key_of(sp, sel_cid[i], lo, hi);
    klo[i] = lo;
    khi[i] = hi;
  }
}

// ---------------------------------------------------------------- LSD radix sort of the kept entries
static constexpr uint32_t SORT_ROUNDS = 16, SORT_TILE = 64 * SORT_ROUNDS;

__device__ __forceinline__ uint32_t sort_digit(uint64_t lo, uint64_t hi, uint64_t c, uint32_t pass, uint32_t klev,
                                               uint64_t cmax) {
  if (pass < klev) return key_digit(lo, hi, 8 * pass);
  return (uint32_t)(((cmax - c) >> (8 * (pass - klev))) & 255);
}

__global__ void __launch_bounds__(64) k_sort_hist(const SelState *st, const uint64_t *klo, const uint64_t *khi,
                                                  const unsigned long long *cnt, uint32_t pass, uint32_t klev,
                                                  uint64_t cmax, uint32_t *hist, uint32_t ntiles) {
  __shared__ uint32_t h[256];
  const uint32_t lane = threadIdx.x, tile = blockIdx.x;
  for (uint32_t d = lane; d < 256; d += 64) h[d] = 0;
  __syncthreads();
  const uint64_t n = st->kprime;
  for (uint32_t r = 0; r < SORT_ROUNDS; r++) {
    const uint64_t i = (uint64_t)tile * SORT_TILE + r * 64 + lane;
    if (i < n) atomicAdd(&h[sort_digit(klo[i], khi[i], cnt[i], pass, klev, cmax)], 1u);
  }
  __syncthreads();
  for (uint32_t d = lane; d < 256; d += 64) hist[(uint64_t)d * ntiles + tile] = h[d];
}

// exclusive scan of hist[256 * ntiles] (digit-major) in one workgroup
__global__ void __launch_bounds__(1024) k_sort_scan(uint32_t *hist, uint64_t len) {
  wg_exclusive_scan<uint32_t>(hist, len, nullptr);
}

__global__ void __launch_bounds__(64) k_sort_scatter(const SelState *st, const uint64_t *klo, const uint64_t *khi,
                                                     const unsigned long long *cnt, uint64_t *olo, uint64_t *ohi,
                                                     unsigned long long *ocnt, uint32_t pass, uint32_t klev,
                                                     uint64_t cmax, const uint32_t *hist, uint32_t ntiles) {
  __shared__ uint32_t base[256];
  const uint32_t lane = threadIdx.x, tile = blockIdx.x;
  for (uint32_t d = lane; d < 256; d += 64) base[d] = hist[(uint64_t)d * ntiles + tile];
  __syncthreads();
  const uint64_t n = st->kprime;
  const unsigned long long lt = (1ull << lane) - 1;
  for (uint32_t r = 0; r < SORT_ROUNDS; r++) {
    const uint64_t i = (uint64_t)tile * SORT_TILE + r * 64 + lane;
    const bool valid = i < n;
    uint64_t lo = 0, hi = 0;
    unsigned long long c = 0;
    uint32_t d = 0;
    if (valid) {
      lo = klo[i];
      hi = khi[i];
      c = cnt[i];
      d = sort_digit(lo, hi, c, pass, klev, cmax);
    }
    unsigned long long eq = __ballot(valid);
    for (uint32_t bit = 0; bit < 8; bit++) {
      const unsigned long long b = __ballot((d >> bit) & 1u);
      eq &= ((d >> bit) & 1u) ? b : ~b;
    }
    const uint32_t rank = (uint32_t)__popcll(eq & lt);
    if (valid) {
      const uint32_t pos = base[d] + rank;
      olo[pos] = lo;
      ohi[pos] = hi;
      ocnt[pos] = c;
    }
    __syncthreads();
    if (valid && (eq >> lane) == 1ull) base[d] += (uint32_t)__popcll(eq);   // highest lane of the group
    __syncthreads();
  }
}

__global__ void k_copy_out(const SelState *st, const uint64_t *klo, const uint64_t *khi, const unsigned long long *cnt,
                           uint64_t *tlo, uint64_t *thi, uint64_t *tcnt) {
  for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < st->kprime; i += (uint64_t)gridDim.x * blockDim.x) {
    tlo[i] = klo[i];
    thi[i] = khi[i];
    tcnt[i] = cnt[i];
  }
}

static uint32_t grid_for(uint64_t n, uint32_t block, uint32_t cap) {
  uint64_t g = (n + block - 1) / block;
  if (g < 1) g = 1;
  if (g > cap) g = cap;
  return (uint32_t)g;
}

// A pass run as the direct-indexed count of every n-gram although the previous table kept only
// part of the (n-1)-grams (Algorithm 3's prefix test then passes most windows): the grams whose
// prefix was not kept are made ineligible (count 0) before the selection, which leaves exactly
// the counts of the filtered pass.  bits: one bit per (n-1)-gram key, set for the kept ones.
__global__ void k_prefix_bits(const uint64_t *keys, uint64_t kept, uint32_t *bits) {
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < kept; i += (uint64_t)gridDim.x * blockDim.x) {
    const uint64_t k = keys[i];
    atomicOr(bits + (k >> 5), 1u << (k & 31));
  }
}
__global__ void k_prefix_mask(void *cnt, int c64, uint64_t nc, uint32_t b, const uint32_t *bits) {
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < nc; i += (uint64_t)gridDim.x * blockDim.x) {
    const uint64_t pre = i >> b;
    if ((bits[pre >> 5] >> (pre & 31)) & 1u) continue;
    if (c64) {
      uint64_t *q = reinterpret_cast<uint64_t *>(cnt) + i;
      if (*q) *q = 0;
    } else {
      uint32_t *q = reinterpret_cast<uint32_t *>(cnt) + i;
      if (*q) *q = 0;
    }
  }
}

hipError_t prefix_mask_enqueue(ig_ctx *c, const uint64_t *prev_keys, uint64_t prev_kept, uint32_t prefix_bits, void *cnt,
                               int c64, uint64_t nc, uint32_t b, uint32_t *bits, hipStream_t s) {
  const uint64_t words = ((1ull << prefix_bits) + 31) / 32;
  hipError_t e = launch_fill_u32(bits, words, 0, s);
  if (e != hipSuccess) return e;
  const uint32_t gmax = (uint32_t)c->n_cu * 8;
  if (prev_kept) {
    const uint32_t g = (uint32_t)std::min<uint64_t>(gmax, (prev_kept + 255) / 256);
    hipLaunchKernelGGL(k_prefix_bits, dim3(g), dim3(256), 0, s, prev_keys, prev_kept, bits);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  const uint32_t g = (uint32_t)std::min<uint64_t>(gmax, (nc + 255) / 256);
  hipLaunchKernelGGL(k_prefix_mask, dim3(g ? g : 1), dim3(256), 0, s, cnt, c64, nc, b, (const uint32_t *)bits);
  return hipGetLastError();
}

int select_reserve(ig_ctx *c, uint64_t nc, uint64_t k_keep) {
  const uint64_t K = k_keep < nc ? k_keep : nc;
  const uint64_t Kc = K ? K : 1;
  const uint64_t ncc = nc ? nc : 1;
  const uint32_t ntiles = (uint32_t)((Kc + SORT_TILE - 1) / SORT_TILE);
  if (dev_reserve(c, c->selstate, sizeof(SelState)) || dev_reserve(c, c->hist, 512 * 8) ||
      dev_reserve(c, c->sel_cid, Kc * 4) || dev_reserve(c, c->sel_cnt, Kc * 8) ||
      dev_reserve(c, c->sel_klo, 2 * Kc * 8) || dev_reserve(c, c->sel_khi, 2 * Kc * 8) ||
      dev_reserve(c, c->sort_tmp, Kc * 8) || dev_reserve(c, c->tie_a, ncc * 4) || dev_reserve(c, c->tie_b, ncc * 4) ||
      dev_reserve(c, c->thist, (uint64_t)256 * ntiles * 4) || dev_reserve(c, c->ts[c->nxt].lo, Kc * 8) ||
      dev_reserve(c, c->ts[c->nxt].hi, Kc * 8) || dev_reserve(c, c->ts[c->nxt].cnt, Kc * 8))
    return IG_ENOMEM;
  return IG_OK;
}

const unsigned long long *select_kept_ptr(ig_ctx *c) {
  return &reinterpret_cast<const SelState *>(c->selstate.p)->kprime;
}

int select_read(ig_ctx *c, uint64_t *kept, uint64_t *distinct) {
  SelState hs;
  if (check_hip(c, hipMemcpyAsync(&hs, c->selstate.p, sizeof hs, hipMemcpyDeviceToHost, c->stream), "select state copy") ||
      check_hip(c, hipStreamSynchronize(c->stream), "select sync"))
    return IG_EDEVICE;
  *kept = hs.kprime;
  *distinct = hs.total;
  return IG_OK;
}

// Enqueue the selection (no host synchronization; buffers from select_reserve).
hipError_t select_enqueue(ig_ctx *c, const SelectParams &sp, uint64_t k_keep, uint32_t key_bits, uint32_t count_bits) {
  hipStream_t s = c->stream;
  const uint64_t K = k_keep < sp.nc ? k_keep : sp.nc;
  const uint64_t Kc = K ? K : 1;
  const uint32_t ntiles = (uint32_t)((Kc + SORT_TILE - 1) / SORT_TILE);
  SelState *st = reinterpret_cast<SelState *>(c->selstate.p);
  unsigned long long *hist = reinterpret_cast<unsigned long long *>(c->hist.p);
  uint32_t *sel_cid = reinterpret_cast<uint32_t *>(c->sel_cid.p);
  unsigned long long *sel_cnt = reinterpret_cast<unsigned long long *>(c->sel_cnt.p);
  uint32_t *ta = reinterpret_cast<uint32_t *>(c->tie_a.p), *tb = reinterpret_cast<uint32_t *>(c->tie_b.p);
  uint32_t *thist = reinterpret_cast<uint32_t *>(c->thist.p);
  const uint32_t G = (uint32_t)c->n_cu * 4;

  hipLaunchKernelGGL(k_sel_reset, dim3(1), dim3(1), 0, s, st);
  hipError_t e = launch_fill_u64(reinterpret_cast<uint64_t *>(hist), 512, 0, s);
  if (e != hipSuccess) return e;
  const uint32_t cl = (count_bits + 7) / 8;
  for (int lev = (int)cl - 1; lev >= 0; lev--) {
    const uint32_t shift = 8u * (uint32_t)lev;
    hipLaunchKernelGGL(k_cnt_hist, dim3(grid_for(sp.nc, 256, G)), dim3(256), 0, s, sp, shift, st, hist);
    hipLaunchKernelGGL(k_cnt_pick, dim3(1), dim3(256), 0, s, st, hist, shift, lev == (int)cl - 1 ? 1 : 0, K);
  }
  hipLaunchKernelGGL(k_collect, dim3(grid_for(sp.nc, 256, G)), dim3(256), 0, s, sp, st, sel_cid, sel_cnt, ta);
  hipLaunchKernelGGL(k_tie_init, dim3(1), dim3(1), 0, s, st);
  const uint32_t kl = (key_bits + 7) / 8;
  for (int lev = (int)kl - 1; lev >= 0; lev--) {
    const uint32_t shift = 8u * (uint32_t)lev;
    const uint32_t gt = grid_for(sp.nc, 256, G);
    hipLaunchKernelGGL(k_key_hist, dim3(gt), dim3(256), 0, s, sp, shift, st, ta, tb, hist);
    hipLaunchKernelGGL(k_hist_copy, dim3(1), dim3(256), 0, s, hist, st);
    hipLaunchKernelGGL(k_key_pick, dim3(1), dim3(256), 0, s, st, hist);
    hipLaunchKernelGGL(k_key_route, dim3(gt), dim3(256), 0, s, sp, shift, st, ta, tb, sel_cid, sel_cnt);
    hipLaunchKernelGGL(k_key_next, dim3(1), dim3(1), 0, s, st, hist);
  }
  hipLaunchKernelGGL(k_tie_final, dim3(grid_for(sp.nc, 256, G)), dim3(256), 0, s, st, ta, tb, sel_cid, sel_cnt);

  uint64_t *klo = reinterpret_cast<uint64_t *>(c->sel_klo.p), *khi = reinterpret_cast<uint64_t *>(c->sel_khi.p);
  unsigned long long *cnt2 = reinterpret_cast<unsigned long long *>(c->sort_tmp.p);
  hipLaunchKernelGGL(k_materialize, dim3(grid_for(Kc, 256, G)), dim3(256), 0, s, sp, st, sel_cid, klo, khi);
  const uint64_t cmax = count_bits >= 64 ? ~0ull : ((1ull << count_bits) - 1);
  const uint32_t npass = kl + cl;
  // ping-pong between (klo, khi, sel_cnt) and (klo + Kc, khi + Kc, cnt2)
  uint64_t *alo = klo, *ahi = khi, *blo = klo + Kc, *bhi = khi + Kc;
  unsigned long long *acnt = sel_cnt, *bcnt = cnt2;
  for (uint32_t pass = 0; pass < npass; pass++) {
    hipLaunchKernelGGL(k_sort_hist, dim3(ntiles), dim3(64), 0, s, st, alo, ahi, acnt, pass, kl, cmax, thist, ntiles);
    hipLaunchKernelGGL(k_sort_scan, dim3(1), dim3(1024), 0, s, thist, (uint64_t)256 * ntiles);
    hipLaunchKernelGGL(k_sort_scatter, dim3(ntiles), dim3(64), 0, s, st, alo, ahi, acnt, blo, bhi, bcnt, pass, kl, cmax,
                       thist, ntiles);
    std::swap(alo, blo);
    std::swap(ahi, bhi);
    std::swap(acnt, bcnt);
  }
  hipLaunchKernelGGL(k_copy_out, dim3(grid_for(Kc, 256, G)), dim3(256), 0, s, st, alo, ahi, acnt,
                     reinterpret_cast<uint64_t *>(c->ts[c->nxt].lo.p), reinterpret_cast<uint64_t *>(c->ts[c->nxt].hi.p),
                     reinterpret_cast<uint64_t *>(c->ts[c->nxt].cnt.p));
  return hipGetLastError();
}

}  // namespace ig
