// Once-per-sequence counting (Eq. 2) without device-scope atomics.
//
// The scan leaves, for every chunk, its chunk-distinct candidate ids ("records")
// in a slab at the chunk's own window positions, and a histogram of their top
// b1 bits.  Counting the sequences that contain each candidate then needs the
// duplicates of (sequence, candidate) across the chunks of one sequence
// removed.  Records are laid out in file order of the chunks, so that every
// candidate range below keeps the records of one sequence together:
//
//   1. exclusive scan of the level-1 histograms ([bucket][chunk], chunk in file
//      order) and per-bucket bases, each bucket padded to a whole number of
//      tiles;
//   2. gather: each chunk's records go to its run in its level-1 bucket, tagged
//      with the sequence id (runs of one bucket follow the file order);
//   3. a stable split of every level-1 bucket on the next b2 bits (per-tile
//      histograms, a scan, and a scatter ranked with wavefront ballots, so the
//      order inside each final bucket is still the file order);
//   4. one workgroup per final bucket of at most 2^low2 candidates counts, in
//      LDS, the distinct sequences of each candidate: a record is new unless
//      the previous record of its candidate came from the same sequence (the
//      sequence ids along a bucket never decrease), with a small per-round hash
//      resolving duplicates that arrive in the same round.  The counts are then
//      written with plain stores: every candidate belongs to exactly one bucket.
//
// Every kernel takes its sizes from device memory (record totals are only known
// after the scan) and loops over fixed grids, so the sequence of launches can
// be captured in a graph.  If the records exceed the reserved capacity, the
// bases kernel raises a status bit, the later kernels return at once, and the
// pass is replayed with larger buffers.
#include "ig_internal.h"

namespace ig {

static constexpr uint32_t TILE = 4096;          // records per level-2 tile
static constexpr uint32_t SCAN_SEG = 4096;      // elements per block of the generic scan
static constexpr uint32_t P2_BLOCK = 512;       // threads of the level-2 kernels
static constexpr uint32_t CNT_BLOCK = 512;      // threads of the count kernel
static constexpr uint32_t CNT_HASH = 1024;      // per-round pair hash slots (>= 2 x CNT_BLOCK)

template <typename R> struct Rec;
template <> struct Rec<uint32_t> {
  __device__ __forceinline__ static uint32_t pack(uint32_t file, uint32_t cl, uint32_t low) { return (file << low) | cl; }
  __device__ __forceinline__ static uint32_t file(uint32_t r, uint32_t low) { return r >> low; }
  __device__ __forceinline__ static uint32_t cl(uint32_t r, uint32_t low) { return low >= 32 ? r : (r & ((1u << low) - 1)); }
};
template <> struct Rec<uint64_t> {
  __device__ __forceinline__ static uint64_t pack(uint32_t file, uint32_t cl, uint32_t) {
    return ((uint64_t)file << 32) | cl;
  }
  __device__ __forceinline__ static uint32_t file(uint64_t r, uint32_t) { return (uint32_t)(r >> 32); }
  __device__ __forceinline__ static uint32_t cl(uint64_t r, uint32_t) { return (uint32_t)r; }
};

// Any status bit means the pass will be replayed: a table overflow stops the scan
// early (so some chunks' counts are stale) and a record overflow leaves no room.
__device__ __forceinline__ bool rec_overflow(const DedupParams &d) {
  return __hip_atomic_load(d.status, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0;
}

// ------------------------------------------------------------------ generic exclusive scan u32 -> u64
__global__ void __launch_bounds__(256) k_xscan_reduce(const uint32_t *in, uint64_t n, uint64_t *part) {
  __shared__ uint64_t s[256];
  const uint64_t b0 = (uint64_t)blockIdx.x * SCAN_SEG;
  uint64_t acc = 0;
  for (uint32_t i = threadIdx.x; i < SCAN_SEG; i += 256)
    if (b0 + i < n) acc += in[b0 + i];
  s[threadIdx.x] = acc;
  __syncthreads();
  for (uint32_t o = 128; o; o >>= 1) {
    if (threadIdx.x < o) s[threadIdx.x] += s[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = s[0];
}

// exclusive scan of np partials in place (one workgroup), total to *total
__global__ void __launch_bounds__(1024) k_xscan_top(uint64_t *part, uint64_t np, uint64_t *total) {
  __shared__ uint64_t s[1024];
  const uint32_t t = threadIdx.x;
  const uint64_t per = (np + 1023) / 1024, lo = t * per, hi = lo + per < np ? lo + per : np;
  uint64_t acc = 0;
  for (uint64_t i = lo; i < hi; i++) acc += part[i];
  s[t] = acc;
  __syncthreads();
  for (uint32_t o = 1; o < 1024; o <<= 1) {
    const uint64_t x = t >= o ? s[t - o] : 0;
    __syncthreads();
    s[t] += x;
    __syncthreads();
  }
  uint64_t run = s[t] - acc;
  for (uint64_t i = lo; i < hi; i++) {
    const uint64_t v = part[i];
    part[i] = run;
    run += v;
  }
  if (t == 1023) *total = s[1023];
}

__global__ void __launch_bounds__(256) k_xscan_apply(const uint32_t *in, uint64_t n, const uint64_t *part, uint64_t *out) {
  __shared__ uint64_t s[256];
  constexpr uint32_t PER = SCAN_SEG / 256;
  const uint64_t b0 = (uint64_t)blockIdx.x * SCAN_SEG + (uint64_t)threadIdx.x * PER;
  uint32_t v[PER];
  uint64_t acc = 0;
  for (uint32_t j = 0; j < PER; j++) {
    v[j] = b0 + j < n ? in[b0 + j] : 0u;
    acc += v[j];
  }
  s[threadIdx.x] = acc;
  __syncthreads();
  for (uint32_t o = 1; o < 256; o <<= 1) {
    const uint64_t x = threadIdx.x >= o ? s[threadIdx.x - o] : 0;
    __syncthreads();
    s[threadIdx.x] += x;
    __syncthreads();
  }
  uint64_t run = part[blockIdx.x] + s[threadIdx.x] - acc;
  for (uint32_t j = 0; j < PER; j++) {
    if (b0 + j < n) out[b0 + j] = run;
    run += v[j];
  }
}

// out[0..n) = exclusive prefix sums of in, out[n] = total
static hipError_t xscan(const uint32_t *in, uint64_t n, uint64_t *part, uint64_t *out, hipStream_t s) {
  const uint64_t nb = (n + SCAN_SEG - 1) / SCAN_SEG;
  if (nb) {
    hipLaunchKernelGGL(k_xscan_reduce, dim3((uint32_t)nb), dim3(256), 0, s, in, n, part);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(k_xscan_top, dim3(1), dim3(1024), 0, s, part, nb, out + n);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || !nb) return e;
  hipLaunchKernelGGL(k_xscan_apply, dim3((uint32_t)nb), dim3(256), 0, s, in, n, part, out);
  return hipGetLastError();
}

// ------------------------------------------------------------------ level-1 bases
// g1 = scan of hist1 laid out [bucket][chunk]; bucket b's records start at
// base1[b] (a multiple of TILE) and end at bend[b].
__global__ void __launch_bounds__(256) k_bases(DedupParams d) {
  __shared__ uint64_t s[256];
  const uint32_t t = threadIdx.x;
  uint64_t tot = 0, pad = 0;
  if (t < d.nb1) {
    tot = d.g1[(uint64_t)(t + 1) * d.nct] - d.g1[(uint64_t)t * d.nct];
    pad = (tot + TILE - 1) / TILE * TILE;
  }
  s[t] = pad;
  __syncthreads();
  for (uint32_t o = 1; o < 256; o <<= 1) {
    const uint64_t x = t >= o ? s[t - o] : 0;
    __syncthreads();
    s[t] += x;
    __syncthreads();
  }
  if (t < d.nb1) {
    d.base1[t] = s[t] - pad;
    d.bend[t] = s[t] - pad + tot;
  }
  if (t == 255) {
    const uint64_t padded = s[255];
    d.base1[d.nb1] = padded;
    d.dscal[0] = d.g1[(uint64_t)d.nb1 * d.nct];   // records
    d.dscal[1] = padded / TILE;                     // tiles
    d.dscal[2] = padded;
    if (padded > d.cap) atomicOr(d.status, ST_REC_OVF);
  }
}

// ------------------------------------------------------------------ level-1 gather
// Each workgroup takes a contiguous range of chunks (file order), so the strided
// reads of g1 for neighbouring chunks share cache lines.
template <typename R1>
__global__ void __launch_bounds__(256) k_gather(DedupParams d) {
  __shared__ uint64_t s_base[256];
  __shared__ uint32_t s_cur[256];
  if (rec_overflow(d)) return;
  const uint32_t tid = threadIdx.x;
  const uint32_t per = (d.nct + gridDim.x - 1) / gridDim.x;
  const uint32_t c0 = blockIdx.x * per, c1 = c0 + per < d.nct ? c0 + per : d.nct;
  R1 *out = reinterpret_cast<R1 *>(d.l1);
  const uint32_t m1 = d.low1 >= 32 ? 0xFFFFFFFFu : ((1u << d.low1) - 1);
  for (uint32_t ci = c0; ci < c1; ci++) {
    const Chunk c = d.chunks[ci];
    const uint32_t n = d.nrec[ci] < c.nsym ? d.nrec[ci] : c.nsym;   // a chunk records at most one per window
    if (n == 0) continue;   // uniform across the workgroup
    if (tid < d.nb1) {
      s_base[tid] = d.base1[tid] + (d.g1[(uint64_t)tid * d.nct + ci] - d.g1[(uint64_t)tid * d.nct]);
      s_cur[tid] = 0;
    }
    __syncthreads();
    const uint32_t *src = d.rec0 + c.s0;
    for (uint32_t i = tid; i < n; i += 256) {
      const uint32_t cid = src[i];
      const uint32_t b = d.low1 >= 32 ? 0u : (cid >> d.low1);
      const uint32_t k = atomicAdd(s_cur + b, 1u);
      const uint64_t at = s_base[b] + k;
      if (at < d.cap) out[at] = Rec<R1>::pack(c.file, cid & m1, d.low1);
    }
    __syncthreads();
  }
}

// bucket of tile t: the last b with base1[b] <= t * TILE (empty buckets have no tiles)
__device__ __forceinline__ uint32_t tile_bucket(const uint64_t *s_base1, uint32_t nb1, uint64_t pos) {
  uint32_t lo = 0, hi = nb1;   // invariant: base1[lo] <= pos < base1[hi]
  while (hi - lo > 1) {
    const uint32_t mid = (lo + hi) >> 1;
    if (s_base1[mid] <= pos) lo = mid;
    else hi = mid;
  }
  return lo;
}

// ------------------------------------------------------------------ level-2 histograms
// hist2 index of (bucket b, digit d2, tile tl of b): (base1[b]/TILE)*nb2 + d2*nt_b + tl,
// so one linear scan gives every record's final position; slots past the last
// tile are zero.
template <typename R1>
__global__ void __launch_bounds__(P2_BLOCK) k_p2_hist(DedupParams d) {
  __shared__ uint64_t s_base1[257];
  __shared__ uint64_t s_bend[256];
  __shared__ uint32_t h[1024];
  if (rec_overflow(d)) return;
  const uint32_t tid = threadIdx.x;
  for (uint32_t i = tid; i <= d.nb1; i += P2_BLOCK) s_base1[i] = d.base1[i];
  for (uint32_t i = tid; i < d.nb1; i += P2_BLOCK) s_bend[i] = d.bend[i];
  __syncthreads();
  const uint64_t ntiles = d.dscal[1];
  const R1 *in = reinterpret_cast<const R1 *>(d.l1);
  const uint32_t dm = d.nb2 - 1;
  for (uint64_t t = blockIdx.x; t < d.ntmax; t += gridDim.x) {
    if (t >= ntiles) {
      for (uint32_t k = tid; k < d.nb2; k += P2_BLOCK) d.hist2[t * d.nb2 + k] = 0;
      continue;
    }
    const uint64_t pos = t * TILE;
    const uint32_t b = tile_bucket(s_base1, d.nb1, pos);
    const uint64_t tb = s_base1[b] / TILE, ntb = (s_base1[b + 1] - s_base1[b]) / TILE, tl = t - tb;
    const uint64_t hi = pos + TILE < s_bend[b] ? pos + TILE : s_bend[b];
    for (uint32_t k = tid; k < d.nb2; k += P2_BLOCK) h[k] = 0;
    __syncthreads();
    for (uint64_t i = pos + tid; i < hi; i += P2_BLOCK) {
      const uint32_t cl = Rec<R1>::cl(in[i], d.low1);
      atomicAdd(h + ((cl >> d.low2) & dm), 1u);
    }
    __syncthreads();
    for (uint32_t k = tid; k < d.nb2; k += P2_BLOCK) d.hist2[tb * d.nb2 + k * ntb + tl] = h[k];
    __syncthreads();
  }
}

// final bucket bounds: fin[b*nb2 + d2] = first position of (b, d2) in l2
__global__ void k_fin(DedupParams d) {
  if (rec_overflow(d)) return;
  const uint32_t nf = d.nb1 * d.nb2;
  for (uint32_t f = blockIdx.x * blockDim.x + threadIdx.x; f <= nf; f += gridDim.x * blockDim.x) {
    if (f == nf) {
      d.fin[nf] = d.g2[d.ntmax * d.nb2];
      continue;
    }
    const uint32_t b = f / d.nb2, d2 = f - b * d.nb2;
    const uint64_t tb = d.base1[b] / TILE, ntb = (d.base1[b + 1] - d.base1[b]) / TILE;
    d.fin[f] = d.g2[tb * d.nb2 + d2 * ntb];
  }
}

// ------------------------------------------------------------------ level-2 stable scatter
template <typename R1, typename R2>
__global__ void __launch_bounds__(P2_BLOCK) k_p2_scatter(DedupParams d) {
  constexpr uint32_t NW = P2_BLOCK / 64;
  __shared__ uint64_t s_base1[257];
  __shared__ uint64_t s_bend[256];
  __shared__ uint64_t run[1024];
  __shared__ uint32_t tot[1024];
  __shared__ uint32_t wcnt[NW][1024];
  if (rec_overflow(d)) return;
  const uint32_t tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  for (uint32_t i = tid; i <= d.nb1; i += P2_BLOCK) s_base1[i] = d.base1[i];
  for (uint32_t i = tid; i < d.nb1; i += P2_BLOCK) s_bend[i] = d.bend[i];
  __syncthreads();
  const uint64_t ntiles = d.dscal[1];
  const R1 *in = reinterpret_cast<const R1 *>(d.l1);
  R2 *out = reinterpret_cast<R2 *>(d.l2);
  const uint32_t dm = d.nb2 - 1;
  const uint32_t m2 = d.low2 >= 32 ? 0xFFFFFFFFu : ((1u << d.low2) - 1);
  const uint64_t lt = (1ull << lane) - 1;
  for (uint64_t t = blockIdx.x; t < ntiles; t += gridDim.x) {
    const uint64_t pos = t * TILE;
    const uint32_t b = tile_bucket(s_base1, d.nb1, pos);
    const uint64_t tb = s_base1[b] / TILE, ntb = (s_base1[b + 1] - s_base1[b]) / TILE, tl = t - tb;
    const uint64_t hi = pos + TILE < s_bend[b] ? pos + TILE : s_bend[b];
    for (uint32_t k = tid; k < d.nb2; k += P2_BLOCK) run[k] = d.g2[tb * d.nb2 + k * ntb + tl];
    for (uint64_t s0 = pos; s0 < hi; s0 += P2_BLOCK) {
      const uint64_t i = s0 + tid;
      const bool valid = i < hi;
      uint32_t file = 0, cl = 0, dg = 0;
      if (valid) {
        const R1 r = in[i];
        file = Rec<R1>::file(r, d.low1);
        cl = Rec<R1>::cl(r, d.low1);
        dg = (cl >> d.low2) & dm;
      }
      for (uint32_t k = tid; k < NW * d.nb2; k += P2_BLOCK) wcnt[k / d.nb2][k % d.nb2] = 0;
      __syncthreads();
      // lanes of this wavefront with the same digit, by ballots over the digit bits
      const uint64_t vm = __ballot(valid);
      uint64_t same = vm;
      for (uint32_t j = 0; (1u << j) < d.nb2; j++) {
        const bool bit = (dg >> j) & 1u;
        const uint64_t bj = __ballot(valid && bit);
        same &= bit ? bj : (vm & ~bj);
      }
      const uint32_t rank = valid ? (uint32_t)__popcll(same & lt) : 0u;
      if (valid && rank == 0) wcnt[w][dg] = (uint32_t)__popcll(same);
      __syncthreads();
      for (uint32_t k = tid; k < d.nb2; k += P2_BLOCK) {
        uint32_t off = 0;
        for (uint32_t ww = 0; ww < NW; ww++) {
          const uint32_t x = wcnt[ww][k];
          wcnt[ww][k] = off;
          off += x;
        }
        tot[k] = off;
      }
      __syncthreads();
      if (valid) {
        const uint64_t at = run[dg] + wcnt[w][dg] + rank;
        if (at < d.cap) out[at] = Rec<R2>::pack(file, cl & m2, d.low2);
      }
      __syncthreads();
      for (uint32_t k = tid; k < d.nb2; k += P2_BLOCK) run[k] += tot[k];
      __syncthreads();
    }
  }
}

// ------------------------------------------------------------------ distinct sequences per candidate
template <typename R2>
__global__ void __launch_bounds__(CNT_BLOCK) k_count(DedupParams d) {
  extern __shared__ __align__(16) uint8_t lds[];
  uint64_t *hk = reinterpret_cast<uint64_t *>(lds);                // CNT_HASH pair keys
  uint32_t *last = reinterpret_cast<uint32_t *>(hk + CNT_HASH);    // 1 + sequence of the latest record
  uint32_t *cnt = last + (1u << d.low2);
  if (rec_overflow(d)) return;
  const uint32_t tid = threadIdx.x;
  const uint32_t cb = 1u << d.low2;
  const R2 *in = reinterpret_cast<const R2 *>(d.l2);
  uint32_t *gcnt = reinterpret_cast<uint32_t *>(d.cnt);
  for (uint32_t k = tid; k < CNT_HASH; k += CNT_BLOCK) hk[k] = 0;
  for (uint32_t k = tid; k < cb; k += CNT_BLOCK) { last[k] = 0; cnt[k] = 0; }
  __syncthreads();
  const uint32_t nf = d.nb1 * d.nb2;
  for (uint32_t f = blockIdx.x; f < nf; f += gridDim.x) {
    const uint64_t cid0 = (uint64_t)f << d.low2;
    if (cid0 >= d.nc) break;   // later buckets are beyond the candidate space (and empty)
    const uint64_t lo = d.fin[f], hi = d.fin[f + 1] < d.cap ? d.fin[f + 1] : d.cap;
    for (uint64_t s0 = lo; s0 < hi; s0 += CNT_BLOCK) {
      const uint64_t i = s0 + tid;
      const bool valid = i < hi;
      uint32_t f1 = 0, cl = 0, lp = 0;
      if (valid) {
        const R2 r = in[i];
        f1 = Rec<R2>::file(r, d.low2) + 1;
        cl = Rec<R2>::cl(r, d.low2);
        lp = last[cl];
      }
      __syncthreads();
      bool won = false;
      uint32_t slot = 0;
      if (valid) {
        const uint64_t key = ((uint64_t)f1 << 32) | cl;
        slot = (uint32_t)(mix64(key) & (CNT_HASH - 1));
        for (;;) {
          const unsigned long long old = atomicCAS(reinterpret_cast<unsigned long long *>(hk + slot), 0ull,
                                                   (unsigned long long)key);
          if (old == 0ull) { won = true; break; }
          if (old == key) break;
          slot = (slot + 1) & (CNT_HASH - 1);
        }
        if (won && lp != f1) atomicAdd(cnt + cl, 1u);
        atomicMax(last + cl, f1);
      }
      __syncthreads();
      if (won) hk[slot] = 0;
      __syncthreads();
    }
    const uint64_t cend = cid0 + cb < d.nc ? cid0 + cb : d.nc;
    for (uint32_t k = tid; k < cb; k += CNT_BLOCK) {
      if (cid0 + k < cend) gcnt[cid0 + k] = cnt[k];
      cnt[k] = 0;
      last[k] = 0;
    }
    __syncthreads();
  }
}

size_t count_lds_bytes(uint32_t low2) { return (size_t)CNT_HASH * 8 + ((size_t)2 << low2) * 4; }

// ------------------------------------------------------------------ host side
DedupShape dedup_shape(uint64_t nc, uint64_t m) {
  DedupShape sh{};
  auto bits_of = [](uint64_t x) { uint32_t b = 0; while (b < 64 && (x >> b)) b++; return b; };
  const uint32_t cbits = std::max<uint32_t>(1, bits_of(nc - 1));
  const uint32_t fbits = std::max<uint32_t>(1, bits_of(m ? m - 1 : 0));
  uint32_t low2 = std::min<uint32_t>(13, cbits);
  uint32_t split = cbits - low2;
  if (split > 18) { low2 = cbits - 18; split = 18; }
  // level 1 as fine as needed to pack its records into 32 bits, at most 8 bits
  uint32_t b1 = (split + 1) / 2;
  if (fbits + cbits > 32) b1 = std::max<uint32_t>(b1, fbits + cbits - 32);
  b1 = std::min<uint32_t>(std::min<uint32_t>(b1, 8), split);
  uint32_t b2 = split - b1;
  if (b2 > 10) { b2 = 10; b1 = split - 10; }
  sh.nb1 = 1u << b1;
  sh.nb2 = 1u << b2;
  sh.low1 = cbits - b1;
  sh.low2 = low2;
  sh.w1 = (fbits + sh.low1 <= 32) ? 4 : 8;
  sh.w2 = (fbits + sh.low2 <= 32) ? 4 : 8;
  return sh;
}

uint64_t dedup_tile() { return TILE; }

hipError_t dedup_enqueue(const DedupParams &d, int n_cu, hipStream_t s) {
  hipError_t e = xscan(d.hist1, (uint64_t)d.nb1 * d.nct, d.scan_tmp, d.g1, s);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_bases, dim3(1), dim3(256), 0, s, d);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  const uint32_t grid = (uint32_t)n_cu * 4;
  if (d.w1 == 4) hipLaunchKernelGGL(k_gather<uint32_t>, dim3(grid), dim3(256), 0, s, d);
  else hipLaunchKernelGGL(k_gather<uint64_t>, dim3(grid), dim3(256), 0, s, d);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  const uint32_t g2 = (uint32_t)n_cu * 4;
  if (d.w1 == 4) hipLaunchKernelGGL(k_p2_hist<uint32_t>, dim3(g2), dim3(P2_BLOCK), 0, s, d);
  else hipLaunchKernelGGL(k_p2_hist<uint64_t>, dim3(g2), dim3(P2_BLOCK), 0, s, d);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  e = xscan(d.hist2, d.ntmax * d.nb2, d.scan_tmp, d.g2, s);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_fin, dim3((d.nb1 * d.nb2 + 256) / 256), dim3(256), 0, s, d);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  if (d.w1 == 4 && d.w2 == 4) hipLaunchKernelGGL((k_p2_scatter<uint32_t, uint32_t>), dim3(g2), dim3(P2_BLOCK), 0, s, d);
  else if (d.w1 == 4) hipLaunchKernelGGL((k_p2_scatter<uint32_t, uint64_t>), dim3(g2), dim3(P2_BLOCK), 0, s, d);
  else if (d.w2 == 4) hipLaunchKernelGGL((k_p2_scatter<uint64_t, uint32_t>), dim3(g2), dim3(P2_BLOCK), 0, s, d);
  else hipLaunchKernelGGL((k_p2_scatter<uint64_t, uint64_t>), dim3(g2), dim3(P2_BLOCK), 0, s, d);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  const size_t lds = count_lds_bytes(d.low2);
  const uint32_t nf = d.nb1 * d.nb2;
  const uint32_t gc = nf < (uint32_t)n_cu * 2 ? nf : (uint32_t)n_cu * 2;
  if (d.w2 == 4) hipLaunchKernelGGL(k_count<uint32_t>, dim3(gc), dim3(CNT_BLOCK), lds, s, d);
  else hipLaunchKernelGGL(k_count<uint64_t>, dim3(gc), dim3(CNT_BLOCK), lds, s, d);
  return hipGetLastError();
}

hipError_t prepare_dedup(uint32_t low2) {
  const int lds = (int)count_lds_bytes(low2);
  hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(k_count<uint32_t>),
                                     hipFuncAttributeMaxDynamicSharedMemorySize, lds);
  if (e == hipSuccess)
    e = hipFuncSetAttribute(reinterpret_cast<const void *>(k_count<uint64_t>), hipFuncAttributeMaxDynamicSharedMemorySize,
                            lds);
  return e;
}

uint64_t dedup_scan_tmp_entries(uint64_t n) { return (n + SCAN_SEG - 1) / SCAN_SEG + 1; }

}  // namespace ig
