// Once-per-sequence counting (Eq. 2) without device-scope atomics.
//
// The scan leaves, for every chunk, its chunk-distinct candidate ids ("records")
// in a slab at the chunk's own window positions, and a histogram of their top
// b1 bits.  Counting the sequences that contain each candidate then needs the
// duplicates of (sequence, candidate) across the chunks of one sequence
// removed.  Records are laid out in file order of the chunks, so that every
// candidate range below keeps the records of one sequence together:
//
//   1. a column scan of the level-1 histograms (rows = chunks in file order) in
//      bucket-major order, and per-bucket bases, each bucket padded to a whole
//      number of tiles;
//   2. gather: each chunk's records go to its run in its level-1 bucket, tagged
//      with the sequence id (runs of one bucket follow the file order);
//   3. a stable split of every level-1 bucket on the next b2 bits (per-tile
//      histograms, a scan, and a scatter ranked with wavefront ballots, so the
//      order inside each final bucket is still the file order);
//   4. one wavefront per final bucket (or per segment of a large bucket, cut at
//      sequence boundaries) counts, in LDS, the distinct sequences of each of
//      its at most 2^low2 candidates: a record is new unless the previous record
//      of its candidate came from the same sequence (sequence ids never decrease
//      along a bucket).  Within a round of 64 records the previous record of
//      the same candidate is found with ballots over the candidate bits.  A
//      bucket counted whole is written with plain stores (every candidate
//      belongs to exactly one bucket); segments add their counts atomically.
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
static constexpr uint32_t SLICE_ROUNDS = TILE / P2_BLOCK;   // records per thread and tile in the level-2 kernels
static constexpr uint32_t NCOL_MAX = 1024;      // chunk groups of the column scan
static constexpr uint32_t SEG = 32768;          // records per counting segment (buckets are cut into segments)
static constexpr uint32_t CNT_LDS = 64 * 1024;  // LDS of one count workgroup

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
// The element count is n, or min(n, ndev[0] * mult) when ndev is given (a count only the device knows).
__device__ __forceinline__ uint64_t scan_len(uint64_t n, const uint64_t *ndev, uint32_t mult) {
  if (!ndev) return n;
  const uint64_t m = ndev[0] * mult;
  return m < n ? m : n;
}

__global__ void __launch_bounds__(256) k_xscan_reduce(const uint32_t *in, uint64_t n0, const uint64_t *ndev, uint32_t mult,
                                                      uint64_t *part) {
  __shared__ uint64_t s[256];
  const uint64_t n = scan_len(n0, ndev, mult);
  const uint64_t b0 = (uint64_t)blockIdx.x * SCAN_SEG;
  if (b0 >= n) return;
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

// exclusive scan of np partials in place (one workgroup), total to *total; with ndev, np and
// the total's position follow the device count (out + n)
__global__ void __launch_bounds__(1024) k_xscan_top(uint64_t *part, uint64_t np, uint64_t *total) {
  wg_exclusive_scan<uint64_t>(part, np, total);
}

__global__ void __launch_bounds__(1024) k_xscan_top_d(uint64_t *part, uint64_t n0, const uint64_t *ndev, uint32_t mult,
                                                      uint64_t *out) {
  const uint64_t n = scan_len(n0, ndev, mult);
  wg_exclusive_scan<uint64_t>(part, (n + SCAN_SEG - 1) / SCAN_SEG, out + n);
}

__global__ void __launch_bounds__(256) k_xscan_apply(const uint32_t *in, uint64_t n0, const uint64_t *ndev, uint32_t mult,
                                                     const uint64_t *part, uint64_t *out) {
  __shared__ uint64_t s[256];
  constexpr uint32_t PER = SCAN_SEG / 256;
  const uint64_t n = scan_len(n0, ndev, mult);
  if ((uint64_t)blockIdx.x * SCAN_SEG >= n) return;
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

// out[0..n) = exclusive prefix sums of in, out[n] = total; n = min(n_max, ndev[0] * mult) when
// ndev is given (the grid covers n_max, blocks past n return at once)
static hipError_t xscan(const uint32_t *in, uint64_t n_max, uint64_t *part, uint64_t *out, hipStream_t s,
                        const uint64_t *ndev = nullptr, uint32_t mult = 1) {
  const uint64_t nb = (n_max + SCAN_SEG - 1) / SCAN_SEG;
  if (nb) {
    hipLaunchKernelGGL(k_xscan_reduce, dim3((uint32_t)nb), dim3(256), 0, s, in, n_max, ndev, mult, part);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(k_xscan_top_d, dim3(1), dim3(1024), 0, s, part, n_max, ndev, mult, out);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || !nb) return e;
  hipLaunchKernelGGL(k_xscan_apply, dim3((uint32_t)nb), dim3(256), 0, s, in, n_max, ndev, mult, part, out);
  return hipGetLastError();
}

// ------------------------------------------------------------------ level-1 column scan
// Column c of hist1 ([chunk][bucket]) summed over chunk group w -> part[b * ncol + w].
__global__ void __launch_bounds__(256) k_col_reduce(DedupParams d) {
  const uint32_t w = blockIdx.x, per = (d.nct + d.ncol - 1) / d.ncol;
  const uint32_t c0 = w * per, c1 = c0 + per < d.nct ? c0 + per : d.nct;
  for (uint32_t b = threadIdx.x; b < d.nb1; b += 256) {
    uint64_t acc = 0;
    for (uint32_t ci = c0; ci < c1; ci++) acc += d.hist1[(uint64_t)ci * d.nb1 + b];
    d.scan_tmp[(uint64_t)b * d.ncol + w] = acc;
  }
}
// after the partials are scanned: g1[ci][b] = records before (b, ci) in bucket-major order
__global__ void __launch_bounds__(256) k_col_apply(DedupParams d) {
  const uint32_t w = blockIdx.x, per = (d.nct + d.ncol - 1) / d.ncol;
  const uint32_t c0 = w * per, c1 = c0 + per < d.nct ? c0 + per : d.nct;
  for (uint32_t b = threadIdx.x; b < d.nb1; b += 256) {
    uint64_t run = d.scan_tmp[(uint64_t)b * d.ncol + w];
    for (uint32_t ci = c0; ci < c1; ci++) {
      d.g1[(uint64_t)ci * d.nb1 + b] = run;
      run += d.hist1[(uint64_t)ci * d.nb1 + b];
    }
  }
}

// ------------------------------------------------------------------ level-1 bases
// Bucket b's records start at base1[b] (a multiple of TILE) and end at bend[b].
__global__ void __launch_bounds__(256) k_bases(DedupParams d) {
  __shared__ uint64_t s[256];
  const uint32_t t = threadIdx.x;
  const uint64_t total = d.scan_tmp[(uint64_t)d.nb1 * d.ncol];
  uint64_t start = 0, tot = 0, pad = 0;
  if (t < d.nb1) {
    start = d.scan_tmp[(uint64_t)t * d.ncol];
    const uint64_t next = t + 1 < d.nb1 ? d.scan_tmp[(uint64_t)(t + 1) * d.ncol] : total;
    tot = next - start;
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
    d.bshift[t] = (s[t] - pad) - start;   // modulo 2^64
  }
  if (t == 255) {
    const uint64_t padded = s[255];
    d.base1[d.nb1] = padded;
    d.dscal[0] = total;
    d.dscal[1] = padded / TILE;
    d.dscal[2] = padded;
    if (padded > d.cap) atomicOr(d.status, ST_REC_OVF);
  }
}

// ------------------------------------------------------------------ level-1 gather
static constexpr uint32_t GATHER_BLOCK = 512;
template <typename R1>
__global__ void __launch_bounds__(GATHER_BLOCK) k_gather(DedupParams d) {
  // Records go through LDS in tiles of GT, counting-sorted by bucket, so that consecutive lanes
  // write consecutive positions of one bucket's run (a direct scatter sends each lane of a store
  // to a different bucket, so to a different cache line).  Larger tiles make longer runs: fewer
  // partly written lines at their ends.
  constexpr uint32_t GB = GATHER_BLOCK, GT = 4096, PER = GT / GB;
  __shared__ uint64_t s_base[256];   // the chunk's first position in each bucket
  __shared__ uint32_t s_cur[256];    // records of the chunk already written per bucket
  __shared__ uint32_t s_h[256];      // the tile's records per bucket
  __shared__ uint32_t s_off[256];    // the tile's first sorted slot per bucket
  __shared__ uint32_t s_wsum[4];
  __shared__ uint32_t s_stage[GT];
  if (rec_overflow(d)) return;
  const uint32_t tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const uint32_t per = (d.nct + gridDim.x - 1) / gridDim.x;
  const uint32_t c0 = blockIdx.x * per, c1 = c0 + per < d.nct ? c0 + per : d.nct;
  R1 *out = reinterpret_cast<R1 *>(d.l1);
  const uint32_t m1 = d.low1 >= 32 ? 0xFFFFFFFFu : ((1u << d.low1) - 1);
  auto bucket = [&](uint32_t cid) {
    uint32_t b = d.low1 >= 32 ? 0u : (cid >> d.low1);
    return b < d.nb1 ? b : d.nb1 - 1;   // (only a corrupt record could exceed the candidate space)
  };
  for (uint32_t ci = c0; ci < c1; ci++) {
    const Chunk c = d.chunks[ci];
    const uint32_t n = d.nrec[ci] < c.nsym ? d.nrec[ci] : c.nsym;   // a chunk records at most one per window
    if (n == 0) continue;   // uniform across the workgroup
    if (tid < d.nb1) {
      s_base[tid] = d.g1[(uint64_t)ci * d.nb1 + tid] + d.bshift[tid];
      s_cur[tid] = 0;
    }
    const uint32_t *src = d.rec0 + c.s0;
    for (uint32_t t0 = 0; t0 < n; t0 += GT) {
      const uint32_t m = n - t0 < GT ? n - t0 : GT;
      if (tid < 256) s_h[tid] = 0;
      __syncthreads();
      // this thread's records of the tile (loads first), their buckets and ranks within them
      uint32_t cid[PER], rk[PER];
#pragma unroll
      for (uint32_t q = 0; q < PER; q++) cid[q] = src[t0 + (q * GB + tid < m ? q * GB + tid : m - 1)];
#pragma unroll
      for (uint32_t q = 0; q < PER; q++)
        rk[q] = q * GB + tid < m ? atomicAdd(s_h + bucket(cid[q]), 1u) : 0u;
      __syncthreads();
      // exclusive scan of the tile's bucket counts (one bucket per thread of the first four
      // wavefronts)
      uint32_t hv = 0, x = 0;
      if (tid < 256) {
        hv = s_h[tid];
        x = hv;
        for (uint32_t off = 1; off < 64; off <<= 1) {
          const uint32_t y = __shfl_up(x, off);
          if (lane >= off) x += y;
        }
        if (lane == 63) s_wsum[w] = x;
      }
      __syncthreads();
      if (tid < 256) {
        uint32_t wb = 0;
        for (uint32_t ww = 0; ww < w; ww++) wb += s_wsum[ww];
        s_off[tid] = wb + x - hv;
      }
      __syncthreads();
#pragma unroll
      for (uint32_t q = 0; q < PER; q++)
        if (q * GB + tid < m) s_stage[s_off[bucket(cid[q])] + rk[q]] = cid[q];
      __syncthreads();
      // sorted slots: slot j of bucket b goes to the chunk's run in b
      for (uint32_t j = tid; j < m; j += GB) {
        const uint32_t v = s_stage[j];
        const uint32_t b = bucket(v);
        const uint64_t at = s_base[b] + s_cur[b] + (j - s_off[b]);
        if (at < d.cap) out[at] = Rec<R1>::pack(c.file, v & m1, d.low1);
      }
      __syncthreads();
      if (tid < d.nb1) s_cur[tid] += s_h[tid];
    }
    __syncthreads();
  }
}

// The level-2 kernels take tiles strided by the grid.  Workgroups are dispatched to the 8 XCDs
// round-robin by id, and neighbouring tiles share the cache lines of their per-digit counts and
// bases (entry d2 * ntb + tl of a bucket): numbered as below, the workgroups of one XCD take
// consecutive tiles, so those lines are filled and read within one L2.  (A bijection of
// [0, grid) when the grid is a multiple of 8; the identity otherwise.)
__device__ __forceinline__ uint32_t xcd_major_block() {
  const uint32_t g = gridDim.x, b = blockIdx.x;
  return g % 8u ? b : (b % 8u) * (g / 8u) + b / 8u;
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
  for (uint64_t t = xcd_major_block(); t < ntiles; t += gridDim.x) {
    const uint64_t pos = t * TILE;
    const uint32_t b = tile_bucket(s_base1, d.nb1, pos);
    const uint64_t tb = s_base1[b] / TILE, ntb = (s_base1[b + 1] - s_base1[b]) / TILE, tl = t - tb;
    const uint64_t hi = pos + TILE < s_bend[b] ? pos + TILE : s_bend[b];
    for (uint32_t k = tid; k < d.nb2; k += P2_BLOCK) h[k] = 0;
    __syncthreads();
    // the tile's loads are issued together (every tile lies inside the padded level-1 array,
    // so they need no bound); records past the bucket's end are not counted
    R1 v[SLICE_ROUNDS];
#pragma unroll
    for (uint32_t q = 0; q < SLICE_ROUNDS; q++) v[q] = in[pos + q * P2_BLOCK + tid];
#pragma unroll
    for (uint32_t q = 0; q < SLICE_ROUNDS; q++)
      if (pos + q * P2_BLOCK + tid < hi) atomicAdd(h + ((Rec<R1>::cl(v[q], d.low1) >> d.low2) & dm), 1u);
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
      d.fin[nf] = d.g2[d.dscal[1] * d.nb2];
      continue;
    }
    const uint32_t b = f / d.nb2, d2 = f - b * d.nb2;
    const uint64_t tb = d.base1[b] / TILE, ntb = (d.base1[b + 1] - d.base1[b]) / TILE;
    d.fin[f] = d.g2[tb * d.nb2 + d2 * ntb];
  }
}

// ------------------------------------------------------------------ level-2 stable scatter
// A tile is cut into one contiguous slice per wavefront (SLICE_ROUNDS rounds of 64 records,
// kept in registers).  Each wavefront counts its slice's digits, one prefix over the
// wavefronts (per digit) gives every wavefront its first position, and each wavefront then
// replays its rounds in order, advancing its own cursors: positions follow the tile order.
// (Registers for 5 wavefronts per SIMD: the tile in flight and the next one's records fit
// without spills, and 2 workgroups per CU are resident.)
template <typename R1, typename R2>
__global__ void __launch_bounds__(P2_BLOCK) __attribute__((amdgpu_waves_per_eu(5))) k_p2_scatter(DedupParams d) {
  constexpr uint32_t NW = P2_BLOCK / 64;
  __shared__ uint64_t s_base1[257];
  __shared__ uint64_t s_bend[256];
  // sized by the digit count (nb2 <= 1024): the tile's first position of each digit, and each
  // wavefront's cursor per digit relative to it
  extern __shared__ __align__(16) uint8_t p2lds[];
  uint64_t *dbase = reinterpret_cast<uint64_t *>(p2lds);
  uint32_t *wcur_ = reinterpret_cast<uint32_t *>(p2lds + (size_t)d.nb2 * 8);
  auto wcur = [&](uint32_t ww, uint32_t k) -> uint32_t & { return wcur_[ww * d.nb2 + k]; };
  // the tile sorted by digit in LDS (stable), written out in order: consecutive lanes then store
  // consecutive positions of one digit's run
  uint32_t *toff = wcur_ + (size_t)NW * d.nb2;                            // the tile's first slot per digit
  R2 *stage = reinterpret_cast<R2 *>(toff + d.nb2 + (d.nb2 & 1));         // TILE records (8-byte aligned)
  uint16_t *sdig = reinterpret_cast<uint16_t *>(stage + TILE);            // their digits
  if (rec_overflow(d)) return;
  const uint32_t tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  for (uint32_t i = tid; i <= d.nb1; i += P2_BLOCK) s_base1[i] = d.base1[i];
  for (uint32_t i = tid; i < d.nb1; i += P2_BLOCK) s_bend[i] = d.bend[i];
  const uint64_t ntiles = d.dscal[1];
  const R1 *in = reinterpret_cast<const R1 *>(d.l1);
  R2 *out = reinterpret_cast<R2 *>(d.l2);
  const uint32_t dm = d.nb2 - 1;
  const uint32_t m2 = d.low2 >= 32 ? 0xFFFFFFFFu : ((1u << d.low2) - 1);
  const uint64_t lt = (1ull << lane) - 1;
  // The next tile's records are loaded into registers while this tile is sorted and written.
  // Every tile lies inside the padded level-1 array (ntiles * TILE records, at most cap, or the
  // pass has stopped above), so the loads need no bound; records past a bucket's end are not used.
  R1 rn[SLICE_ROUNDS];
  auto load_tile = [&](uint64_t tt) {
    const uint64_t i0 = tt * TILE + (uint64_t)w * SLICE_ROUNDS * 64 + lane;
#pragma unroll
    for (uint32_t q = 0; q < SLICE_ROUNDS; q++) rn[q] = in[i0 + q * 64];
  };
  const uint32_t vb = xcd_major_block();
  if (vb < ntiles) load_tile(vb);
  for (uint64_t t = vb; t < ntiles; t += gridDim.x) {
    for (uint32_t k = tid; k < NW * d.nb2; k += P2_BLOCK) wcur_[k] = 0;
    __syncthreads();
    const uint64_t pos = t * TILE;
    const uint32_t b = tile_bucket(s_base1, d.nb1, pos);
    const uint64_t tb = s_base1[b] / TILE, ntb = (s_base1[b + 1] - s_base1[b]) / TILE, tl = t - tb;
    const uint64_t hi = pos + TILE < s_bend[b] ? pos + TILE : s_bend[b];
    const uint64_t s0 = pos + (uint64_t)w * SLICE_ROUNDS * 64;
    // per round only the record and its digit-match mask stay in registers (sequence, candidate
    // and digit are decoded again in the replay)
    // (of the digit match only this lane's rank in its group and the group's size are kept)
    R1 rr[SLICE_ROUNDS];
    uint32_t rs[SLICE_ROUNDS];   // rank | size << 8
    // pass 1: this wavefront's digit counts
#pragma unroll
    for (uint32_t q = 0; q < SLICE_ROUNDS; q++) {
      const uint64_t i = s0 + q * 64 + lane;
      const bool valid = i < hi;
      rr[q] = valid ? rn[q] : (R1)0;
      const uint32_t rd = (Rec<R1>::cl(rr[q], d.low1) >> d.low2) & dm;
      const uint64_t same = wave_match(rd, d.b2bits, valid);
      rs[q] = (uint32_t)__popcll(same & lt) | ((uint32_t)__popcll(same) << 8);
      if (valid && (rs[q] & 0xFFu) == 0) wcur(w, rd) += rs[q] >> 8;
    }
    __syncthreads();
    // per digit: the tile's first position, each wavefront's offset from it, the digit's total
    for (uint32_t k = tid; k < d.nb2; k += P2_BLOCK) {
      dbase[k] = d.g2[tb * d.nb2 + (uint64_t)k * ntb + tl];
      uint32_t off = 0;
      for (uint32_t ww = 0; ww < NW; ww++) {
        const uint32_t x = wcur(ww, k);
        wcur(ww, k) = off;
        off += x;
      }
      toff[k] = off;
    }
    __syncthreads();
    // (issued after this tile's last global loads, the reads of its digit bases above: a wait
    // for those would otherwise wait for these too)
    if (t + gridDim.x < ntiles) load_tile(t + gridDim.x);
    // exclusive scan of the digit totals (one wavefront, nb2 / 64 consecutive digits per lane)
    if (w == 0) {
      const uint32_t per = (d.nb2 + 63) / 64, k0 = lane * per, k1 = k0 + per < d.nb2 ? k0 + per : d.nb2;
      uint32_t sum = 0;
      for (uint32_t k = k0; k < k1; k++) sum += toff[k];
      uint32_t x = sum;
      for (uint32_t off = 1; off < 64; off <<= 1) {
        const uint32_t y = __shfl_up(x, off);
        if (lane >= off) x += y;
      }
      uint32_t run = x - sum;
      for (uint32_t k = k0; k < k1; k++) {
        const uint32_t v = toff[k];
        toff[k] = run;
        run += v;
      }
    }
    __syncthreads();
    // pass 2: replay in order
#pragma unroll
    for (uint32_t q = 0; q < SLICE_ROUNDS; q++) {
      const uint64_t i = s0 + q * 64 + lane;
      const bool valid = i < hi;
      const uint32_t rc = Rec<R1>::cl(rr[q], d.low1), rd = (rc >> d.low2) & dm;
      if (valid) {
        const uint32_t slot = toff[rd] + wcur(w, rd) + (rs[q] & 0xFFu);
        stage[slot] = Rec<R2>::pack(Rec<R1>::file(rr[q], d.low1), rc & m2, d.low2);
        sdig[slot] = (uint16_t)rd;
      }
      // every lane has read its cursor before the group's first lane advances it
      __builtin_amdgcn_wave_barrier();
      if (valid && (rs[q] & 0xFFu) == 0) wcur(w, rd) += rs[q] >> 8;
      __builtin_amdgcn_wave_barrier();
    }
    __syncthreads();
    const uint32_t tlen = (uint32_t)(hi > pos ? hi - pos : 0);
    for (uint32_t j = tid; j < tlen; j += P2_BLOCK) {
      const uint32_t dg = sdig[j];
      const uint64_t at = dbase[dg] + (j - toff[dg]);
      if (at < d.cap) out[at] = stage[j];
    }
    __syncthreads();
  }
}

// ------------------------------------------------------------------ distinct sequences per candidate
template <typename R2>
__device__ __forceinline__ uint32_t rec_file(const R2 *in, uint64_t i, uint32_t low2) {
  return Rec<R2>::file(in[i], low2);
}

// first index in [x, hi) whose sequence differs from the record at x - 1 (lo and hi map to themselves)
template <typename R2>
__device__ uint64_t snap_to_sequence(const R2 *in, uint64_t lo, uint64_t hi, uint64_t x, uint32_t low2) {
  if (x <= lo || x >= hi) return x <= lo ? lo : hi;
  const uint32_t fprev = rec_file(in, x - 1, low2);
  uint64_t a = x, b = hi;   // first index with sequence > fprev lies in [a, b]
  while (a < b) {
    const uint64_t mid = a + ((b - a) >> 1);
    if (rec_file(in, mid, low2) > fprev) b = mid;
    else a = mid + 1;
  }
  return a;
}

// segments per final bucket (0 beyond the candidate space)
__global__ void k_nseg(DedupParams d) {
  if (rec_overflow(d)) return;
  const uint32_t nf = d.nb1 * d.nb2;
  for (uint32_t f = blockIdx.x * blockDim.x + threadIdx.x; f < nf; f += gridDim.x * blockDim.x) {
    const uint64_t cid0 = (uint64_t)f << d.low2;
    const uint64_t lo = d.fin[f], hi = d.fin[f + 1];
    const uint64_t size = hi > lo ? hi - lo : 0;
    d.nseg[f] = cid0 >= d.nc ? 0u : (uint32_t)(size > SEG ? (size + SEG - 1) / SEG : 1);
  }
}

// One wavefront per segment (segments of one bucket are cut at sequence
// boundaries); the waves of a workgroup work independently.  Per candidate a wavefront keeps
// 1 + the sequence of its latest record and its count: 32-bit each, or (NARROW, fewer than
// 65535 sequences) a 16-bit sequence and a 16-bit count packed two to a word (a count never
// exceeds the number of sequences, so a half never carries into its neighbour).  Half the LDS
// per wavefront doubles the wavefronts per CU.
template <typename R2, int NARROW>
__global__ void __launch_bounds__(512) k_count(DedupParams d) {
  extern __shared__ __align__(16) uint8_t lds[];
  const uint32_t lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
  const uint32_t cb = 1u << d.low2;
  uint32_t *last = reinterpret_cast<uint32_t *>(lds) + (size_t)wave * 2 * cb;   // 1 + sequence of the latest record
  uint32_t *cnt = last + cb;
  uint16_t *last16 = reinterpret_cast<uint16_t *>(lds + (size_t)wave * 4 * cb);
  uint32_t *cnt2 = reinterpret_cast<uint32_t *>(lds + (size_t)wave * 4 * cb + 2 * cb);
  if (rec_overflow(d)) return;
  const R2 *in = reinterpret_cast<const R2 *>(d.l2);
  uint32_t *gcnt = reinterpret_cast<uint32_t *>(d.cnt);
  const uint64_t lt = (1ull << lane) - 1;
  const uint32_t nf = d.nb1 * d.nb2;
  const uint64_t nsegs = d.seg0[nf];
  for (uint64_t g = (uint64_t)blockIdx.x * nw + wave; g < nsegs; g += (uint64_t)gridDim.x * nw) {
    // bucket of segment g: the last f with seg0[f] <= g
    uint32_t fl = 0, fh = nf;
    while (fh - fl > 1) {
      const uint32_t mid = (fl + fh) >> 1;
      if (d.seg0[mid] <= g) fl = mid;
      else fh = mid;
    }
    const uint32_t f = fl;
    const uint64_t j = g - d.seg0[f], nseg = d.seg0[f + 1] - d.seg0[f];
    const uint64_t cid0 = (uint64_t)f << d.low2;
    const uint64_t lo = d.fin[f], hi = d.fin[f + 1] < d.cap ? d.fin[f + 1] : d.cap;
    const uint64_t size = hi > lo ? hi - lo : 0;
    const uint64_t a = snap_to_sequence(in, lo, hi, lo + size * j / nseg, d.low2);
    const uint64_t b = snap_to_sequence(in, lo, hi, lo + size * (j + 1) / nseg, d.low2);
    // nothing to count: an empty bucket (its counters were zero-filled before the scan), or one
    // sequence spans this cut and the neighbouring segment has it.  Skipping here also keeps
    // the clamped ring loads below inside [a, b).
    if (a >= b) continue;
    if (NARROW) {
      for (uint32_t k = lane; k < cb; k += 64) last16[k] = 0;
      for (uint32_t k = lane; k < cb / 2; k += 64) cnt2[k] = 0;
    } else {
      for (uint32_t k = lane; k < cb; k += 64) { last[k] = 0; cnt[k] = 0; }
    }
    // a ring of KR rounds in registers: the loads of the next KR - 1 rounds are in flight while
    // a round is processed (2 wavefronts per SIMD leave the latency to the wavefront itself)
    // (loads are unconditional, at an index clamped into the segment: a conditional load would
    // be waited for where its branch joins)
    constexpr uint32_t KR = 4;
    R2 buf[KR];
#pragma unroll
    for (uint32_t q = 0; q < KR; q++) buf[q] = in[a + q * 64 + lane < b ? a + q * 64 + lane : b - 1];
    for (uint64_t s00 = a; s00 < b; s00 += KR * 64) {
#pragma unroll
    for (uint32_t q = 0; q < KR; q++) {
      const uint64_t s0 = s00 + q * 64;   // rounds past b run with every lane invalid
      const bool valid = s0 + lane < b;
      const R2 r = buf[q];
      buf[q] = in[s0 + KR * 64 + lane < b ? s0 + KR * 64 + lane : b - 1];
      uint32_t f1 = 0, cl = 0;
      if (valid) {
        f1 = Rec<R2>::file(r, d.low2) + 1;
        cl = Rec<R2>::cl(r, d.low2);
      }
      const uint32_t lp = valid ? (NARROW ? (uint32_t)last16[cl] : last[cl]) : 0u;
      // lanes holding the same candidate: each valid lane writes its lane number into the
      // candidate's entry and reads back the one that stayed, a lane of its own group, so
      // matching that 6-bit leader groups the lanes as matching the candidate would.  The
      // entry gets its sequence back below from the group's highest lane.
      // (atomic accesses: the read must not be answered from this lane's own write)
      uint32_t leader = 0;
      if (valid) {
        if (NARROW) {
          __hip_atomic_store(last16 + cl, (uint16_t)lane, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WAVEFRONT);
          leader = __hip_atomic_load(last16 + cl, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WAVEFRONT);
        } else {
          __hip_atomic_store(last + cl, lane, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WAVEFRONT);
          leader = __hip_atomic_load(last + cl, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WAVEFRONT);
        }
      }
      const uint64_t same = wave_match(leader, 6, valid);
      const uint64_t below = same & lt;
      const uint32_t pred = below ? 63u - (uint32_t)__clzll((unsigned long long)below) : lane;
      const uint32_t fpred = (uint32_t)__shfl((int)f1, (int)pred);
      const bool isnew = valid && (below ? fpred != f1 : lp != f1);
      const bool islast = valid && (same >> lane) == 1ull;   // highest lane of its group
      if (NARROW) {
        if (isnew) atomicAdd(cnt2 + (cl >> 1), 1u << ((cl & 1u) * 16));
        if (islast) last16[cl] = (uint16_t)f1;
      } else {
        if (isnew) atomicAdd(cnt + cl, 1u);
        if (islast) last[cl] = f1;
      }
    }
    }
    const uint64_t cend = cid0 + cb < d.nc ? cid0 + cb : d.nc;
    for (uint32_t k = lane; k < cb; k += 64) {
      if (cid0 + k >= cend) break;
      const uint32_t ck = NARROW ? (cnt2[k >> 1] >> ((k & 1u) * 16)) & 0xFFFFu : cnt[k];
      if (nseg == 1) gcnt[cid0 + k] = ck;
      else if (ck) atomicAdd(gcnt + cid0 + k, ck);
    }
  }
}

static uint32_t count_waves(uint32_t low2, bool narrow) {
  const size_t per_wave = (size_t)(narrow ? 4 : 8) << low2;
  size_t w = CNT_LDS / per_wave;
  if (w > 8) w = 8;
  return w ? (uint32_t)w : 1u;
}
static size_t count_lds(uint32_t low2, bool narrow) {
  return (size_t)count_waves(low2, narrow) * ((size_t)(narrow ? 4 : 8) << low2);
}
size_t count_lds_bytes(uint32_t low2) { return count_lds(low2, false); }

// ------------------------------------------------------------------ host side
DedupShape dedup_shape(uint64_t nc, uint64_t m) {
  DedupShape sh{};
  auto bits_of = [](uint64_t x) { uint32_t b = 0; while (b < 64 && (x >> b)) b++; return b; };
  const uint32_t cbits = std::max<uint32_t>(1, bits_of(nc - 1));
  const uint32_t fbits = std::max<uint32_t>(1, bits_of(m ? m - 1 : 0));
  uint32_t low2 = std::min<uint32_t>(11, cbits);   // 2^11 candidates: 16 KB of LDS per wavefront
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
uint32_t dedup_ncol(uint32_t nct) { return std::max<uint32_t>(1, std::min<uint32_t>(NCOL_MAX, nct)); }

hipError_t dedup_enqueue(const DedupParams &d, int n_cu, hipStream_t s) {
  hipError_t e;
  hipLaunchKernelGGL(k_col_reduce, dim3(d.ncol), dim3(256), 0, s, d);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  const uint64_t np = (uint64_t)d.nb1 * d.ncol;
  hipLaunchKernelGGL(k_xscan_top, dim3(1), dim3(1024), 0, s, d.scan_tmp, np, d.scan_tmp + np);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  hipLaunchKernelGGL(k_col_apply, dim3(d.ncol), dim3(256), 0, s, d);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  hipLaunchKernelGGL(k_bases, dim3(1), dim3(256), 0, s, d);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  // 4 workgroups of 8 wavefronts per CU (all resident at its register and LDS use): each walks
  // its chunks one after another, and the others hide the latency of each chunk's first loads
  const uint32_t grid = (uint32_t)n_cu * 4;
  if (d.w1 == 4) hipLaunchKernelGGL(k_gather<uint32_t>, dim3(grid), dim3(GATHER_BLOCK), 0, s, d);
  else hipLaunchKernelGGL(k_gather<uint64_t>, dim3(grid), dim3(GATHER_BLOCK), 0, s, d);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  const uint32_t g2 = (uint32_t)n_cu * 4;
  if (d.w1 == 4) hipLaunchKernelGGL(k_p2_hist<uint32_t>, dim3(g2), dim3(P2_BLOCK), 0, s, d);
  else hipLaunchKernelGGL(k_p2_hist<uint64_t>, dim3(g2), dim3(P2_BLOCK), 0, s, d);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  e = xscan(d.hist2, d.ntmax * d.nb2, d.scan_tmp, d.g2, s, d.dscal + 1, d.nb2);   // live tiles only
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_fin, dim3((d.nb1 * d.nb2 + 256) / 256), dim3(256), 0, s, d);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  const size_t p2l = (size_t)d.nb2 * 8 + (size_t)(P2_BLOCK / 64) * d.nb2 * 4 + (size_t)(d.nb2 + (d.nb2 & 1)) * 4 +
                     (size_t)TILE * d.w2 + (size_t)TILE * 2;
  if (d.w1 == 4 && d.w2 == 4) hipLaunchKernelGGL((k_p2_scatter<uint32_t, uint32_t>), dim3(g2), dim3(P2_BLOCK), p2l, s, d);
  else if (d.w1 == 4) hipLaunchKernelGGL((k_p2_scatter<uint32_t, uint64_t>), dim3(g2), dim3(P2_BLOCK), p2l, s, d);
  else if (d.w2 == 4) hipLaunchKernelGGL((k_p2_scatter<uint64_t, uint32_t>), dim3(g2), dim3(P2_BLOCK), p2l, s, d);
  else hipLaunchKernelGGL((k_p2_scatter<uint64_t, uint64_t>), dim3(g2), dim3(P2_BLOCK), p2l, s, d);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  // segments of at most SEG records, cut at sequence boundaries, so that a hot bucket is shared out
  const uint32_t nf = d.nb1 * d.nb2;
  hipLaunchKernelGGL(k_nseg, dim3((nf + 255) / 256), dim3(256), 0, s, d);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  e = xscan(d.nseg, nf, d.scan_tmp, d.seg0, s);
  if (e != hipSuccess) return e;
  const bool nar = d.narrow != 0;
  const uint32_t wv = count_waves(d.low2, nar);
  const uint32_t gc = (uint32_t)n_cu * 2;
  const size_t lds = count_lds(d.low2, nar);
  if (d.w2 == 4) {
    if (nar) hipLaunchKernelGGL((k_count<uint32_t, 1>), dim3(gc), dim3(64 * wv), lds, s, d);
    else hipLaunchKernelGGL((k_count<uint32_t, 0>), dim3(gc), dim3(64 * wv), lds, s, d);
  } else {
    if (nar) hipLaunchKernelGGL((k_count<uint64_t, 1>), dim3(gc), dim3(64 * wv), lds, s, d);
    else hipLaunchKernelGGL((k_count<uint64_t, 0>), dim3(gc), dim3(64 * wv), lds, s, d);
  }
  return hipGetLastError();
}

hipError_t prepare_dedup(uint32_t low2) {
  const int l0 = (int)count_lds(low2, false), l1 = (int)count_lds(low2, true);
  const void *fns[4] = {reinterpret_cast<const void *>(k_count<uint32_t, 0>), reinterpret_cast<const void *>(k_count<uint64_t, 0>),
                        reinterpret_cast<const void *>(k_count<uint32_t, 1>), reinterpret_cast<const void *>(k_count<uint64_t, 1>)};
  hipError_t e = hipSuccess;
  for (int i = 0; i < 4 && e == hipSuccess; i++)
    e = hipFuncSetAttribute(fns[i], hipFuncAttributeMaxDynamicSharedMemorySize, i < 2 ? l0 : l1);
  // the level-2 scatter stages a tile: up to 1024 digits and 8-byte records need about 84 KB
  const void *p2[4] = {reinterpret_cast<const void *>(k_p2_scatter<uint32_t, uint32_t>),
                       reinterpret_cast<const void *>(k_p2_scatter<uint32_t, uint64_t>),
                       reinterpret_cast<const void *>(k_p2_scatter<uint64_t, uint32_t>),
                       reinterpret_cast<const void *>(k_p2_scatter<uint64_t, uint64_t>)};
  for (int i = 0; i < 4 && e == hipSuccess; i++)
    e = hipFuncSetAttribute(p2[i], hipFuncAttributeMaxDynamicSharedMemorySize, 96 * 1024);
  return e;
}

uint64_t dedup_scan_tmp_entries(uint64_t n) { return (n + SCAN_SEG - 1) / SCAN_SEG + 1; }

}  // namespace ig
