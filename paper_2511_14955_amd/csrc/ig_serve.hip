// Serving loop: continuous batching of featurize / count requests against the
// retained table (the featurization step of Figure 1, run as requests arrive).
//
// Memory.  At start the loop takes one device arena of max_inflight_bytes.
// Every launch carves one region of it (first fit, 256-byte aligned) for its
// inputs, per-sequence bitmaps and outputs, and gives it back when the launch
// has finished; nothing else is allocated on the device while serving, so the
// arena is the HBM budget of everything in flight.
//
// Scheduling.  A dispatcher thread owns n_streams launch slots (one stream,
// one completion event and pinned host staging each).  Submitted requests
// wait in a FIFO queue.  Whenever a slot is free, the dispatcher admits
// requests from the head of the queue while the region the batch needs still
// fits the largest free block of the arena (up to max_batch requests), packs
// them into one batch, and launches copy-in, featurize, row extraction,
// column counts and copy-out on the slot's stream.  Requests that arrive while
// batches run are admitted as soon as a slot and arena space free up; batches
// on different streams overlap on the device.  FIFO admission never lets a
// later request overtake an earlier one.  A request that could not fit even
// an empty arena completes at once with IG_ENOMEM.
#include <time.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <thread>
#include <vector>

#include "ig_internal.h"

namespace ig {

static inline uint64_t al256(uint64_t x) { return (x + 255) & ~255ull; }

// additive sizes of a batch; the device region is a function of them
struct Sums {
  uint64_t syms = 0, m = 0, nchunks = 0, out_cap = 0, ncount = 0;
  void add(const Sums &o) {
    syms += o.syms; m += o.m; nchunks += o.nchunks; out_cap += o.out_cap; ncount += o.ncount;
  }
};

struct Layout {
  uint64_t data, offs, ch, bm, nnz, ptr, ind, col, total, data_bytes;
};

static Layout layout_of(const Sums &s, uint32_t bits, uint64_t words) {
  Layout L{};
  uint64_t o = 0;
  L.data_bytes = (((s.syms * bits + 7) / 8 + 15) & ~15ull) + 64;   // staging reads run up to 16 bytes past the end
  L.data = o; o += al256(L.data_bytes);
  L.offs = o; o += al256((s.m + 1) * 8);
  L.ch = o;   o += al256(std::max<uint64_t>(1, s.nchunks) * sizeof(Chunk));
  L.bm = o;   o += al256(std::max<uint64_t>(1, s.m * words) * 4);
  L.nnz = o;  o += al256(std::max<uint64_t>(1, s.m) * 8);
  L.ptr = o;  o += al256((s.m + 1) * 8);
  L.ind = o;  o += al256(std::max<uint64_t>(1, s.out_cap) * 4);
  L.col = o;  o += al256(std::max<uint64_t>(1, s.ncount * words * 32) * 4);
  L.total = o;
  return L;
}

// first-fit allocator over the device arena, free blocks coalesced
struct Arena {
  uint64_t size = 0;
  std::map<uint64_t, uint64_t> free;   // offset -> length
  void reset(uint64_t n) { size = n; free.clear(); if (n) free[0] = n; }
  uint64_t largest() const {
    uint64_t b = 0;
    for (auto &kv : free) b = std::max(b, kv.second);
    return b;
  }
  bool alloc(uint64_t n, uint64_t *off) {
    for (auto it = free.begin(); it != free.end(); ++it)
      if (it->second >= n) {
        *off = it->first;
        const uint64_t rest = it->second - n, at = it->first + n;
        free.erase(it);
        if (rest) free[at] = rest;
        return true;
      }
    return false;
  }
  void release(uint64_t off, uint64_t n) {
    auto it = free.emplace(off, n).first;
    auto nx = std::next(it);
    if (nx != free.end() && it->first + it->second == nx->first) {
      it->second += nx->second;
      free.erase(nx);
    }
    if (it != free.begin()) {
      auto pv = std::prev(it);
      if (pv->first + pv->second == it->first) {
        pv->second += it->second;
        free.erase(it);
      }
    }
  }
};

struct SReq {
  uint64_t tag;
  int kind;
  double t_arrival;
  std::vector<uint8_t> data;    // packed symbols, as submitted
  std::vector<uint64_t> offs;   // m+1, relative to data
  Sums sz;
};

struct SRes {
  ig_result r;
  std::vector<int32_t> cols;
  std::vector<uint64_t> counts;
};

struct SSlot {
  hipStream_t stream = nullptr;
  hipEvent_t done = nullptr;
  bool busy = false;
  std::vector<SReq *> reqs;
  std::vector<uint64_t> file0;  // first batch sequence of each request, + total
  Sums sz;
  Layout lay{};
  uint64_t off = 0;             // region in the arena
  uint8_t *h = nullptr;         // pinned staging, grow only
  size_t h_cap = 0;
};

struct Server {
  ig_serve_config cfg;
  std::mutex mu;
  std::condition_variable cv;
  std::deque<SReq *> queue;
  std::deque<SRes *> done;
  std::vector<SSlot> slots;
  std::thread th;
  bool stop = false;
  uint64_t pending = 0;        // submitted, not yet completed
  uint64_t inflight = 0;       // arena bytes held by running batches
  uint64_t running = 0;        // launches running
  DevBuf arena_buf;
  Arena arena;
  ig_serve_stats st{};
};

static double now_s() {
  timespec ts;
  clock_gettime(CLOCK_MONOTONIC, &ts);
  return (double)ts.tv_sec + 1e-9 * (double)ts.tv_nsec;
}

// exclusive scan of nnz (m values) into indptr (m+1), one workgroup
__global__ void __launch_bounds__(1024) k_batch_scan(const uint64_t *nnz, uint64_t m, uint64_t *indptr) {
  __shared__ uint64_t s[1024];
  const uint32_t t = threadIdx.x;
  const uint64_t per = (m + 1023) / 1024, lo = t * per, hi = lo + per < m ? lo + per : m;
  uint64_t acc = 0;
  for (uint64_t i = lo; i < hi; i++) acc += nnz[i];
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
    indptr[i] = run;
    run += nnz[i];
  }
  if (t == 1023) indptr[m] = s[1023];
}

// pinned staging of a batch: copy-in (data, offsets, chunks), then copy-out
// (indptr, indices, column counts) mirroring the device region's tail
struct HostLayout {
  uint64_t offs, ch, out, total;
};

static HostLayout host_layout(const Layout &L, const Sums &s) {
  HostLayout H{};
  H.offs = al256(L.data_bytes);
  H.ch = H.offs + al256((s.m + 1) * 8);
  H.out = H.ch + al256(std::max<uint64_t>(1, s.nchunks) * sizeof(Chunk));
  H.total = H.out + (L.total - L.ptr);
  return H;
}

// pack and launch one batch on its slot (dispatcher thread)
static int launch_batch(ig_ctx *c, Server *sv, SSlot &sl) {
  hipStream_t s = sl.stream;
  const uint64_t words = (c->kept + 31) / 32;
  const uint32_t b = c->cfg.symbol_bits;
  const Layout &L = sl.lay;
  const uint64_t m = sl.sz.m;
  const HostLayout H = host_layout(L, sl.sz);
  if (sl.h_cap < H.total) {
    if (sl.h) (void)hipHostFree(sl.h);
    sl.h = nullptr;
    sl.h_cap = 0;
    const size_t want = H.total + H.total / 4 + 4096;
    if (hipHostMalloc(reinterpret_cast<void **>(&sl.h), want, hipHostMallocDefault) != hipSuccess) {
      (void)hipGetLastError();
      sl.h = nullptr;
      return IG_ENOMEM;
    }
    sl.h_cap = want;
  }
  uint8_t *h_data = sl.h;
  uint64_t *h_offs = reinterpret_cast<uint64_t *>(sl.h + H.offs);
  Chunk *h_ch = reinterpret_cast<Chunk *>(sl.h + H.ch);
  uint8_t *h_out = sl.h + H.out;

  // the batch: the requests' sequences one after the other, featurize
  // requests first so that their rows are the first m_feat of the batch
  std::stable_partition(sl.reqs.begin(), sl.reqs.end(), [](const SReq *r) { return r->kind == IG_REQ_FEATURIZE; });
  uint64_t m_feat = 0;
  for (SReq *r : sl.reqs)
    if (r->kind == IG_REQ_FEATURIZE) m_feat += r->offs.size() - 1;
  std::memset(h_data, 0, L.data_bytes);
  const uint64_t CH = c->lc.chunk_syms;
  uint64_t f = 0, g = 0, nch = 0;
  h_offs[0] = 0;
  sl.file0.clear();
  for (SReq *r : sl.reqs) {
    sl.file0.push_back(f);
    const uint64_t base = g, syms = r->offs.back();
    if (b == 8) {
      if (syms) std::memcpy(h_data + base, r->data.data(), syms);
    } else {
      for (uint64_t i = 0; i < syms; i++) {
        const uint32_t v = (r->data[i >> 2] >> (6 - 2 * (i & 3))) & 3u;
        const uint64_t q = base + i;
        h_data[q >> 2] |= (uint8_t)(v << (6 - 2 * (q & 3)));
      }
    }
    for (size_t i = 0; i + 1 < r->offs.size(); i++, f++) {
      const uint64_t a = base + r->offs[i], len = r->offs[i + 1] - r->offs[i];
      h_offs[f + 1] = base + r->offs[i + 1];
      for (uint64_t q = 0; q < len; q += CH)
        h_ch[nch++] = Chunk{a + q, (uint32_t)f, (uint32_t)std::min<uint64_t>(CH, len - q), len > CH ? 1u : 0u, 0u};
    }
    g += syms;
  }
  sl.file0.push_back(f);

  uint8_t *dev = reinterpret_cast<uint8_t *>(sv->arena_buf.p) + sl.off;
  uint32_t *d_bm = reinterpret_cast<uint32_t *>(dev + L.bm);
  uint64_t *d_nnz = reinterpret_cast<uint64_t *>(dev + L.nnz);
  uint64_t *d_ptr = reinterpret_cast<uint64_t *>(dev + L.ptr);
  int32_t *d_ind = reinterpret_cast<int32_t *>(dev + L.ind);
  uint32_t *d_col = reinterpret_cast<uint32_t *>(dev + L.col);

  hipError_t e = hipMemcpyAsync(dev + L.data, h_data, L.data_bytes, hipMemcpyHostToDevice, s);
  if (e == hipSuccess) e = hipMemcpyAsync(dev + L.offs, h_offs, (m + 1) * 8, hipMemcpyHostToDevice, s);
  if (e == hipSuccess && nch) e = hipMemcpyAsync(dev + L.ch, h_ch, nch * sizeof(Chunk), hipMemcpyHostToDevice, s);
  if (e == hipSuccess && m * words) e = launch_fill_u32(d_bm, m * words, 0, s);
  FeatBatch fb{dev + L.data, reinterpret_cast<const uint64_t *>(dev + L.offs), m,
               reinterpret_cast<const Chunk *>(dev + L.ch), (uint32_t)nch, d_bm, (uint32_t)words};
  if (e == hipSuccess && words && m) e = launch_featurize(c, fb, s);
  // sparse rows of the featurize sequences: count, scan, write
  if (e == hipSuccess && m_feat) {
    if (words) e = launch_rows(d_bm, m_feat, (uint32_t)words, d_nnz, nullptr, nullptr, 0, 1, s);
    else e = launch_fill_u64(d_nnz, m_feat, 0, s);
    if (e == hipSuccess) {
      hipLaunchKernelGGL(k_batch_scan, dim3(1), dim3(1024), 0, s, d_nnz, m_feat, d_ptr);
      e = hipGetLastError();
    }
    if (e == hipSuccess && words && sl.sz.out_cap)
      e = launch_rows(d_bm, m_feat, (uint32_t)words, nullptr, d_ptr, d_ind, sl.sz.out_cap, 0, s);
  }
  // column counts of each count request over its own sequences
  uint64_t ci = 0;
  for (size_t q = 0; q < sl.reqs.size() && e == hipSuccess; q++) {
    if (sl.reqs[q]->kind != IG_REQ_COUNT) continue;
    uint32_t *col = d_col + ci * words * 32;
    if (words) {
      e = launch_fill_u32(col, words * 32, 0, s);
      if (e == hipSuccess)
        e = launch_col_counts(d_bm + sl.file0[q] * words, sl.file0[q + 1] - sl.file0[q], (uint32_t)words,
                              (uint32_t)c->kept, col, s);
    }
    ci++;
  }
  if (e == hipSuccess && m_feat) e = hipMemcpyAsync(h_out, d_ptr, (m_feat + 1) * 8, hipMemcpyDeviceToHost, s);
  if (e == hipSuccess && sl.sz.out_cap)
    e = hipMemcpyAsync(h_out + (L.ind - L.ptr), d_ind, sl.sz.out_cap * 4, hipMemcpyDeviceToHost, s);
  if (e == hipSuccess && ci && words)
    e = hipMemcpyAsync(h_out + (L.col - L.ptr), d_col, ci * words * 32 * 4, hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipEventRecord(sl.done, s);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    (void)hipStreamSynchronize(s);
    return IG_EDEVICE;
  }
  return IG_OK;
}

// turn a finished (or failed) slot into results; no lock held
static void collect(ig_ctx *c, SSlot &sl, int status, std::vector<SRes *> &out) {
  const uint64_t kept = c->kept, words = (kept + 31) / 32;
  const Layout &L = sl.lay;
  const uint8_t *h_out = status == IG_OK ? sl.h + host_layout(L, sl.sz).out : nullptr;
  const uint64_t *h_ptr = reinterpret_cast<const uint64_t *>(h_out);
  const int32_t *h_ind = reinterpret_cast<const int32_t *>(h_out + (L.ind - L.ptr));
  const uint32_t *h_col = reinterpret_cast<const uint32_t *>(h_out + (L.col - L.ptr));
  const double t = now_s();
  uint64_t ci = 0;
  for (size_t q = 0; q < sl.reqs.size(); q++) {
    SReq *r = sl.reqs[q];
    SRes *res = new SRes();
    res->r.tag = r->tag;
    res->r.kind = r->kind;
    res->r.status = status;
    res->r.t_arrival = r->t_arrival;
    if (status == IG_OK) {
      if (r->kind == IG_REQ_FEATURIZE) {
        if (words) res->cols.assign(h_ind + h_ptr[sl.file0[q]], h_ind + h_ptr[sl.file0[q + 1]]);
      } else {
        if (words) {
          const uint32_t *col = h_col + ci * words * 32;
          for (uint64_t j = 0; j < kept; j++)
            if (col[j]) {
              res->cols.push_back((int32_t)j);
              res->counts.push_back(col[j]);
            }
        }
        ci++;
      }
    }
    res->r.n = res->cols.size();
    res->r.t_done = t;
    out.push_back(res);
    delete r;
  }
  sl.reqs.clear();
}

static void complete(Server *sv, SSlot &sl, std::vector<SRes *> &fin) {
  std::lock_guard<std::mutex> lk(sv->mu);
  for (SRes *r : fin) sv->done.push_back(r);
  sv->st.completed += fin.size();
  sv->pending -= fin.size();
  sv->arena.release(sl.off, sl.lay.total);
  sv->inflight -= sl.lay.total;
  sv->running--;
  sl.busy = false;
  sv->cv.notify_all();
}

static void dispatcher(ig_ctx *c, Server *sv) {
  (void)hipSetDevice(c->cfg.device);
  const uint64_t words = (c->kept + 31) / 32;
  const uint32_t bits = c->cfg.symbol_bits;
  std::vector<SRes *> fin;
  for (;;) {
    // finished launches
    bool any_busy = false;
    for (SSlot &sl : sv->slots) {
      if (!sl.busy) continue;
      const hipError_t q = hipEventQuery(sl.done);
      if (q == hipErrorNotReady) { any_busy = true; continue; }
      if (q != hipSuccess) (void)hipGetLastError();
      fin.clear();
      collect(c, sl, q == hipSuccess ? IG_OK : IG_EDEVICE, fin);
      complete(sv, sl, fin);
    }
    SSlot *slot = nullptr;
    for (SSlot &sl : sv->slots)
      if (!sl.busy) { slot = &sl; break; }
    {
      std::unique_lock<std::mutex> lk(sv->mu);
      if (sv->stop && sv->queue.empty() && !any_busy) break;
      if (slot) {
        // admission: FIFO while the batch's region fits the largest free block
        const uint64_t room = sv->arena.largest();
        Sums acc;
        while (!sv->queue.empty() && slot->reqs.size() < sv->cfg.max_batch) {
          SReq *r = sv->queue.front();
          if (layout_of(r->sz, bits, words).total > sv->arena.size) {
            sv->queue.pop_front();
            SRes *res = new SRes();
            res->r.tag = r->tag;
            res->r.kind = r->kind;
            res->r.status = IG_ENOMEM;
            res->r.t_arrival = r->t_arrival;
            res->r.t_done = now_s();
            sv->done.push_back(res);
            sv->st.rejected++;
            sv->st.completed++;
            sv->pending--;
            delete r;
            continue;
          }
          Sums t = acc;
          t.add(r->sz);
          if (layout_of(t, bits, words).total > room) break;
          acc = t;
          sv->queue.pop_front();
          slot->reqs.push_back(r);
        }
        if (!slot->reqs.empty()) {
          slot->sz = acc;
          slot->lay = layout_of(acc, bits, words);
          // the region fits the largest free block, so first fit finds it
          (void)sv->arena.alloc(slot->lay.total, &slot->off);
          sv->inflight += slot->lay.total;
          sv->running++;
          sv->st.peak_inflight_bytes = std::max(sv->st.peak_inflight_bytes, sv->inflight);
          sv->st.peak_running = std::max(sv->st.peak_running, sv->running);
          sv->st.launches++;
          for (SReq *r : slot->reqs) sv->st.bytes_in += r->data.size();
        }
      }
      if (!slot || slot->reqs.empty()) {
        // nothing to launch now: wait for a submission, or look at running launches again shortly
        sv->cv.wait_for(lk, std::chrono::microseconds(any_busy ? 20 : 1000));
        continue;
      }
    }
    slot->busy = true;
    const int rc = launch_batch(c, sv, *slot);
    if (rc != IG_OK) {
      fin.clear();
      collect(c, *slot, rc, fin);
      complete(sv, *slot, fin);
    }
  }
}

void serve_teardown(ig_ctx *c) {
  if (!c || !c->server) return;
  Server *sv = reinterpret_cast<Server *>(c->server);
  {
    std::lock_guard<std::mutex> lk(sv->mu);
    sv->stop = true;
  }
  sv->cv.notify_all();
  if (sv->th.joinable()) sv->th.join();
  for (SSlot &sl : sv->slots) {
    if (sl.stream) (void)hipStreamSynchronize(sl.stream);
    if (sl.h) (void)hipHostFree(sl.h);
    if (sl.done) (void)hipEventDestroy(sl.done);
    if (sl.stream) (void)hipStreamDestroy(sl.stream);
  }
  dev_release(c, sv->arena_buf);
  for (SReq *r : sv->queue) delete r;
  for (SRes *r : sv->done) delete r;
  delete sv;
  c->server = nullptr;
}

}  // namespace ig

using namespace ig;

extern "C" {

double ig_serve_now(void) { return now_s(); }

int ig_serve_start(ig_ctx *c, const ig_serve_config *scfg) {
  if (!c || !scfg) return IG_EINVAL;
  if (c->sticky) return set_error(c, IG_EDEVICE, "context has a sticky device error: %s", c->err.c_str());
  if (c->server) return set_error(c, IG_ESTATE, "serving loop already running");
  if (c->fresh || !c->loaded) return set_error(c, IG_ESTATE, "no retained table to serve");
  if (scfg->n_streams < 1 || scfg->n_streams > 8 || scfg->max_batch < 1 || scfg->max_inflight_bytes < 65536 ||
      scfg->queue_capacity == 0)
    return set_error(c, IG_EINVAL, "bad serving configuration");
  if (check_hip(c, hipStreamSynchronize(c->stream), "serve start sync")) return IG_EDEVICE;
  Server *sv = new Server();
  sv->cfg = *scfg;
  c->server = sv;
  const uint64_t asz = scfg->max_inflight_bytes & ~255ull;
  if (int rc = dev_reserve(c, sv->arena_buf, asz)) {
    serve_teardown(c);
    return rc;
  }
  sv->arena.reset(asz);
  sv->slots.resize(scfg->n_streams);
  for (SSlot &sl : sv->slots) {
    // default-priority, non-blocking streams
    if (hipStreamCreateWithFlags(&sl.stream, hipStreamNonBlocking) != hipSuccess ||
        hipEventCreateWithFlags(&sl.done, hipEventDisableTiming) != hipSuccess) {
      (void)hipGetLastError();
      serve_teardown(c);
      return set_error(c, IG_EDEVICE, "could not create serving streams");
    }
  }
  sv->th = std::thread(dispatcher, c, sv);
  return IG_OK;
}

int ig_submit(ig_ctx *c, int kind, const void *data, uint64_t data_bytes, const uint64_t *sym_offsets, uint64_t m,
              uint64_t tag, double t_arrival) {
  if (!c) return IG_EINVAL;
  Server *sv = reinterpret_cast<Server *>(c->server);
  if (!sv) return IG_ESTATE;
  if ((kind != IG_REQ_FEATURIZE && kind != IG_REQ_COUNT) || !sym_offsets || sym_offsets[0] != 0 || m == 0 ||
      (kind == IG_REQ_FEATURIZE && m != 1) || m >= 0xFFFFFFFFull)
    return IG_EINVAL;
  for (uint64_t i = 0; i < m; i++)
    if (sym_offsets[i + 1] < sym_offsets[i]) return IG_EINVAL;
  const uint32_t b = c->cfg.symbol_bits;
  const uint64_t need = (sym_offsets[m] * b + 7) / 8;
  if (data_bytes < need || (need && !data)) return IG_EINVAL;
  SReq *r = new SReq();
  r->tag = tag;
  r->kind = kind;
  r->t_arrival = t_arrival;
  if (need) r->data.assign(reinterpret_cast<const uint8_t *>(data), reinterpret_cast<const uint8_t *>(data) + need);
  r->offs.assign(sym_offsets, sym_offsets + m + 1);
  const uint64_t CH = c->lc.chunk_syms;
  const uint32_t n = c->n_prev;
  uint64_t cap = 0;
  r->sz.syms = sym_offsets[m];
  r->sz.m = m;
  for (uint64_t i = 0; i < m; i++) {
    const uint64_t len = sym_offsets[i + 1] - sym_offsets[i];
    r->sz.nchunks += (len + CH - 1) / CH;
    if (len >= n) cap += std::min<uint64_t>(c->kept, len - n + 1);
  }
  r->sz.out_cap = kind == IG_REQ_FEATURIZE ? cap : 0;
  r->sz.ncount = kind == IG_REQ_COUNT ? 1 : 0;
  std::lock_guard<std::mutex> lk(sv->mu);
  if (sv->stop || sv->pending >= sv->cfg.queue_capacity) {
    delete r;
    return IG_EBUSY;
  }
  sv->queue.push_back(r);
  sv->pending++;
  sv->st.submitted++;
  sv->cv.notify_all();
  return IG_OK;
}

int ig_poll(ig_ctx *c, ig_result *res, uint64_t max, int32_t *cols, uint64_t *counts, uint64_t cap, uint64_t *out_off,
            uint64_t *n_out) {
  if (!c || !n_out || (max && !res)) return IG_EINVAL;
  *n_out = 0;
  Server *sv = reinterpret_cast<Server *>(c->server);
  if (!sv) return IG_ESTATE;
  std::lock_guard<std::mutex> lk(sv->mu);
  uint64_t used = 0, k = 0;
  if (out_off) out_off[0] = 0;
  while (k < max && !sv->done.empty()) {
    SRes *r = sv->done.front();
    const uint64_t nn = r->cols.size();
    if (used + nn > cap || (nn && !cols)) {
      if (k == 0) {
        res[0] = r->r;   // tells the caller how much room the oldest result needs
        return IG_ETRUNC;
      }
      break;
    }
    if (nn) {
      std::memcpy(cols + used, r->cols.data(), nn * 4);
      if (counts && r->counts.size() == nn) std::memcpy(counts + used, r->counts.data(), nn * 8);
    }
    res[k] = r->r;
    used += nn;
    k++;
    if (out_off) out_off[k] = used;
    sv->done.pop_front();
    delete r;
  }
  *n_out = k;
  return IG_OK;
}

int ig_serve_stop(ig_ctx *c) {
  if (!c) return IG_EINVAL;
  if (!c->server) return IG_ESTATE;
  serve_teardown(c);
  return IG_OK;
}

int ig_serve_get_stats(ig_ctx *c, ig_serve_stats *st) {
  if (!c || !st) return IG_EINVAL;
  Server *sv = reinterpret_cast<Server *>(c->server);
  if (!sv) return IG_ESTATE;
  std::lock_guard<std::mutex> lk(sv->mu);
  *st = sv->st;
  return IG_OK;
}

}  // extern "C"
