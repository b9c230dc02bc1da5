// Autotuner for the scan's launch shape: chunk length (symbols per work item),
// workgroup size, and the LDS de-duplication set.  Each candidate runs the
// real pass on the loaded corpus (then the chain is rewound); the fastest
// device pass wins.  Every candidate must return the same table, which the
// tuner checks.  Results can be cached in the file named by IG_TUNE_CACHE,
// keyed by device, corpus shape and pass.
#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>
#include <vector>

#include "ig_internal.h"

using namespace ig;

static std::string tune_key(ig_ctx *c, uint32_t n, uint64_t k_keep) {
  hipDeviceProp_t prop{};
  (void)hipGetDeviceProperties(&prop, c->cfg.device);
  char buf[512];
  snprintf(buf, sizeof buf, "%s|cu%d|b%u|f%d|m%llu|s%llu|n%u|k%llu", prop.gcnArchName, c->n_cu, c->cfg.symbol_bits,
           (int)c->cfg.freq, (unsigned long long)c->m, (unsigned long long)c->total_syms, n, (unsigned long long)k_keep);
  for (char *q = buf; *q; q++)
    if (*q == ' ') *q = '_';
  return buf;
}

// A launch shape the scan supports: whole wavefronts per workgroup, a power-of-two LDS set of at
// least one slot per thread (the set's hashing and its flush assume both), chunk length in range.
static bool shape_ok(uint32_t chunk_syms, uint32_t block, uint32_t set_cap, uint32_t wg_per_cu) {
  return chunk_syms >= 1024 && chunk_syms <= 65536 && (block == 256 || block == 512 || block == 1024) &&
         set_cap >= 1024 && set_cap <= 32768 && (set_cap & (set_cap - 1)) == 0 && set_cap >= block &&
         (wg_per_cu == 1 || wg_per_cu == 2);
}

// The last line for `key` whose shape is valid (a stale or edited line is ignored).
static bool cache_lookup(const std::string &key, LaunchCfg *lc) {
  const char *path = getenv("IG_TUNE_CACHE");
  if (!path) return false;
  FILE *f = fopen(path, "r");
  if (!f) return false;
  char line[1024];
  bool found = false;
  while (fgets(line, sizeof line, f)) {
    char k[600];
    unsigned cs, bl, sc, wp, ml, fw;
    if (sscanf(line, "%599s %u %u %u %u %u %u", k, &cs, &bl, &sc, &wp, &ml, &fw) == 7 && key == k &&
        shape_ok(cs, bl, sc, wp) && ml >= 1 && ml <= 3 && fw >= 1024 && fw <= 16384 && (fw & (fw - 1)) == 0) {
      lc->chunk_syms = cs;
      lc->block = bl;
      lc->set_cap = sc;
      lc->grid_per_cu = wp;
      lc->map_log2 = ml;
      lc->filt_max_words = fw;
      found = true;
    }
  }
  fclose(f);
  return found;
}

static void cache_store(const std::string &key, const LaunchCfg &lc) {
  const char *path = getenv("IG_TUNE_CACHE");
  if (!path) return;
  FILE *f = fopen(path, "a");
  if (!f) return;
  fprintf(f, "%s %u %u %u %u %u %u\n", key.c_str(), lc.chunk_syms, lc.block, lc.set_cap, lc.grid_per_cu, lc.map_log2,
          lc.filt_max_words);
  fclose(f);
}

extern "C" int ig_autotune(ig_ctx *c, uint32_t n, uint64_t k_keep, ig_tune_report *rep) {
  if (!c) return IG_EINVAL;
  if (c->sticky) return set_error(c, IG_EDEVICE, "context has a sticky device error: %s", c->err.c_str());
  if (c->server) return set_error(c, IG_ESTATE, "serving loop is running");
  if (!c->loaded) return set_error(c, IG_ESTATE, "no corpus loaded");
  if (rep) std::memset(rep, 0, sizeof *rep);
  const std::string key = tune_key(c, n, k_keep);
  const LaunchCfg start = c->lc;
  LaunchCfg cached = start;
  if (cache_lookup(key, &cached)) {
    c->lc = cached;
    if (cached.chunk_syms != start.chunk_syms) {
      int rc = rebuild_chunks(c);
      if (rc) return rc;
    }
    if (cached.map_log2 != start.map_log2 || cached.filt_max_words != start.filt_max_words) {
      int rc = reindex_current(c);
      if (rc) return rc;
    }
    if (rep) {
      rep->n_candidates = 1;
      rep->cand[0].chunk_syms = cached.chunk_syms;
      rep->cand[0].block = cached.block;
      rep->cand[0].set_cap = cached.set_cap;
      rep->cand[0].wg_per_cu = cached.grid_per_cu;
      rep->cand[0].map_slots_log2 = cached.map_log2;
      rep->cand[0].filter_max_words = cached.filt_max_words;
      rep->cand[0].pass_ms = -1.0;
      rep->best = 0;
      rep->identical = 1;
      rep->from_cache = 1;
    }
    return IG_OK;
  }
  // Chunk lengths are multiples of 1024 symbols (per-thread window runs of chunk / 1024, made
  // odd); 512-thread blocks are kept as a fallback for small corpora, and the largest LDS set
  // only with the shorter chunks.  Shapes that do not fit the pass's LDS are skipped.
  std::vector<LaunchCfg> cands;
  for (uint32_t cs : {15360u, 16384u, 19456u, 23552u, 27648u, 31744u})
    for (uint32_t bl : {512u, 1024u})
      for (uint32_t sc : {4096u, 8192u, 16384u}) {
        if (bl == 512 && cs > 16384) continue;
        if (sc == 16384 && cs > 16384) continue;
        LaunchCfg lc = start;
        lc.chunk_syms = cs;
        lc.block = bl;
        lc.set_cap = sc;
        cands.push_back(lc);
      }
  std::vector<uint64_t> ref_lo, ref_hi, ref_cnt;
  std::vector<ig_key> keys;
  std::vector<uint64_t> counts;
  int identical = 1;
  bool have_ref = false;
  uint32_t cur_chunk = c->lc.chunk_syms;
  uint32_t nrep = 0;
  // Run pass n (twice, keeping the faster) with launch shape `lc` and compare its table with the
  // first candidate's.  Returns the pass time, -1 when the shape does not fit the pass, or
  // -2 - rc on another error.
  auto trial = [&](const LaunchCfg &lc) -> double {
    const bool retable = lc.map_log2 != c->lc.map_log2 || lc.filt_max_words != c->lc.filt_max_words;
    c->lc = lc;
    if (lc.chunk_syms != cur_chunk) {
      int rc = rebuild_chunks(c);
      if (rc) return -2.0 + rc;
      cur_chunk = lc.chunk_syms;
    }
    if (retable) {
      int rc = reindex_current(c);
      if (rc) return -2.0 + rc;
    }
    double ms = 1e30;
    for (int rep_i = 0; rep_i < 2; rep_i++) {
      int rc = ig_pass(c, n, k_keep);
      if (rc == IG_EINVAL) return -1.0;   // launch shape does not fit this pass
      if (rc) return -2.0 + rc;
      if (c->last.set_cap < lc.set_cap) {   // ran only with a smaller LDS set: unusable here
        rc = ig_rewind(c);
        return rc ? -2.0 + rc : -1.0;
      }
      ms = std::min(ms, c->last.pass_ms);
      if (rep_i == 0) {
        const uint64_t kept = c->kept;
        keys.resize(kept ? kept : 1);
        counts.resize(kept ? kept : 1);
        uint64_t got = 0;
        rc = ig_topk(c, kept, keys.data(), counts.data(), &got);
        if (rc) return -2.0 + rc;
        if (!have_ref) {
          have_ref = true;
          for (uint64_t j = 0; j < got; j++) {
            ref_lo.push_back(keys[j].lo);
            ref_hi.push_back(keys[j].hi);
            ref_cnt.push_back(counts[j]);
          }
        } else {
          bool same = got == ref_cnt.size();
          for (uint64_t j = 0; same && j < got; j++)
            same = keys[j].lo == ref_lo[j] && keys[j].hi == ref_hi[j] && counts[j] == ref_cnt[j];
          if (!same) identical = 0;
        }
      }
      rc = ig_rewind(c);
      if (rc) return -2.0 + rc;
    }
    return ms;
  };
  auto record = [&](const LaunchCfg &lc, double ms) {
    if (!rep || nrep >= IG_TUNE_MAX) { nrep++; return; }
    rep->cand[nrep].chunk_syms = lc.chunk_syms;
    rep->cand[nrep].block = lc.block;
    rep->cand[nrep].set_cap = lc.set_cap;
    rep->cand[nrep].wg_per_cu = lc.grid_per_cu;
    rep->cand[nrep].map_slots_log2 = lc.map_log2;
    rep->cand[nrep].filter_max_words = lc.filt_max_words;
    rep->cand[nrep].pass_ms = ms;
    rep->n_candidates = ++nrep;
  };
  auto restore = [&](int code, const char *msg) {
    const LaunchCfg now = c->lc;
    c->lc = start;
    if (cur_chunk != start.chunk_syms) (void)rebuild_chunks(c);
    if (now.map_log2 != start.map_log2 || now.filt_max_words != start.filt_max_words) (void)reindex_current(c);
    return msg ? set_error(c, code, "%s", msg) : code;
  };
  // stage 1: the launch shape, with the starting table sizes
  int best = -1;
  uint32_t win_idx = 0;   // the winner's entry in the report
  double best_ms = 1e30;
  for (size_t i = 0; i < cands.size(); i++) {
    const double ms = trial(cands[i]);
    if (ms <= -2.0) return restore((int)(ms + 2.0), nullptr);
    record(cands[i], ms);
    if (ms >= 0 && ms < best_ms) {
      best_ms = ms;
      best = (int)i;
      win_idx = nrep - 1;
    }
  }
  if (best < 0) return restore(IG_EINVAL, "no launch shape fits this pass");
  // stage 2: the table sizes (map load, filter image) with that launch shape
  LaunchCfg win = cands[best];
  for (uint32_t ml : {1u, 2u})
    for (uint32_t fw : {8192u, 16384u}) {
      LaunchCfg lc = cands[best];
      lc.map_log2 = ml;
      lc.filt_max_words = fw;
      if (ml == start.map_log2 && fw == start.filt_max_words) continue;   // measured in stage 1
      const double ms = trial(lc);
      if (ms <= -2.0) return restore((int)(ms + 2.0), nullptr);
      record(lc, ms);
      if (ms >= 0 && ms < best_ms) {
        best_ms = ms;
        win = lc;
        win_idx = nrep - 1;
      }
    }
  // stage 3: two workgroups per CU, which needs a workgroup's LDS to fit half a CU: the Bloom
  // image in L2 (an LDS cap of 1024 words sends it there) and a smaller LDS set, with shorter
  // chunks or the winner's, and 512- or 1024-thread workgroups (512 threads give each thread a
  // run twice as long: passes that read the Bloom image in L2 for every window run faster so)
  const uint32_t win_cs = win.chunk_syms, win_ml = win.map_log2;
  const uint32_t s3_chunks[3] = {12288u, 16384u, win_cs};
  const int n3 = (win_cs == 12288u || win_cs == 16384u) ? 2 : 3;
  for (int ci = 0; ci < n3; ci++)
    for (uint32_t bl : {512u, 1024u}) {
      const uint32_t cs = s3_chunks[ci];
      LaunchCfg lc = win;
      lc.chunk_syms = cs;
      lc.block = bl;
      lc.set_cap = 4096;
      lc.grid_per_cu = 2;
      lc.map_log2 = win_ml;
      lc.filt_max_words = 1024;
      const double ms = trial(lc);
      if (ms <= -2.0) return restore((int)(ms + 2.0), nullptr);
      record(lc, ms);
      if (ms >= 0 && ms < best_ms) {
        best_ms = ms;
        win = lc;
        win_idx = nrep - 1;
      }
    }
  // the winner's chunks and index
  {
    const LaunchCfg now = c->lc;
    c->lc = win;
    if (win.chunk_syms != cur_chunk) {
      int rc = rebuild_chunks(c);
      if (rc) return rc;
    }
    if (win.map_log2 != now.map_log2 || win.filt_max_words != now.filt_max_words) {
      int rc = reindex_current(c);
      if (rc) return rc;
    }
  }
  if (rep) rep->best = win_idx;
  if (rep) rep->identical = identical;
  if (!identical) return set_error(c, IG_EDEVICE, "launch shapes gave different tables");
  cache_store(key, c->lc);
  return IG_OK;
}

extern "C" int ig_get_launch(const ig_ctx *c, uint32_t *chunk_syms, uint32_t *block, uint32_t *set_cap,
                             uint32_t *wg_per_cu) {
  if (!c) return IG_EINVAL;
  if (chunk_syms) *chunk_syms = c->lc.chunk_syms;
  if (block) *block = c->lc.block;
  if (set_cap) *set_cap = c->lc.set_cap;
  if (wg_per_cu) *wg_per_cu = c->lc.grid_per_cu;
  return IG_OK;
}

extern "C" int ig_set_launch(ig_ctx *c, uint32_t chunk_syms, uint32_t block, uint32_t set_cap, uint32_t wg_per_cu) {
  if (!c) return IG_EINVAL;
  if (c->server) return set_error(c, IG_ESTATE, "serving loop is running");
  if (!shape_ok(chunk_syms, block, set_cap, wg_per_cu)) return set_error(c, IG_EINVAL, "bad launch shape");
  c->lc.grid_per_cu = wg_per_cu;
  const bool rechunk = chunk_syms != c->lc.chunk_syms;
  c->lc.chunk_syms = chunk_syms;
  c->lc.block = block;
  c->lc.set_cap = set_cap;
  if (rechunk && c->loaded) return rebuild_chunks(c);
  return IG_OK;
}

static bool tables_ok(const ig_table_shape &t) {
  return t.map_slots_log2 >= 1 && t.map_slots_log2 <= 3 && t.filter_bits_per_key >= 4 && t.filter_bits_per_key <= 32 &&
         t.filter_max_words >= 1024 && t.filter_max_words <= 16384 && (t.filter_max_words & (t.filter_max_words - 1)) == 0 &&
         (t.sparse_slots == 0 || (t.sparse_slots >= 1024 && t.sparse_slots <= (1ull << 31) &&
                                  (t.sparse_slots & (t.sparse_slots - 1)) == 0));
}

extern "C" int ig_get_tables(const ig_ctx *c, ig_table_shape *t) {
  if (!c || !t) return IG_EINVAL;
  std::memset(t, 0, sizeof *t);
  t->map_slots_log2 = c->lc.map_log2;
  t->filter_bits_per_key = c->lc.bloom_bits;
  t->filter_max_words = c->lc.filt_max_words;
  t->sparse_slots = c->tkey_slots;
  t->record_capacity = c->rec_cap;
  return IG_OK;
}

extern "C" int ig_set_tables(ig_ctx *c, const ig_table_shape *t) {
  if (!c || !t) return IG_EINVAL;
  if (c->sticky) return set_error(c, IG_EDEVICE, "context has a sticky device error: %s", c->err.c_str());
  if (c->server) return set_error(c, IG_ESTATE, "serving loop is running");
  if (!tables_ok(*t)) return set_error(c, IG_EINVAL, "bad table shape");
  if (hipSetDevice(c->cfg.device) != hipSuccess) return set_error(c, IG_EDEVICE, "hipSetDevice");
  const bool reindex = t->map_slots_log2 != c->lc.map_log2 || t->filter_bits_per_key != c->lc.bloom_bits ||
                       t->filter_max_words != c->lc.filt_max_words;
  c->lc.map_log2 = t->map_slots_log2;
  c->lc.bloom_bits = t->filter_bits_per_key;
  c->lc.filt_max_words = t->filter_max_words;
  if (t->sparse_slots) c->tkey_slots = t->sparse_slots;
  if (t->record_capacity) {
    const uint64_t T = dedup_tile();
    c->rec_cap = (t->record_capacity + T - 1) / T * T;
    c->rec_floor = true;
  }
  return reindex ? reindex_current(c) : IG_OK;
}
